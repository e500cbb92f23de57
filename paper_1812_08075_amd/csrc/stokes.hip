// DG Stokes operator (placeholder until the kernel lands).
#include "internal.h"

namespace dgi {
void stokes_setup(dg_mesh&) {}
hipError_t stokes_apply(const dg_mesh&, const double*, double*, hipStream_t) { return hipErrorNotSupported; }
}  // namespace dgi
