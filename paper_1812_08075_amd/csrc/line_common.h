// Device-side helpers shared by the line-structured kernels of the axis-aligned
// diffusion-reaction operators: the padded LDS layout of a cell block, the
// decoding of a block's chunk from the sweep table, and reads and writes of
// the 1D lines of a cell in each direction.
#pragma once

#include "internal.h"

namespace dgi {

// LDS layout of one cell block: node (i0, i1, i2) at i0 + S1 i1 + S2 i2,
// cells NP apart. Padded strides break the power-of-two bank patterns of the
// three line directions.
template <int P>
struct Layout {
  static constexpr int S1 = P, S2 = P * P, NP = P * P * P;
};
template <>
struct Layout<4> {
  static constexpr int S1 = 4, S2 = 19, NP = 76;
};
template <>
struct Layout<6> {
  static constexpr int S1 = 6, S2 = 39, NP = 244;
};
template <>
struct Layout<7> {
  static constexpr int S1 = 7, S2 = 52, NP = 369;
};
template <>
struct Layout<8> {
  static constexpr int S1 = 9, S2 = 72, NP = 576;
};

struct BlockCoord {
  int ex0, ey, ez;  // x index of the chunk's first cell, y and z of its row
};

// Coordinates of this hardware block's chunk (table built on the host: sweep
// order, XCD-aware renumbering).
__device__ __forceinline__ BlockCoord block_coord(const uint32_t* __restrict__ blocks) {
  const uint32_t w0 = blocks[2 * blockIdx.x], w1 = blocks[2 * blockIdx.x + 1];
  BlockCoord c;
  c.ex0 = (int)(w0 & 0xffffu);
  c.ey = (int)(w0 >> 16);
  c.ez = (int)w1;
  return c;
}

// Position of a block's chunk in the plain order (x chunks, then y, then z):
// where the block writes its partial sums, so that a reduction adds them in
// the same order whatever sweep order ran the blocks.
template <typename A>
__device__ __forceinline__ int64_t chunk_slot(const BlockCoord& bc, const A& a, int eb) {
  return ((int64_t)bc.ez * a.n[1] + bc.ey) * a.nchunk + bc.ex0 / eb;
}

// Copies the calling thread's share of its cell into the padded LDS layout:
// the thread that owns the lines (ta, tb) of cell le moves the P nodes
// (ta, tb, 0..P-1), one z-plane apart. Per load the lanes of a cell read one
// contiguous plane of it.
template <int P, typename T>
__device__ __forceinline__ void load_cell_column(T* __restrict__ s, const T* __restrict__ g, uint32_t gbase,
                                                 int le, int ta, int tb) {
  constexpr int L = P * P, N = P * P * P;
  using Ly = Layout<P>;
  const T* __restrict__ gc = g + gbase + (le * N + ta + P * tb);
  T* __restrict__ sc = s + le * Ly::NP + ta + Ly::S1 * tb;
#pragma unroll
  for (int j = 0; j < P; ++j) sc[j * Ly::S2] = gc[j * L];
}

// Reads the line of direction DIR at (ta, tb) of LDS cell block `sc`.
template <int P, typename T, int DIR>
__device__ __forceinline__ void lds_line(const T* __restrict__ sc, int ta, int tb, T* v) {
  using Ly = Layout<P>;
  const int off = DIR == 0 ? Ly::S1 * ta + Ly::S2 * tb : (DIR == 1 ? ta + Ly::S2 * tb : ta + Ly::S1 * tb);
  constexpr int S = DIR == 0 ? 1 : (DIR == 1 ? Ly::S1 : Ly::S2);
#pragma unroll
  for (int j = 0; j < P; ++j) v[j] = sc[off + j * S];
}

// Reads the line of direction DIR at (ta, tb) of the global cell block at `base`.
template <int P, typename T, int DIR>
__device__ __forceinline__ void global_line(const T* __restrict__ g, uint32_t base, int ta, int tb, T* v) {
  constexpr int L = P * P;
  const T* __restrict__ gl = g + base + (DIR == 0 ? P * ta + L * tb : (DIR == 1 ? ta + L * tb : ta + P * tb));
  constexpr int S = DIR == 0 ? 1 : (DIR == 1 ? P : L);
#pragma unroll
  for (int j = 0; j < P; ++j) v[j] = gl[j * S];
}

// Neighbour lines of direction DIR for both sides (x-neighbours inside the
// chunk come from LDS, everything else from global memory / L2).
template <int P, typename T, int DIR>
__device__ __forceinline__ void neighbor_lines(const T* __restrict__ s, const T* __restrict__ g, uint32_t e,
                                               int le, int nvalid, int ecd, int nd, uint32_t estride, int ta,
                                               int tb, T (*nb)[P], bool* has) {
  constexpr int N = P * P * P;
  using Ly = Layout<P>;
  has[0] = ecd > 0;
  has[1] = ecd < nd - 1;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    if (!has[side]) {
#pragma unroll
      for (int j = 0; j < P; ++j) nb[side][j] = T(0);
      continue;
    }
    const int lnb = side ? le + 1 : le - 1;
    if (DIR == 0 && lnb >= 0 && lnb < nvalid) {
      lds_line<P, T, 0>(s + lnb * Ly::NP, ta, tb, nb[side]);
    } else {
      const uint32_t en = side ? e + estride : e - estride;
      global_line<P, T, DIR>(g, en * N, ta, tb, nb[side]);
    }
  }
}

template <int P, typename T, int DIR>
__device__ __forceinline__ void lds_store_line(T* __restrict__ sc, int ta, int tb, const T* v) {
  using Ly = Layout<P>;
  const int off = DIR == 0 ? Ly::S1 * ta + Ly::S2 * tb : (DIR == 1 ? ta + Ly::S2 * tb : ta + Ly::S1 * tb);
  constexpr int S = DIR == 0 ? 1 : (DIR == 1 ? Ly::S1 : Ly::S2);
#pragma unroll
  for (int j = 0; j < P; ++j) sc[off + j * S] = v[j];
}

}  // namespace dgi
