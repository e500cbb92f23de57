"""Benchmark of the sum-factorized DG operator apply on one MI355X.

One step = one matrix-free FP64 application y = A x of the Q3 SIPG
diffusion-reaction operator on the 64^3 axis-aligned mesh (16,777,216 DOFs),
inputs resident in HBM; the step runs the matrix-core kernel k_apply_q3_mfma.
Consecutive steps rotate over four (x, y) buffer pairs (1.07 GB, beyond the
256 MB MALL), so every step reads x from and writes y to HBM. `ms_per_step`
is the median over trials of the mean of the timed steps of each trial.
The JSON line reports DOFs/s of that step, the roofline of the apply kernel
(HBM-bound: 16 B/DOF compulsory traffic), the achieved bandwidth of a plain
device copy on the same box, and the CPU oracle's block-sparse SpMV as a
baseline; `extra` carries the other workloads (the same step with one buffer
pair, FP32 apply, kappa apply and adjoint, Q5 applies, Stokes, Section 5.2's
benchmark operator, the preconditioner, the FP64-CG vs FP32-refinement solve),
each timed the same way, with 30 ms of further untimed calls after the warm-up
(a row's fresh buffers are otherwise still being touched for the first time in
its first trial).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_applies(fn, steps, warmup, stream, trials=3, warm_ms=0.0):
    """ms per call of fn(): `trials` runs of `steps` calls, each bracketed by a
    device synchronization and timed with HIP events recorded on the stream the
    kernels are launched on; returns (median over trials, per-trial list).
    Untimed before the trials: `warmup` calls, then (warm_ms > 0) further calls
    until warm_ms milliseconds of them have run, at most 2000 calls."""
    import statistics
    import time as _time
    import torch
    for _ in range(warmup):
        fn()
    if warm_ms > 0:
        torch.cuda.synchronize()
        t0, done = _time.perf_counter(), 0
        while done < 2000 and (_time.perf_counter() - t0) * 1e3 < warm_ms:
            for _ in range(10):
                fn()
            done += 10
            torch.cuda.synchronize()
    per = []
    for _ in range(trials):
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(steps):
            fn()
        end.record(stream)
        torch.cuda.synchronize()
        per.append(start.elapsed_time(end) / steps)
    return statistics.median(per), per


def copy_reference():
    """Achieved HBM bandwidth of a plain device copy of 134 MB (torch's copy
    kernel), timed like the applies: the same-box reference for the fractions.
    `gbs` rotates 4 source/destination pairs (1.07 GB, beyond the 256 MB MALL),
    the reuse pattern of the benchmark step; `gbs_one_pair` copies one pair
    over and over (the MALL serves part of it)."""
    import torch
    n = 16777216
    src = [torch.ones(n, dtype=torch.float64, device="cuda") for _ in range(4)]
    dst = [torch.empty_like(src[0]) for _ in range(4)]
    stream = torch.cuda.current_stream()
    out = {}
    for key, npair in (("", 4), ("_one_pair", 1)):
        it = [0]

        def step():
            i = it[0] % npair
            it[0] += 1
            dst[i].copy_(src[i])

        ms, _ = time_applies(step, 40, 4, stream)
        out["ms" + key] = round(ms, 5)
        out["gbs" + key] = 2 * n * 8 / (ms * 1e-3) / 1e9
    return out


def rates(info, ms, prec, nbytes=None, flops=None, per=None):
    t = ms * 1e-3
    b = info.bytes_apply[prec] if nbytes is None else nbytes
    f = info.flops_apply if flops is None else flops
    peak_f = FP64_PEAK_TFLOPS if prec == 0 else FP32_PEAK_TFLOPS
    out = {
        "ms": round(ms, 5),
        "dofs_per_s": info.ndofs / t,
        "hbm_gbs": b / t / 1e9,
        "hbm_frac": b / t / 1e9 / HBM_PEAK_GBS,
        "gflops_model": f / t / 1e9,
        "flop_frac_model": f / t / 1e12 / peak_f,
    }
    if per is not None:
        out["ms_trials"] = [round(v, 5) for v in per]
    return out


def bench_apply(dg, w, prec, steps, warmup, nbuf=4, n=None, trials=3, problem=None, warm_ms=0.0):
    """Times dg_apply on workload w. Consecutive calls rotate over `nbuf`
    (x, y[, kappa]) buffer sets: 4 sets of the full-size vectors exceed the
    256 MB MALL, so every call reads and writes HBM (nbuf = 1: one set, the
    MALL serves part of it)."""
    import torch
    import workloads
    desc = dg.desc_from_workload(w, n=n)
    if problem is not None:
        desc.problem = problem
        if problem == dg.DG_PROBLEM_DIFFREAC_PAPER:
            desc.c = 10.0  # Section 5.2's reaction coefficient
    mesh = dg.Mesh(desc)
    dt = torch.float64 if prec == dg.DG_F64 else torch.float32
    ww = w if n is None else w.scaled(n)
    x0 = torch.from_numpy(workloads.inputs(ww, "x")).to("cuda", dt)
    xs = [x0] + [x0.clone() for _ in range(nbuf - 1)]
    ys = [torch.empty_like(x0) for _ in range(nbuf)]
    kaps = [None] * nbuf
    if w.kappa_mode:
        k0 = torch.from_numpy(workloads.inputs(ww, "kappa")).to("cuda", dt)
        kaps = [k0] + [k0.clone() for _ in range(nbuf - 1)]
    stream = torch.cuda.current_stream()
    it = [0]

    def step():
        i = it[0] % nbuf
        it[0] += 1
        dg.dg_apply(mesh.handle, prec, xs[i], ys[i], kaps[i], stream)

    ms, per = time_applies(step, steps, warmup, stream, trials, warm_ms)
    return mesh, ms, per


def bench_residual(dg, w, steps, warmup, trials=3, nbuf=4, warm_ms=0.0):
    """dg_residual (Section 5.2's full residual, source and Dirichlet data
    terms included) on workload w's mesh with the paper's operator."""
    import torch
    import workloads
    desc = dg.desc_from_workload(w)
    desc.problem = dg.DG_PROBLEM_DIFFREAC_PAPER
    desc.c = 10.0
    mesh = dg.Mesh(desc)
    u0 = torch.from_numpy(workloads.inputs(w, "x")).cuda()
    us = [u0] + [u0.clone() for _ in range(nbuf - 1)]
    rs = [torch.empty_like(u0) for _ in range(nbuf)]
    stream = torch.cuda.current_stream()
    it = [0]

    def step():
        i = it[0] % nbuf
        it[0] += 1
        dg.dg_residual(mesh.handle, dg.DG_F64, us[i], rs[i], stream)

    ms, per = time_applies(step, steps, warmup, stream, trials, warm_ms)
    return mesh, ms, per


def bench_adjoint(dg, w, steps, warmup, trials=3, nbuf=2, warm_ms=0.0):
    """A^T g and dL/dkappa; 2 rotating sets of (g, u, kappa, A^T g, dkappa)
    (1.1 GB at Q4 48^3) keep every call in HBM."""
    import torch
    import workloads
    mesh = dg.Mesh(dg.desc_from_workload(w))
    g = torch.from_numpy(workloads.inputs(w, "g")).cuda()
    u = torch.from_numpy(workloads.inputs(w, "u")).cuda()
    kap = torch.from_numpy(workloads.inputs(w, "kappa")).cuda()
    sets = [(g, u, kap)] + [(g.clone(), u.clone(), kap.clone()) for _ in range(nbuf - 1)]
    outs = [(torch.empty_like(g), torch.empty_like(kap)) for _ in range(nbuf)]
    stream = torch.cuda.current_stream()
    it = [0]

    def step():
        i = it[0] % nbuf
        it[0] += 1
        gg, uu, kk = sets[i]
        dg.dg_apply_adjoint(mesh.handle, dg.DG_F64, gg, uu, kk, outs[i][0], outs[i][1], stream)

    ms, per = time_applies(step, steps, warmup, stream, trials, warm_ms)
    info = mesh.info
    return rates(info, ms, 0, nbytes=info.bytes_adjoint, flops=info.flops_adjoint, per=per)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def host_threads():
    """Threads the CPU baseline may use: the OpenMP setting of the host if any
    (a shared host states the process's CPU share there), else the CPUs this
    process may run on."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(int(env), avail)) if env.isdigit() and int(env) > 0 else avail


def cpu_baseline(trials=5, reps=5, single_reps=1):
    """The oracle's SpMV of the Q3 operator on the full 64^3 benchmark mesh:
    the block-sparse matrix assembled by full quadrature (one block row per
    cell, blocks stored once per boundary class) applied by the oracle's C
    routine with its block rows split over the host threads; median over
    `trials` runs of `reps` applies, and the same with one thread."""
    import statistics
    import numpy as np
    import workloads
    from oracle import ScalarDG, problem_from_workload
    from oracle.blocks import CBlockMatvec
    w = workloads.WORKLOADS[2]
    t0 = time.perf_counter()
    A = ScalarDG(problem_from_workload(w)).assemble("dedup")
    mv = CBlockMatvec(A)
    t_asm = time.perf_counter() - t0
    x = workloads.inputs(w, "x")
    y = np.empty_like(x)
    nthr = host_threads()

    def median_rate(threads, nrep, ntrial):
        mv(x, threads, y)
        times = []
        for _ in range(ntrial):
            t = time.perf_counter()
            for _ in range(nrep):
                mv(x, threads, y)
            times.append((time.perf_counter() - t) / nrep)
        return w.ndofs / statistics.median(times), statistics.median(times)

    rate, sec = median_rate(nthr, reps, trials)
    rate1, sec1 = median_rate(1, single_reps, 1)
    return {"value": rate, "unit": "DOFs/s", "cores": nthr, "kind": "oracle",
            "sample": f"Q3 SIPG block-sparse SpMV (oracle/spmv.c, OpenMP over block rows) on the full 64^3 mesh, "
                      f"{w.ndofs} DOFs, median of {trials} x {reps} applies ({sec * 1e3:.0f} ms each); "
                      f"blocks assembled by full quadrature once per boundary class in {t_asm:.1f} s (not timed); "
                      f"host: {os.cpu_count()} logical CPUs, {cpu_model()}",
            "value_1thread": rate1, "ms_1thread": sec1 * 1e3}


def bench_precond(dg, w, prec, steps, warmup, trials=3, nbuf=4, warm_ms=0.0):
    """z = P r with the block-Jacobi preconditioner (fast diagonalization):
    read r, write z, 12 p^4 + p^3 flops per cell; 4 rotating (r, z) pairs."""
    import torch
    import workloads
    mesh = dg.Mesh(dg.desc_from_workload(w))
    dt = torch.float64 if prec == dg.DG_F64 else torch.float32
    r0 = torch.from_numpy(workloads.inputs(w, "x")).to("cuda", dt)
    rs = [r0] + [r0.clone() for _ in range(nbuf - 1)]
    zs = [torch.empty_like(r0) for _ in range(nbuf)]
    stream = torch.cuda.current_stream()
    it = [0]

    def step():
        i = it[0] % nbuf
        it[0] += 1
        dg.dg_precond_apply(mesh.handle, prec, rs[i], zs[i], stream)

    ms, per = time_applies(step, steps, warmup, stream, trials, warm_ms)
    info = mesh.info
    p = info.p
    es = 8 if prec == dg.DG_F64 else 4
    return rates(info, ms, prec, nbytes=2.0 * es * info.ndofs, flops=info.nelem * (12.0 * p ** 4 + p ** 3), per=per)


def bench_solve(dg, rtol=1e-10):
    """Q5 40^3 manufactured sin problem, all to the same true relative
    residual from x0 = 0: FP64 CG; the FP32-apply refinement schemes; FP64 CG
    preconditioned by s steps of the Chebyshev iteration on the FP32 operator
    (and, as the baseline of that scheme, on the FP64 operator); each
    unpreconditioned and with the block-Jacobi preconditioner."""
    import torch
    import workloads
    w = workloads.WORKLOADS[5]
    mesh = dg.Mesh(dg.desc_from_workload(w))
    xyz = dg.dg_mesh_qpoints(mesh.handle)
    fq = torch.from_numpy(workloads.sin_forcing(xyz, w.c)).cuda()
    del xyz
    b = torch.empty(mesh.ndofs, dtype=torch.float64, device="cuda")
    dg.dg_load_vector(mesh.handle, dg.DG_F64, fq, b)
    out = {}
    sol = {}
    # inner tolerance / reliable-update drop / Chebyshev steps per mode, chosen by a sweep at this size
    inner = {"cg_f64": 1e-5, "ir_f32": 1e-5, "ru_f32": 0.1, "ir_f32_bj": 1e-3}
    degree = {"cheb_f64": 12, "cheb_f32": 12, "cheb_f64_bj": 8, "cheb_f32_bj": 8}
    runs = []
    for pc, suffix in ((dg.DG_PRECOND_NONE, ""), (dg.DG_PRECOND_BLOCK_JACOBI, "_bj")):
        for base, mode in (("cg_f64", dg.DG_SOLVE_CG_F64), ("ir_f32", dg.DG_SOLVE_IR_F32),
                           ("ru_f32", dg.DG_SOLVE_RU_F32), ("cheb_f64", dg.DG_SOLVE_CHEB_F64),
                           ("cheb_f32", dg.DG_SOLVE_CHEB_F32)):
            runs.append((base + suffix, base, mode, pc))
    for name, base, mode, pc in runs:
        log(f"solve {name}")
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, info = dg.dg_solve(mesh.handle, mode, b, x, rtol=rtol, inner_rtol=inner.get(name, inner["cg_f64"]),
                               maxit=200000, max_outer=20, check_every=10, precond=pc,
                               cheb_degree=degree.get(name, 0))
        el = time.perf_counter() - t0
        out[name] = {"status": st, "seconds": el, "iterations": info.iterations, "outer": info.outer,
                     "true_rel_residual": info.rel_residual}
        if base.startswith("cheb"):
            out[name].update({"inner_applies": info.inner_applies, "degree": degree[name],
                              "lambda_max": info.lambda_max})
        sol[name] = x
    for suffix in ("", "_bj"):
        ref = "cg_f64" + suffix
        for base in ("ir_f32", "ru_f32", "cheb_f64", "cheb_f32"):
            name = base + suffix
            out[f"speedup_{name}_over_{ref}"] = out[ref]["seconds"] / out[name]["seconds"]
            d = sol[name] - sol["cg_f64"]
            out[f"rel_diff_{name}_vs_cg_f64"] = float(torch.linalg.norm(d) / torch.linalg.norm(sol["cg_f64"]))
    out["speedup_cg_f64_bj_over_cg_f64"] = out["cg_f64"]["seconds"] / out["cg_f64_bj"]["seconds"]
    out["speedup_cheb_f32_bj_over_cg_f64"] = out["cg_f64"]["seconds"] / out["cheb_f32_bj"]["seconds"]
    out["workload"] = w.name
    return out


def measured_traffic(kernel_file, key):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when the kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    src = os.path.join(ROOT, "paper_1812_08075_amd", "csrc", kernel_file)
    try:
        rec = json.load(open(path))[key]
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except (OSError, KeyError, ValueError):
        return None
    return rec["traffic_bytes"] if rec.get("source_sha256_16") == sha else None


def executed_flop_frac(ms, kernel_file, key):
    """FP64 flops the kernel executes per launch (rocprofv3 instruction counters
    in profiles/counters.json: 64 lanes x (add + mul + 2 fma + trans) per VALU
    FP64 instruction, 512 per v_mfma_f64_4x4x4f64) over the launch time, as a
    fraction of the FP64 peak; None when the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "counters.json")
    src = os.path.join(ROOT, "paper_1812_08075_amd", "csrc", kernel_file)
    try:
        rec = json.load(open(path))[key]
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("source_sha256_16") != sha:
        return None
    return rec["fp64_flops"] / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--trials", type=int, default=5, help="timed trials of --steps steps each (median reported)")
    ap.add_argument("--no-extra", action="store_true", help="only the headline step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the Q5 40^3 FP64-CG vs FP32-refinement solve comparison")
    ap.add_argument("--only", choices=["stokes", "q4", "q5", "f32", "paper", "precond"], default=None,
                    help="run one secondary workload only (for profiling), no JSON line")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed region, copy the 134 MB input vector 5 times with torch's copy "
                         "kernel (a known-size reference for HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the multi-GPU sharding of the apply is a design note, "
              "not built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1812_08075_amd as dg
    import workloads

    K, W, T = args.steps, args.warmup, args.trials
    w2, w3, w4, w5 = (workloads.WORKLOADS[i] for i in (2, 3, 4, 5))
    if args.only is not None:
        if args.only == "stokes":
            _, ms, _ = bench_apply(dg, w3, dg.DG_F64, K, W, trials=1)
            log(f"{w3.name}: {ms * 1e3:.1f} us per apply")
        elif args.only == "q4":
            _, ms, _ = bench_apply(dg, w4, dg.DG_F64, K, W, trials=1)
            log(f"{w4.name}: {ms * 1e3:.1f} us per apply")
            r = bench_adjoint(dg, w4, K, W, trials=1)
            log(f"{w4.name} adjoint: {r['ms'] * 1e3:.1f} us")
        elif args.only == "q5":
            for prec in (dg.DG_F64, dg.DG_F32):
                _, ms, _ = bench_apply(dg, w5, prec, K, W, trials=1)
                log(f"{w5.name} precision {prec}: {ms * 1e3:.1f} us per apply")
        elif args.only == "f32":
            _, ms, _ = bench_apply(dg, w2, dg.DG_F32, K, W, trials=1)
            log(f"{w2.name} FP32: {ms * 1e3:.1f} us per apply")
        elif args.only == "paper":
            _, ms, _ = bench_apply(dg, w2, dg.DG_F64, K, W, trials=1, problem=dg.DG_PROBLEM_DIFFREAC_PAPER)
            log(f"Section 5.2 operator on {w2.name}: {ms * 1e3:.1f} us per apply")
            _, ms, _ = bench_residual(dg, w2, K, W, trials=1)
            log(f"Section 5.2 residual on {w2.name}: {ms * 1e3:.1f} us")
        elif args.only == "precond":
            for prec in (dg.DG_F64, dg.DG_F32):
                r = bench_precond(dg, w5, prec, K, W, trials=1)
                log(f"{w5.name} block-Jacobi precision {prec}: {r['ms'] * 1e3:.1f} us")
        return

    log(f"headline: {w2.name} FP64 apply, 4 rotating buffer pairs, {T} trials x {K} steps")
    mesh, ms, per = bench_apply(dg, w2, dg.DG_F64, K, W, nbuf=4, trials=T)
    info = mesh.info
    r64 = rates(info, ms, 0, per=per)
    if args.copy_probe:
        src = torch.from_numpy(workloads.inputs(w2, "x")).cuda()
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    extra = {"apply_q3_f64": r64}

    if not args.no_extra:
        # the secondary rows: after their W warm-up calls, further untimed calls
        # for XW ms (fresh buffers, first touches), then the trials
        XW = 30.0
        extra["hbm_copy_reference"] = copy_reference()
        log("Q3 FP64, one buffer pair (the MALL serves part of x and y)")
        _, ms_w, per_w = bench_apply(dg, w2, dg.DG_F64, K, W, nbuf=1, warm_ms=XW)
        extra["apply_q3_f64_one_pair"] = rates(info, ms_w, 0, per=per_w)
        log("Q3 FP32")
        _, ms32, per32 = bench_apply(dg, w2, dg.DG_F32, K, W, warm_ms=XW)
        extra["apply_q3_f32"] = rates(info, ms32, 1, per=per32)
        log("Q5 FP64 / FP32")
        m5, ms5, per5 = bench_apply(dg, w5, dg.DG_F64, K, W, warm_ms=XW)
        extra["apply_q5_f64"] = rates(m5.info, ms5, 0, per=per5)
        _, ms5f, per5f = bench_apply(dg, w5, dg.DG_F32, K, W, warm_ms=XW)
        extra["apply_q5_f32"] = rates(m5.info, ms5f, 1, per=per5f)
        log("Stokes Q3/Q2 32^3 perturbed FP64")
        m3, ms3, per3 = bench_apply(dg, w3, dg.DG_F64, K, W, warm_ms=XW)
        extra["apply_stokes_f64"] = rates(m3.info, ms3, 0, per=per3)
        # the model's flops assume the paper's sum-factorized kernels; the
        # executed count (instruction counters) includes the geometry recomputed
        # at every point
        extra["apply_stokes_f64"]["fp64_flop_frac_executed"] = executed_flop_frac(
            ms3, "stokes.hip", "k_stokes_apply_q3q2_32cube_perturbed")
        del m3
        log("Q4 FP64 with kappa per point")
        m4, ms4, per4 = bench_apply(dg, w4, dg.DG_F64, K, W, warm_ms=XW)
        extra["apply_q4_kappa_f64"] = rates(m4.info, ms4, 0, per=per4)
        log("Q4 FP64 adjoint (A^T g and dL/dkappa)")
        extra["adjoint_q4_kappa_f64"] = bench_adjoint(dg, w4, K, W, warm_ms=XW)
        del m4, m5
        log("Section 5.2 operator (K = x x^T + I, c = 10) on the Q3 64^3 mesh: Jacobian action and full residual")
        mp, msp, perp = bench_apply(dg, w2, dg.DG_F64, K, W, problem=dg.DG_PROBLEM_DIFFREAC_PAPER, warm_ms=XW)
        extra["apply_paper_q3_f64"] = rates(mp.info, msp, 0, per=perp)
        _, msr, perr = bench_residual(dg, w2, K, W, warm_ms=XW)
        extra["residual_paper_q3_f64"] = rates(mp.info, msr, 0, per=perr)
        extra["paper_context"] = "Section 5.2 reports 40-60% of FP64 peak for one full apply on Haswell/Skylake"
        del mp
        log("Q5 block-Jacobi preconditioner FP64 / FP32")
        extra["precond_q5_f64"] = bench_precond(dg, w5, dg.DG_F64, K, W, warm_ms=XW)
        extra["precond_q5_f32"] = bench_precond(dg, w5, dg.DG_F32, K, W, warm_ms=XW)
    if not args.no_solve and not args.no_extra:
        extra["solve_q5_40cube"] = bench_solve(dg)

    out = {
        "metric": "DOFs/s per DG operator apply (FP64 vs FP32+refine) + % roofline, Q3-Q5",
        "value": r64["dofs_per_s"],
        "unit": "DOFs/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded uniform[-1,1] DOF vector)",
        "config": {"workload": w2.name, "k": w2.k, "m": w2.m, "mesh": f"{w2.n}^3", "ndofs": int(info.ndofs),
                   "penalty": "3k(k+1)/h", "theta": -1.0, "parallelism": "single GPU",
                   "buffers": "4 rotating (x, y) pairs", "timing": f"median of {T} trials x {K} steps"},
        "roofline": {"bound": "hbm", "achieved": r64["hbm_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r64["hbm_frac"],
                     "traffic": measured_traffic("apply_mfma.hip", "k_apply_q3_mfma_64cube_f64"),
                     "kernel": "k_apply_q3_mfma",
                     "algorithmic_bytes_per_launch": info.bytes_apply[0],
                     "fp64_flop_frac_model": r64["flop_frac_model"],
                     "fp64_flop_frac_executed": executed_flop_frac(ms, "apply_mfma.hip",
                                                                   "k_apply_q3_mfma_64cube_f64")},
        "extra": extra,
    }
    if not args.no_cpu:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
