"""Benchmark of the LoMaC-SLAR time step on one MI355X.

Workload: 2D2V strong Landau damping (alpha = 0.5, k = 0.5) on a 128^4 grid,
x in [0, 4 pi)^2, v in [-6, 6]^2, tolerance 1e-5, rank cap 60, dt = 0.2,
third-order exponential integrator (three SLAR calls per step), LoMaC with
JFNK (BE start, BDF2 after), FP32 sampling contractions, FP64 elsewhere.

A step is one pass of the whole path: three cross approximations with their
SL-FD sampling, three truncations, the field solves, the LoMaC closure, the
Newton--Krylov macroscopic solve and the correction.  Inputs (the HT state)
are resident in HBM before the timed region starts.

Prints one JSON line: sampled SL-FD entries per second over the timed steps
(value), time per step, the roofline position of the dominant kernel and the
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}   # MI355X dense matrix-core peaks
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hbm_traffic_k_aca_col_stronglandau2d_128.md")
# sources that define the column-fiber kernel; the counter-measured traffic
# is reported only for the source state it was measured on
KERNEL_SOURCES = ["aca.h", "frame_sampler.h", "sl_device.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2606_29027_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per column-fiber launch from the committed rocprofv3 counter
    summary, or None when the kernel sources changed since it was taken."""
    try:
        vals = {}
        with open(TRAFFIC_SUMMARY) as fh:
            for line in fh:
                if ":" in line and line.split(":")[0].strip() in ("source_sha256", "traffic_bytes_per_launch"):
                    k, v = line.split(":", 1)
                    vals[k.strip()] = v.strip().strip("`")
        if vals.get("source_sha256") != kernel_source_hash():
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


BATCH_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hbm_traffic_batched_cross_64.md")
BATCH_SOURCES = ("batch_kernels.h", "aca.h", "frame_sampler.h", "sl_device.h")


def measured_batch_traffic():
    """HBM bytes per step of the batched cross approximation (FETCH_SIZE +
    WRITE_SIZE over its launches in the timed steps, calibrated), from the
    committed counter summary, or None when its kernels changed since."""
    try:
        vals = {}
        with open(BATCH_TRAFFIC_SUMMARY) as fh:
            for line in fh:
                if ":" in line and line.split(":")[0].strip() in ("source_sha256", "traffic_bytes_per_step"):
                    k, v = line.split(":", 1)
                    vals[k.strip()] = v.strip().strip("`")
        h = hashlib.sha256()
        for fn in BATCH_SOURCES:
            with open(os.path.join(ROOT, "paper_2606_29027_amd", "csrc", fn), "rb") as fh:
                h.update(fh.read())
        if vals.get("source_sha256") != h.hexdigest():
            return None
        return float(vals["traffic_bytes_per_step"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["f32", "f64"], default="f32")
    ap.add_argument("--n", type=int, default=128, help="cells per dimension")
    ap.add_argument("--nested-config", default="stronglandau2d",
                    help="2D2V workload whose state the nested workload compares the samplers on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--nested-dtype", choices=["auto", "f32", "f64"], default="auto",
                    help="frame-table precision of the nested workload")
    ap.add_argument("--cpu-seconds", type=float, default=18.0)
    ap.add_argument("--variants", default="plain,spectral,learned",
                    help="comma list of macro solvers to time: plain, spectral, learned "
                         "(the last one listed is the headline)")
    ap.add_argument("--workload", choices=["stronglandau2d", "batched", "samplers", "nested"], default="stronglandau2d",
                    help="batched: 64 independent 1D1V/2D2V Landau instances of uneven size")
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--no-tune", action="store_true", help="batched: keep the default launch configuration")
    ap.add_argument("--no-batched", action="store_true",
                    help="default workload: leave out the batched-instances leg of the line")
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--no-other-precision", action="store_true",
                    help="skip the short run of the step with the other table precision")
    ap.add_argument("--no-samplers", action="store_true", help="skip the r = 60 entry-sampler records")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before timing, run one device copy of this size (for counter calibration)")
    return ap.parse_args()


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, budget_s: float):
    """The CPU oracle on a bounded sample of the workload, at all host
    threads and at one BLAS thread:

    * SL-FD entries/s of the frame-form evaluation (the algorithm the GPU's
      cross approximation runs: both frame gathers and an r-term dot
      product) and of the leaf-to-root HT contraction, on whole row fibers
      of a rank-60 orthogonal 128^4 state (graded singular values, seed 21),
      first RK sub-flow (tau = dt / 3) in the initial state's field;
    * seconds per time step of the 64^4 weak-Landau workload (its first
      steps; the 128^4 steps take the oracle hours).

    value = frame-form entries/s at all threads.  Each timing runs for
    about budget_s / 6 seconds."""
    import slar_inputs as SI
    from oracle import feet as FT
    from oracle import ht as HT
    from oracle import step as ST
    from threadpoolctl import threadpool_info, threadpool_limits
    nthreads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    o = ST.Oracle(p)
    E = o.efield(SI.initial_ht(p))
    F = SI.graded_ht(p.n, 60, 60, 0.85, seed=21)
    X = HT.x_frame(F)
    P = np.tensordot(HT.v_frame(F), F["root"], axes=([2], [1]))
    Nx = int(np.prod(p.n[: p.dx])); Nv = int(np.prod(p.n[p.dx:]))
    slot = budget_s / 6.0

    def fibers(fn):
        done, fib = 0, 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < slot:
            idx = o._idx(np.full(Nv, fib * 997 % Nx), np.arange(Nv))
            foot = FT.feet(idx, p.lo, p.hi, p.n, p.dx, 2, p.dt / 3.0, 1.0, E)
            rows, wts = FT.stencils(foot, idx, p.lo, p.hi, p.n, 3, 2, p.dx)
            fn(rows, wts)
            done += Nv
            fib += 1
        return done / (time.perf_counter() - t0), fib

    def cfg2_steps(nsteps):
        q = SI.config("landau2d")
        oq = ST.Oracle(q, probes=SI.probe_indices(64 * 64, 64 * 64, 64, 1234))
        t0 = time.perf_counter()
        oq.run(SI.initial_ht(q), nsteps)
        return (time.perf_counter() - t0) / nsteps

    res = {}
    for label, lim in (("threads_all", nthreads), ("threads_1", 1)):
        with threadpool_limits(limits=lim):
            fr, nf = fibers(lambda r, w: HT.sample_frames(X, P, r, w))
            ct, nc = fibers(lambda r, w: HT.sample(F, r, w))
            st = cfg2_steps(2 if lim > 1 else 1)
        res[label] = {"frame_entries_per_s": fr, "contraction_entries_per_s": ct,
                      "cfg2_64_4_s_per_step": st, "fibers": [nf, nc]}
    return {"value": res["threads_all"]["frame_entries_per_s"], "unit": "entries/s",
            "cores": int(nthreads), "kind": "oracle",
            "sample": f"row fibers of {Nv} SL-FD entries of a rank-60 orthogonal 128^4 state, first RK "
                      "sub-flow of the workload, frame-form evaluation (the GPU cross's algorithm), "
                      "FP64 NumPy; plus the leaf-to-root contraction and 64^4 weak-Landau steps",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "blas_threads": int(nthreads),
            "threads_all": res["threads_all"], "threads_1": res["threads_1"]}


def cpu_baseline_batched(problems, budget_s: float):
    """The CPU oracle on a bounded sample of the batched workload: whole row
    fibers of the instances' initial states at their first RK sub-flow (each
    instance in its own field), frame-form evaluation, instances taken in
    turn until budget_s has passed; entries/s at all host threads."""
    import slar_inputs as SI
    from oracle import feet as FT
    from oracle import ht as HT
    from oracle import step as ST
    from threadpoolctl import threadpool_info
    nthreads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    done, fib, inst, cache = 0, 0, set(), {}
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        q = fib % len(problems)
        p = problems[q]
        if q not in cache:
            o = ST.Oracle(p)
            F = SI.initial_ht(p)
            V = HT.v_frame(F)
            cache[q] = (o, o.efield(F), HT.x_frame(F), np.tensordot(V, F["root"], axes=([V.ndim - 1], [1])))
        o, E, X, P = cache[q]
        Nx = int(np.prod(p.n[: p.dx])); Nv = int(np.prod(p.n[p.dx:]))
        idx = o._idx(np.full(Nv, (fib * 997) % Nx), np.arange(Nv))
        foot = FT.feet(idx, p.lo, p.hi, p.n, p.dx, 2, p.dt / 3.0, 1.0, E)
        rows, wts = FT.stencils(foot, idx, p.lo, p.hi, p.n, 3, 2, p.dx)
        HT.sample_frames(X, P, rows, wts)
        done += Nv
        fib += 1
        inst.add(q)
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "entries/s", "cores": int(nthreads), "kind": "oracle",
            "sample": f"{fib} row fibers ({done} SL-FD entries) over {len(inst)} of the instances' initial "
                      "states, first RK sub-flow, frame-form evaluation, FP64 NumPy",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count()}


def batched_run(args, steps, warmup, cpu_seconds=None):
    """64 independent Landau instances (1D1V or 2D2V, N per dimension from
    {32, 48, 64, 96, 128}) advanced together: one SLAR_VP step of every
    instance per step; value = sampled entries of all instances per second.
    Returns the record of the batched workload."""
    import torch
    import slar_inputs as SI
    from paper_2606_29027_amd.batch import BatchSolver

    problems = SI.batched_instances(args.instances)
    probes = []
    for q, p in enumerate(problems):
        Nx = int(np.prod(p.n[: p.dx])); Nv = int(np.prod(p.n[p.dx:]))
        probes.append(SI.probe_indices(Nx, Nv, 64, 1000 + q))
    b = BatchSolver(problems, probes=probes)
    b.set_initial([SI.initial_ht(p) for p in problems])
    tuned = None
    t_tune = time.perf_counter()
    if not args.no_tune:
        tuned = b.tune(reps=2)
    t_tune = time.perf_counter() - t_tune
    for _ in range(warmup):
        b.step()
    torch.cuda.synchronize()
    if args.calib_copy_mib > 0:
        # marks the start of the timed steps in a counter trace
        a = torch.ones(args.calib_copy_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        c = torch.empty_like(a)
        c.copy_(a)
        torch.cuda.synchronize()
        del a, c
    n0 = len(b.stats)
    b.batch.timing_reset()
    b.tphase = {k: 0.0 for k in b.tphase}
    t0 = time.perf_counter()
    for _ in range(steps):
        b.step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tim = b.batch.timing()
    samples = sum(st["samples"] for st in b.stats[n0:])
    # algorithmic bytes of the batched cross approximations: per sampled
    # entry both FP32 stencil gathers (3^dx rows of X, 3^dv rows of P, ldt
    # columns), the 8-byte write and 16 k bytes of earlier cross vectors
    # (k taken at half the final rank of the call)
    by = 0.0
    for st in b.stats[n0:]:
        for q, p in enumerate(problems):
            rx = 3 ** p.dx
            r = st["src_ranks"][q]
            ldt = (r + 3) & ~3
            by += st["samples_q"][q] * (2.0 * rx * ldt * 4 + 8 + 16 * st["ranks"][q] / 2.0)
    achieved = by / (tim["cross_ms"] * 1e-3) / 1e9 if tim["cross_ms"] > 0 else 0.0
    n1 = sum(1 for p in problems if p.dx == 1)
    traffic = measured_batch_traffic()
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "batched cross approximation (prep + row + col launches, graph replays)",
            "algorithmic_bytes_per_step": by / steps, "cross_ms_per_step": tim["cross_ms"] / steps}
    if traffic and tim["cross_ms"] > 0:
        hbm = traffic / (tim["cross_ms"] / steps * 1e-3) / 1e9
        roof["hbm_measured_GBps"] = hbm
        roof["hbm_measured_frac"] = hbm / HBM_PEAK_GBS
    out = {
        "metric": "HT-SL sampled entries/s & time/step, batched independent instances",
        "value": samples / elapsed,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": 1e3 * elapsed / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(problems)} independent Landau instances ({n1} 1D1V, {len(problems) - n1} 2D2V), "
                               "N per dim from {32,48,64,96,128}, tol 1e-6, rmax 40, dt 0.1, CF3, FP32 tables",
                   "tuned": tuned, "tune_seconds": t_tune,
                   "cross_ms_per_step": tim["cross_ms"] / steps,
                   "graph_chunks_per_step": tim["chunks"] / steps,
                   "host_phase_ms_per_step": {k: 1e3 * v / steps for k, v in b.tphase.items()}},
        "roofline": roof,
        "cpu_baseline": None,
    }
    del b
    torch.cuda.synchronize()
    if cpu_seconds:
        out["cpu_baseline"] = cpu_baseline_batched(problems, cpu_seconds)
    return out


def batched_main(args):
    out = batched_run(args, args.steps, args.warmup, None if args.no_cpu_baseline else args.cpu_seconds / 3.0)
    print(json.dumps(out))


def nested_main(args):
    """Nested HT cross against HTACA on one SL-FD update of a 2D2V workload
    (--nested-config, default strong Landau; 128^4 unless --n): the state
    after two steps of the workload, the first CF3 sub-flow of the next
    step (RK4 frozen-field feet, tau = dt / 3, the state's own field).
    HTACA (slar_cross_update, rank cap 60) and the nested cross
    (slar_nested_cross, rank cap 64, 64 seeded probes) both sample through
    the same frame tables (--nested-dtype; auto: FP64 below tol 1e-5, where
    FP32 table noise exceeds the probe threshold, else FP32); each is timed with events on the stream (three runs
    after one warm-up, the median reported), and its approximation is
    compared with the exact update (FP64 tables) at 4096 seeded random
    entries.  One JSON line."""
    import torch
    import slar_inputs as SI
    from paper_2606_29027_amd import lib as L
    from paper_2606_29027_amd.solver import Solver
    n = args.n
    p = SI.config(args.nested_config, n=n)
    Nx = n * n
    s = Solver(p, L.F32, probes=SI.probe_indices(Nx, Nx, 64, 1234), precond=1)
    s.set_initial(SI.initial_ht(p))
    for _ in range(2):
        s.step()
    src = s.state
    E1 = s.efield(src, s.E[0]).clone()
    adv = L.make_adv(2, p.dt / 3.0, 1.0, E1)
    g, ws = s.grid, s.ws
    rng = np.random.default_rng(4321)
    probes4 = np.stack([rng.integers(0, n, 64) for _ in range(4)], 1).astype(np.int32)
    seed = (0, 0, n // 2, n // 2)
    kmax = 64
    T = {"leaves": [torch.zeros(n * kmax, dtype=torch.float64, device="cuda") for _ in range(4)],
         "B12": torch.zeros(kmax ** 3, dtype=torch.float64, device="cuda"),
         "B34": torch.zeros(kmax ** 3, dtype=torch.float64, device="cuda"),
         "root": torch.zeros(kmax ** 2, dtype=torch.float64, device="cuda")}
    H = L.HT()
    H.d, H.dtype = 4, L.F64
    for m in range(4):
        H.leaf[m] = T["leaves"][m].data_ptr()
    H.B12, H.B34, H.root = T["B12"].data_ptr(), T["B34"].data_ptr(), T["root"].data_ptr()

    def timed(fn):
        fn()
        ms = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            out = fn()
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return sorted(ms)[1], out

    dt = {"f32": L.F32, "f64": L.F64}.get(args.nested_dtype, L.F64 if p.tol < 1e-5 else L.F32)
    ms_h, (lr, ih, sth) = timed(lambda: L.slar_cross_update(g, src, adv, dt, p.tol, 60, s.probes, s.U, s.V, ws))
    ms_n, (inn, stn) = timed(lambda: L.slar_nested_cross(g, src, adv, dt, p.tol, kmax, probes4, seed, H, ws))
    # accuracy at random entries against the exact update (FP64 tables)
    idx = SI.random_requests(p.n, 4096, seed=99)
    idx_d = torch.as_tensor(idx, dtype=torch.int32, device="cuda")
    exact = torch.zeros(4096, dtype=torch.float64, device="cuda")
    L.slar_frame_sample(g, src, adv, L.F64, idx_d, exact, ws)
    I = torch.as_tensor(idx[:, 0] * n + idx[:, 1], device="cuda")
    J = torch.as_tensor(idx[:, 2] * n + idx[:, 3], device="cuda")
    k = lr.k
    approx_h = (s.U[:k][:, I] * s.V[:k][:, J]).sum(0)
    approx_n = torch.zeros(4096, dtype=torch.float64, device="cuda")
    L.slar_ht_sample(g, H, L.make_adv(0, 0.0), idx_d, approx_n)
    torch.cuda.synchronize()
    rel = lambda a: float(torch.linalg.norm(a - exact) / torch.linalg.norm(exact))   # noqa: E731
    print(json.dumps({
        "workload": f"nested HT cross vs HTACA, one SL-FD update of the {args.nested_config} {n}^4 state "
                    "after two steps (first CF3 sub-flow), %s tables, tol %g" % ("FP64" if dt == L.F64 else "FP32",
                                                                                  p.tol),
        "htaca": {"ms": ms_h, "samples": int(ih.samples), "rank": int(ih.rank), "converged": int(ih.converged),
                  "status": int(sth), "rel_err_4096": rel(approx_h)},
        "nested": {"ms": ms_n, "samples": int(inn.samples), "ranks": list(inn.rank), "sweeps": int(inn.sweeps),
                   "probe_rounds": int(inn.probe_rounds), "converged": int(inn.converged), "status": int(stn),
                   "rel_err_4096": rel(approx_n)}}))
    return 0


def sampler_case(r, steps, p=None, E=None, idx=None):
    """Entry-evaluation rates of a random HT of uniform rank r on the 128^4
    grid (orthonormal leaves, Gaussian transfer tensors, seed 1000 + r),
    2^20 uniform random requests (seed 1234), the first sub-flow of the
    strong-Landau workload: the leaf-to-root contraction (slar_ht_sample,
    matrix cores) and the frame-table sampler (slar_frame_sample, its FP64
    -> table copy included), FP32 and FP64, timed with HIP events on the
    launch stream.  Returns one record per (sampler, dtype)."""
    import torch
    import slar_inputs as SI
    from paper_2606_29027_amd import lib as L
    from paper_2606_29027_amd.solver import Solver
    if p is None:
        p = SI.config("stronglandau2d", n=128)
    if E is None:
        s0 = Solver(p, L.F64)              # field of the initial state, by the library's Poisson solve
        s0.set_initial(SI.initial_ht(p))
        E = s0.efield(s0.state, s0.E[0]).clone()
        del s0
    S = 1 << 20
    if idx is None:
        idx = torch.as_tensor(SI.random_requests(p.n, S, seed=1234), dtype=torch.int32, device="cuda")
    g = L.make_grid(p)
    ws = L.Workspace(g, 64)
    adv = L.make_adv(2, p.dt / 3.0, 1.0, E)
    Nx = 128 * 128

    def timed(fn):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / steps

    F = SI.random_ht(4, p.n, (r,) * 6, seed=1000 + r)
    T64 = {"leaves": [torch.as_tensor(U, device="cuda") for U in F["leaves"]],
           "root": torch.as_tensor(F["root"], device="cuda"),
           "B12": torch.as_tensor(F["B12"].reshape(r * r, r), device="cuda"),
           "B34": torch.as_tensor(F["B34"].reshape(r * r, r), device="cuda")}
    H64 = L.make_ht(T64, 4, L.F64)
    X = torch.zeros(Nx, 72, dtype=torch.float64, device="cuda")
    P = torch.zeros(Nx, 72, dtype=torch.float64, device="cuda")
    Fr = L.slar_frames_from_ht(g, H64, L.frames(X, P, 0), ws)
    out_recs = []
    for prec in ("f32", "f64"):
        tdt = torch.float32 if prec == "f32" else torch.float64
        T = {k: ([x.to(tdt) for x in v] if isinstance(v, list) else v.to(tdt)) for k, v in T64.items()}
        H = L.make_ht(T, 4, L.F32 if prec == "f32" else L.F64)
        out = torch.zeros(S, dtype=tdt, device="cuda")
        dt = timed(lambda: L.slar_ht_sample(g, H, adv, idx, out))
        flops = 2.0 * (4 * 3 * r + 2 * r ** 3 + r * r) * S
        out_recs.append({"sampler": "ht_contraction", "dtype": prec, "rank": r, "entries": S,
                         "entries_per_s": S / dt, "ms": 1e3 * dt, "tflops": flops / dt / 1e12,
                         "frac_of_mfma_peak": flops / dt / 1e12 / MFMA_PEAK_TFLOPS[prec]})
        outd = torch.zeros(S, dtype=torch.float64, device="cuda")
        dtc = L.F32 if prec == "f32" else L.F64
        dt = timed(lambda: L.slar_frame_sample(g, Fr, adv, dtc, idx, outd, ws))
        ldt = (r + 3) & ~3
        by = S * (2.0 * 9 * ldt * (4 if prec == "f32" else 8) + 8 + 16)
        out_recs.append({"sampler": "frame_tables", "dtype": prec, "rank": r, "entries": S,
                         "entries_per_s": S / dt, "ms": 1e3 * dt, "gather_GBps": by / dt / 1e9})
    return out_recs


def samplers_main(args):
    """Entry-evaluation microbenchmark on the 128^4 grid (sampler_case) for
    ranks 8 to 60; prints one JSON line per case: entries/s, and the
    contraction's flops against the dense matrix-core peak of its dtype, or
    the tables' algorithmic gather bytes (mostly L2 hits: 2 x 2.4 MB tables
    at r = 60) per second."""
    import torch
    import slar_inputs as SI
    from paper_2606_29027_amd import lib as L
    from paper_2606_29027_amd.solver import Solver
    p = SI.config("stronglandau2d", n=128)
    s0 = Solver(p, L.F64)
    s0.set_initial(SI.initial_ht(p))
    E = s0.efield(s0.state, s0.E[0]).clone()
    del s0
    idx = torch.as_tensor(SI.random_requests(p.n, 1 << 20, seed=1234), dtype=torch.int32, device="cuda")
    for r in (8, 16, 24, 32, 40, 48, 60):
        for rec in sampler_case(r, args.steps, p, E, idx):
            print(json.dumps(rec), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU runs are not part of this build",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        return batched_main(args)
    if args.workload == "nested":
        return nested_main(args)
    if args.workload == "samplers":
        return samplers_main(args)
    import torch
    import slar_inputs as SI
    from paper_2606_29027_amd import lib as L
    from paper_2606_29027_amd.solver import Solver

    p = SI.config("stronglandau2d", n=args.n)
    Nx = int(np.prod(p.n[: p.dx])); Nv = int(np.prod(p.n[p.dx:]))
    probes = SI.probe_indices(Nx, Nv, 64, 1234)
    prec = L.F32 if args.precision == "f32" else L.F64
    pc_code = {"plain": 0, "spectral": 1, "learned": 2}
    if args.calib_copy_mib > 0:
        a = torch.ones(args.calib_copy_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    def run_variant(name, vprec, steps, warmup):
        cnn = None
        if name == "learned":
            from paper_2606_29027_amd import cnn as CNN
            cnn = CNN.load_trained(p)
        s = Solver(p, vprec, probes=probes, precond=pc_code[name], cnn=cnn, strict=False)
        s.set_initial(SI.initial_ht(p))
        for _ in range(warmup):
            s.step()
        torch.cuda.synchronize()
        n0 = len(s.stats)
        infos = []
        # every 8th cross iteration carries dispatch events: the average
        # kernel duration without the ~2 ms per step that timing every
        # dispatch adds to the pipeline
        L.slar_timing_enable(s.ws, True, every=8)
        s.tphase = {k: 0.0 for k in s.tphase}
        step_ms = []
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            infos.append(s.step())          # ends with a device synchronisation
            step_ms.append(1e3 * (time.perf_counter() - ts))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        nconv = sum(1 for i in infos if i.get("converged"))
        if nconv < len(infos):
            print(f"bench.py: {name}: {len(infos) - nconv} of {len(infos)} timed steps did not reach the "
                  "Newton tolerance", file=sys.stderr, flush=True)
        tim = L.slar_timing_read(s.ws)
        L.slar_timing_enable(s.ws, False)
        samples = sum(st["samples"] for st in s.stats[n0:])
        # fiber-kernel time of all iterations: sampled average per launch
        # times the iterations that ran
        n_it = sum(st["iters"] for st in s.stats[n0:])
        per_it = (tim["row_ms"] / max(tim["row_launches"], 1) + tim["col_ms"] / max(tim["col_launches"], 1))
        kern_s = n_it * per_it * 1e-3
        phase = {k: 1e3 * v / steps for k, v in s.tphase.items()}
        phase["other"] = 1e3 * elapsed / steps - sum(phase.values())
        rec = {"value": samples / elapsed, "ms_per_step": 1e3 * elapsed / steps,
               "median_ms_per_step": float(np.median(step_ms)),
               "converged_steps": nconv, "timed_steps": len(infos),
               "t_end": round((warmup + steps) * p.dt, 6),
               "samples_per_step": samples / steps,
               "entries_per_s_cross": samples / (s.tphase["cross"] or float("nan")),
               "entries_per_s_fiber_kernels": samples / kern_s if kern_s > 0 else None,
               "phase_ms_per_step": phase,
               "newton_krylov": [[i.get("newton"), i.get("krylov")] for i in infos],
               "ranks": [st["ranks"] for st in s.stats[-3:]], "timing": tim}
        del s
        return rec

    runs = {}
    for name in [v for v in args.variants.split(",") if v]:
        runs[name] = run_variant(name, prec, args.steps, args.warmup)
    head = [v for v in args.variants.split(",") if v][-1]
    H = runs[head]
    tim = H.pop("timing")
    for r in runs.values():
        r.pop("timing", None)
    # dominant sampling kernel: whichever fiber kernel took more time
    which = "row" if tim["row_ms"] >= tim["col_ms"] else "col"
    ms, nl, by = tim[which + "_ms"], tim[which + "_launches"], tim[which + "_bytes"]
    achieved = (by / nl) / (ms / nl * 1e-3) / 1e9 if nl > 0 and ms > 0 else 0.0
    traffic = measured_traffic() if which == "col" else None
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": traffic,
                "kernel": "k_aca_row" if which == "row" else "k_aca_col",
                "avg_launch_us": 1e3 * ms / nl if nl else None, "launches": int(nl),
                "algorithmic_bytes_per_launch": by / nl if nl else None}
    if traffic and nl and ms > 0:
        # the counters' HBM bytes over the same launch time: most of the
        # algorithmic gather bytes hit the L1 and L2 caches, so the kernel is
        # bound by the latency of its dependent phases, not by HBM bandwidth
        hbm = traffic / (ms / nl * 1e-3) / 1e9
        roofline["hbm_measured_GBps"] = hbm
        roofline["hbm_measured_frac"] = hbm / HBM_PEAK_GBS
        # share of the gathered bytes served by the L1/L2 caches (the rest is HBM)
        roofline["cache_share_of_algorithmic_bytes"] = 1.0 - traffic / (by / nl)
        roofline["limiter"] = "latency of dependent phases (gathers served from the L1/L2 caches)"
    out = {
        "metric": "HT-SL sampled entries/s & time/step, 2D2V 128^4, learned vs plain at 1e-6",
        "value": H["value"],
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": H["ms_per_step"],
        "median_ms_per_step": H["median_ms_per_step"],
        "all_converged": H["converged_steps"] == H["timed_steps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == L.F32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"2D2V strong Landau alpha=0.5 k=0.5, {p.n[0]}^4, tol 1e-5, rmax 60, "
                               f"dt 0.2, CF3 + LoMaC/JFNK (BDF2), macro solver: {head}",
                   "variants": runs},
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not args.no_other_precision:
        # the same step with the other table precision (the headline macro
        # solver), a shorter run
        other = L.F64 if prec == L.F32 else L.F32
        o = run_variant(head, other, 3, 2)
        o.pop("timing", None)
        o["dtype"] = "f64" if other == L.F64 else "f32"
        out["config"]["other_precision"] = {k: o[k] for k in ("dtype", "value", "ms_per_step", "median_ms_per_step",
                                                              "converged_steps", "timed_steps", "t_end",
                                                              "samples_per_step", "entries_per_s_cross",
                                                              "entries_per_s_fiber_kernels", "phase_ms_per_step",
                                                              "newton_krylov")}
    if not args.no_samplers:
        # the entry samplers at the workload's rank cap (r = 60): the
        # paper's leaf-to-root contraction on the matrix cores and the
        # frame-table gathers, FP32 and FP64
        out["config"]["samplers_r60"] = sampler_case(60, 10)
    if not args.no_batched:
        # the batched-instances workload, measured in the same run
        b = batched_run(args, args.batched_steps, 1, None if args.no_cpu_baseline else args.cpu_seconds / 3.0)
        out["config"]["batched"] = {k: b[k] for k in ("metric", "value", "unit", "steps", "warmup", "ms_per_step",
                                                      "dtype", "config", "roofline", "cpu_baseline")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
