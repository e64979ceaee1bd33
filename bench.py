"""Benchmark: KKT solves per second of the all-at-once Stokes control problem.

One step = one complete solve of A x = b (eq. FinalA) to a true relative
residual of 1e-8 with flexible GMRES preconditioned by the block-circulant
preconditioner with per-frequency inner GMRES (Algorithm 2), on the
N = 128 quads, nt = 256, T = 1, nu = 1, beta = 1e-4 Stokes workload (75.1M
unknowns, inputs resident in HBM before timing starts).

Prints one JSON line (see the keys below).  ``--gpus`` above 1 is refused:
this build runs on one GPU.

``--config 4`` measures the batched form instead: the 64-problem mix of
``workloads.batch_mix`` (N in {32, 64, 128}, nt in {32, ..., 256}, log-uniform
beta, nu in {1, 1/50, 1/100}, Stokes and Oseen) solved with FP32 inner /
FP64 outer solves by the concurrent runner of ``paper_2405_18964_amd.batch``;
one step = one pass over the whole mix, value = aggregate solves/s.

``--config 5`` measures the served form: the Poisson request stream of
``workloads.serve_stream`` (``--requests`` requests, N capped by
``--serve-max-n``).  A closed-loop pass (all requests at once) measures the
capacity C; the timed open-loop pass releases request k at its arrival time
scaled to the rate rho * C (``--rho``) and reports p50/p99 arrival-to-
completion latency beside solves/s.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# The roofline kernel: the finest-grid post-smoothing sweep of the velocity
# multigrid (the largest share of device time in the Stokes solve);
# template arguments <arithmetic, convection table, forward sweep, prolongation>.


def sweep_kernel(fp64: bool, oseen: bool) -> str:
    return f"k_q2_sweep<{'double' if fp64 else 'float'},{'true' if oseen else 'false'},false,true>"


# HBM traffic of that kernel from two rocprofv3 --pmc passes over one solve of
# this workload (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch at the finest
# grid), each scaled by what the same counter reads for a 1 GiB device copy in
# the same process.  Valid only for the kernel source they were taken on:
# reported as null once that file changes (or before they are taken).
SWEEP_SOURCE = os.path.join(ROOT, "paper_2405_18964_amd", "csrc", "q2_tiles.hip")
SWEEP_PMC = {"kernel": "k_q2_sweep<double,false,false,true>",
             "source_sha256": "2e972e25d279af992d70cb6a44fbf622b8d1c0048c0d6ad1b8b2b9f983a0b544",
             "fetch_kib": 468560.3, "fetch_scale": 2.0, "write_kib": 422822.4, "write_scale": 1.0}


def sweep_traffic_bytes(kernel=None):
    import hashlib
    if SWEEP_PMC is None or (kernel is not None and kernel != SWEEP_PMC["kernel"]):
        return None
    with open(SWEEP_SOURCE, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != SWEEP_PMC["source_sha256"]:
            return None
    return 1024.0 * (SWEEP_PMC["fetch_kib"] * SWEEP_PMC["fetch_scale"] + SWEEP_PMC["write_kib"] * SWEEP_PMC["write_scale"])


def method_precond_bytes(w, csize: int, n_all: int) -> float:
    """Algorithmic bytes of one linear preconditioner application counted
    per pass of the unfused method (every pass a separate sweep over its
    fields): a V(1,1) cycle is 10.5 field passes per level (smoothing 3,
    residual/restriction 2.25, prolongation/correction 2.25, smoothing 3)
    times 4/3 for the hierarchy, four cycles 56; ten Chebyshev steps 40; the
    time FFT pair reads and writes the canonical vector twice (4 n_all
    doubles).  Per kept frequency, in fields of interior nodes (a velocity
    field: two components; complex entries of csize bytes):
      Stokes (Algorithm 1): 2 x 56 velocity + 2 x (56 + 40 + 3) pressure;
      Oseen (Algorithm 3):  6 Uzawa steps x 167 velocity + 2 velocity + 201 pressure.
    The library's own byte model counts the passes as implemented (the
    prolongation fused into the post-smoothing load, the first cycle's
    pre-smoothing reading no x), which is what HBM actually moves."""
    import workloads as W
    nf = w.nt // 2 + 1
    nv = (2 * w.N - 1) ** 2                 # interior Q2 nodes per component
    npr = (w.N + 1) ** 2                    # Q1 nodes
    vf, pf = 2 * nv * csize, npr * csize    # one velocity field, one pressure field
    if w.flow == W.STOKES:
        per = 2 * 56 * vf + 2 * (56 + 40 + 3) * pf
    else:
        per = (6 * (4 + 42 + 4 + 56 + 2 + 56 + 3) + 2) * vf + (80 + 6 + 112 + 3) * pf
    return nf * per + 4.0 * n_all * 8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 3; 1 for --config 4 and 5)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2,
                    help="workload: 1, 2 (single Stokes problem), 3 (single Oseen problem), "
                         "4 (batched 64-problem mix) or 5 (served request stream)")
    ap.add_argument("--batch-count", type=int, default=64, help="problems of the batched mix (--config 4)")
    ap.add_argument("--workers", type=int, default=4, help="concurrent problems on the device (--config 4, 5)")
    ap.add_argument("--fused-workers", type=int, default=4, help="concurrent fused groups (--config 4)")
    ap.add_argument("--requests", type=int, default=256, help="requests of the served stream (--config 5)")
    ap.add_argument("--rho", type=str, default="0.8",
                    help="comma-separated arrival rates / capacity, one open-loop pass each (--config 5)")
    ap.add_argument("--capacity", type=float, default=None,
                    help="--config 5: capacity in solves/s measured earlier (skips the closed-loop pass)")
    ap.add_argument("--slice-cycles", type=int, default=1,
                    help="--config 5: FGMRES restart cycles per turn before a slot is recycled (0: whole solves)")
    ap.add_argument("--serve-max-n", type=int, default=256, help="largest grid of the served stream (--config 5)")
    ap.add_argument("--z-fp32", action="store_true",
                    help="--config 4, 5: keep the outer FGMRES basis in FP32 (options.z_fp32)")
    ap.add_argument("--stokes-inner", choices=["gmres", "minres"], default="gmres",
                    help="--config 4, 5: inner solver of the Stokes jobs (the Oseen jobs keep GMRES)")
    ap.add_argument("--graphs", action="store_true",
                    help="--config 4, 5: replay block preconditioner applications from HIP graphs (options.graphs)")
    ap.add_argument("--compare", action="store_true",
                    help="--config 4: also solve the mix one problem at a time (FP32-inner and FP64)")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default=None,
                    help="inner arithmetic of the timed solves (default: fp64 for Stokes, fp32 for Oseen)")
    ap.add_argument("--inner", choices=["gmres", "linear", "minres"], default="gmres",
                    help="inner treatment of the frequency blocks: GMRES (Algorithm 2), one application of the "
                         "linear preconditioner (Algorithm 1, outer GMRES(30)), or MINRES on the Stokes blocks")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precond-reps", type=int, default=5)
    ap.add_argument("--no-fp32", action="store_true", help="skip the solve in the other precision mode")
    ap.add_argument("--no-minres", action="store_true", help="skip the extra MINRES (Algorithm 1) solve")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one device copy of 1 GiB first (reference for HBM byte counters)")
    return ap.parse_args()


def _host_cores() -> int:
    """Cores this process may use on the host (the CPU share of one GPU is at
    most 16 cores on the GPU hosts), whatever the machine's total."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_block_worker(args):
    """One pool worker: the oracle's nonlinear block solve of frequency j
    (Algorithm 2 / its Oseen analogue: T transforms, inner GMRES with the
    block preconditioner, the block matvec and Gram-Schmidt) capped at one
    inner iteration, on one BLAS thread.  Returns (seconds, applications of
    the block preconditioner and block matrix it made)."""
    w, j = args
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle.kkt import Problem as OP
    from oracle.precond import OseenPreconditioner, Settings, StokesPreconditioner

    with threadpool_limits(limits=1):
        wind = W.wind_nodal(w.N) if w.flow == W.OSEEN else None
        op = OP.from_workload(w, wind)
        st = Settings(inner_maxit=1, inner_restart=1)
        if w.flow == W.STOKES:
            pc = StokesPreconditioner(op, st, freqs=[j])
            pc.W_mg(j)                                  # multigrid set-up outside the timing
        else:
            pc = OseenPreconditioner(op, wind, st, freqs=[j])
            pc.Q_mgs(j)
        rng = np.random.default_rng(j)
        r = [rng.standard_normal(n) + 1j * rng.standard_normal(n) for n in (op.nv, op.nv, op.nP, op.nP)]
        t0 = time.perf_counter()
        pc.block_apply(j, *r, nonlinear=True)
        # GMRES capped at one iteration: one Arnoldi step (preconditioner,
        # block matrix, Gram-Schmidt), the update through the preconditioner
        # and the residual through the block matrix
        return time.perf_counter() - t0, 2


def cpu_sample(w) -> dict:
    """Time the FP64 oracle on the host, before the GPU is touched.

    The per-frequency block solves are the oracle's parallel part (the paper
    distributes frequency blocks over processes, section 5.3): one pool worker
    per host core, each timing one frequency's nonlinear block solve capped at
    one inner iteration, all workers at once so they share memory bandwidth as
    a full run would.  The serial parts -- the time FFT pair over the whole
    vector, one all-at-once matvec and one step of the outer modified
    Gram-Schmidt -- are timed after the pool on one core."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import circulant as circ
    from oracle.kkt import Problem as OP

    cores = _host_cores()
    nf = w.nt // 2 + 1
    js = sorted({int(round(i * (nf - 1) / max(cores - 1, 1))) for i in range(cores)})
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(len(js)) as pool:
        res = pool.map(_oracle_block_worker, [(w, j) for j in js], chunksize=1)
    t_pool = time.perf_counter() - t0
    t_app = float(np.mean([t / k for t, k in res]))     # one block preconditioner + block matvec, under load
    with threadpool_limits(limits=1):
        op = OP.from_workload(w, W.wind_nodal(w.N) if w.flow == W.OSEEN else None)
        x = np.random.default_rng(0).standard_normal(2 * op.nt * op.n)
        t1 = time.perf_counter()
        circ.time_ifft(op, circ.time_fft(op, x))
        t_fft = time.perf_counter() - t1
        t1 = time.perf_counter()
        y = op.kkt_apply(x)
        t_mv = time.perf_counter() - t1
        t1 = time.perf_counter()
        hdot = np.vdot(x, y)
        y -= hdot * x
        t_mgs = time.perf_counter() - t1
    return {"cores": cores, "cpu_model": _cpu_model(), "t_block_app": t_app, "t_fft_pair": t_fft,
            "t_matvec": t_mv, "t_mgs_step": t_mgs, "frequencies_sampled": js, "pool_seconds": t_pool,
            "seconds_measured": t_pool + t_fft + t_mv + t_mgs}


def cpu_baseline(w, smp: dict, outer_its: int, inner_mean: float, restart: int = 10) -> dict:
    """Oracle solves/s extrapolated from the sample: per outer iteration the
    oracle's preconditioner transforms the vector, solves all nt frequency
    blocks (it does not use the conjugate symmetry of real data) with
    inner_mean + 1 block preconditioner and block matrix applications each,
    spread over the pool, and makes one all-at-once matvec and a Gram-Schmidt
    step against half a restart cycle's basis on average; plus the final
    residual."""
    cores = smp["cores"]
    waves = math.ceil(w.nt / cores)
    per_outer = (smp["t_fft_pair"] + waves * (inner_mean + 1.0) * smp["t_block_app"] + smp["t_matvec"]
                 + (restart + 1) / 2.0 * smp["t_mgs_step"])
    t_solve = outer_its * per_outer + smp["t_matvec"]
    kind = "Stokes (Algorithm 2)" if w.flow == 0 else "Oseen (Algorithm 3 inside GMRES)"
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "cpu_model": smp["cpu_model"], "extrapolated": True,
            "sample": (f"FP64 oracle on {cores} host cores ({smp['cpu_model']}): {len(smp['frequencies_sampled'])} "
                       f"per-frequency {kind} block solves of the N={w.N}, nt={w.nt} workload in a process pool "
                       f"(one inner iteration each: {smp['t_block_app']:.2f} s per block preconditioner + block "
                       f"matrix application under full load), one time-FFT pair ({smp['t_fft_pair']:.2f} s), "
                       f"all-at-once matvec ({smp['t_matvec']:.2f} s) and Gram-Schmidt step "
                       f"({smp['t_mgs_step']:.2f} s) on one core; extrapolated to {outer_its} outer iterations x "
                       f"{w.nt} frequency blocks x ({inner_mean:.1f} inner + 1) applications over {cores} cores"),
            "seconds_measured": smp["seconds_measured"], "seconds_per_solve": t_solve}


def _pct(lat, q):
    s = sorted(lat)
    return s[min(len(s) - 1, max(0, int(math.ceil(q * len(s))) - 1))]


def _timed_solve(gp, b, x):
    """One solve from x = 0 timed with host clocks around a synchronised
    call; returns (seconds, stats, converged)."""
    import torch
    x.zero_()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, st, ok = gp.solve(b, x)
    torch.cuda.synchronize()
    return time.perf_counter() - t1, st, ok


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Device-to-device copy of `nbytes` (read + write = 2 x nbytes of HBM
    traffic), timed with events after one untimed copy: the attainable
    streaming rate that the roofline kernel's fraction is also read against."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"GBs": 2 * nbytes / (ms * 1e-3) / 1e9, "bytes_per_copy": 2 * nbytes, "avg_ms": ms, "reps": reps,
            "frac_of_peak": 2 * nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def main():
    args = parse()
    if args.steps is None:
        args.steps = 1 if args.config in (4, 5) else 3
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (no multi-GPU path)"}))
        sys.exit(2)
    import workloads as W

    if args.config not in (4, 5):
        w = W.config(args.config)
        # the oracle sample runs first, in forked workers, before the GPU is touched
        smp = None if args.no_cpu_baseline else cpu_sample(w)
    import numpy as np
    import torch

    import paper_2405_18964_amd as P

    if args.config == 4:
        return bench_batch(args)
    if args.config == 5:
        return bench_serve(args)
    precision = args.precision or ("fp32" if w.flow == W.OSEEN else "fp64")
    prec = P.PREC_FP64 if precision == "fp64" else P.PREC_FP32_INNER
    inner = {"gmres": P.INNER_GMRES, "linear": P.INNER_LINEAR, "minres": P.INNER_MINRES}[args.inner]
    flow = "Stokes" if w.flow == W.STOKES else "Oseen"
    solver_opts = dict(inner=inner, max_outer=400 if args.inner == "linear" else 60,
                       restart=30 if args.inner == "linear" else 10)
    gp = P.Problem.from_workload(w, precision=prec, **solver_opts)
    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    vd = torch.from_numpy(W.desired_state(w)).cuda()
    b = gp.assemble_rhs(vd)
    x = gp.empty()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    ws_main = gp.workspace_bytes
    print(f"[bench] {w.name} n_all={gp.n_all} workspace={gp.workspace_bytes / 1e9:.1f} GB", file=sys.stderr,
          flush=True)
    for i in range(args.warmup):
        x.zero_()
        _, st, ok = gp.solve(b, x)
        print(f"[bench] warmup {i}: {st['outer_iterations']} its, {st['seconds']:.2f} s", file=sys.stderr,
              flush=True)
    lat, stats = [], []
    gp.profile_enable(True)          # HIP events around the finest-grid smoother launches
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        x.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _, st, ok = gp.solve(b, x)
        e1.record(stream)
        e1.synchronize()
        if not ok:
            raise SystemExit(f"solve did not converge: {st}")
        lat.append(e0.elapsed_time(e1) / 1e3)
        stats.append(st)
        print(f"[bench] step {i}: {st['outer_iterations']} its, inner mean {st['inner_iterations_mean']:.1f}, "
              f"{lat[-1]:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if w.N > 16:
        kt = gp.profile_read()
    else:                            # no finest-grid tile sweeps to time (one-launch small V-cycle)
        kt = {"avg_ms": 0.0, "launches": 0, "algorithmic_bytes": 0.0,
              "post": {"avg_ms": 0.0, "launches": 0, "algorithmic_bytes": 0.0}}
    gp.profile_enable(False)
    # independent check of the last solution: true residual through the KKT matvec
    rel = float(torch.linalg.norm(b - gp.kkt_apply(x)) / torch.linalg.norm(b))
    x_main = x.clone()
    # linear preconditioner application (Algorithm 1 / Algorithm 3): model bytes / time
    lp = P.Problem.from_workload(w, inner=P.INNER_LINEAR, precision=prec)
    z = lp.empty()
    lp.precond_apply(b, z)
    torch.cuda.synchronize()
    pc_lat = []
    for _ in range(args.precond_reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lp.precond_apply(b, z)
        e1.record(stream)
        e1.synchronize()
        pc_lat.append(e0.elapsed_time(e1) / 1e3)
    t_pc = sum(pc_lat) / len(pc_lat)
    pc_bytes = stats[-1]["precond_model_bytes"]
    mb_pc = method_precond_bytes(w, 16 if precision == "fp64" else 8, gp.n_all)
    del lp, z
    outer = int(np.mean([s["outer_iterations"] for s in stats]))
    inner_mean = float(np.mean([s["inner_iterations_mean"] for s in stats]))
    phases = {k: float(np.mean([s["phase_seconds"][k] for s in stats])) for k in P.PHASES}
    out = {
        "metric": "KKT solves/sec to 1e-8 residual and preconditioner-apply HBM GB/s; p50/p99",
        "value": args.steps / wall,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32-inner/f64-outer",
        "data": "synthetic",
        "config": {"workload": f"{flow} control, Q2-Q1 on {w.N}x{w.N} quads of the unit square, nt={w.nt}, "
                               f"T={w.T}, nu={w.nu:g}, beta={w.beta:g}"
                               + (", wind w=(2y(1-x^2), -2x(1-y^2))" if w.flow == W.OSEEN else "")
                               + f", {gp.n_all} unknowns (canonical)",
                   "solver": f"FGMRES({solver_opts['restart']}) + block-circulant preconditioner, "
                             f"inner={args.inner}" + (", coarse-level viscosity on the Q_j multigrid"
                                                       if w.flow == W.OSEEN else ""),
                   "precision": precision},
        "latency_s": {"p50": _pct(lat, 0.5), "p99": _pct(lat, 0.99), "all": lat},
        "iterations": {"outer": outer, "inner_mean": inner_mean,
                       "inner_max": int(max(s["inner_iterations_max"] for s in stats))},
        "final_rel_residual": rel,
        "phase_seconds": phases,
        "solve_model_bytes": float(np.mean([s["model_bytes"] for s in stats])),
        "precond_apply": {"ms": 1e3 * t_pc, "p50_ms": 1e3 * _pct(pc_lat, 0.5), "p99_ms": 1e3 * _pct(pc_lat, 0.99),
                          "model_bytes": pc_bytes, "model_GBs": pc_bytes / t_pc / 1e9,
                          "frac_of_hbm_peak": pc_bytes / t_pc / 1e9 / HBM_PEAK_GBS,
                          "method_model_bytes": mb_pc, "method_model_GBs": mb_pc / t_pc / 1e9,
                          "method_model_frac": mb_pc / t_pc / 1e9 / HBM_PEAK_GBS,
                          "note": "model_bytes: passes as implemented (what HBM moves); method_model_bytes: the "
                                  "unfused method's passes (prolongation/correction and first-cycle x reads "
                                  "counted), the same work"},
    }
    post = kt["post"]
    cp = copy_bandwidth(torch)
    if post["launches"] == 0:
        # N <= 16: the whole velocity hierarchy runs in the one-launch small
        # V-cycle and the working set sits in the 256 MB Infinity Cache, so
        # the run reports latencies only (no HBM roofline fraction)
        note = "working set resident in the Infinity Cache (no finest-grid tile sweeps): latency only"
        out["precond_apply"].update(model_GBs=None, frac_of_hbm_peak=None, method_model_GBs=None,
                                    method_model_frac=None, note=note)
        out["roofline"] = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
                           "traffic": None, "note": note}
        out["hbm_copy"] = cp
    else:
        achieved = post["algorithmic_bytes"] / (post["avg_ms"] * 1e-3) / 1e9
        kname = sweep_kernel(precision == "fp64", w.flow == W.OSEEN)
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS,
                           "traffic": sweep_traffic_bytes(kname),
                           "kernel": kname + " (finest-grid post-smoothing sweep of the velocity multigrid "
                                     "with the prolonged coarse correction, all kept frequencies; the kernel with "
                                     "the largest share of device time)",
                           "avg_launch_ms": post["avg_ms"], "launches_timed": post["launches"],
                           "algorithmic_bytes_per_launch": post["algorithmic_bytes"]}
        out["hbm_copy"] = dict(cp, roofline_kernel_frac_of_copy=achieved / cp["GBs"])
        pre_gbs = kt["algorithmic_bytes"] / (kt["avg_ms"] * 1e-3) / 1e9
        out["pre_smoothing_sweep"] = {"avg_launch_ms": kt["avg_ms"], "launches_timed": kt["launches"],
                                      "algorithmic_bytes_per_launch": kt["algorithmic_bytes"],
                                      "achieved_GBs": pre_gbs, "frac": pre_gbs / HBM_PEAK_GBS}
    if not args.no_fp32:
        # the other precision mode on the same right-hand side, and the
        # difference of the two solutions (the FP32-inner result's error
        # against the FP64 form, both at the 1e-8 true residual)
        del gp
        torch.cuda.empty_cache()
        other = "fp32" if precision == "fp64" else "fp64"
        go = P.Problem.from_workload(w, precision=P.PREC_FP32_INNER if other == "fp32" else P.PREC_FP64,
                                     **solver_opts)
        _timed_solve(go, b, x)                       # warm-up
        t_o, st_o, ok_o = _timed_solve(go, b, x)
        r_o = float(torch.linalg.norm(b - go.kkt_apply(x)) / torch.linalg.norm(b))
        x32, x64 = (x, x_main) if other == "fp32" else (x_main, x)
        err = float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))
        out["fp32_inner" if other == "fp32" else "fp64_reference"] = {
            "solves_per_s": 1.0 / t_o, "seconds": t_o, "converged": bool(ok_o), "final_rel_residual": r_o,
            "outer": st_o["outer_iterations"], "inner_mean": st_o["inner_iterations_mean"]}
        out["fp32_inner_vs_fp64"] = {
            "rel_error_2norm": err,
            "note": "||x_fp32inner - x_fp64|| / ||x_fp64|| for this right-hand side; multigrid, Chebyshev, "
                    "Uzawa and inner GMRES in FP32, outer FGMRES, residuals and coarsest-grid inverses in FP64"}
        print(f"[bench] {other} solve: {st_o['outer_iterations']} its, {t_o:.2f} s, rel. difference {err:.2e}",
              file=sys.stderr, flush=True)
        del go
    if not args.no_minres and precision == "fp64" and w.flow == W.STOKES:
        # paper variant: MINRES with the linear preconditioner (Algorithm 1), FP64
        gm = P.Problem.from_workload(w, inner=P.INNER_LINEAR, outer=P.OUTER_MINRES, precision=P.PREC_FP64,
                                     max_outer=800)
        tm, stm, okm = _timed_solve(gm, b, x)
        rm = float(torch.linalg.norm(b - gm.kkt_apply(x)) / torch.linalg.norm(b))
        out["minres_linear_fp64"] = {"solves_per_s": 1.0 / tm, "seconds": tm, "converged": bool(okm),
                                     "final_rel_residual": rm, "iterations": stm["outer_iterations"],
                                     "note": "MINRES on the symmetric all-at-once matrix with the symmetric "
                                             "positive definite linear preconditioner (Algorithm 1), FP64"}
        print(f"[bench] MINRES + Algorithm 1 (FP64): {stm['outer_iterations']} its, {tm:.2f} s",
              file=sys.stderr, flush=True)
        del gm
    if not args.no_minres and precision == "fp64" and w.flow == W.STOKES and args.inner == "gmres":
        # paper variant: Algorithm 2 with MINRES in place of the inner GMRES, FP64
        gi = P.Problem.from_workload(w, inner=P.INNER_MINRES, precision=P.PREC_FP64, max_outer=60)
        _timed_solve(gi, b, x)                       # warm-up
        ti, sti, oki = _timed_solve(gi, b, x)
        ri = float(torch.linalg.norm(b - gi.kkt_apply(x)) / torch.linalg.norm(b))
        out["inner_minres_fp64"] = {"solves_per_s": 1.0 / ti, "seconds": ti, "converged": bool(oki),
                                    "final_rel_residual": ri, "outer": sti["outer_iterations"],
                                    "inner_mean": sti["inner_iterations_mean"],
                                    "workspace_GB": gi.workspace_bytes / 1e9,
                                    "workspace_GB_inner_gmres": ws_main / 1e9,
                                    "note": "FGMRES(10) with MINRES on the Stokes blocks Z_j (preconditioned by "
                                            "P~_j) in place of the inner GMRES of Algorithm 2, FP64"}
        print(f"[bench] inner MINRES (FP64): {sti['outer_iterations']} its, inner mean "
              f"{sti['inner_iterations_mean']:.1f}, {ti:.2f} s, workspace {gi.workspace_bytes / 1e9:.1f} GB",
              file=sys.stderr, flush=True)
        del gi
    if not args.no_minres and w.flow == W.STOKES:
        # the same solve with the pressure part of P~_j on a second stream
        go = P.Problem.from_workload(w, precision=prec, pressure_stream=1, **solver_opts)
        _timed_solve(go, b, x)                       # warm-up
        to, sto, oko = _timed_solve(go, b, x)
        same = bool(torch.equal(x, x_main))
        out["pressure_stream"] = {"solves_per_s": 1.0 / to, "seconds": to, "converged": bool(oko),
                                  "identical_to_value_solve": same,
                                  "note": "options.pressure_stream = 1: K_p multigrid and M_p Chebyshev on a second "
                                          "stream beside the velocity multigrid (same results)"}
        print(f"[bench] pressure part on a second stream: {to:.2f} s, identical {same}", file=sys.stderr, flush=True)
        del go
    if smp is not None:
        out["cpu_baseline"] = cpu_baseline(w, smp, outer, inner_mean, solver_opts["restart"])
    print(json.dumps(out), flush=True)


def _stokes_inner(args, w, P):
    """Per-job option overrides: the inner MINRES for Stokes jobs when asked."""
    return {"inner": P.INNER_MINRES} if args.stokes_inner == "minres" and w.flow == 0 else {}


def bench_batch(args):
    """Batched form: the 64-problem mix, fused (groups of the same grid and
    flow in one handle, group size and smoother per class from the
    autotuner), with --compare also the concurrent form (one problem per
    stream) and one problem at a time (FP32-inner and the plain FP64 form)."""
    import torch

    import paper_2405_18964_amd as P
    import workloads as W
    from paper_2405_18964_amd.batch import autotune, job_bytes, run, run_fused

    mix = W.batch_mix(args.batch_count)
    jobs = [{"N": w.N, "nt": w.nt, "T": w.T, "nu": w.nu, "beta": w.beta, "flow": w.flow,
             "wind": W.wind_nodal(w.N) if w.flow == W.OSEEN else None, "vd": W.desired_state(w),
             "options": _stokes_inner(args, w, P)} for w in mix]
    opts = dict(inner=P.INNER_GMRES, precision=P.PREC_FP32_INNER, max_outer=60, z_fp32=int(args.z_fp32),
                graphs=int(args.graphs))
    job_mem = sum(job_bytes(j, **opts) for j in jobs)
    print(f"[bench] batched mix of {len(jobs)} problems, {sum(w.n_all for w in mix) / 1e9:.2f}e9 unknowns, "
          f"{job_mem / 1e9:.0f} GB of job memory", file=sys.stderr, flush=True)
    small = sorted(range(len(jobs)), key=lambda k: job_bytes(jobs[k], **opts))[:args.workers]
    for i in range(args.warmup):                           # module loading, allocator warm-up
        run([jobs[k] for k in small], workers=args.workers, **opts)
    t0 = time.perf_counter()
    plan = autotune(jobs, **opts)
    t_tune = time.perf_counter() - t0
    for key, v in sorted(plan.items()):
        print(f"[bench] autotune N={key[0]} {'Oseen' if key[1] else 'Stokes'}: group size {v['size']}, "
              f"smoother {'global' if v['smoother'] else 'tiled'}", file=sys.stderr, flush=True)

    def progress(tag):
        def cb(k, r):
            print(f"[bench] {tag}: job {k} ({mix[k].name}, nt={mix[k].nt}) done at {r['end']:.2f} s"
                  f"{'' if r['converged'] else ' NOT CONVERGED'}", file=sys.stderr, flush=True)
        return cb

    walls, outs = [], []
    for i in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = run_fused(jobs, plan, workers=args.fused_workers, checksum=True, on_done=progress(f"fused {i}"), **opts)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        outs.append(out)
        print(f"[bench] fused step {i}: {walls[-1]:.2f} s, converged {sum(r['converged'] for r in out)}/{len(out)}",
              file=sys.stderr, flush=True)
    out = outs[-1]
    wall = sum(walls)
    lat = [r["end"] - r["start"] for r in out]
    res = {
        "metric": "KKT solves/sec to 1e-8 residual (batched mix, aggregate); p50/p99 per-solve latency",
        "value": len(jobs) * args.steps / wall,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-inner/f64-outer",
        "data": "synthetic",
        "config": {"workload": f"{len(jobs)} independent Stokes/Oseen control problems (N in {{32,64,128}}, "
                               "nt in {32,...,256}, log-uniform beta in [1e-6,1e-2], nu in {1,1/50,1/100})",
                   "solver": "FGMRES(10) + block-circulant preconditioner with inner GMRES per frequency; "
                             "fused groups of the same grid and flow (one batch of every per-frequency kernel, "
                             f"lockstep FGMRES), {args.fused_workers} groups concurrent"},
        "converged": int(sum(r["converged"] for r in out)),
        "latency_s": {"p50": _pct(lat, 0.5), "p99": _pct(lat, 0.99)},
        "autotune": {"seconds": t_tune,
                     "plan": {f"N{k[0]}_{'oseen' if k[1] else 'stokes'}": {"size": v["size"], "smoother":
                              "global" if v["smoother"] else "tiled", "fused_beats_side_by_side": v["fused_wins"]}
                              for k, v in sorted(plan.items())},
                     "trials": {f"N{k[0]}_{'oseen' if k[1] else 'stokes'}": {"fused": v["trials"],
                                                                            "side_by_side": v["concurrent"]}
                                for k, v in sorted(plan.items())}},
        "groups": len({r["group"] for r in out}),
        "job_memory_GB": job_mem / 1e9,
        "z_fp32": bool(args.z_fp32),
        "graphs": bool(args.graphs),
        "stokes_inner": args.stokes_inner,
    }
    if args.compare:
        for name, prec, workers in (("concurrent_fp32_inner", P.PREC_FP32_INNER, args.workers),
                                    ("sequential_fp32_inner", P.PREC_FP32_INNER, 1),
                                    ("sequential_fp64", P.PREC_FP64, 1)):
            o = dict(opts, precision=prec, z_fp32=opts["z_fp32"] if prec == P.PREC_FP32_INNER else 0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            seq = run(jobs, workers=workers, checksum=True, on_done=progress(name), **o)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            res[name] = {"solves_per_s": len(jobs) / t, "seconds": t, "workers": workers,
                         "converged": int(sum(r["converged"] for r in seq))}
            if name == "concurrent_fp32_inner":
                tiled = [k for k in range(len(jobs)) if plan[(jobs[k]["N"], jobs[k]["flow"])]["smoother"] == 0]
                res["fused_identical_to_concurrent"] = {
                    "tiled_classes": len(tiled),
                    "identical": int(sum(out[k]["digest"] == seq[k]["digest"] for k in tiled))}
            print(f"[bench] {name}: {t:.2f} s", file=sys.stderr, flush=True)
    print(json.dumps(res), flush=True)


def bench_serve(args):
    """Served form: Poisson arrivals at rho times the measured capacity,
    slots recycled at FGMRES restart boundaries (``--slice-cycles``)."""
    import torch

    import paper_2405_18964_amd as P
    import workloads as W
    from paper_2405_18964_amd.batch import run

    stream = W.serve_stream(args.requests, max_N=args.serve_max_n)

    def jobs_at(rate):
        return [{"N": w.N, "nt": w.nt, "T": w.T, "nu": w.nu, "beta": w.beta, "flow": w.flow,
                 "wind": W.wind_nodal(w.N) if w.flow == W.OSEEN else None, "vd": W.desired_state(w),
                 "arrival": (a / rate if rate else 0.0), "options": _stokes_inner(args, w, P)} for w, a in stream]
    opts = dict(inner=P.INNER_GMRES, precision=P.PREC_FP32_INNER, max_outer=60, z_fp32=int(args.z_fp32),
                graphs=int(args.graphs))

    def progress(tag):
        def cb(k, r):
            w = stream[k][0]
            print(f"[bench] {tag}: request {k} ({w.name}, nt={w.nt}) {r['end'] - r['arrival']:.2f} s after arrival, "
                  f"{r['slices']} turns", file=sys.stderr, flush=True)
        return cb

    closed = None
    if args.capacity:
        cap = args.capacity
    else:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        closed = run(jobs_at(None), workers=args.workers, checksum=True, slice_cycles=args.slice_cycles,
                     on_done=progress("closed loop"), **opts)
        cap = len(stream) / (time.perf_counter() - t0)
        print(f"[bench] closed loop: capacity {cap:.3f} solves/s", file=sys.stderr, flush=True)
    rates = {}
    for rho in [float(r) for r in args.rho.split(",")] if args.rho else []:
        rate = rho * cap
        print(f"[bench] open loop at rho={rho}: {rate:.3f} requests/s", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        out = run(jobs_at(rate), workers=args.workers, checksum=True, slice_cycles=args.slice_cycles,
                  on_done=progress(f"rho={rho}"), **opts)
        wall = time.perf_counter() - t0
        lat = [r["end"] - r["arrival"] for r in out]
        rates[str(rho)] = {"arrival_rate_per_s": rate, "solves_per_s": len(stream) / wall, "seconds": wall,
                           "latency_s": {"p50": _pct(lat, 0.5), "p99": _pct(lat, 0.99)},
                           "queue_s": {"p50": _pct([r["start"] - r["arrival"] for r in out], 0.5),
                                       "p99": _pct([r["start"] - r["arrival"] for r in out], 0.99)},
                           "converged": int(sum(r["converged"] for r in out)),
                           "turns_mean": sum(r["slices"] for r in out) / len(out)}
        if closed is not None:
            rates[str(rho)]["identical_to_closed_loop"] = int(sum(a["digest"] == b["digest"]
                                                                  for a, b in zip(closed, out)))
    first = next(iter(rates.values())) if rates else None
    res = {
        "metric": "served KKT solves/sec to 1e-8 residual; p50/p99 arrival-to-completion latency",
        "value": first["solves_per_s"] if first else cap,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": 1e3 * (first["seconds"] if first else len(stream) / cap),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-inner/f64-outer",
        "data": "synthetic",
        "config": {"workload": f"{len(stream)} Poisson-arrival Stokes/Oseen control requests (N in 32..."
                               f"{args.serve_max_n}, nt in 32...256, log-uniform beta, nu in {{1,1/50,1/100}}), "
                               f"{args.workers} worker streams, slots recycled every {args.slice_cycles} FGMRES "
                               "restart cycle(s)"},
        "capacity_solves_per_s": cap,
        "capacity_measured": closed is not None,
        "rates": rates,
    }
    if closed is not None:
        res["closed_loop_converged"] = int(sum(r["converged"] for r in closed))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
