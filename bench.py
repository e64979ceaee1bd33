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

# HBM traffic of the dominant kernel (finest-grid pre-smoothing sweep) from two
# rocprofv3 --pmc passes over one solve of this workload (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch at the finest grid), each scaled by what the
# same counter reads for a 1 GiB device copy in the same process (FETCH_SIZE
# 524330.3 KiB, WRITE_SIZE 1048576 KiB).  Valid only for the kernel source they
# were taken on: reported as null once that file changes.
SWEEP_SOURCE = os.path.join(ROOT, "paper_2405_18964_amd", "csrc", "q2_tiles.hip")
SWEEP_PMC = {"source_sha256": "2e972e25d279af992d70cb6a44fbf622b8d1c0048c0d6ad1b8b2b9f983a0b544",
             "fetch_kib": 363452.0, "fetch_scale": 1048576.0 / 524330.3,
             "write_kib": 420161.8, "write_scale": 1.0}


def sweep_traffic_bytes():
    import hashlib
    with open(SWEEP_SOURCE, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != SWEEP_PMC["source_sha256"]:
            return None
    return 1024.0 * (SWEEP_PMC["fetch_kib"] * SWEEP_PMC["fetch_scale"] + SWEEP_PMC["write_kib"] * SWEEP_PMC["write_scale"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 3; 1 for --config 4 and 5)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2,
                    help="workload: 1, 2 (single Stokes problem) or 4 (batched 64-problem mix)")
    ap.add_argument("--batch-count", type=int, default=64, help="problems of the batched mix (--config 4)")
    ap.add_argument("--workers", type=int, default=4, help="concurrent problems on the device (--config 4)")
    ap.add_argument("--requests", type=int, default=32, help="requests of the served stream (--config 5)")
    ap.add_argument("--rho", type=float, default=0.8, help="arrival rate / measured capacity (--config 5)")
    ap.add_argument("--serve-max-n", type=int, default=128, help="largest grid of the served stream (--config 5)")
    ap.add_argument("--compare", action="store_true",
                    help="--config 4: also solve the mix one problem at a time (FP32-inner and FP64)")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--inner", choices=["gmres", "linear"], default="gmres")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precond-reps", type=int, default=5)
    ap.add_argument("--no-fp32", action="store_true", help="skip the extra FP32-inner solve")
    ap.add_argument("--no-minres", action="store_true", help="skip the extra MINRES (Algorithm 1) solve")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one device copy of 1 GiB first (reference for HBM byte counters)")
    return ap.parse_args()


def precond_model_bytes(N: int, nt: int, n_vcycles: int, n_cheb: int, csize: int) -> dict:
    """Compulsory HBM bytes of one linear preconditioner application
    (Algorithm 1): every kernel pass reads/writes each field it touches once.

    Field sizes per kept frequency (nf = nt/2 + 1): 4 complex Q2 grids (velocity
    of both blocks) and 2 complex Q1 grids (pressure).  Per multigrid level
    (sizes shrink by 4, so a cycle costs 4/3 of its finest level): the
    pre-smoothing sweep reads x, b and writes x (3 passes; 2 in the first cycle,
    which starts from x = 0), the post-smoothing sweep reads x, the coarse
    correction and b and writes x (3 + 1/4).  Between them the Q2 levels run
    one fused residual/restriction pass (reads x, b, writes the coarse rhs:
    2 + 1/4), the Q1 levels a residual (3) and a restriction (1 + 1/4): 8.5
    (Q2) and 10.5 (Q1) passes per level.  A Chebyshev step reads x_k, x_{k-1},
    b, writes x_{k+1}; the first reads b and writes x_1, the second has no
    x_0 to read (4 n - 3 passes for n steps).  The FFT pair reads and writes the canonical vector and
    the frequency vector once each."""
    nf = nt // 2 + 1
    nq2, np2 = (2 * N + 1) ** 2, (N + 1) ** 2
    FV = 4 * nf * nq2 * csize          # velocity frequency fields
    FP = 2 * nf * np2 * csize          # pressure frequency fields
    L = 2 * nq2 + np2
    canon = 2 * nt * L * 8
    freq = FV + FP
    mg_w = (8.5 * n_vcycles - 1.0) * 4.0 / 3.0 * FV
    mg_k = (10.5 * n_vcycles - 1.0) * 4.0 / 3.0 * FP
    cheb = (1 + 4 * (n_cheb - 1)) * FP
    schur = 2 * FP + 3 * FP            # unpin copy, combine
    fft = 2 * (canon + freq)
    total = mg_w + mg_k + cheb + schur + fft
    return {"total": total, "mg_velocity": mg_w, "mg_pressure": mg_k, "chebyshev": cheb, "fft": fft,
            "velocity_field_bytes": FV}


def cpu_baseline(w, outer_its: int, inner_mean: float, budget_s: float = 15.0) -> dict:
    """Time the oracle's per-frequency block solve P~_j^{-1} at the full grid
    size on the host and extrapolate to one KKT solve with the iteration
    counts the GPU solve used (each outer iteration applies P~_j^{-1} to
    (inner_mean + 1) vectors per frequency for all nt frequencies)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.kkt import Problem as OP
    from oracle.precond import StokesPreconditioner

    with threadpool_limits(limits=1):
        op = OP.from_workload(w)
        freqs = [1, w.nt // 4, w.nt // 2]
        pc = StokesPreconditioner(op, freqs=freqs)
        rng = np.random.default_rng(0)
        n = op.nv
        for j in freqs:
            pc.W_mg(j)                                   # set-up outside the timing
        samples = 0
        t_used = 0.0
        while t_used < budget_s:                         # bounded sample: ~budget_s of CPU work
            j = freqs[samples % len(freqs)]
            s1 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
            s2 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
            s3 = rng.standard_normal(op.nP) + 1j * rng.standard_normal(op.nP)
            s4 = rng.standard_normal(op.nP) + 1j * rng.standard_normal(op.nP)
            t0 = time.perf_counter()
            pc.ptilde_inv(j, s1, s2, s3, s4)
            t_used += time.perf_counter() - t0
            samples += 1
    t_block = t_used / samples
    t_solve = outer_its * (inner_mean + 1.0) * w.nt * t_block
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"{samples} per-frequency P~_j applications of the FP64 oracle at N={w.N} "
                       f"({t_block:.2f} s each, BLAS threads 1), extrapolated to {outer_its} outer x "
                       f"({inner_mean:.1f} inner + 1) x {w.nt} frequencies; FFTs and matvecs omitted"),
            "seconds_measured": t_used}


def main():
    args = parse()
    if args.steps is None:
        args.steps = 1 if args.config in (4, 5) else 3
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (no multi-GPU path)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2405_18964_amd as P
    import workloads as W

    if args.config == 4:
        return bench_batch(args)
    if args.config == 5:
        return bench_serve(args)
    w = W.config(args.config)
    prec = P.PREC_FP64 if args.precision == "fp64" else P.PREC_FP32_INNER
    inner = P.INNER_GMRES if args.inner == "gmres" else P.INNER_LINEAR
    gp = P.Problem.from_workload(w, inner=inner, precision=prec, max_outer=60 if args.inner == "gmres" else 400,
                                 restart=10 if args.inner == "gmres" else 30)
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
    print(f"[bench] {w.name} n_all={gp.n_all} workspace={gp.workspace_bytes / 1e9:.1f} GB", file=sys.stderr,
          flush=True)
    for i in range(args.warmup):
        x.zero_()
        _, st, ok = gp.solve(b, x)
        print(f"[bench] warmup {i}: {st['outer_iterations']} its, {st['seconds']:.2f} s", file=sys.stderr,
              flush=True)
    lat, stats = [], []
    gp.profile_enable(True)          # HIP events around the dominant kernel's launches
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
    kt = gp.profile_read()
    gp.profile_enable(False)
    # independent check of the last solution: true residual through the KKT matvec
    r = b - gp.kkt_apply(x)
    rel = float(torch.linalg.norm(r) / torch.linalg.norm(b))
    # linear preconditioner application: model bytes / time
    lp = P.Problem.from_workload(w, inner=P.INNER_LINEAR, precision=prec)
    z = lp.empty()
    lp.precond_apply(b, z)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.precond_reps):
        lp.precond_apply(b, z)
    e1.record(stream)
    e1.synchronize()
    t_pc = e0.elapsed_time(e1) / 1e3 / args.precond_reps
    csize = 16 if args.precision == "fp64" else 8
    model = precond_model_bytes(w.N, w.nt, 4, 10, csize)
    del lp
    lat_sorted = sorted(lat)
    p50 = lat_sorted[len(lat) // 2]
    p99 = lat_sorted[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)]
    outer = int(np.mean([s["outer_iterations"] for s in stats]))
    inner_mean = float(np.mean([s["inner_iterations_mean"] for s in stats]))
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
        "dtype": "f64" if args.precision == "fp64" else "f32-inner/f64-outer",
        "data": "synthetic",
        "config": {"workload": f"Stokes control, Q2-Q1 on {w.N}x{w.N} quads, nt={w.nt}, T={w.T}, nu={w.nu}, "
                               f"beta={w.beta}, {gp.n_all} unknowns (canonical)",
                   "solver": f"FGMRES(10) + block-circulant preconditioner, inner={args.inner}",
                   "precision": args.precision},
        "latency_s": {"p50": p50, "p99": p99, "all": lat},
        "iterations": {"outer": outer, "inner_mean": inner_mean,
                       "inner_max": int(max(s["inner_iterations_max"] for s in stats))},
        "final_rel_residual": rel,
        "precond_apply": {"ms": 1e3 * t_pc, "model_bytes": model["total"],
                          "model_GBs": model["total"] / t_pc / 1e9,
                          "frac_of_hbm_peak": model["total"] / t_pc / 1e9 / HBM_PEAK_GBS},
    }
    achieved = kt["algorithmic_bytes"] / (kt["avg_ms"] * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS, "traffic": sweep_traffic_bytes(),
                       "kernel": "k_q2_sweep<double,false,true,false> (finest-grid pre-smoothing sweep of the "
                                 "velocity multigrid, all kept frequencies)",
                       "avg_launch_ms": kt["avg_ms"], "launches_timed": kt["launches"],
                       "algorithmic_bytes_per_launch": kt["algorithmic_bytes"]}
    if not args.no_fp32 and args.precision == "fp64":
        del gp
        torch.cuda.empty_cache()
        g32 = P.Problem.from_workload(w, inner=inner, precision=P.PREC_FP32_INNER, max_outer=60, restart=10)
        x.zero_()
        g32.solve(b, x)                                  # warm-up
        x.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, st32, ok32 = g32.solve(b, x)
        torch.cuda.synchronize()
        t32 = time.perf_counter() - t1
        r32 = float(torch.linalg.norm(b - g32.kkt_apply(x)) / torch.linalg.norm(b))
        out["fp32_inner"] = {"solves_per_s": 1.0 / t32, "seconds": t32, "converged": bool(ok32),
                             "final_rel_residual": r32, "outer": st32["outer_iterations"],
                             "inner_mean": st32["inner_iterations_mean"],
                             "note": "multigrid, Chebyshev, Uzawa and inner GMRES in FP32; outer FGMRES, "
                                     "residuals and the coarsest-grid inverses in FP64"}
        del g32
    if not args.no_minres and args.precision == "fp64" and w.flow == W.STOKES:
        # paper variant: MINRES with the linear preconditioner (Algorithm 1), FP64
        gm = P.Problem.from_workload(w, inner=P.INNER_LINEAR, outer=P.OUTER_MINRES, precision=P.PREC_FP64,
                                     max_outer=800)
        x.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, stm, okm = gm.solve(b, x)
        torch.cuda.synchronize()
        tm = time.perf_counter() - t1
        rm = float(torch.linalg.norm(b - gm.kkt_apply(x)) / torch.linalg.norm(b))
        out["minres_linear_fp64"] = {"solves_per_s": 1.0 / tm, "seconds": tm, "converged": bool(okm),
                                     "final_rel_residual": rm, "iterations": stm["outer_iterations"],
                                     "note": "MINRES on the symmetric all-at-once matrix with the symmetric "
                                             "positive definite linear preconditioner (Algorithm 1), FP64"}
        print(f"[bench] MINRES + Algorithm 1 (FP64): {stm['outer_iterations']} its, {tm:.2f} s",
              file=sys.stderr, flush=True)
        del gm
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, outer, inner_mean)
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """Batched form: the 64-problem mix through the concurrent runner."""
    import torch

    import paper_2405_18964_amd as P
    import workloads as W
    from paper_2405_18964_amd.batch import job_bytes, run

    mix = W.batch_mix(args.batch_count)
    jobs = [{"N": w.N, "nt": w.nt, "T": w.T, "nu": w.nu, "beta": w.beta, "flow": w.flow,
             "wind": W.wind_nodal(w.N) if w.flow == W.OSEEN else None, "vd": W.desired_state(w)} for w in mix]
    opts = dict(inner=P.INNER_GMRES, precision=P.PREC_FP32_INNER, max_outer=60)
    print(f"[bench] batched mix of {len(jobs)} problems, {sum(w.n_all for w in mix) / 1e9:.2f}e9 unknowns, "
          f"{sum(job_bytes(j, **opts) for j in jobs) / 1e9:.0f} GB of job memory", file=sys.stderr, flush=True)
    small = sorted(range(len(jobs)), key=lambda k: job_bytes(jobs[k], **opts))[:args.workers]
    for i in range(args.warmup):                           # module loading, allocator warm-up
        run([jobs[k] for k in small], workers=args.workers, **opts)
    def progress(tag):
        def cb(k, r):
            print(f"[bench] {tag}: job {k} ({mix[k].name}, nt={mix[k].nt}) {r['end'] - r['start']:.2f} s"
                  f"{'' if r['converged'] else ' NOT CONVERGED'}", file=sys.stderr, flush=True)
        return cb

    walls, outs = [], []
    for i in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = run(jobs, workers=args.workers, checksum=True, on_done=progress(f"step {i}"), **opts)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        outs.append(out)
        print(f"[bench] step {i}: {walls[-1]:.2f} s, converged {sum(r['converged'] for r in out)}/{len(out)}",
              file=sys.stderr, flush=True)
    out = outs[-1]
    wall = sum(walls)
    lat = sorted(r["end"] - r["start"] for r in out)
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
                               "nt in {32,...,256}, log-uniform beta in [1e-6,1e-2], nu in {1,1/50,1/100}), "
                               f"{args.workers} concurrent on one GPU",
                   "solver": "FGMRES(10) + block-circulant preconditioner with inner GMRES per frequency"},
        "converged": int(sum(r["converged"] for r in out)),
        "latency_s": {"p50": lat[len(lat) // 2], "p99": lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)]},
    }
    if args.compare:
        for name, prec in (("sequential_fp32_inner", P.PREC_FP32_INNER), ("sequential_fp64", P.PREC_FP64)):
            o = dict(opts, precision=prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            seq = run(jobs, workers=1, checksum=True, on_done=progress(name), **o)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            res[name] = {"solves_per_s": len(jobs) / t, "seconds": t,
                         "converged": int(sum(r["converged"] for r in seq))}
            if prec == P.PREC_FP32_INNER:
                res["identical_to_sequential"] = int(sum(a["digest"] == b["digest"] for a, b in zip(seq, out)))
            print(f"[bench] {name}: {t:.2f} s", file=sys.stderr, flush=True)
    print(json.dumps(res), flush=True)


def bench_serve(args):
    """Served form: Poisson arrivals at rho times the measured capacity."""
    import torch

    import paper_2405_18964_amd as P
    import workloads as W
    from paper_2405_18964_amd.batch import run

    stream = W.serve_stream(args.requests, max_N=args.serve_max_n)

    def jobs_at(rate):
        return [{"N": w.N, "nt": w.nt, "T": w.T, "nu": w.nu, "beta": w.beta, "flow": w.flow,
                 "wind": W.wind_nodal(w.N) if w.flow == W.OSEEN else None, "vd": W.desired_state(w),
                 "arrival": (a / rate if rate else 0.0)} for w, a in stream]
    opts = dict(inner=P.INNER_GMRES, precision=P.PREC_FP32_INNER, max_outer=60)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    def progress(tag):
        def cb(k, r):
            w = stream[k][0]
            print(f"[bench] {tag}: request {k} ({w.name}, nt={w.nt}) {r['end'] - r['start']:.2f} s",
                  file=sys.stderr, flush=True)
        return cb

    closed = run(jobs_at(None), workers=args.workers, checksum=True, on_done=progress("closed loop"), **opts)
    cap = len(stream) / (time.perf_counter() - t0)
    rate = args.rho * cap
    print(f"[bench] closed loop: capacity {cap:.3f} solves/s; open loop at {rate:.3f} requests/s",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    out = run(jobs_at(rate), workers=args.workers, checksum=True, on_done=progress("open loop"), **opts)
    wall = time.perf_counter() - t0
    lat = sorted(r["end"] - r["arrival"] for r in out)
    same = int(sum(a["digest"] == b["digest"] for a, b in zip(closed, out)))
    res = {
        "metric": "served KKT solves/sec to 1e-8 residual; p50/p99 arrival-to-completion latency",
        "value": len(stream) / wall,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": 1e3 * wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-inner/f64-outer",
        "data": "synthetic",
        "config": {"workload": f"{len(stream)} Poisson-arrival Stokes/Oseen control requests (N in 32..."
                               f"{args.serve_max_n}, nt in 32...256), rate {args.rho} x measured capacity, "
                               f"{args.workers} concurrent on one GPU"},
        "capacity_solves_per_s": cap,
        "arrival_rate_per_s": rate,
        "latency_s": {"p50": lat[len(lat) // 2], "p99": lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)]},
        "converged": int(sum(r["converged"] for r in out)),
        "identical_to_closed_loop": same,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
