"""Many control problems on one GPU: concurrent solves under a memory budget,
and a served request stream with slots recycled at restart boundaries.

``run(jobs, workers, budget_bytes, slice_cycles)`` admits jobs in arrival
order while their device memory (workspace, right-hand side, solution,
desired state) fits the budget, and ``workers`` host threads, each with its
own HIP stream, solve them: whole (``slice_cycles`` = 0) or a few FGMRES
restart cycles per turn, round robin over the admitted jobs, whose Krylov
state stays in device memory between turns.  Kernels of different problems
overlap on the device; every kernel and reduction of a solve depends only on
its own problem and a sliced solve makes the same iterates as an
uninterrupted one, so each result equals that of a lone solve.  The compute
runs in the HIP library (``pintoc_solve``); this module only schedules.

A job is a dict with the problem data of :class:`Problem` (``N, nt, T, nu,
beta, flow, wind``), the desired state ``vd`` (array of shape
``[nt, 2, (2N+1)^2]``) and optionally ``arrival`` (seconds after the start).
"""
from __future__ import annotations

import threading
import time

from ._lib import Problem

_PROBLEM_KEYS = ("N", "nt", "T", "nu", "beta", "flow", "wind")


def job_bytes(job, **options) -> int:
    """Device bytes a job holds while it runs (workspace + four vectors)."""
    import ctypes as C

    from ._lib import Desc, _check, default_options, library
    import numpy as np
    wind = job.get("wind")
    w = None if wind is None else np.ascontiguousarray(np.asarray(wind, dtype=np.float64).reshape(-1))
    d = Desc(job["N"], job["nt"], job.get("T", 1.0), job["nu"], job["beta"], job.get("flow", 0),
             None if w is None else w.ctypes.data_as(C.POINTER(C.c_double)))
    o = default_options(**options)
    h = C.c_void_p()
    lib = library()
    _check(lib.pintoc_problem_create(C.byref(d), C.byref(o), C.byref(h)), "pintoc_problem_create")
    try:
        ws = int(lib.pintoc_workspace_bytes(h))
        n_all = int(lib.pintoc_vector_length(h))
    finally:
        lib.pintoc_problem_destroy(h)
    nq2 = (2 * job["N"] + 1) ** 2
    return ws + 8 * (2 * n_all + job["nt"] * 2 * nq2)


def run(jobs, workers: int = 4, budget_bytes: int | None = None, keep_solutions: bool = False,
        checksum: bool = False, on_done=None, device="cuda", slice_cycles: int = 0, **options):
    """Solve every job; returns one record per job (in job order) with the
    stats of its solve, its arrival, start and end times (seconds after the
    start of the run), the device bytes it held, the number of slices it ran
    in, with ``keep_solutions`` its solution copied to host memory (numpy) and
    with ``checksum`` a BLAKE2b digest of the solution's bytes (to compare
    runs without keeping them).  ``on_done(k, record)`` is called (from a
    worker thread) as job k ends.

    Scheduling.  A job is admitted in arrival order once it has arrived and
    its device memory fits the budget left; the worker that admits it creates
    and binds the problem and assembles the right-hand side, and the job joins
    the ready queue.  Each of the ``workers`` host threads owns a HIP stream
    and repeatedly takes the job at the head of the ready queue.  With
    ``slice_cycles`` = 0 it solves the job to the end; with ``slice_cycles`` =
    c > 0 it runs c FGMRES restart cycles (``pintoc_solve`` with a cycle
    budget, resumed on the next turn) and, if the job is not finished, puts it
    back at the tail of the queue: the worker's slot is recycled at a restart
    boundary, so requests that arrive while long solves run start at once and
    every admitted request progresses.  A paused job keeps its problem,
    workspace and vectors (its Krylov state) in device memory between turns;
    each turn completes before the next starts (the library synchronises the
    stream), so a job may move between worker streams.  The iterates of a
    sliced solve equal those of an uninterrupted one, so each result is the
    same alone, in a batch and served."""
    import collections
    import hashlib

    import numpy as np
    import torch

    n = len(jobs)
    need = [job_bytes(j, **options) for j in jobs]
    # blocks the caching allocator keeps for streams of earlier runs are of no
    # use to this run's streams: return them before measuring the free memory
    torch.cuda.synchronize(device)
    torch.cuda.empty_cache()
    if budget_bytes is None:
        free, _ = torch.cuda.mem_get_info(device)
        budget_bytes = int(0.85 * free)
    if n and max(need) > budget_bytes:
        raise ValueError(f"a job needs {max(need)} bytes, more than the budget {budget_bytes}")
    order = sorted(range(n), key=lambda k: (jobs[k].get("arrival", 0.0), k))
    out = [None] * n
    lock = threading.Condition()
    ready = collections.deque()                          # admitted jobs: [k, problem, b, x, turns, start]
    state = {"next": 0, "free": budget_bytes, "error": None, "done": 0}
    t0 = time.perf_counter()

    def admit_one():
        """Under the lock: index of the next job if it has arrived and fits, else None."""
        if state["next"] >= n:
            return None
        k = order[state["next"]]
        if jobs[k].get("arrival", 0.0) > time.perf_counter() - t0 or need[k] > state["free"]:
            return None
        state["next"] += 1
        state["free"] -= need[k]
        return k

    def next_wait():
        if state["next"] >= n:
            return 0.05
        k = order[state["next"]]
        return min(max(jobs[k].get("arrival", 0.0) - (time.perf_counter() - t0), 0.0), 0.05) or 0.05

    def setup(k, stream):
        job = jobs[k]
        start = time.perf_counter() - t0
        with torch.cuda.stream(stream):
            p = Problem(job["N"], job["nt"], job.get("T", 1.0), job["nu"], job["beta"],
                        job.get("flow", 0), job.get("wind"), device=device, **options)
            vd = torch.as_tensor(np.ascontiguousarray(job["vd"], dtype=np.float64)).to(device)
            b = p.assemble_rhs(vd)
            x = p.empty()
            stream.synchronize()
        return [k, p, b, x, 0, start]

    def finish(item, st, ok, stream):
        k, p, b, x, turns, start = item
        with torch.cuda.stream(stream):
            sol = x.cpu().numpy() if (keep_solutions or checksum) else None
        digest = hashlib.blake2b(sol.tobytes(), digest_size=16).hexdigest() if checksum else None
        p.close()
        end = time.perf_counter() - t0
        out[k] = {"stats": st, "converged": ok, "arrival": jobs[k].get("arrival", 0.0), "start": start,
                  "end": end, "bytes": need[k], "slices": turns, "digest": digest,
                  "solution": sol if keep_solutions else None}

    def worker():
        stream = torch.cuda.Stream(device=device)          # default priority
        while True:
            item, k_new = None, None
            with lock:
                while True:
                    if state["error"] is not None or state["done"] >= n:
                        return
                    k_new = admit_one()
                    if k_new is not None:
                        break
                    if ready:
                        item = ready.popleft()
                        break
                    lock.wait(timeout=next_wait())
            try:
                if k_new is not None:
                    item = setup(k_new, stream)
                k, p, b, x = item[0], item[1], item[2], item[3]
                with torch.cuda.stream(stream):
                    _, st, ok = p.solve(b, x, cycle_budget=slice_cycles, resume=item[4] > 0)
                item[4] += 1
                if st["paused"]:
                    with lock:
                        ready.append(item)
                        lock.notify_all()
                    continue
                finish(item, st, ok, stream)
                del item, p, b, x
            except BaseException as e:                      # noqa: BLE001 - reported to the caller
                with lock:
                    state["error"] = e
                    lock.notify_all()
                return
            with lock:
                state["free"] += need[k]
                state["done"] += 1
                lock.notify_all()
            if on_done is not None:
                on_done(k, out[k])

    threads = [threading.Thread(target=worker, daemon=True) for _ in range(max(1, workers))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize(device)
    ready.clear()
    torch.cuda.empty_cache()
    if state["error"] is not None:
        raise state["error"]
    return out


def _member_of(job):
    return {"N": job["N"], "nt": job["nt"], "T": job.get("T", 1.0), "nu": job["nu"], "beta": job["beta"],
            "flow": job.get("flow", 0), "wind": job.get("wind")}


def autotune(jobs, sizes=(1, 2, 4, 8, 16), smoothers=None, budget_bytes=None, device="cuda", reps=2,
             keep: float = 0.85, **options) -> dict:
    """Pick, per class of jobs with the same (N, flow), the group size and the
    smoother of the fused form by measurement: for every candidate that fits
    the memory budget, one group of that many of the class's jobs (linear
    preconditioner, the options' precision) applies its fused preconditioner
    ``reps`` times.  The pick is the smallest group whose member applications
    per second reach ``keep`` times the best candidate's: the fused
    application runs beside other groups on other streams, and a group's
    members converge at different outer iterations (those that finish sit
    out while the rest iterate), so beyond the knee a larger group gains
    little throughput and loses concurrency.  Returns
    {(N, flow): {"size", "smoother", "trials": [...]}}."""
    import numpy as np
    import torch

    from ._lib import INNER_LINEAR, SMOOTHER_GLOBAL, SMOOTHER_TILED, Group, group_bytes

    smoothers = (SMOOTHER_TILED, SMOOTHER_GLOBAL) if smoothers is None else smoothers
    if budget_bytes is None:
        torch.cuda.synchronize(device)
        torch.cuda.empty_cache()
        free, _ = torch.cuda.mem_get_info(device)
        budget_bytes = int(0.5 * free)
    tune_opts = {k: v for k, v in options.items() if k in ("precision", "n_vcycles", "n_cheb", "n_uzawa", "mu_uzawa")}
    classes = {}
    for j in jobs:
        classes.setdefault((j["N"], j.get("flow", 0)), []).append(j)
    out = {}
    for key, cj in classes.items():
        trials = []
        for sm in smoothers:
            for g in sizes:
                if g > len(cj):
                    break
                members = [_member_of(j) for j in cj[:g]]
                opts = dict(tune_opts, inner=INNER_LINEAR, smoother=sm)
                need = group_bytes(members, **opts) + sum(8 * 2 * (2 * m["nt"] * (2 * (2 * m["N"] + 1) ** 2
                                                                                  + (m["N"] + 1) ** 2))
                                                          for m in members)
                if need > budget_bytes:
                    break
                grp = Group(members, device=device, **opts)
                rs = [torch.randn(grp.n_all[k], dtype=torch.float64, device=device) for k in range(g)]
                grp.precond_apply(rs)                                   # warm-up
                torch.cuda.synchronize(device)
                t0 = time.perf_counter()
                for _ in range(reps):
                    grp.precond_apply(rs)
                torch.cuda.synchronize(device)
                dt = (time.perf_counter() - t0) / reps
                trials.append({"size": g, "smoother": int(sm), "seconds": dt, "member_apps_per_s": g / dt})
                grp.close()
                del grp, rs
                torch.cuda.empty_cache()
        best = max(t["member_apps_per_s"] for t in trials)
        pick = min((t for t in trials if t["member_apps_per_s"] >= keep * best),
                   key=lambda t: (t["size"], t["smoother"]))
        out[key] = {"size": pick["size"], "smoother": pick["smoother"], "trials": trials}
    return out


def run_fused(jobs, plan=None, workers: int = 2, budget_bytes: int | None = None, checksum: bool = False,
              keep_solutions: bool = False, on_done=None, device="cuda", **options):
    """The fused batched form: jobs with the same (N, flow) are solved in
    groups (``pintoc_group_*``: one batch of every per-frequency kernel, FGMRES
    in lockstep), the group size and smoother per class from ``plan`` (see
    ``autotune``; default: groups of 4, tiled smoother).  ``workers`` host
    threads, each with its own stream, run groups concurrently while their
    device memory fits the budget.  Returns one record per job, as ``run``
    (with the group it ran in)."""
    import hashlib

    import numpy as np
    import torch

    from ._lib import Group, group_bytes

    n = len(jobs)
    classes = {}
    for k, j in enumerate(jobs):
        classes.setdefault((j["N"], j.get("flow", 0)), []).append(k)
    groups = []
    for key, ks in classes.items():
        size = plan[key]["size"] if plan and key in plan else 4
        sm = plan[key]["smoother"] if plan and key in plan else 0
        for i in range(0, len(ks), size):
            groups.append((ks[i:i + size], sm))
    torch.cuda.synchronize(device)
    torch.cuda.empty_cache()
    if budget_bytes is None:
        free, _ = torch.cuda.mem_get_info(device)
        budget_bytes = int(0.85 * free)

    def vec_bytes(j):
        return 8 * (2 * 2 * j["nt"] * (2 * (2 * j["N"] + 1) ** 2 + (j["N"] + 1) ** 2) + j["nt"] * 2 * (2 * j["N"] + 1) ** 2)

    need = []
    for ks, sm in groups:
        members = [_member_of(jobs[k]) for k in ks]
        need.append(group_bytes(members, smoother=sm, **options) + sum(vec_bytes(jobs[k]) for k in ks))
    if groups and max(need) > budget_bytes:
        raise ValueError(f"a group needs {max(need)} bytes, more than the budget {budget_bytes}")
    # largest groups first: they bound the makespan
    order = sorted(range(len(groups)), key=lambda g: -need[g])
    out = [None] * n
    lock = threading.Condition()
    state = {"next": 0, "free": budget_bytes, "error": None}
    t0 = time.perf_counter()

    def worker():
        stream = torch.cuda.Stream(device=device)          # default priority
        while True:
            with lock:
                while True:
                    if state["error"] is not None or state["next"] >= len(order):
                        return
                    gi = order[state["next"]]
                    if need[gi] <= state["free"]:
                        state["next"] += 1
                        state["free"] -= need[gi]
                        break
                    lock.wait(timeout=0.05)
            ks, sm = groups[gi]
            start = time.perf_counter() - t0
            try:
                with torch.cuda.stream(stream):
                    g = Group([_member_of(jobs[k]) for k in ks], device=device, smoother=sm, **options)
                    bs = []
                    for i, k in enumerate(ks):
                        vd = torch.as_tensor(np.ascontiguousarray(jobs[k]["vd"], dtype=np.float64)).to(device)
                        bs.append(g.assemble_rhs(i, vd))
                    xs, sts, oks = g.solve(bs)
                    stream.synchronize()
                    end = time.perf_counter() - t0
                    for i, k in enumerate(ks):
                        sol = xs[i].cpu().numpy() if (keep_solutions or checksum) else None
                        digest = hashlib.blake2b(sol.tobytes(), digest_size=16).hexdigest() if checksum else None
                        out[k] = {"stats": sts[i], "converged": oks[i], "arrival": 0.0, "start": start, "end": end,
                                  "bytes": need[gi], "group": gi, "group_size": len(ks), "digest": digest,
                                  "solution": sol if keep_solutions else None}
                    g.close()
                    del g, bs, xs
            except BaseException as e:                      # noqa: BLE001 - reported to the caller
                with lock:
                    state["error"] = e
                    lock.notify_all()
                return
            with lock:
                state["free"] += need[gi]
                lock.notify_all()
            if on_done is not None:
                for k in ks:
                    on_done(k, out[k])

    threads = [threading.Thread(target=worker, daemon=True) for _ in range(max(1, workers))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize(device)
    torch.cuda.empty_cache()
    if state["error"] is not None:
        raise state["error"]
    return out
