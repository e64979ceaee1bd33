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


def job_options(job, options):
    """The run's options with the job's own ``job["options"]`` (if any) on top:
    e.g. ``{"inner": INNER_MINRES}`` for the Stokes jobs of a mixed list."""
    return dict(options, **job.get("options", {}))


def job_layout(job, **options):
    """(workspace bytes, canonical vector length) of a job (host-side set-up only)."""
    import ctypes as C

    from ._lib import Desc, _check, default_options, library
    import numpy as np
    wind = job.get("wind")
    w = None if wind is None else np.ascontiguousarray(np.asarray(wind, dtype=np.float64).reshape(-1))
    d = Desc(job["N"], job["nt"], job.get("T", 1.0), job["nu"], job["beta"], job.get("flow", 0),
             None if w is None else w.ctypes.data_as(C.POINTER(C.c_double)))
    o = default_options(**job_options(job, options))
    h = C.c_void_p()
    lib = library()
    _check(lib.pintoc_problem_create(C.byref(d), C.byref(o), C.byref(h)), "pintoc_problem_create")
    try:
        ws = int(lib.pintoc_workspace_bytes(h))
        n_all = int(lib.pintoc_vector_length(h))
    finally:
        lib.pintoc_problem_destroy(h)
    return ws, n_all


_ALIGN = 4096


def _up(v):
    return (v + _ALIGN - 1) // _ALIGN * _ALIGN


def _pieces(job, ws, n_all):
    """Byte sizes of a job's workspace, b, x and desired state in its arena chunk."""
    nq2 = (2 * job["N"] + 1) ** 2
    return [_up(ws), _up(8 * n_all), _up(8 * n_all), _up(8 * job["nt"] * 2 * nq2)]


def job_bytes(job, **options) -> int:
    """Device bytes a job holds while it runs (workspace + three vectors)."""
    ws, n_all = job_layout(job, **options)
    return sum(_pieces(job, ws, n_all))


class _Arena:
    """First-fit allocator over one device allocation made at the start of a
    run: jobs of very different sizes (up to ~120 GB) come and go, and
    carving them from one arena keeps the caching allocator of the framework
    out of it (its per-stream pools and split blocks left large requests
    without room although the budget had it).  Freed ranges coalesce."""

    def __init__(self, nbytes, device):
        import torch
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.free = [(0, nbytes)]                         # sorted (offset, size)

    def largest(self):
        return max((s for _, s in self.free), default=0)

    def alloc(self, n):
        for i, (o, s) in enumerate(self.free):
            if s >= n:
                if s == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (o + n, s - n)
                return o
        return None

    def release(self, o, n):
        self.free.append((o, n))
        self.free.sort()
        merged = []
        for a, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == a:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((a, s))
        self.free = merged


def run(jobs, workers: int = 4, budget_bytes: int | None = None, keep_solutions: bool = False,
        checksum: bool = False, on_done=None, device="cuda", slice_cycles: int = 0, **options):
    """Solve every job; returns one record per job (in job order) with the
    stats of its solve, its arrival, start and end times (seconds after the
    start of the run), the device bytes it held, the number of slices it ran
    in, with ``keep_solutions`` its solution copied to host memory (numpy) and
    with ``checksum`` a BLAKE2b digest of the solution's bytes (to compare
    runs without keeping them).  ``on_done(k, record)`` is called (from a
    worker thread) as job k ends.

    Scheduling.  The run makes one device allocation of the budget (capped
    at what all jobs together need) and carves each job's memory (workspace,
    right-hand side, iterate, desired state) from it first-fit.  A job is
    admitted in arrival order once it has arrived and a free range of that
    arena holds it; the worker that admits it creates
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
    same alone, in a batch and served.  A job's ``options`` entry (a dict)
    overrides the run's options for that job."""
    import collections
    import hashlib

    import numpy as np
    import torch

    n = len(jobs)
    lay = [job_layout(j, **options) for j in jobs]
    pieces = [_pieces(j, ws, n_all) for j, (ws, n_all) in zip(jobs, lay)]
    need = [sum(pc) for pc in pieces]
    # blocks the caching allocator keeps for streams of earlier runs are of no
    # use to this run: return them before measuring the free memory
    torch.cuda.synchronize(device)
    torch.cuda.empty_cache()
    if budget_bytes is None:
        free, _ = torch.cuda.mem_get_info(device)
        budget_bytes = int(0.85 * free) // _ALIGN * _ALIGN
    if n and max(need) > budget_bytes:
        raise ValueError(f"a job needs {max(need)} bytes, more than the budget {budget_bytes}")
    arena = _Arena(min(budget_bytes, sum(need)) if n else _ALIGN, device)
    order = sorted(range(n), key=lambda k: (jobs[k].get("arrival", 0.0), k))
    out = [None] * n
    lock = threading.Condition()
    ready = collections.deque()                          # admitted jobs: [k, problem, b, x, turns, start, offset]
    state = {"next": 0, "error": None, "done": 0}
    offset = [None] * n
    t0 = time.perf_counter()

    def admit_one():
        """Under the lock: index of the next job if it has arrived and a free
        range of the arena holds it, else None (arrival order is kept)."""
        if state["next"] >= n:
            return None
        k = order[state["next"]]
        if jobs[k].get("arrival", 0.0) > time.perf_counter() - t0:
            return None
        o = arena.alloc(need[k])
        if o is None:
            return None
        offset[k] = o
        state["next"] += 1
        return k

    def next_wait():
        if state["next"] >= n:
            return 0.05
        k = order[state["next"]]
        return min(max(jobs[k].get("arrival", 0.0) - (time.perf_counter() - t0), 0.0), 0.05) or 0.05

    def setup(k, stream):
        """Problem, right-hand side and initial guess of job k in its arena range
        [workspace | b | x | desired state]."""
        job = jobs[k]
        start = time.perf_counter() - t0
        ws, n_all = lay[k]
        o = offset[k]
        views = []
        for sz in pieces[k]:
            views.append(arena.buf[o:o + sz])
            o += sz
        b = views[1][:8 * n_all].view(torch.float64)
        x = views[2][:8 * n_all].view(torch.float64)
        nq2 = (2 * job["N"] + 1) ** 2
        vd = views[3][:8 * job["nt"] * 2 * nq2].view(torch.float64)
        with torch.cuda.stream(stream):
            p = Problem(job["N"], job["nt"], job.get("T", 1.0), job["nu"], job["beta"], job.get("flow", 0),
                        job.get("wind"), device=device, workspace=views[0], **job_options(job, options))
            vd.copy_(torch.as_tensor(np.ascontiguousarray(job["vd"], dtype=np.float64)).reshape(-1))
            x.zero_()
            p.assemble_rhs(vd, b)
            stream.synchronize()
        return [k, p, b, x, 0, start]

    def finish(item, st, ok, stream):
        k, p, b, x, turns, start = item
        with torch.cuda.stream(stream):
            sol = x.cpu().numpy() if (keep_solutions or checksum) else None
            stream.synchronize()
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
                arena.release(offset[k], need[k])
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
    del arena
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
    ``reps`` times, and the same members as lone problems apply theirs on
    streams of their own, side by side.  The pick is the smallest group whose
    member applications per second reach ``keep`` times the best candidate's
    (size 1 -- no fusion -- where the lone problems side by side are faster
    than that group): the fused
    application runs beside other groups on other streams, and a group's
    members converge at different outer iterations (those that finish sit
    out while the rest iterate), so beyond the knee a larger group gains
    little throughput and loses concurrency.  Returns
    {(N, flow): {"size", "smoother", "trials", "concurrent", "fused_wins"}}."""
    import numpy as np
    import torch

    from ._lib import INNER_LINEAR, SMOOTHER_GLOBAL, SMOOTHER_TILED, Group, Problem, group_bytes

    smoothers = (SMOOTHER_TILED, SMOOTHER_GLOBAL) if smoothers is None else smoothers
    if budget_bytes is None:
        torch.cuda.synchronize(device)
        torch.cuda.empty_cache()
        free, _ = torch.cuda.mem_get_info(device)
        budget_bytes = int(0.5 * free)
    tune_opts = {k: v for k, v in options.items()
                 if k in ("precision", "n_vcycles", "n_cheb", "n_uzawa", "mu_uzawa", "graphs")}
    classes = {}
    for j in jobs:
        classes.setdefault((j["N"], j.get("flow", 0)), []).append(j)
    out = {}
    for key, cj in classes.items():
        trials, concurrent = [], []
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
                del grp
                if sm == smoothers[0] and g > 1:
                    # the same members as lone problems on streams of their own
                    lone = [Problem(device=device, **m, **opts) for m in members]
                    streams = [torch.cuda.Stream(device=device) for _ in members]
                    zs = [q.empty() for q in lone]

                    def issue():
                        for q, st, r, z in zip(lone, streams, rs, zs):
                            with torch.cuda.stream(st):
                                q.precond_apply(r, z)
                    issue()
                    torch.cuda.synchronize(device)
                    t0 = time.perf_counter()
                    for _ in range(reps):
                        issue()
                    torch.cuda.synchronize(device)
                    dt = (time.perf_counter() - t0) / reps
                    concurrent.append({"size": g, "seconds": dt, "member_apps_per_s": g / dt})
                    for q in lone:
                        q.close()
                    del lone, zs
                del rs
                torch.cuda.empty_cache()
        best = max(t["member_apps_per_s"] for t in trials)
        pick = min((t for t in trials if t["member_apps_per_s"] >= keep * best),
                   key=lambda t: (t["size"], t["smoother"]))
        # fusion pays only where it beats the same members running side by side
        conc = [c for c in concurrent if c["size"] == pick["size"]]
        fused_wins = not conc or pick["member_apps_per_s"] > conc[0]["member_apps_per_s"]
        out[key] = {"size": pick["size"] if fused_wins else 1, "smoother": pick["smoother"], "trials": trials,
                    "concurrent": concurrent, "fused_wins": fused_wins}
    return out


def run_fused(jobs, plan=None, workers: int = 2, budget_bytes: int | None = None, checksum: bool = False,
              keep_solutions: bool = False, on_done=None, device="cuda", **options):
    """The fused batched form: jobs with the same (N, flow) are solved in
    groups (``pintoc_group_*``: one batch of every per-frequency kernel, FGMRES
    in lockstep), the group size and smoother per class from ``plan`` (see
    ``autotune``; default: groups of 4, tiled smoother).  ``workers`` host
    threads, each with its own stream, run groups concurrently while their
    device memory fits the budget.  Per-job ``options`` overrides must agree
    within an (N, flow) class (the group takes its first job's).  Returns one
    record per job, as ``run`` (with the group it ran in)."""
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
        need.append(group_bytes(members, smoother=sm, **job_options(jobs[ks[0]], options))
                    + sum(vec_bytes(jobs[k]) for k in ks))
    if groups and max(need) > budget_bytes:
        raise ValueError(f"a group needs {max(need)} bytes, more than the budget {budget_bytes}")
    # groups in the order of their first job (as ``run`` admits jobs)
    order = sorted(range(len(groups)), key=lambda g: min(groups[g][0]))
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
                    g = Group([_member_of(jobs[k]) for k in ks], device=device, smoother=sm,
                              **job_options(jobs[ks[0]], options))
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
