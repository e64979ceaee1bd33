"""Many control problems on one GPU: concurrent solves under a memory budget.

``run(jobs, workers, budget_bytes)`` keeps up to ``workers`` problems on the
device at once.  Each worker is a host thread with its own HIP stream; it takes
the next job in arrival order once the job has arrived and its device memory
(workspace, right-hand side, solution, desired state) fits the budget left,
then creates and binds the problem, assembles the right-hand side, solves and
releases the memory.  Kernels of different problems overlap on the device;
every kernel and reduction of a solve depends only on its own problem, so each
result equals that of a lone solve.  The compute runs in the HIP library
(``pintoc_solve`` per job); this module only schedules.

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
        checksum: bool = False, on_done=None, device="cuda", **options):
    """Solve every job; returns one record per job (in job order) with the
    stats of its solve, its arrival, start and end times (seconds after the
    start of the run), the device bytes it held, with ``keep_solutions`` its
    solution copied to host memory (numpy) and with ``checksum`` a BLAKE2b
    digest of the solution's bytes (to compare runs without keeping them).
    ``on_done(k, record)`` is called (from the worker thread) as job k ends."""
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
    state = {"next": 0, "free": budget_bytes, "error": None}
    t0 = time.perf_counter()

    def worker():
        stream = torch.cuda.Stream(device=device)          # default priority
        while True:
            with lock:
                while True:
                    if state["error"] is not None or state["next"] >= n:
                        return
                    k = order[state["next"]]
                    wait = jobs[k].get("arrival", 0.0) - (time.perf_counter() - t0)
                    if wait <= 0 and need[k] <= state["free"]:
                        state["next"] += 1
                        state["free"] -= need[k]
                        break
                    lock.wait(timeout=max(wait, 0.0) if wait > 0 else 0.05)
            start = time.perf_counter() - t0
            try:
                job = jobs[k]
                with torch.cuda.stream(stream):
                    p = Problem(job["N"], job["nt"], job.get("T", 1.0), job["nu"], job["beta"],
                                job.get("flow", 0), job.get("wind"), device=device, **options)
                    vd = torch.as_tensor(np.ascontiguousarray(job["vd"], dtype=np.float64)).to(device)
                    b = p.assemble_rhs(vd)
                    x, st, ok = p.solve(b)
                    stream.synchronize()
                    sol = x.cpu().numpy() if (keep_solutions or checksum) else None
                    digest = hashlib.blake2b(sol.tobytes(), digest_size=16).hexdigest() if checksum else None
                    if not keep_solutions:
                        sol = None
                    p.close()
                    del p, vd, b, x
                end = time.perf_counter() - t0
                out[k] = {"stats": st, "converged": ok, "arrival": job.get("arrival", 0.0), "start": start,
                          "end": end, "bytes": need[k], "solution": sol, "digest": digest}
            except BaseException as e:                      # noqa: BLE001 - reported to the caller
                with lock:
                    state["error"] = e
                    lock.notify_all()
                return
            with lock:
                state["free"] += need[k]
                lock.notify_all()
            if on_done is not None:
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
