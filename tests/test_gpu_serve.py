"""Served form: requests that arrive while others run, slots recycled at
FGMRES restart boundaries, each result equal to its lone solve and checked
by the oracle.

* ``pintoc_solve`` paused after every restart cycle and resumed until it
  converges gives the uninterrupted solve's iterate bit for bit, with the
  same iteration count.
* ``batch.run`` with staggered arrivals, two worker streams and one restart
  cycle per turn (Stokes and Oseen requests of N = 8..32 that spend several
  turns each, interleaved): every result equals its lone solve bit for bit,
  and the oracle recomputes each one's true residual (at most 1e-8).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    import paper_2405_18964_amd as P
    P.library()
    return P


def _job(w, arrival):
    return {"N": w.N, "nt": w.nt, "T": w.T, "nu": w.nu, "beta": w.beta, "flow": w.flow,
            "wind": W.wind_nodal(w.N) if w.flow == W.OSEEN else None, "vd": W.desired_state(w),
            "arrival": arrival}


MIX = [W.small(W.STOKES, 32, 16, beta=1e-4, seed=11),
       W.Workload(W.OSEEN, 32, 8, 1.0, 0.01, 1e-3, 12, 1.0),
       W.small(W.STOKES, 16, 32, beta=1e-3, seed=13),
       W.Workload(W.OSEEN, 16, 16, 1.0, 0.02, 1e-2, 14, 1.5),
       W.small(W.STOKES, 8, 16, beta=1e-2, seed=15)]
OPTS = dict(inner=1, max_outer=200, restart=5)   # inner GMRES (Algorithm 2 / its Oseen analogue), short cycles


def test_paused_and_resumed_solve_equals_uninterrupted(lib):
    w = MIX[0]
    print(f"pause/resume {w.name}", flush=True)
    gp = lib.Problem.from_workload(w, **OPTS)
    b = gp.assemble_rhs(torch.from_numpy(W.desired_state(w)).cuda())
    x_ref, st_ref, ok_ref = gp.solve(b)
    x = gp.empty()
    _, st, ok = gp.solve(b, x, cycle_budget=1)
    turns = 1
    while st["paused"]:
        _, st, ok = gp.solve(b, x, cycle_budget=1, resume=True)
        turns += 1
    torch.cuda.synchronize()
    print(f"  {turns} turns, {st['outer_iterations']} its (uninterrupted {st_ref['outer_iterations']})", flush=True)
    assert ok and ok_ref and turns >= 2
    assert st["outer_iterations"] == st_ref["outer_iterations"]
    assert torch.equal(x, x_ref)
    with pytest.raises(RuntimeError):
        gp.solve(b, x, resume=True)              # nothing paused any more


def test_served_stream_results_equal_lone_solves_and_pass_the_oracle(lib):
    from oracle.kkt import Problem as OP
    from paper_2405_18964_amd.batch import run
    jobs = [_job(w, a) for w, a in zip(MIX, (0.0, 0.05, 0.1, 0.15, 0.3))]
    print("lone solves", flush=True)
    lone = run([dict(j, arrival=0.0) for j in jobs], workers=1, checksum=True, **OPTS)
    print("served: 2 workers, one restart cycle per turn", flush=True)
    served = run(jobs, workers=2, slice_cycles=1, checksum=True, keep_solutions=True, **OPTS)
    for k, (w, a, r) in enumerate(zip(MIX, lone, served)):
        op = OP.from_workload(w, W.wind_nodal(w.N) if w.flow == W.OSEEN else None)
        bo = op.rhs(W.desired_state(w))
        x = op.to_compact(r["solution"])
        res = np.linalg.norm(bo - op.kkt_apply(x)) / np.linalg.norm(bo)
        print(f"  {w.name}: {r['slices']} turns, start {r['start']:.2f} s, end {r['end']:.2f} s, "
              f"oracle residual {res:.2e}, same as lone: {a['digest'] == r['digest']}", flush=True)
        assert r["converged"] and a["converged"]
        assert a["digest"] == r["digest"]
        assert res <= 1e-8
        assert r["start"] >= r["arrival"]
    assert max(r["slices"] for r in served) >= 3
