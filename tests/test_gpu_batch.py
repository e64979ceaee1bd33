"""Batched solves: several problems concurrently on one GPU.

Each result must be the same alone and in the mix.  Every kernel and reduction
of a solve depends only on its own problem and runs in a fixed order, so the
solutions agree bit for bit (the tolerance is zero) and the iteration counts
are equal; each batched solve also reaches the true residual 1e-8.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MIX = [W.small(W.STOKES, 8, 16, beta=1e-2, seed=1),
       W.small(W.OSEEN, 8, 16, beta=1e-4, nu=0.1, seed=2),
       W.small(W.STOKES, 16, 32, beta=1e-4, seed=3),
       W.small(W.OSEEN, 16, 8, beta=1e-3, nu=0.5, seed=4)]


@pytest.fixture(scope="module")
def lib():
    import paper_2405_18964_amd as P
    P.library()
    return P


def _problem(lib, w, **opts):
    return lib.Problem.from_workload(w, inner=lib.INNER_GMRES, max_outer=200, **opts)


def _alone(lib, w, **opts):
    p = _problem(lib, w, **opts)
    b = p.assemble_rhs(torch.from_numpy(W.desired_state(w)).cuda())
    x, st, ok = p.solve(b)
    torch.cuda.synchronize()
    return x.cpu().numpy(), st, ok


@pytest.mark.parametrize("precision", [0, 1])
def test_solve_batch_equals_single(lib, precision):
    print(f"solve_batch mix of {len(MIX)} precision={precision}", flush=True)
    alone = [_alone(lib, w, precision=precision) for w in MIX]
    probs = [_problem(lib, w, precision=precision) for w in MIX]
    bs = [p.assemble_rhs(torch.from_numpy(W.desired_state(w)).cuda()) for p, w in zip(probs, MIX)]
    res = lib.solve_batch(probs, bs)
    torch.cuda.synchronize()
    for (xa, sa, oka), (xb, sb, okb) in zip(alone, res):
        assert oka and okb and sb["rel_residual"] <= 1e-8
        assert sa["outer_iterations"] == sb["outer_iterations"]
        assert np.array_equal(xa, xb.cpu().numpy())


def test_batch_runner_budget(lib):
    """Two workers under a budget that fits only one job at a time for the
    larger problems: every job still runs, and each result equals its lone solve."""
    from paper_2405_18964_amd.batch import job_bytes, run
    print("batch runner", flush=True)
    jobs = [{"N": w.N, "nt": w.nt, "T": w.T, "nu": w.nu, "beta": w.beta, "flow": w.flow,
             "wind": W.wind_nodal(w.N) if w.flow == W.OSEEN else None, "vd": W.desired_state(w)} for w in MIX]
    opts = dict(inner=lib.INNER_GMRES, max_outer=200)
    need = [job_bytes(j, **opts) for j in jobs]
    out = run(jobs, workers=2, budget_bytes=max(need) + min(need), keep_solutions=True, **opts)
    for w, rec in zip(MIX, out):
        xa, sa, oka = _alone(lib, w)
        assert rec["converged"] and oka
        assert np.array_equal(rec["solution"], xa)
        assert rec["end"] > rec["start"] >= 0
