"""Captured block-preconditioner applications (options.graphs = 1).

The launch sequence of a block preconditioner application is captured into a
HIP graph once per set of buffers and replayed.  A replay runs the same
kernels with the same arguments, so results must equal the eager launches
bit for bit -- checked on every replay, with other eager work and host
synchronisations between the replays:
* linear preconditioner (Algorithm 1 / Algorithm 3), Stokes and Oseen, FP64
  and FP32 inner, five replays each interleaved with another problem's eager
  applications;
* whole solves with inner GMRES (Algorithm 2 / its Oseen analogue), where the
  replayed graphs see a different convergence mask (device data) on every
  inner iteration, against the eager solve;
* on the legacy default stream the library launches eagerly (no capture).
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


CASES = [(W.small(W.STOKES, 32, 16, beta=1e-3, seed=81), "fp64"),
         (W.Workload(W.OSEEN, 16, 16, 1.0, 0.02, 1e-2, 82, 1.0), "fp64"),
         (W.small(W.STOKES, 16, 32, beta=1e-4, seed=83), "fp32"),
         (W.Workload(W.OSEEN, 32, 8, 1.0, 0.05, 1e-3, 84, 1.0), "fp32")]


@pytest.mark.parametrize("w,precision", CASES, ids=lambda c: getattr(c, "name", str(c)))
def test_linear_replays_equal_eager(lib, w, precision):
    prec = lib.PREC_FP64 if precision == "fp64" else lib.PREC_FP32_INNER
    print(f"graph replays, linear, {w.name} {precision}", flush=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        eager = lib.Problem.from_workload(w, precision=prec)
        graph = lib.Problem.from_workload(w, precision=prec, graphs=1)
        other = lib.Problem.from_workload(W.small(W.STOKES, 8, 16), precision=prec)
        r = torch.from_numpy(W.random_canonical(w.N, w.nt, seed=5)).cuda()
        ro = torch.from_numpy(W.random_canonical(8, 16, seed=6)).cuda()
        ref = eager.precond_apply(r)
        for k in range(5):
            z = graph.precond_apply(r)
            other.precond_apply(ro)                 # eager work between the replays
            stream.synchronize()
            assert torch.equal(z, ref), f"replay {k} differs"
            r2 = r * (1.0 + 0.1 * k)                # new data in the same buffer each time
            r.copy_(r2)
            ref = eager.precond_apply(r)
        torch.cuda.synchronize()


@pytest.mark.parametrize("w,precision", CASES[:2], ids=lambda c: getattr(c, "name", str(c)))
def test_gmres_solve_with_graphs_equals_eager(lib, w, precision):
    prec = lib.PREC_FP64 if precision == "fp64" else lib.PREC_FP32_INNER
    opts = dict(inner=lib.INNER_GMRES, precision=prec, max_outer=100)
    print(f"graph replays, inner GMRES solve, {w.name}", flush=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        vd = torch.from_numpy(W.desired_state(w)).cuda()
        pe = lib.Problem.from_workload(w, **opts)
        b = pe.assemble_rhs(vd)
        xe, ste, oke = pe.solve(b)
        pg = lib.Problem.from_workload(w, graphs=1, **opts)
        for rep in range(2):                        # second solve replays the graphs of the first
            xg, stg, okg = pg.solve(b)
            stream.synchronize()
            print(f"  solve {rep}: {stg['outer_iterations']} its (eager {ste['outer_iterations']}), "
                  f"identical {torch.equal(xg, xe)}", flush=True)
            assert oke and okg and torch.equal(xg, xe)
            assert stg["inner_counts"] == ste["inner_counts"]


def test_default_stream_launches_eagerly(lib):
    w = W.small(W.STOKES, 16, 16, beta=1e-3, seed=85)
    a = lib.Problem.from_workload(w)
    g = lib.Problem.from_workload(w, graphs=1)
    r = torch.from_numpy(W.random_canonical(w.N, w.nt, seed=7)).cuda()
    assert torch.equal(a.precond_apply(r), g.precond_apply(r))
