"""Inner MINRES on the Stokes blocks (options.inner = PINTOC_INNER_MINRES).

The variant of Algorithm 2 that solves the real symmetric Z_j of section 3.2
with preconditioned MINRES and the Hermitian positive definite P~_j,
against the oracle's StokesPreconditioner with inner_solver="minres":

* one nonlinear preconditioner application: per-frequency step counts equal
  to the oracle's and the output within 1e-10 (FP64) -- at N = 8 and 16 in the
  small-grid multigrid kernels, at N = 32 (two ragged 48-node tiles) with the
  tiled smoother against the oracle's tiled variant;
* full solves (FGMRES outside) reach the true residual 1e-8, recomputed by
  the oracle, in FP64 and with FP32 inner solves;
* the workspace holds seven block vectors instead of the GMRES basis.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

Q2_TILE, Q1_TILE = 48, 32           # the library's tiled smoother (include/pintoc.h)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def lib():
    import paper_2405_18964_amd as P
    P.library()
    return P


@pytest.mark.parametrize("N,nt,beta", [(8, 16, 1e-2), (16, 8, 1e-4), (32, 8, 1e-3)])
def test_precond_minres_parity(lib, N, nt, beta):
    from oracle.kkt import Problem as OP
    from oracle.precond import Settings, StokesPreconditioner
    from oracle.smoothers import Tiling
    print(f"precond inner minres N={N} nt={nt}", flush=True)
    w = W.small(W.STOKES, N, nt, beta=beta)
    op = OP.from_workload(w)
    gp = lib.Problem.from_workload(w, inner=lib.INNER_MINRES)
    r = W.random_canonical(N, nt, seed=21)
    z = _host(gp.precond_apply(_dev(r)))
    counts = gp.last_inner_iterations()
    pc = StokesPreconditioner(op, Settings(inner_solver="minres", tiling=Tiling(Q2_TILE, Q1_TILE)))
    ref = op.to_canonical(pc.apply(op.to_compact(r), nonlinear=True))
    oracle_counts = [pc.inner_its[j] for j in range(nt // 2 + 1)]
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    print(f"  counts {counts}, rel error {err:.2e}", flush=True)
    assert counts == oracle_counts
    assert err <= 1e-10
    assert np.all(z[~W.canonical_mask(N, nt)] == 0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_solve_inner_minres(lib, precision):
    from oracle.kkt import Problem as OP
    w = W.small(W.STOKES, 16, 32, beta=1e-4)
    print(f"solve inner minres {w.name} {precision}", flush=True)
    prec = lib.PREC_FP64 if precision == "fp64" else lib.PREC_FP32_INNER
    gm = lib.Problem.from_workload(w, inner=lib.INNER_GMRES, precision=prec)
    gp = lib.Problem.from_workload(w, inner=lib.INNER_MINRES, precision=prec)
    assert gp.workspace_bytes < gm.workspace_bytes
    b = gp.assemble_rhs(_dev(W.desired_state(w)))
    x, st, ok = gp.solve(b)
    assert ok and st["rel_residual"] <= 1e-8
    xg, sg, okg = gm.solve(gm.assemble_rhs(_dev(W.desired_state(w))))
    op = OP.from_workload(w)
    xh, bh = _host(x), _host(b)
    res = np.linalg.norm(bh - op.to_canonical(op.kkt_apply(op.to_compact(xh)))) / np.linalg.norm(bh)
    diff = np.linalg.norm(xh - _host(xg)) / np.linalg.norm(_host(xg))
    print(f"  outer {st['outer_iterations']} (GMRES inner {sg['outer_iterations']}), inner mean "
          f"{st['inner_iterations_mean']:.1f} (GMRES {sg['inner_iterations_mean']:.1f}), oracle residual {res:.2e}, "
          f"difference from the GMRES-inner solution {diff:.2e}, workspace {gp.workspace_bytes / 2**20:.0f} MiB "
          f"(GMRES {gm.workspace_bytes / 2**20:.0f} MiB)", flush=True)
    assert res <= 1e-8
    assert diff <= 1e-6


def test_group_inner_minres_equals_lone(lib):
    """Fused group (two Stokes members of one grid): the per-frequency MINRES
    runs over the members' frequencies in one batch; every member's result
    equals its lone solve bit for bit."""
    print("group inner minres", flush=True)
    ws = [W.small(W.STOKES, 16, 16, beta=1e-3), W.small(W.STOKES, 16, 32, beta=1e-4)]
    opts = dict(inner=lib.INNER_MINRES)
    members = [{"N": w.N, "nt": w.nt, "T": w.T, "nu": w.nu, "beta": w.beta, "flow": w.flow} for w in ws]
    g = lib.Group(members, **opts)
    bs = [g.assemble_rhs(i, _dev(W.desired_state(w))) for i, w in enumerate(ws)]
    xs, sts, oks = g.solve(bs)
    for i, w in enumerate(ws):
        gp = lib.Problem.from_workload(w, **opts)
        x, st, ok = gp.solve(gp.assemble_rhs(_dev(W.desired_state(w))))
        assert oks[i] and ok
        assert sts[i]["outer_iterations"] == st["outer_iterations"]
        assert np.array_equal(_host(xs[i]), _host(x))
