"""GPU parity of the Oseen path (section 4, Algorithm 3) against the oracle.

Wind w = (2y(1-x^2), -2x(1-y^2)) as Q2 nodal values.  Same bars as the
Stokes tests: all-at-once matrix 1e-13; one application of P~_j^(UZ) (6 Uzawa
steps, 4 V-cycles per multigrid solve, 10 Chebyshev steps) 1e-10; GMRES mode
with identical inner counts 1e-10; small solves to a true residual of 1e-8.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


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


def _pair(lib, N, nt, nu, beta, **opts):
    from oracle.kkt import Problem as OP
    w = W.Workload(W.OSEEN, N, nt, 1.0, nu, beta, 0, 1.0)
    wind = W.wind_nodal(N)
    return w, wind, OP.from_workload(w, wind), lib.Problem.from_workload(w, **opts)


CASES = [(4, 8, 0.1, 1e-2), (8, 16, 0.01, 1e-4), (16, 32, 0.01, 1e-4)]


@pytest.mark.parametrize("N,nt,nu,beta", CASES)
def test_oseen_kkt_apply_parity(lib, N, nt, nu, beta):
    print(f"oseen kkt N={N} nt={nt}", flush=True)
    w, wind, op, gp = _pair(lib, N, nt, nu, beta)
    xc = W.random_canonical(N, nt, seed=13)
    y = _host(gp.kkt_apply(_dev(xc)))
    ref = op.to_canonical(op.kkt_apply(op.to_compact(xc)))
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("N,nt,nu,beta", CASES)
def test_oseen_precond_linear_parity(lib, N, nt, nu, beta):
    from oracle.precond import OseenPreconditioner
    print(f"oseen precond N={N} nt={nt}", flush=True)
    w, wind, op, gp = _pair(lib, N, nt, nu, beta)
    r = W.random_canonical(N, nt, seed=7)
    z = _host(gp.precond_apply(_dev(r)))
    ref = op.to_canonical(OseenPreconditioner(op, wind).apply(op.to_compact(r), nonlinear=False))
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)
    assert np.all(z[~W.canonical_mask(N, nt)] == 0)


@pytest.mark.parametrize("N,nt,nu,beta", CASES[1:])
def test_oseen_precond_gmres_parity(lib, N, nt, nu, beta):
    from oracle.precond import OseenPreconditioner
    print(f"oseen precond gmres N={N} nt={nt}", flush=True)
    w, wind, op, gp = _pair(lib, N, nt, nu, beta, inner=lib.INNER_GMRES)
    r = op.to_canonical(op.rhs(W.desired_state(w)))
    z = _host(gp.precond_apply(_dev(r)))
    pc = OseenPreconditioner(op, wind)
    ref = op.to_canonical(pc.apply(op.to_compact(r), nonlinear=True))
    assert gp.last_inner_iterations() == [pc.inner_its[j] for j in range(nt // 2 + 1)]
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_oseen_solve_small(lib, precision):
    from oracle.kkt import Problem as OP
    N, nt = 8, 16
    print(f"oseen solve N={N} nt={nt} {precision}", flush=True)
    prec = lib.PREC_FP64 if precision == "fp64" else lib.PREC_FP32_INNER
    w, wind, op, gp = _pair(lib, N, nt, 0.1, 1e-4, inner=lib.INNER_GMRES, precision=prec)
    b = gp.assemble_rhs(_dev(W.desired_state(w)))
    x, st, ok = gp.solve(b)
    assert ok and st["rel_residual"] <= 1e-8
    xh, bh = _host(x), _host(b)
    res = np.linalg.norm(bh - op.to_canonical(op.kkt_apply(op.to_compact(xh)))) / np.linalg.norm(bh)
    assert res <= 1e-8
    xs = op.to_canonical(op.solve_direct(op.to_compact(bh)))
    assert np.linalg.norm(xh - xs) <= 1e-5 * np.linalg.norm(xs)


def test_oseen_precond_single_frequency_full_size(lib):
    """Full size of the Oseen workload (N=128, nt=128, nu=1/100, beta=1e-4):
    a residual with one temporal Fourier mode is checked against the oracle's
    block j and nt-j alone."""
    from oracle.precond import OseenPreconditioner, Settings
    from oracle.smoothers import Tiling   # the library's tiled smoother (include/pintoc.h)
    w = W.config(3)
    j = 21
    print(f"oseen precond full size mode j={j}", flush=True)
    wind = W.wind_nodal(w.N)
    gp = lib.Problem.from_workload(w)
    r = W.single_frequency_canonical(w.N, w.nt, j, seed=4)
    z = _host(gp.precond_apply(_dev(r)))
    from oracle.kkt import Problem as OP
    op = OP.from_workload(w, wind)
    pc = OseenPreconditioner(op, wind, Settings(tiling=Tiling(48, 32)), freqs=[j, w.nt - j])
    ref = op.to_canonical(pc.apply(op.to_compact(r), nonlinear=False))
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)


def test_oseen_solve_full_size_oracle_residual(lib):
    """The Oseen workload (N=128, nt=128, nu=1/100, beta=1e-4) with FP32 inner
    solves and FP64 outer FGMRES: the true residual of the GPU solution,
    recomputed by the oracle's level-by-level all-at-once product (with the
    convection operator) against the oracle's right-hand side, is at most 1e-8
    of ||b||."""
    from oracle.kkt import Problem as OP
    w = W.config(3)
    print(f"oseen full-size solve {w.name}", flush=True)
    wind = W.wind_nodal(w.N)
    vd = W.desired_state(w)
    gp = lib.Problem.from_workload(w, inner=lib.INNER_GMRES, precision=lib.PREC_FP32_INNER, max_outer=60)
    x, st, ok = gp.solve(gp.assemble_rhs(_dev(vd)))
    assert ok and st["rel_residual"] <= 1e-8
    xh = _host(x)
    del x, gp
    torch.cuda.empty_cache()
    op = OP.from_workload(w, wind)
    bo = op.rhs(vd)
    rel = np.linalg.norm(bo - op.kkt_apply(op.to_compact(xh))) / np.linalg.norm(bo)
    print(f"oracle residual {rel:.3e}, library {st['rel_residual']:.3e}", flush=True)
    assert rel <= 1e-8
    assert abs(rel - st["rel_residual"]) <= 1e-3 * st["rel_residual"]
