"""GPU parity on the paper's own test problems (section 5) on [-1, 1]^2.

* section 5.1, Stokes with a known solution: right-hand side from forcing,
  Dirichlet and initial data, all-at-once matrix and linear preconditioner
  on the square of side 2 against the oracle (1e-13 / 1e-10); the tight
  solve against the oracle's sparse direct solve; GPU solves on three grids
  converge to the known state (each solve's true residual recomputed by the
  oracle).
* section 5.2, the lid-driven cavity Oseen problem (two-vortex wind, lid,
  wedge initial velocity): the same parity checks and solves.
"""
import numpy as np
import pytest

import workloads as W
from workloads import paper_problems as PP

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


def _data(kind, N, nt):
    return PP.stokes_exact(N, nt) if kind == "stokes" else PP.cavity(N, nt)


def _oracle(d):
    from oracle.kkt import Problem as OP
    return OP(d.N, d.nt, d.T, d.nu, d.beta, d.wind, domain=d.domain)


def _gpu(lib, d, **opts):
    return lib.Problem(d.N, d.nt, d.T, d.nu, d.beta, d.flow, d.wind, domain=d.domain, **opts)


def _rhs(gp, d):
    return gp.assemble_rhs_data(_dev(d.vd), _dev(d.f), _dev(d.h), _dev(d.v0))


@pytest.mark.parametrize("kind", ["stokes", "cavity"])
def test_rhs_and_matvec_parity(lib, kind):
    d = _data(kind, 8, 8)
    print(f"{kind} rhs/matvec N=8 nt=8", flush=True)
    op, gp = _oracle(d), _gpu(lib, d)
    b = _host(_rhs(gp, d))
    ref = op.to_canonical(op.rhs_data(d.vd, d.f, d.h, d.v0))
    eb = np.abs(b - ref).max() / np.abs(ref).max()
    x = W.random_canonical(d.N, d.nt, seed=7)
    y = _host(gp.kkt_apply(_dev(x)))
    yr = op.to_canonical(op.kkt_apply(op.to_compact(x)))
    ey = np.abs(y - yr).max() / np.abs(yr).max()
    print(f"  rhs {eb:.2e}, matvec {ey:.2e}", flush=True)
    assert eb <= 1e-13 and ey <= 1e-13


@pytest.mark.parametrize("N", [8, 32])
@pytest.mark.parametrize("kind", ["stokes", "cavity"])
def test_linear_preconditioner_parity(lib, kind, N):
    """The library applies the unit-square preconditioner with nu / 4, w / 2
    between the domain scalings; the oracle builds it from the matrices of
    the square of side 2."""
    from oracle.precond import OseenPreconditioner, Settings, StokesPreconditioner
    from oracle.smoothers import Tiling
    d = _data(kind, N, 8)
    print(f"{kind} linear preconditioner N={N} nt=8", flush=True)
    op, gp = _oracle(d), _gpu(lib, d)
    r = W.random_canonical(N, 8, seed=9)
    z = _host(gp.precond_apply(_dev(r)))
    st = Settings(tiling=Tiling(48, 32))
    pc = StokesPreconditioner(op, st) if d.flow == 0 else OseenPreconditioner(op, d.wind, st)
    ref = op.to_canonical(pc.apply(op.to_compact(r)))
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    print(f"  rel error {err:.2e}", flush=True)
    assert err <= 1e-10


@pytest.mark.parametrize("kind", ["stokes", "cavity"])
def test_tight_solve_against_direct(lib, kind):
    d = _data(kind, 8, 8)
    print(f"{kind} tight solve N=8 nt=8", flush=True)
    op, gp = _oracle(d), _gpu(lib, d, restart=30, max_outer=900, tol=1e-12)
    b = _rhs(gp, d)
    x, st, ok = gp.solve(b)
    xs = op.to_canonical(op.solve_direct(op.rhs_data(d.vd, d.f, d.h, d.v0)))
    xh = _host(x)
    err = np.linalg.norm(xh - xs) / np.linalg.norm(xs)
    print(f"  {st['outer_iterations']} its, residual {st['rel_residual']:.2e}, error against sparse LU {err:.2e}",
          flush=True)
    assert ok and err <= 1e-9


def _l2_state_error(op, d, xh):
    V = op.full_velocity(op.to_compact(xh), d.h, d.v0)
    M2 = op.ops.full["M2"]
    ev = V[1:] - d.exact["v"][1:]
    num = sum(ev[k, c] @ (M2 @ ev[k, c]) for k in range(d.nt) for c in range(2))
    den = sum(d.exact["v"][k + 1, c] @ (M2 @ d.exact["v"][k + 1, c]) for k in range(d.nt) for c in range(2))
    return np.sqrt(num / den)


def test_stokes_exact_solution_gpu_convergence(lib):
    """Section 5.1 solved on the GPU (nonlinear preconditioner, FP64) on
    grids N = 16, 32, 64 with nt = 2N: every solve reaches the 1e-8 true
    residual (recomputed by the oracle) and the state error against the
    known solution falls by at least 1.8 per refinement (backward Euler is
    first order in tau)."""
    errs = []
    for N in (16, 32, 64):
        d = PP.stokes_exact(N, 2 * N)
        print(f"stokes exact N={N} nt={2 * N}", flush=True)
        gp = _gpu(lib, d, inner=lib.INNER_GMRES, max_outer=100)
        b = _rhs(gp, d)
        x, st, ok = gp.solve(b)
        bh, xh = _host(b), _host(x)
        del gp, b, x
        torch.cuda.empty_cache()
        op = _oracle(d)
        res = np.linalg.norm(bh - op.to_canonical(op.kkt_apply(op.to_compact(xh)))) / np.linalg.norm(bh)
        errs.append(_l2_state_error(op, d, xh))
        print(f"  {st['outer_iterations']} its, oracle residual {res:.2e}, state error {errs[-1]:.3e}", flush=True)
        assert ok and res <= 1e-8
    assert errs[0] / errs[1] >= 1.8 and errs[1] / errs[2] >= 1.8


def test_cavity_solve_full_grid(lib):
    """Section 5.2 at N = 64, nt = 32 with the nonlinear preconditioner and
    FP32 inner solves: true residual 1e-8, recomputed by the oracle."""
    d = PP.cavity(64, 32)
    print("cavity N=64 nt=32 fp32-inner", flush=True)
    gp = _gpu(lib, d, inner=lib.INNER_GMRES, precision=lib.PREC_FP32_INNER, max_outer=100)
    b = _rhs(gp, d)
    x, st, ok = gp.solve(b)
    bh, xh = _host(b), _host(x)
    op = _oracle(d)
    res = np.linalg.norm(bh - op.to_canonical(op.kkt_apply(op.to_compact(xh)))) / np.linalg.norm(bh)
    print(f"  {st['outer_iterations']} its, inner mean {st['inner_iterations_mean']:.1f}, oracle residual {res:.2e}",
          flush=True)
    assert ok and res <= 1e-8
