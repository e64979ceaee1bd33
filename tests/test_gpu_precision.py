"""Mixed precision: FP32 block solves inside the FP64 outer FGMRES.

The per-frequency work (FFT output, multigrid, Chebyshev, inner GMRES) runs
in FP32 while the outer FGMRES, its orthogonalisation, residual
recomputation and the KKT matrix stay FP64, so the outer loop acts as
iterative refinement.  The Q2 multigrid kernels compute in FP32 as well.
Tolerances: one preconditioner application agrees with the FP64 oracle to
1e-5 relative (FP32 rounding, unit 6e-8, over a few hundred dependent
operations of multigrid cycles whose residuals are ~cond(A) times smaller
than their terms; measured 5e-8 to 6e-8 here); solves still reach a true
residual of 1e-8 and agree with the FP64 direct solution to 1e-5.
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


@pytest.mark.parametrize("N,nt,beta", [(8, 16, 1e-2), (16, 32, 1e-4)])
def test_precond_linear_fp32(lib, N, nt, beta):
    from oracle.kkt import Problem as OP
    from oracle.precond import StokesPreconditioner
    print(f"fp32 precond N={N} nt={nt}", flush=True)
    w = W.small(W.STOKES, N, nt, beta=beta)
    op = OP.from_workload(w)
    gp = lib.Problem.from_workload(w, precision=lib.PREC_FP32_INNER)
    r = W.random_canonical(N, nt, seed=5)
    z = _host(gp.precond_apply(_dev(r)))
    ref = op.to_canonical(StokesPreconditioner(op).apply(op.to_compact(r)))
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    print(f"  relative error vs FP64 oracle: {err:.2e}")
    assert err <= 1e-5


@pytest.mark.parametrize("inner", ["linear", "gmres"])
def test_solve_fp32_inner_reaches_fp64_tolerance(lib, inner):
    from oracle.kkt import Problem as OP
    w = W.config(1)
    print(f"fp32 solve {w.name} inner={inner}", flush=True)
    mode = lib.INNER_GMRES if inner == "gmres" else lib.INNER_LINEAR
    gp = lib.Problem.from_workload(w, inner=mode, precision=lib.PREC_FP32_INNER, restart=30, max_outer=300)
    b = gp.assemble_rhs(_dev(W.desired_state(w)))
    x, st, ok = gp.solve(b)
    assert ok and st["rel_residual"] <= 1e-8
    op = OP.from_workload(w)
    xh, bh = _host(x), _host(b)
    res = np.linalg.norm(bh - op.to_canonical(op.kkt_apply(op.to_compact(xh)))) / np.linalg.norm(bh)
    assert res <= 1e-8
    xs = op.to_canonical(op.solve_direct(op.to_compact(bh)))
    err = np.linalg.norm(xh - xs) / np.linalg.norm(xs)
    print(f"  outer its {st['outer_iterations']}, error vs FP64 direct solve {err:.2e}")
    assert err <= 1e-5
