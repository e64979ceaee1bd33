"""Outer FGMRES in the frequency domain (PINTOC_OUTER_FGMRES_FREQ; section
3.1, Theorem 1: A = P_C + corner term, so the Fourier-transformed matrix is
the blocks G_j plus two time samples spread over all frequencies, and the
iterations need no FFT).

The scaled spectra make the Krylov method the time-domain FGMRES in another
orthonormal basis, so it takes the same number of outer iterations (within
one, for rounding at the stopping test) and reaches the same solution:
* tight solves of small Stokes and Oseen problems against the oracle's sparse
  direct solve (1e-9);
* solves at 1e-8 whose true residual the oracle recomputes, in FP64 and with
  FP32 inner solves (Stokes), iteration counts against the time-domain FGMRES.
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


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("flow", [W.STOKES, W.OSEEN])
def test_tight_solve_against_direct(lib, flow):
    from oracle.kkt import Problem as OP
    w = W.config(1) if flow == W.STOKES else W.Workload(W.OSEEN, 8, 8, 1.0, 0.1, 1e-2, 5, 1.0)
    print(f"frequency-domain FGMRES, tight, {w.name}", flush=True)
    gp = lib.Problem.from_workload(w, outer=lib.OUTER_FGMRES_FREQ, restart=30, max_outer=900, tol=1e-12)
    b = gp.assemble_rhs(torch.from_numpy(W.desired_state(w)).cuda())
    x, st, ok = gp.solve(b)
    op = OP.from_workload(w, W.wind_nodal(w.N) if flow == W.OSEEN else None)
    bh, xh = _host(b), _host(x)
    xs = op.to_canonical(op.solve_direct(op.to_compact(bh)))
    err = np.linalg.norm(xh - xs) / np.linalg.norm(xs)
    print(f"  {st['outer_iterations']} its, residual {st['rel_residual']:.2e}, error against sparse LU {err:.2e}",
          flush=True)
    assert ok and st["rel_residual"] <= 1e-12 and err <= 1e-9
    assert np.all(xh[~W.canonical_mask(w.N, w.nt)] == 0)


CASES = [(W.small(W.STOKES, 16, 32, beta=1e-4, seed=71), "fp64", 1),
         (W.small(W.STOKES, 32, 32, beta=1e-3, seed=72), "fp32", 1),
         (W.Workload(W.OSEEN, 16, 16, 1.0, 0.02, 1e-3, 73, 1.0), "fp64", 1),
         (W.small(W.STOKES, 16, 16, beta=1e-2, seed=74), "fp64", 0)]


@pytest.mark.parametrize("w,precision,inner", CASES, ids=lambda c: getattr(c, "name", str(c)))
def test_solve_matches_time_domain_fgmres(lib, w, precision, inner):
    from oracle.kkt import Problem as OP
    prec = lib.PREC_FP64 if precision == "fp64" else lib.PREC_FP32_INNER
    restart = 10 if inner else 30
    print(f"frequency-domain FGMRES {w.name} {precision} inner={'gmres' if inner else 'linear'}", flush=True)
    opts = dict(inner=inner, precision=prec, restart=restart, max_outer=400)
    gt = lib.Problem.from_workload(w, **opts)
    b = gt.assemble_rhs(torch.from_numpy(W.desired_state(w)).cuda())
    xt, stt, okt = gt.solve(b)
    del gt
    gf = lib.Problem.from_workload(w, outer=lib.OUTER_FGMRES_FREQ, **opts)
    xf, stf, okf = gf.solve(b)
    op = OP.from_workload(w, W.wind_nodal(w.N) if w.flow == W.OSEEN else None)
    bh, xh = _host(b), _host(xf)
    res = np.linalg.norm(bh - op.to_canonical(op.kkt_apply(op.to_compact(xh)))) / np.linalg.norm(bh)
    print(f"  time domain {stt['outer_iterations']} its, frequency domain {stf['outer_iterations']} its, "
          f"oracle residual {res:.2e} (library {stf['rel_residual']:.2e})", flush=True)
    assert okt and okf and res <= 1e-8
    assert abs(stf["outer_iterations"] - stt["outer_iterations"]) <= 1
