"""Pins of the oracle on the paper's own test problems (section 5) and of the
square-domain scaling.

* The section 5.1 data fix the continuous optimum: the state and adjoint
  equations of section 2.1 and both divergence constraints are checked
  pointwise by finite differences, so a transcription error in the data
  (desired state, forcing, known solution) fails here.
* The oracle's discrete solution with those data (general right-hand side,
  [-1, 1]^2, sparse direct solve) converges to the known state: the relative
  space-time L2 error drops by at least 8 from (N, nt) = (4, 8) to (8, 16)
  (measured 5.4e-3 -> 3.6e-4), and leaving out any one datum (initial
  velocity, Dirichlet values, forcing or desired state) breaks that.
* A square of side l equals the unit square's system with nu / l^2 and wind
  w / l up to the row and column scalings D_r, D_c (the identity the library
  uses for non-unit squares), checked on assembled matrices.
* With only a desired state that vanishes on the boundary the general
  right-hand side equals the homogeneous one.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle.kkt import Problem
from workloads import paper_problems as PP


def test_section51_data_satisfy_the_optimality_system():
    rng = np.random.default_rng(0)
    beta, T, eps = 1e-2, 1.0, 1e-4
    x = rng.uniform(-0.95, 0.95, size=20)
    y = rng.uniform(-0.95, 0.95, size=20)
    t = rng.uniform(0.05, 0.95, size=20)
    F = lambda dx, dy, dt: PP.stokes_exact_fields(x + dx, y + dy, t + dt, T, beta)
    c0 = F(0, 0, 0)
    xp, xm, yp, ym, tp, tm = F(eps, 0, 0), F(-eps, 0, 0), F(0, eps, 0), F(0, -eps, 0), F(0, 0, eps), F(0, 0, -eps)

    def lap(k):
        return (xp[k] + xm[k] + yp[k] + ym[k] - 4 * c0[k]) / eps ** 2

    def grad(k):
        return np.stack([(xp[k] - xm[k]) / (2 * eps), (yp[k] - ym[k]) / (2 * eps)])

    def div(k):
        return (xp[k][0] - xm[k][0] + yp[k][1] - ym[k][1]) / (2 * eps)

    state = (tp["v"] - tm["v"]) / (2 * eps) - lap("v") + grad("p") - c0["lambda"] / beta - c0["f"]
    adjoint = -(tp["lambda"] - tm["lambda"]) / (2 * eps) - lap("lambda") + grad("mu") - (c0["vd"] - c0["v"])
    scale = 1.0 + np.abs(c0["v"]) + np.abs(c0["f"]) + np.abs(c0["vd"])
    assert np.all(np.abs(state) <= 1e-4 * scale), np.abs(state / scale).max()
    assert np.all(np.abs(adjoint) <= 1e-4 * scale), np.abs(adjoint / scale).max()
    assert np.all(np.abs(div("v")) <= 1e-6 * (1 + np.abs(c0["v"]).max()))
    assert np.all(np.abs(div("lambda")) <= 1e-8)
    # the boundary and terminal conditions of the adjoint (section 2.1)
    e = PP.stokes_exact_fields(np.array([-1.0, 1.0, 0.3, 0.3]), np.array([0.2, -0.4, -1.0, 1.0]), 0.5, T, beta)
    assert np.abs(e["lambda"]).max() == 0.0
    assert np.abs(PP.stokes_exact_fields(x, y, T, T, beta)["lambda"]).max() == 0.0


def _state_error(N, nt, drop=None):
    d = PP.stokes_exact(N, nt, T=1.0, beta=1e-2)
    P = Problem(N, nt, d.T, d.nu, d.beta, domain=d.domain)
    data = dict(vd=d.vd, f=d.f, h=d.h, v0=d.v0)
    if drop:
        data[drop] = None
    b = P.rhs_data(**data)
    x = P.solve_direct(b)
    assert np.linalg.norm(b - P.kkt_apply(x)) <= 1e-12 * np.linalg.norm(b)
    V = P.full_velocity(x, d.h, d.v0)
    M2 = P.ops.full["M2"]
    ev = V[1:] - d.exact["v"][1:]
    num = sum(ev[k, c] @ (M2 @ ev[k, c]) for k in range(nt) for c in range(2))
    den = sum(d.exact["v"][k + 1, c] @ (M2 @ d.exact["v"][k + 1, c]) for k in range(nt) for c in range(2))
    return np.sqrt(num / den)


@pytest.mark.slow
def test_stokes_exact_solution_discretisation_converges():
    e1, e2 = _state_error(4, 8), _state_error(8, 16)
    print(f"relative L2 state error {e1:.3e} -> {e2:.3e}")
    assert e2 <= 5e-4 and e1 / e2 >= 8.0


@pytest.mark.slow
@pytest.mark.parametrize("drop", ["v0", "h", "f", "vd"])
def test_leaving_out_a_datum_breaks_convergence(drop):
    e1, e2 = _state_error(4, 8, drop), _state_error(8, 16, drop)
    print(f"without {drop}: {e1:.3e} -> {e2:.3e}")
    assert e2 >= 3e-3 and e1 / e2 < 4.0


@pytest.mark.parametrize("flow", [W.STOKES, W.OSEEN])
def test_square_of_side_l_is_a_scaled_unit_square(flow):
    N, nt, T, nu, beta, l = 4, 4, 1.0, 0.03, 1e-2, 2.0
    wind = PP.cavity_wind(N) if flow == W.OSEEN else None
    A = Problem(N, nt, T, nu, beta, wind, domain=(-1.0, -1.0, 1.0, 1.0)).kkt_matrix()
    Au = Problem(N, nt, T, nu / l ** 2, beta, None if wind is None else wind / l).kkt_matrix()
    P = Problem(N, nt, T, nu, beta)
    nv = P.nv
    lev_r = np.concatenate([np.full(nv, l * l), np.full(P.nP, l)])
    lev_c = np.concatenate([np.ones(nv), np.full(P.nP, 1.0 / l)])
    Dr = sp.diags(np.tile(lev_r, 2 * nt))
    Dc = sp.diags(np.tile(lev_c, 2 * nt))
    diff = (A - Dr @ Au @ Dc).tocoo()
    assert np.abs(diff.data).max(initial=0.0) <= 1e-13 * np.abs(A.data).max()


def test_rhs_data_reduces_to_the_homogeneous_rhs():
    w = W.small(W.STOKES, 4, 8)
    P = Problem.from_workload(w)
    vd = W.desired_state(w)
    assert np.allclose(P.rhs_data(vd=vd), P.rhs(vd), rtol=0, atol=1e-15)
    assert np.abs(P.rhs_data()).max() == 0.0
