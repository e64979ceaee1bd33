"""Pins of the oracle's preconditioners (sections 2.3, 3.2-3.4, 4) and solvers."""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import circulant as circ
from oracle.fem import Operators
from oracle.kkt import Problem
from oracle.krylov import fgmres, gmres
from oracle.mg import Levels, ScalarMG, coarse_viscosity
from oracle.precond import OseenPreconditioner, StokesPreconditioner, stokes_constants
from oracle.smoothers import (Q1_MASS_BOUNDS, Q2_MASS_BOUNDS, ColouredSOR, TiledSOR, chebyshev,
                              chebyshev_error_bound, colours_q1, colours_q2, tiles_of)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def golden_bounds():
    out = {}
    for line in open(os.path.join(GOLD, "bounds.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, val = line.split()[:2]
        out[name] = float(val)
    return out


@pytest.fixture(scope="module")
def stokes4():
    w = W.small(W.STOKES, 4, 8, beta=1e-2)
    P = Problem.from_workload(w)
    return w, P, StokesPreconditioner(P)


def test_golden_bounds_closed_forms():
    g = golden_bounds()
    assert abs(g["phat_lower"] - 1 / np.sqrt(12)) < 1e-15
    assert abs(g["phat_upper"] - (1 + np.sqrt(5)) / 2) < 1e-15
    assert g["uzawa_mu"] == (g["pw_lower"] + g["pw_upper"]) / 2


@pytest.mark.parametrize("j", [0, 1, 3, 4, 7])
def test_gj_factorisation(stokes4, j):
    """P9: G_j = T_l Z_j T_r (eq. GJTransformation) with c1 = d_r / sqrt(tau^2/beta
    + d_c^2); T_l^H = T_r; the inverse transforms invert T_l and T_r."""
    _, P, pc = stokes4
    Tl, Z, Tr = pc.T_matrices(j)
    G = circ.G_block(P, pc.d[j])
    assert abs(Tl @ Z @ Tr - G).max() < 1e-14
    assert abs(Tl.conj().T - Tr).max() < 1e-15
    rng = np.random.default_rng(j)
    n = Tl.shape[0]
    r = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    cut = np.cumsum([P.nv, P.nv, P.nP])
    s = np.concatenate(pc.t_left_inv(j, *np.split(r, cut)))
    assert np.allclose(Tl @ s, r, atol=1e-13)
    y = np.concatenate(pc.t_right_inv(j, *np.split(r, cut)))
    assert np.allclose(Tr @ y, r, atol=1e-13)


def test_printed_c1_does_not_factorise(stokes4):
    """The constant c1 as printed (d_c not squared) breaks G_j = T_l Z_j T_r
    for j with d_c != +-1, which is why the squared form is used."""
    _, P, pc = stokes4
    j = 1
    dr, dc, c1, c2 = pc.constants(j)
    c1_printed = dr / np.sqrt(P.tau ** 2 / P.beta + dc)
    assert abs(c1 - dr * c2 / P.tau) < 1e-15
    assert abs(c1_printed - c1) > 1e-3 * abs(c1)


@pytest.mark.parametrize("j", [0, 2, 4])
def test_phat_bounds(stokes4, j):
    """P10, eq. (SchurComplementHatBounds): |eig(P^_j^{-1} Z_j)| in
    [1/sqrt(12), (1+sqrt(5))/2] with W_j = (1+c1)M + c2 L and exact B W^{-1} B^T."""
    g = golden_bounds()
    _, P, pc = stokes4
    o = P.ops
    _, _, c1, c2 = pc.constants(j)
    Wj = ((1 + c1) * o.M + c2 * o.L).toarray()
    B = o.B.toarray()
    S = B @ np.linalg.solve(Wj, B.T)
    Ph = sla.block_diag(Wj, Wj, S, S)
    ev = np.abs(np.linalg.eigvals(np.linalg.solve(Ph, pc.Z_matrix(j).toarray())))
    assert ev.min() >= g["phat_lower"] - 1e-10
    assert ev.max() <= g["phat_upper"] + 1e-10


def test_stokes_schur_commutator_algebra(stokes4):
    """P15: M_p ((1+c1) M_p + c2 nu K_p)^{-1} K_p = ((1+c1) K_p^{-1} + nu c2 M_p^{-1})^{-1}."""
    _, P, pc = stokes4
    o = P.ops
    _, _, c1, c2 = pc.constants(3)
    Mp, Kp = o.Mp.toarray(), o.Kp.toarray()
    lhs = Mp @ np.linalg.solve((1 + c1) * Mp + c2 * P.nu * Kp, Kp)
    rhs = np.linalg.inv((1 + c1) * np.linalg.inv(Kp) + P.nu * c2 * np.linalg.inv(Mp))
    assert np.allclose(lhs, rhs, rtol=1e-10, atol=1e-12)


def _pin_ops(N):
    o = Operators(N, 1.0)
    np2 = o.grid.np2
    R = np.eye(np2)[1:]
    Lmap = np.eye(np2) - np.outer(np.ones(np2), np.eye(np2)[0])     # y - y0 * 1
    return o, R, Lmap


def test_pinned_inverse_identity():
    """For any S whose left and right kernels are the constant pressures,
    (R S R^T)^{-1} = R L S^+ L^T R^T with L = I - 1 e0^T (the identity used to
    carry the commutator Schur approximation onto the pinned space)."""
    N = 4
    o, R, Lmap = _pin_ops(N)
    Bfull = np.hstack([o.full["Bx"].toarray() @ o.grid.Rv().T.toarray(),
                       o.full["By"].toarray() @ o.grid.Rv().T.toarray()])
    Wd = (1.3 * o.M + 0.2 * o.L).toarray()
    S = Bfull @ np.linalg.solve(Wd, Bfull.T)
    lhs = np.linalg.inv(R @ S @ R.T)
    rhs = R @ Lmap @ np.linalg.pinv(S) @ Lmap.T @ R.T
    assert np.allclose(lhs, rhs, rtol=1e-9, atol=1e-9 * np.abs(lhs).max())


@pytest.mark.parametrize("N", [4, 8])
def test_pinned_schur_spectrum_h_robust(N):
    """With the mass term transported by the identity above, eig(S^^{-1} S)
    stays in [0.2, 1] (no h-dependent outlier from the pressure pin)."""
    w = W.small(W.STOKES, N, 8, beta=1e-2)
    P = Problem.from_workload(w)
    pc = StokesPreconditioner(P, freqs=[1])
    o = P.ops
    _, _, c1, c2 = pc.constants(1)
    Wj = ((1 + c1) * o.M + c2 * o.L).toarray()
    B = o.B.toarray()
    S = B @ np.linalg.solve(Wj, B.T)
    np2 = o.grid.np2
    R = np.eye(np2)[1:]
    Lmap = np.eye(np2) - np.outer(np.ones(np2), np.eye(np2)[0])
    MNi = Lmap @ np.linalg.inv(o.full["M1"].toarray()) @ Lmap.T
    Shinv = (1 + c1) * np.linalg.inv(o.Kp.toarray()) + P.nu * c2 * (R @ MNi @ R.T)
    ev = np.linalg.eigvals(Shinv @ S).real
    assert ev.min() > 0.2 and ev.max() < 1.0 + 1e-10


@pytest.mark.parametrize("j", [0, 1, 3])
def test_pearson_wathen_bounds_complex(j):
    """P11, eq. (SchurComplementPearsonWathen): for G_j^(1,1) (Oseen, complex
    d_j) eig(S^^{-1} S) in [1/2, 1] with S^ = tau^{-1} Q_j M^{-1} Q_j^H."""
    g = golden_bounds()
    N = 4
    w = W.small(W.OSEEN, N, 8, beta=1e-2, nu=0.1)
    P = Problem.from_workload(w, W.wind_nodal(N))
    o, tau, beta = P.ops, P.tau, P.beta
    d = circ.d_closed_form(P.nt)[j]
    M, L = o.M.toarray(), o.L.toarray()
    Psi = d * M + tau * L
    S = (tau / beta) * M + Psi @ np.linalg.solve(tau * M, Psi.conj().T)
    Q = Psi + tau / np.sqrt(beta) * M
    Sh = Q @ np.linalg.solve(M, Q.conj().T) / tau
    ev = np.linalg.eigvals(np.linalg.solve(Sh, S))
    assert np.abs(ev.imag).max() < 1e-9
    assert ev.real.min() >= g["pw_lower"] - 1e-9 and ev.real.max() <= g["pw_upper"] + 1e-9


def test_uzawa_exact_components():
    """P14: with exact M^ = M and S^ = S and mu = 1, Uzawa from zero gives the
    exact x2 after one step and the exact x1 after two (eq. Uzawa11 signs)."""
    N = 2
    w = W.small(W.OSEEN, N, 4, beta=1e-2, nu=0.1)
    wind = W.wind_nodal(N)
    P = Problem.from_workload(w, wind)
    pc = OseenPreconditioner(P, wind, freqs=[1])
    o, tau, beta = P.ops, P.tau, P.beta
    j = 1
    d = pc.d[j]
    M, L = o.M.toarray(), o.L.toarray()
    Psi = d * M + tau * L
    S = (tau / beta) * M + Psi @ np.linalg.solve(tau * M, Psi.conj().T)
    G11 = np.block([[tau * M, Psi.conj().T], [Psi, -(tau / beta) * M]])
    rng = np.random.default_rng(0)
    b = rng.standard_normal(2 * P.nv) + 1j * rng.standard_normal(2 * P.nv)
    x = np.linalg.solve(G11, b)
    Minv = lambda v: np.linalg.solve(M, v)
    Sinv = lambda v: np.linalg.solve(S, v)
    x1, x2 = pc.uzawa(j, b[:P.nv], b[P.nv:], Minv, Sinv, mu=1.0, steps=1)
    assert np.allclose(x2, x[P.nv:], atol=1e-10 * np.abs(x).max())
    x1, x2 = pc.uzawa(j, b[:P.nv], b[P.nv:], Minv, Sinv, mu=1.0, steps=2)
    assert np.allclose(x1, x[:P.nv], atol=1e-10 * np.abs(x).max())
    # with the Pearson-Wathen S^ and mu = 3/4 the error contracts by <= 1/3 per step
    Q = Psi + tau / np.sqrt(beta) * M
    Sh = Q @ np.linalg.solve(M, Q.conj().T) / tau
    Shinv = lambda v: np.linalg.solve(Sh, v)
    errs = []
    for k in (3, 4):
        _, x2 = pc.uzawa(j, b[:P.nv], b[P.nv:], Minv, Shinv, mu=0.75, steps=k)
        errs.append(np.linalg.norm(x2 - x[P.nv:]))
    assert errs[1] <= errs[0] / 3 + 1e-12


@pytest.mark.parametrize("fam,bounds", [("q2", Q2_MASS_BOUNDS), ("q1", Q1_MASS_BOUNDS)])
def test_chebyshev_error_bound(fam, bounds):
    """P12: after k steps the M-norm error is at most 1/T_k(1/sigma) (4.18e-4
    for Q2, 1.95e-3 for Q1 at k = 10) of the initial error."""
    o = Operators(6, 1.0)
    A = o.Ms if fam == "q2" else o.Mp
    rng = np.random.default_rng(1)
    for _ in range(3):
        b = rng.standard_normal(A.shape[0])
        xe = spla.spsolve(A.tocsc(), b)
        for k in (1, 2, 5, 10):
            e = chebyshev(A, b, k, bounds) - xe
            en = np.sqrt(e @ (A @ e)) / np.sqrt(xe @ (A @ xe))
            assert en <= chebyshev_error_bound(k, bounds) * (1 + 1e-9)
    assert abs(chebyshev_error_bound(10, Q2_MASS_BOUNDS) - 4.18e-4) < 1e-6
    assert abs(chebyshev_error_bound(10, Q1_MASS_BOUNDS) - 1.95e-3) < 1e-5


def test_colour_classes_independent():
    """The multicolour SOR colour classes are independent sets (checked by the
    constructor) and a symmetric sweep pair is a symmetric operator."""
    for N in (2, 4):
        o = Operators(N, 1.0, W.wind_nodal(N))
        for A, col in ((o.Ms + o.Ks + o.Ns, colours_q2(o.grid)), (o.Kp + o.Mp, colours_q1(o.grid))):
            sor = ColouredSOR(A, col)
            assert sor.ncol == (9 if col.size == o.grid.nV else 4)
        A = (o.Ms + 0.3 * o.Ks).tocsr()
        sor = ColouredSOR(A, colours_q2(o.grid))
        n = A.shape[0]
        Sm = np.zeros((n, n))
        for k in range(n):
            e = np.zeros(n); e[k] = 1.0
            Sm[:, k] = sor.backward(e, sor.forward(e, np.zeros(n)))
        assert np.allclose(Sm, Sm.T, atol=1e-13)


@pytest.mark.parametrize("N", [4, 8])
def test_galerkin_equals_rediscretised(N):
    """P13: P^T A_fine P equals the coarse operator for M, K, N(w) (Q2 interior)
    and the unconstrained Q1 matrices, since the spaces are nested and the
    quadrature exact."""
    wind = W.wind_nodal(N)
    lv = Levels(N, wind)
    P2, P1 = lv.P2[0], lv.P1[0]
    f, c = lv.ops[0], lv.ops[1]
    for Af, Ac in ((f.Ms, c.Ms), (f.Ks, c.Ks), (f.Ns, c.Ns)):
        assert abs(P2.T @ Af @ P2 - Ac).max() < 1e-13
    for key in ("K1", "M1", "N1"):
        assert abs(P1.T @ f.full[key] @ P1 - c.full[key]).max() < 1e-13


def test_prolongation_reproduces_polynomials():
    """Q2 interpolation reproduces quadratics, Q1 reproduces bilinears."""
    from oracle.mg import prolong_1d_q1, prolong_1d_q2
    Nc = 4
    xc = np.arange(2 * Nc + 1) / (2 * Nc)
    xf = np.arange(4 * Nc + 1) / (4 * Nc)
    q = lambda x: 1 - 3 * x + 2 * x * x
    assert np.allclose(prolong_1d_q2(Nc) @ q(xc), q(xf), atol=1e-14)
    xc1, xf1 = np.arange(Nc + 1) / Nc, np.arange(2 * Nc + 1) / (2 * Nc)
    assert np.allclose(prolong_1d_q1(Nc) @ (2 - xc1), 2 - xf1, atol=1e-14)


def test_multigrid_converges_and_is_symmetric():
    """A V-cycle is a contraction on W_j and on the unconstrained K_N (modulo
    constants; the rate has no closed form, the cycle operator itself is pinned
    by test_vcycle_equals_error_propagation_formula), exact on the coarsest
    grid, and symmetric; the pinned K_p^{-1} comes out through
    R L K_N^+ L^T R^T."""
    N = 8
    lv = Levels(N)
    rng = np.random.default_rng(0)
    mg = ScalarMG(lv, "q2", 1.1, 0.05)
    A = mg.A[0]
    b = rng.standard_normal(A.shape[0])
    xe = spla.spsolve(A.tocsc(), b)
    errs = [np.linalg.norm(mg.solve(b, c) - xe) for c in (1, 2, 4)]
    assert errs[0] < 0.3 * np.linalg.norm(xe) and errs[2] < 0.05 * errs[0]
    n = A.shape[0]
    Mx = np.column_stack([mg.solve(np.eye(n)[k], 1) for k in range(n)])
    assert np.allclose(Mx, Mx.T, atol=1e-12 * np.abs(Mx).max())
    # pressure Laplacian through the unconstrained hierarchy
    w = W.small(W.STOKES, N, 4)
    pc = StokesPreconditioner(Problem.from_workload(w), freqs=[0])
    Kp = pc.P.ops.Kp
    bp = rng.standard_normal(Kp.shape[0])
    xe = spla.spsolve(Kp.tocsc(), bp)
    errs = []
    for c in (1, 2, 4):
        pc.s.n_vcycles = c
        errs.append(np.linalg.norm(pc.stiff_p_inv(bp) - xe) / np.linalg.norm(xe))
    assert errs[0] < 0.1 and errs[2] < 1e-3
    coarse = ScalarMG(Levels(2), "q2", 1.0, 1.0)
    b = rng.standard_normal(coarse.A[0].shape[0])
    assert np.allclose(coarse.A[0] @ coarse.solve(b, 1), b, atol=1e-13)


def _vcycle_error_operator(mg, l):
    """Textbook error propagation of one V(1,1) cycle from level l, built from
    dense matrices: E_l = S_b (I - P (I - E_{l+1}) C_{l+1} P^T A_l) S_f, where
    S_f / S_b are the error operators of the forward / backward sweeps (their
    columns are sweeps of unit vectors with b = 0), C the coarse solution
    operator (dense inverse; Q1: node 0 held at zero) and E = 0 on the
    coarsest level."""
    A = mg.A[l].toarray()
    n = A.shape[0]
    Id = np.eye(n)
    Sf = np.column_stack([mg.sor[l].forward(np.zeros(n, complex), Id[:, k].astype(complex)) for k in range(n)])
    Sb = np.column_stack([mg.sor[l].backward(np.zeros(n, complex), Id[:, k].astype(complex)) for k in range(n)])
    P = mg.lv.prolong(mg.fam, l).toarray()
    Ac = mg.A[l + 1].toarray()
    nc = Ac.shape[0]
    if l + 1 == len(mg.A) - 1:
        C = np.zeros((nc, nc), complex)
        if mg.pin_coarse:
            C[1:, 1:] = np.linalg.inv(Ac[1:, 1:])
        else:
            C = np.linalg.inv(Ac)
        coarse = C
    else:
        Ec = _vcycle_error_operator(mg, l + 1)
        coarse = (np.eye(nc) - Ec) @ np.linalg.inv(Ac)
    return Sb @ (Id - P @ coarse @ P.T @ A) @ Sf


@pytest.mark.parametrize("N,fam,conv", [(4, "q2", False), (4, "q2", True), (8, "q2", True), (4, "q1", False),
                                        (8, "q1", True)])
def test_vcycle_equals_error_propagation_formula(N, fam, conv):
    """V-cycle operator pinned to the two-/three-grid error propagation formula:
    one cycle from x = 0 gives (I - E) A^{-1} b and two cycles (I - E^2) A^{-1} b,
    with E composed from dense smoother, transfer and coarse operators.  A
    dropped coarse correction, a restriction by P instead of P^T, a sign error
    in the residual or swapped sweep directions each break the identity."""
    wind = W.wind_nodal(N) if conv else None
    lv = Levels(N, wind)
    mg = ScalarMG(lv, fam, 0.9 + 0.4j, 0.07 - 0.02j, eta=(0.3 + 0.1j) if conv else 0.0,
                  eta_t=(0.05 - 0.2j) if conv else 0.0)
    A = mg.A[0].toarray()
    n = A.shape[0]
    rng = np.random.default_rng(11)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    if fam == "q1":
        b -= b.mean()                                       # consistent for the singular-free shifted operator too
    E = _vcycle_error_operator(mg, 0)
    xe = np.linalg.solve(A, b)
    for cycles, Ek in ((1, E), (2, E @ E)):
        x = mg.solve(b, cycles)
        ref = xe - Ek @ xe
        assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(xe)


def test_vcycle_error_formula_with_level_viscosity():
    """The same pin with a different diffusion coefficient on every level
    (the coarse-level viscosity of the convection-diffusion hierarchies)."""
    N = 8
    lv = Levels(N, W.wind_nodal(N))
    mg = ScalarMG(lv, "q2", 0.9 + 0.4j, 0.07, eta=0.3, gamma_levels=[0.07, 0.21, 0.5])
    assert not np.allclose(mg.A[1].toarray(), ScalarMG(lv, "q2", 0.9 + 0.4j, 0.07, eta=0.3).A[1].toarray())
    A = mg.A[0].toarray()
    rng = np.random.default_rng(12)
    b = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    E = _vcycle_error_operator(mg, 0)
    xe = np.linalg.solve(A, b)
    x = mg.solve(b, 2)
    assert np.linalg.norm(x - (xe - E @ E @ xe)) <= 1e-11 * np.linalg.norm(xe)


def test_coarse_viscosity_closed_form():
    """nu_l = max(nu, |w|_max h_l / 4) below the finest level; the workload
    wind (2y(1-x^2), -2x(1-y^2)) peaks at |w| = 2 in the corners (0,1), (1,0)."""
    lv = Levels(8, W.wind_nodal(8))
    assert lv.wind_max == pytest.approx(2.0, abs=1e-15)
    got = coarse_viscosity(0.01, 2.0, [128, 64, 32, 16, 8, 4, 2])
    assert got == pytest.approx([0.01, 0.01, 1 / 64, 1 / 32, 1 / 16, 1 / 8, 1 / 4], rel=1e-15)
    # diffusion-dominated: every level keeps nu (the plain rediscretised hierarchy)
    assert coarse_viscosity(1.0, 2.0, [64, 32, 16, 8, 4, 2]) == [1.0] * 6
    assert Levels(4).wind_max == 0.0


def test_coarse_viscosity_makes_convective_vcycle_contract():
    """A convection-dominated shifted operator (nu = 0.01, tau = 1/64,
    beta = 4.7e-3, j = 0): V-cycles on the plainly rediscretised hierarchy
    diverge after two cycles, with the coarse-level viscosity every cycle
    contracts."""
    N, tau, nu, beta = 32, 1.0 / 64, 0.01, 4.7e-3
    lv = Levels(N, W.wind_nodal(N))
    a = tau / np.sqrt(beta)
    g = [tau * v for v in coarse_viscosity(nu, lv.wind_max, lv.sizes)]
    plain = ScalarMG(lv, "q2", a, tau * nu, eta=tau)
    visc = ScalarMG(lv, "q2", a, tau * nu, eta=tau, gamma_levels=g)
    A = plain.A[0]
    assert abs(A - visc.A[0]).max() == 0.0                 # the finest operator is the true one
    rng = np.random.default_rng(3)
    b = A @ (rng.standard_normal(A.shape[0]) + 0j)

    def history(mg):
        x, out = np.zeros_like(b), []
        for _ in range(8):
            x = mg.vcycle(0, b, x)
            out.append(np.linalg.norm(b - A @ x) / np.linalg.norm(b))
        return out

    hp, hv = history(plain), history(visc)
    assert hp[7] > hp[1] and hp[7] > 1.0
    assert all(hv[k + 1] < hv[k] for k in range(7)) and hv[7] < 2e-3


def test_linear_stokes_preconditioner_symmetric(stokes4):
    """P16: Algorithm 1 with symmetric V-cycles is a symmetric operator."""
    _, P, pc = stokes4
    rng = np.random.default_rng(4)
    x, y = rng.standard_normal(P.n_all), rng.standard_normal(P.n_all)
    a, b = x @ pc.apply(y), y @ pc.apply(x)
    assert abs(a - b) <= 1e-12 * abs(a)


def test_conjugate_symmetry_of_frequency_outputs(stokes4):
    """P18: for real r, y_hat_{nt-j} = conj(y_hat_j) (linear and nonlinear)."""
    _, P, pc = stokes4
    r = np.random.default_rng(6).standard_normal(P.n_all)
    for nl in (False, True):
        out = pc.freq_domain(r, nonlinear=nl)
        for j in range(1, P.nt // 2):
            for a, b in zip(out[j], out[P.nt - j]):
                assert np.allclose(a, np.conj(b), atol=1e-12 * np.abs(a).max())


@pytest.mark.slow
def test_fgmres_stokes_nonlinear_matches_direct():
    """Outer FGMRES(10) with Algorithm 2 reaches 1e-8 and agrees with the
    direct solve; inner GMRES counts stay moderate (section 5.1.2 behaviour)."""
    w = W.config(1)
    P = Problem.from_workload(w)
    b = P.rhs(W.desired_state(w))
    A = P.kkt_matrix()
    pc = StokesPreconditioner(P)
    x, its, hist = fgmres(lambda v: A @ v, lambda v: pc.apply(v, True), b, 1e-8, restart=10, maxit=40)
    assert hist[-1] <= 1e-8 and its <= 12
    assert np.mean(list(pc.inner_its.values())) < 40
    xs = P.solve_direct(b)
    assert np.linalg.norm(x - xs) <= 1e-5 * np.linalg.norm(xs)


def test_fgmres_oseen_nonlinear_small():
    """Oseen: FGMRES with GMRES(G_j, P~_j^(UZ)) converges to 1e-8."""
    N = 4
    w = W.Workload(W.OSEEN, N, 8, 1.0, 0.1, 1e-4, 0, 1.0)
    wind = W.wind_nodal(N)
    P = Problem.from_workload(w, wind)
    b = P.rhs(W.desired_state(w))
    A = P.kkt_matrix()
    pc = OseenPreconditioner(P, wind)
    x, its, hist = fgmres(lambda v: A @ v, lambda v: pc.apply(v, True), b, 1e-8, restart=10, maxit=40)
    assert hist[-1] <= 1e-8


def test_gmres_matches_direct_solution():
    rng = np.random.default_rng(0)
    n = 40
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, its, _ = gmres(lambda v: A @ v, None, b, 1e-12, restart=n, maxit=n)
    assert np.linalg.norm(A @ x - b) <= 1e-11 * np.linalg.norm(b)
    x, its, _ = fgmres(lambda v: A @ v, lambda v: v / 3, b.real, 1e-12, restart=5, maxit=200)
    assert np.linalg.norm(A @ x - b.real) <= 1e-11 * np.linalg.norm(b.real)


def _brute_tiled_sweep(A, b, x, colours, tiles, order):
    """Node-by-node definition: inside a tile, colours in ``order``; a node
    sees the current values of its own tile and the sweep-start values of
    other tiles."""
    A = A.toarray()
    x0 = x.copy()
    x = x.copy()
    for t in np.unique(tiles):
        for c in order:
            for i in np.flatnonzero((tiles == t) & (colours == c)):
                y = np.where(tiles == t, x, x0)
                x[i] = x[i] + (b[i] - A[i] @ y) / A[i, i]
    return x


@pytest.mark.parametrize("T", [2, 4, 48])
def test_tiled_sor_matches_definition(T):
    """The tiled sweep equals the node-by-node definition (several tiles for
    small T) and, with a single tile, plain multicolour Gauss-Seidel."""
    N = 4
    o = Operators(N, 1.0, W.wind_nodal(N))
    g = o.grid
    iy, ix = np.divmod(g.v_interior, g.nq)
    tiles = tiles_of(ix, iy, g.nq, T)
    col = colours_q2(g)
    A = (1.3 * o.Ms + 0.2 * o.Ks + 0.1 * o.Ns).tocsr()
    rng = np.random.default_rng(T)
    b, x = rng.standard_normal(g.nV), rng.standard_normal(g.nV)
    sor = TiledSOR(A, col, tiles)
    assert np.allclose(sor.forward(b, x.copy()), _brute_tiled_sweep(A, b, x, col, tiles, range(9)), atol=1e-13)
    assert np.allclose(sor.backward(b, x.copy()), _brute_tiled_sweep(A, b, x, col, tiles, range(8, -1, -1)),
                       atol=1e-13)
    if T >= g.nq:
        assert np.allclose(sor.forward(b, x.copy()), ColouredSOR(A, col).forward(b, x.copy()), atol=1e-14)
    # Q1 unconstrained grid, 4 colours
    iy1, ix1 = np.divmod(np.arange(g.np2), g.np1)
    t1 = tiles_of(ix1, iy1, g.np1, max(T // 2, 2))
    c1 = 2 * (iy1 % 2) + ix1 % 2
    A1 = (o.full["K1"] + 0.5 * o.full["M1"]).tocsr()
    b1, x1 = rng.standard_normal(g.np2), rng.standard_normal(g.np2)
    assert np.allclose(TiledSOR(A1, c1, t1).forward(b1, x1.copy()),
                       _brute_tiled_sweep(A1, b1, x1, c1, t1, range(4)), atol=1e-13)


def test_tiled_sor_symmetric_pair():
    N = 8
    o = Operators(N, 1.0)
    g = o.grid
    iy, ix = np.divmod(g.v_interior, g.nq)
    A = (o.Ms + 0.3 * o.Ks).tocsr()
    sor = TiledSOR(A, colours_q2(g), tiles_of(ix, iy, g.nq, 4))
    n = g.nV
    Sm = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n); e[k] = 1.0
        Sm[:, k] = sor.backward(e, sor.forward(e, np.zeros(n)))
    assert np.allclose(Sm, Sm.T, atol=1e-13)


def test_minres_iterate_is_the_krylov_minimiser():
    """The k-th preconditioned MINRES iterate minimises ||b - A x|| in the
    norm of the SPD preconditioner P over the Krylov space span{P b, (P A) P b,
    ...}: checked against that definition by a dense least-squares solve (the
    history entry |eta_k| / gamma_1 is the same minimum, relative to ||b||_P)."""
    from oracle.krylov import minres
    rng = np.random.default_rng(5)
    n = 30
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    A = Q @ np.diag(np.concatenate([rng.uniform(1, 3, 18), -rng.uniform(0.5, 2, 12)])) @ Q.T
    B = rng.standard_normal((n, n))
    P = np.linalg.inv(B @ B.T + n * np.eye(n)) * n
    b = rng.standard_normal(n)
    Lc = np.linalg.cholesky(P)
    for k in range(1, 7):
        x, its, hist, _ = minres(lambda v: A @ v, lambda v: P @ v, b, 0.0, maxit=k)
        assert its == k
        K = np.zeros((n, k))
        K[:, 0] = P @ b
        for j in range(1, k):
            K[:, j] = P @ (A @ K[:, j - 1])
        K = np.linalg.qr(K)[0]
        y = np.linalg.lstsq(Lc.T @ (A @ K), Lc.T @ b, rcond=None)[0]
        xr = K @ y
        assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr)
        r = b - A @ xr
        assert hist[-1] == pytest.approx(np.sqrt(r @ P @ r) / np.sqrt(b @ P @ b), rel=1e-9)


def test_minres_complex_iterate_is_the_krylov_minimiser():
    """With complex vectors, a real symmetric indefinite matrix and a Hermitian
    positive definite preconditioner P (the setting of the Stokes blocks Z_j
    with P~_j), the k-th MINRES iterate minimises ||b - A x|| in the P-norm
    over span{P b, (P A) P b, ...}: checked by a dense least-squares solve.
    Dropping the conjugate in either inner product breaks it."""
    from oracle.krylov import minres
    rng = np.random.default_rng(8)
    n = 24
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    A = Q @ np.diag(np.concatenate([rng.uniform(1, 3, 14), -rng.uniform(0.5, 2, 10)])) @ Q.T
    B = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    P = np.linalg.inv(B @ B.conj().T + n * np.eye(n)) * n
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    Lc = np.linalg.cholesky(P)                     # P = Lc Lc^H
    for k in range(1, 7):
        x, its, hist, _ = minres(lambda v: A @ v, lambda v: P @ v, b, 0.0, maxit=k)
        assert its == k
        K = np.zeros((n, k), complex)
        K[:, 0] = P @ b
        for j in range(1, k):
            K[:, j] = P @ (A @ K[:, j - 1])
        K = np.linalg.qr(K)[0]
        y = np.linalg.lstsq(Lc.conj().T @ (A @ K), Lc.conj().T @ b, rcond=None)[0]
        xr = K @ y
        assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr)
        r = b - A @ xr
        assert hist[-1] == pytest.approx(np.sqrt(np.vdot(r, P @ r).real / np.vdot(b, P @ b).real), rel=1e-9)


def test_minres_inner_solver_on_stokes_blocks(stokes4):
    """The inner MINRES variant of Algorithm 2 rests on Z_j being real
    symmetric and P~_j (with exact inner inverses here) Hermitian positive
    definite on complex frequency vectors; MINRES then stops with the
    P~_j-norm of the residual below the tolerance times that of s_j, and at a
    tight tolerance it reaches the direct solution.  The nonlinear
    preconditioner with the variant records its inner counts."""
    from oracle.krylov import minres
    from oracle.precond import Settings, StokesPreconditioner
    w, P, _ = stokes4
    pc = StokesPreconditioner(P, Settings(exact=True, inner_solver="minres"))
    cut = np.cumsum([P.nv, P.nv, P.nP])
    rng = np.random.default_rng(9)
    for j in (0, 1, P.nt // 2):
        Z = pc.Z_matrix(j)
        Zd = Z.toarray() if hasattr(Z, "toarray") else np.asarray(Z)
        assert np.isrealobj(Zd)
        assert np.abs(Zd - Zd.T).max() <= 1e-12 * np.abs(Zd).max()
        n = Zd.shape[0]
        Pm = np.column_stack([np.concatenate(pc.ptilde_inv(j, *np.split(e.astype(complex), cut)))
                              for e in np.eye(n)])
        assert np.abs(Pm - Pm.conj().T).max() <= 1e-10 * np.abs(Pm).max()
        assert np.linalg.eigvalsh((Pm + Pm.conj().T) / 2).min() > 0
        s_ = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        for tol in (1e-2, 1e-11):
            x, its, hist, _ = minres(lambda v: Zd @ v, lambda v: Pm @ v, s_, tol, 400)
            r = s_ - Zd @ x
            assert np.sqrt(np.vdot(r, Pm @ r).real) <= tol * np.sqrt(np.vdot(s_, Pm @ s_).real) * (1 + 1e-6)
        xd = np.linalg.solve(Zd, s_)
        assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
        pc.block_apply(j, *np.split(s_, cut), nonlinear=True)
        assert pc.inner_its[j] > 0


def test_minres_stokes_linear_preconditioner(stokes4):
    """Algorithm 1 is symmetric positive definite on the Stokes problem, so
    MINRES applies; restarted on the true residual it reaches 1e-8 and agrees
    with the sparse direct solve."""
    from oracle.krylov import minres_restarted
    w, P, pc = stokes4
    A = P.kkt_matrix()
    b = P.rhs(W.desired_state(w))
    rng = np.random.default_rng(6)
    y = rng.standard_normal(P.n_all)
    assert y @ pc.apply(y) > 0
    x, its, hist = minres_restarted(lambda v: A @ v, lambda v: pc.apply(v), b, 1e-8)
    assert hist[-1] <= 1e-8 and its < 200
    xd = P.solve_direct(b)
    assert np.linalg.norm(x - xd) <= 1e-6 * np.linalg.norm(xd)
