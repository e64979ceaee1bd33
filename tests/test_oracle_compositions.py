"""Pins of the oracle's block compositions against dense evaluations of the
paper's definitions (CPU).

With every inner approximation replaced by the inverse it stands for
(``Settings(exact=True)``: multigrid and Chebyshev become sparse LU solves),
the four compositions of the oracle must equal dense matrices built here from
the paper's formulas, written in their printed (product) form rather than in
the form the oracle applies:

* ``StokesPreconditioner.ptilde_inv``: diag(W_j, W_j, S^_j, S^_j)^{-1} of
  section 3.2, W_j = M + c_{j,1} M + c_{j,2} L and
  S^_j = M_p (M_p + c_{j,1} M_p + c_{j,2} L_p)^{-1} K_p;
* ``OseenPreconditioner.shat11_inv``: the inverse of the Schur block
  (1/tau) Q_j M^{-1} Q_j^H of P_j^(1,1) (section 4);
* ``OseenPreconditioner.schur_inv``: the inverse of the three-factor S^_j of
  section 4, [[0, tau M_p], [tau M_p, 0]] H_p^{-1} [[0, tau K_p], [tau K_p, 0]];
* ``OseenPreconditioner.puz_inv``: the second step of Algorithm 3,
  (y3, y4) = -S^_j^{-1}((r3, r4) - G_j^(2,1) (y1, y2)), with G_j^(2,1) cut
  out of the assembled block of eq. (SubBlockG).

The pressure pin (node (0,0) removed) enters as in the oracle's reading: the
commutator forms are built on the unconstrained Q1 space, where K_p is
singular with the constants as kernel, and carried to the pinned space with
R (drops node 0) and L = I - 1 e_0^T.  For Stokes the dense side takes the
Moore-Penrose pseudo-inverse of the whole unconstrained product R L S^+ L^T R^T,
so it shares no step with the oracle's sum-of-inverses evaluation; for Oseen
it inverts the three factors separately (pseudo-inverse for K_p) and
multiplies dense block matrices.

Each pin is shown to be sharp by planted mistakes (a subclass with one
plausible slip -- c_1 for 1 + c_1, the two arguments swapped, conj(d)
dropped, L_p for L_p^T, Q^{-1} and Q^{-H} swapped, y1 and y2 swapped in the
divergence terms, a sign) that each must fail the same comparison.
"""
import numpy as np
import pytest

import workloads as W
from oracle import circulant as circ
from oracle.kkt import Problem
from oracle.precond import OseenPreconditioner, Settings, StokesPreconditioner

TOL = 1e-10


def _dense(A):
    return A.toarray() if hasattr(A, "toarray") else np.asarray(A)


def _rl(n):
    """R (drop node 0) and L = I - 1 e_0^T on n unconstrained Q1 nodes."""
    R = np.eye(n)[1:]
    L = np.eye(n)
    L[:, 0] -= 1.0
    return R, L


def _rand(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ------------------------------------------------------------------ Stokes
@pytest.fixture(scope="module")
def stokes():
    w = W.small(W.STOKES, 4, 8, beta=1e-2)
    P = Problem.from_workload(w)
    return P


def _stokes_dense(P, pc, j):
    """diag(W_j, W_j, S^_j, S^_j)^{-1} from the product forms of section 3.2."""
    o = P.ops
    _, _, c1, c2 = pc.constants(j)
    Wd = _dense(o.M + c1 * o.M + c2 * o.L)                 # W_j = M + c1 M + c2 L
    MN, KN = _dense(o.full["M1"]), _dense(o.full["K1"])
    LpN = P.nu * KN                                         # L_p = nu K_p (Stokes)
    S_N = MN @ np.linalg.solve(MN + c1 * MN + c2 * LpN, KN)  # M_p (M_p + c1 M_p + c2 L_p)^{-1} K_p
    R, L = _rl(MN.shape[0])
    Sinv = R @ L @ np.linalg.pinv(S_N) @ L.T @ R.T
    return np.linalg.inv(Wd), Sinv


def _check_ptilde(P, pc, js):
    rng = np.random.default_rng(3)
    worst = 0.0
    for j in js:
        Winv, Sinv = _stokes_dense(P, pc, j)
        s = [_rand(rng, P.nv), _rand(rng, P.nv), _rand(rng, P.nP), _rand(rng, P.nP)]
        x = pc.ptilde_inv(j, *s)
        ref = (Winv @ s[0], Winv @ s[1], Sinv @ s[2], Sinv @ s[3])
        worst = max(worst, max(_rel(a, b) for a, b in zip(x, ref)))
    return worst


JS = [0, 1, 3, 4]        # d_j = 0, complex, complex, d_j = 2 (nt = 8)


def test_ptilde_inv_equals_dense_definition(stokes):
    pc = StokesPreconditioner(stokes, Settings(exact=True))
    assert _check_ptilde(stokes, pc, JS) <= TOL


class _PtildeC1(StokesPreconditioner):
    """Planted: c1 in place of 1 + c1 in the Schur part."""

    def ptilde_inv(self, j, s1, s2, s3, s4):
        _, _, c1, c2 = self.constants(j)
        x1, x2, _, _ = super().ptilde_inv(j, s1, s2, s3, s4)
        Z = self.unpin_in(np.stack([s3, s4], axis=1))
        Y = self.pin_out(c1 * self.mg_Kp.solve(Z, 4) + self.P.nu * c2 * self.cheb_MN(Z))
        return x1, x2, Y[:, 0], Y[:, 1]


class _PtildeNoNu(StokesPreconditioner):
    """Planted: the viscosity dropped from the mass term of S^_j^{-1}."""

    def ptilde_inv(self, j, s1, s2, s3, s4):
        _, _, c1, c2 = self.constants(j)
        x1, x2, _, _ = super().ptilde_inv(j, s1, s2, s3, s4)
        Z = self.unpin_in(np.stack([s3, s4], axis=1))
        Y = self.pin_out((1 + c1) * self.mg_Kp.solve(Z, 4) + c2 * self.cheb_MN(Z))
        return x1, x2, Y[:, 0], Y[:, 1]


class _PtildeSwapW(StokesPreconditioner):
    """Planted: W_j built as (1 + c2) M + c1 L (constants exchanged)."""

    def W_mg(self, j):
        from oracle.mg import ExactSolve
        _, _, c1, c2 = self.constants(j)
        o = self.P.ops
        return ExactSolve((1 + c2) * o.Ms + c1 * self.P.nu * o.Ks)


@pytest.mark.parametrize("mutant", [_PtildeC1, _PtildeSwapW])
def test_ptilde_pin_catches_planted_mistakes(stokes, mutant):
    pc = mutant(stokes, Settings(exact=True))
    assert _check_ptilde(stokes, pc, JS) > 1e-3


def test_ptilde_pin_catches_dropped_viscosity():
    """With nu = 1 the viscosity slip is invisible, so this mutant is checked
    on a problem with nu != 1."""
    P = Problem(4, 8, 1.0, 0.3, 1e-2)
    assert _check_ptilde(P, StokesPreconditioner(P, Settings(exact=True)), JS) <= TOL
    assert _check_ptilde(P, _PtildeNoNu(P, Settings(exact=True)), JS) > 1e-3


# ------------------------------------------------------------------- Oseen
@pytest.fixture(scope="module")
def oseen():
    N, nt = 4, 8
    w = W.Workload(W.OSEEN, N, nt, 1.0, 0.1, 1e-2, 0, 1.0)
    wind = W.wind_nodal(N)
    P = Problem.from_workload(w, wind)
    return P, wind


def _oseen_mats(P, d):
    o, tau, beta = P.ops, P.tau, P.beta
    M = _dense(o.M)
    Lv = _dense(o.L)                                         # L = nu K + N(w), both components
    Q = d * M + tau * Lv + tau / np.sqrt(beta) * M           # Q_j of section 4
    return M, Q


def _check_shat11(P, pc, js):
    rng = np.random.default_rng(4)
    worst = 0.0
    for j in js:
        M, Q = _oseen_mats(P, pc.d[j])
        Shat = (Q @ np.linalg.solve(M, Q.conj().T)) / P.tau   # (1/tau) Q M^{-1} Q^H
        y = _rand(rng, P.nv)
        worst = max(worst, _rel(pc.shat11_inv(j, y), np.linalg.solve(Shat, y)))
    return worst


def test_shat11_inv_equals_dense_definition(oseen):
    P, wind = oseen
    pc = OseenPreconditioner(P, wind, Settings(exact=True))
    assert _check_shat11(P, pc, JS) <= TOL


class _Shat11Swapped(OseenPreconditioner):
    """Planted: Q^{-1} and Q^{-H} applied in the wrong order."""

    def shat11_inv(self, j, y):
        mgQ, mgQH = self.Q_mgs(j)
        t = self._vec(lambda v: mgQH.solve(v, 4), y)
        t = self.P.ops.M @ t
        return self.P.tau * self._vec(lambda v: mgQ.solve(v, 4), t)


def test_shat11_pin_catches_swapped_factors(oseen):
    P, wind = oseen
    assert _check_shat11(P, _Shat11Swapped(P, wind, Settings(exact=True)), JS) > 1e-3


def _schur_dense(P, d):
    """S^_j^{-1} of section 4 as the reversed product of the inverses of its
    three factors, [[0, tau K_p], [tau K_p, 0]]^{-1} H_p [[0, tau M_p],
    [tau M_p, 0]]^{-1}, with the pinned-space reading applied factor by factor:
    K_p^{-1} -> R L K_N^+ L^T R^T (pseudo-inverse of the unconstrained pressure
    Laplacian), M_p^{-1} -> M_N^{-1} L^T R^T and H_p formed on the unconstrained
    space and restricted by R.  (The product of the unconstrained factors is not
    consistent here: the wind is not tangential on the unit square's boundary,
    so N_p^T 1 != 0 and the first-row output of H_p need not sum to zero.)"""
    o, tau, beta = P.ops, P.tau, P.beta
    MN, KN = _dense(o.full["M1"]), _dense(o.full["K1"])
    LN = P.nu * KN + _dense(o.full["N1"])
    R, L = _rl(MN.shape[0])
    Kt = R @ L @ np.linalg.pinv(KN) @ L.T @ R.T              # pinned (K_p)^{-1}
    Mt = np.linalg.inv(MN) @ L.T @ R.T                        # (M_p)^{-1} into the unconstrained space
    Hp = np.block([[tau * MN, np.conj(d) * MN + tau * LN.T], [d * MN + tau * LN, -(tau / beta) * MN]])
    Zk, Zm = np.zeros_like(Kt), np.zeros_like(Mt)
    Jk_inv = np.block([[Zk, Kt / tau], [Kt / tau, Zk]])
    Jm_inv = np.block([[Zm, Mt / tau], [Mt / tau, Zm]])
    return Jk_inv @ np.kron(np.eye(2), R) @ Hp @ Jm_inv


def _check_schur(P, pc, js):
    rng = np.random.default_rng(5)
    worst = 0.0
    for j in js:
        Sinv = _schur_dense(P, pc.d[j])
        a, b = _rand(rng, P.nP), _rand(rng, P.nP)
        y3, y4 = pc.schur_inv(j, a, b)
        worst = max(worst, _rel(np.concatenate([y3, y4]), Sinv @ np.concatenate([a, b])))
    return worst


def test_schur_inv_equals_dense_definition(oseen):
    P, wind = oseen
    pc = OseenPreconditioner(P, wind, Settings(exact=True))
    assert _check_schur(P, pc, JS) <= TOL


class _SchurArgsSwapped(OseenPreconditioner):
    def schur_inv(self, j, a, b):
        return super().schur_inv(j, b, a)


class _SchurNoConj(OseenPreconditioner):
    """Planted: d and conj(d) exchanged between the off-diagonal blocks of H_p."""

    def schur_inv(self, j, a, b):
        d = self.d[j]
        self.d = self.d.copy()
        self.d[j] = np.conj(d)          # makes the (1,2) entry d and the (2,1) entry conj(d)
        try:
            return super().schur_inv(j, a, b)
        finally:
            self.d[j] = d


class _SchurNoTranspose(OseenPreconditioner):
    """Planted: L_p in place of L_p^T in the (1,2) block of H_p."""

    def schur_inv(self, j, a, b):
        o, tau, beta = self.P.ops, self.P.tau, self.P.beta
        d = self.d[j]
        MN = self.MN
        LN = (self.P.nu * o.full["K1"] + o.full["N1"]).tocsr()
        Zs = self.cheb_MN(self.unpin_in(np.stack([b, a], axis=1))) / tau
        z1, z2 = Zs[:, 0], Zs[:, 1]
        u1 = tau * (MN @ z1) + np.conj(d) * (MN @ z2) + tau * (LN @ z2)
        u2 = d * (MN @ z1) + tau * (LN @ z1) - (tau / beta) * (MN @ z2)
        U = self.stiff_p_inv(np.stack([u2[1:], u1[1:]], axis=1)) / tau
        return U[:, 0], U[:, 1]


@pytest.mark.parametrize("mutant", [_SchurArgsSwapped, _SchurNoConj, _SchurNoTranspose])
def test_schur_pin_catches_planted_mistakes(oseen, mutant):
    P, wind = oseen
    assert _check_schur(P, mutant(P, wind, Settings(exact=True)), [1, 3]) > 1e-3


def _check_puz(P, pc, js):
    rng = np.random.default_rng(6)
    nv, nP = P.nv, P.nP
    worst = 0.0
    for j in js:
        G = circ.G_block(P, pc.d[j]).toarray()
        G21 = G[2 * nv:, :2 * nv]                          # divergence rows of eq. (SubBlockG)
        r = [_rand(rng, nv), _rand(rng, nv), _rand(rng, nP), _rand(rng, nP)]
        y1, y2, y3, y4 = pc.puz_inv(j, *r)
        u1, u2 = pc.uzawa(j, r[0], r[1])                    # first step (pinned separately)
        assert _rel(np.concatenate([y1, y2]), np.concatenate([u1, u2])) == 0.0
        rhs = np.concatenate([r[2], r[3]]) - G21 @ np.concatenate([y1, y2])
        ref = -_schur_dense(P, pc.d[j]) @ rhs
        worst = max(worst, _rel(np.concatenate([y3, y4]), ref))
    return worst


def test_puz_inv_second_step_equals_dense_definition(oseen):
    P, wind = oseen
    pc = OseenPreconditioner(P, wind, Settings(exact=True))
    assert _check_puz(P, pc, JS) <= TOL


class _PuzSwapped(OseenPreconditioner):
    """Planted: y1 and y2 exchanged in the divergence terms."""

    def puz_inv(self, j, r1, r2, r3, r4):
        o, tau = self.P.ops, self.P.tau
        y1, y2 = self.uzawa(j, r1, r2)
        y3, y4 = self.schur_inv(j, r3 - tau * (o.B @ y1), r4 - tau * (o.B @ y2))
        return y1, y2, -y3, -y4


class _PuzSign(OseenPreconditioner):
    """Planted: the leading minus of the Schur step dropped."""

    def puz_inv(self, j, r1, r2, r3, r4):
        y1, y2, y3, y4 = super().puz_inv(j, r1, r2, r3, r4)
        return y1, y2, -y3, -y4


@pytest.mark.parametrize("mutant", [_PuzSwapped, _PuzSign])
def test_puz_pin_catches_planted_mistakes(oseen, mutant):
    P, wind = oseen
    assert _check_puz(P, mutant(P, wind, Settings(exact=True)), [1, 3]) > 1e-3


def test_exact_block_triangular_preconditioner_is_nilpotent(oseen):
    """With the (1,1) block solved exactly (Uzawa with exact M and S, mu = 1,
    two steps: eq. Uzawa11 is then exact, as P14 pins) and S^_j replaced by
    the true pressure Schur complement S_j of section 4, Algorithm 3 is the
    inverse of the block lower triangular matrix [[G11, 0], [G21, -S_j]], so
    (P^{-1} G_j - I)^2 = 0: a check of the whole composition against the
    saddle-point theory it rests on."""
    P, wind = oseen
    nv, nP = P.nv, P.nP
    j = 1
    pc = OseenPreconditioner(P, wind, Settings(exact=True))
    G = circ.G_block(P, pc.d[j]).toarray()
    G11, G12, G21 = G[:2 * nv, :2 * nv], G[:2 * nv, 2 * nv:], G[2 * nv:, :2 * nv]
    S = G21 @ np.linalg.solve(G11, G12)                    # true Schur complement
    Minv = np.linalg.inv(_dense(P.ops.M))
    M = _dense(P.ops.M)
    A12 = G11[:nv, nv:]
    A21 = G11[nv:, :nv]
    S11 = -(G11[nv:, nv:] - A21 @ np.linalg.solve(P.tau * M, A12))   # exact Schur of G11 (negated)

    class Exact(OseenPreconditioner):
        def schur_inv(self, jj, a, b):
            y = np.linalg.solve(S, np.concatenate([a, b]))
            return y[:nP], y[nP:]

    pe = Exact(P, wind, Settings(exact=True, mu_uzawa=1.0, n_uzawa=2))
    Sinv11 = np.linalg.inv(S11)
    cols = []
    for k in range(G.shape[0]):
        e = np.zeros(G.shape[0], complex)
        e[k] = 1.0
        g = G @ e
        y = pe.uzawa(j, g[:nv], g[nv:2 * nv], Minv=lambda v: Minv @ v, Sinv=lambda v: Sinv11 @ v)
        a = g[2 * nv:2 * nv + nP] - P.tau * (P.ops.B @ y[1])
        b = g[2 * nv + nP:] - P.tau * (P.ops.B @ y[0])
        y3, y4 = pe.schur_inv(j, a, b)
        cols.append(np.concatenate([y[0], y[1], -y3, -y4]))
    E = np.array(cols).T - np.eye(G.shape[0])
    assert np.abs(E @ E).max() <= 1e-8 * max(1.0, np.abs(E).max())
    assert np.abs(E).max() > 1e-3                          # not trivially the identity
