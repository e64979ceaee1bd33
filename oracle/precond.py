"""Block-circulant preconditioners for the all-at-once KKT system.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Stokes (section 3.2-3.4).  Each frequency block factors as
G_j = T_l Z_j T_r (eq. GJTransformation) with

    T_l = [[sqrt(tau) I, 0, 0, 0],
           [i d_c/sqrt(tau) I, sqrt(tau)/c2 I, 0, 0],
           [0, 0, sqrt(tau) c2 I, 0],
           [0, 0, i d_c c2/sqrt(tau) I, sqrt(tau) I]]
    T_r = [[sqrt(tau) I, -i d_c/sqrt(tau) I, 0, 0],
           [0, sqrt(tau)/c2 I, 0, 0],
           [0, 0, sqrt(tau) c2 I, -i d_c c2/sqrt(tau) I],
           [0, 0, 0, sqrt(tau) I]]
    Z_j = [[M, c1 M + c2 L, 0, B^T], [c1 M + c2 L, -M, B^T, 0],
           [0, B, 0, 0], [B, 0, 0, 0]]

with d_r = Re d_j, d_c = Im d_j, c2 = (1/beta + d_c^2/tau^2)^(-1/2) and
c1 = d_r / sqrt(tau^2/beta + d_c^2).  Reading: the printed c1 has d_c under
the root; the factorisation holds only with d_c^2 (equivalently c1 =
d_r c2 / tau), which is what is used here.

Z_j is preconditioned by P~_j = diag(W_j, W_j, S^_j, S^_j) with
W_j = (1 + c1) M + c2 L and the commutator Schur approximation
S^_j^{-1} = (1 + c1) K_p^{-1} + nu c2 M_p^{-1} (section 3.2).  The solver tree
of section 3.4: W_j^{-1} by 4 multigrid V-cycles, K_p^{-1} by 4 V-cycles and
M_p^{-1} by 10 Chebyshev steps.

Pressure pin (reading).  The commutator argument is made on the unconstrained
pressure space, where S = B W^{-1} B^T and K_p share the constants as kernel.
It is carried to the pinned space by the exact identity
(R S R^T)^{-1} = R L S^+ L^T R^T  (R drops node 0, L = I - 1 e_0^T), i.e.
S^_j^{-1} r = R L [(1 + c1) K_N^+ + nu c2 M_N^{-1}] L^T R^T r  with the
unconstrained Q1 matrices K_N, M_N.  Building M_p^{-1} and K_p^{-1} from the
pinned matrices instead leaves an h^2-small outlier in eig(S^^{-1} S) that
drives the inner GMRES counts up without bound as h -> 0.

* Algorithm 1 (linear):   FFT -> T_l^{-1} -> P~_j^{-1} -> T_r^{-1} -> inverse FFT.
* Algorithm 2 (nonlinear): the middle step is GMRES(Z_j, P~_j, tol eps).
  Reading: the inner preconditioner is P~_j (the practical one), not P^_j.
  Variant (Settings.inner_solver = "minres"): preconditioned MINRES on the
  real symmetric Z_j with the Hermitian positive definite P~_j, stopped when
  the P~_j-norm of the residual is below eps times that of the right-hand
  side.

Oseen (section 4, Algorithm 3).  No T transforms; each frequency block G_j is
preconditioned by P~_j^(UZ):
    (y1, y2) = k steps of the inexact Uzawa iteration (eq. Uzawa11) on
               G_j^(1,1) from zero, with M^^{-1} = Chebyshev(M) and
               S^^{-1} = tau Q_j^{-H} M Q_j^{-1},
               Q_j = d_j M + tau L + tau/sqrt(beta) M  (4 V-cycles each);
    (y3, y4) = -S^_j^{-1}((r3, r4) - tau (B y2, B y1)) with the commutator
               approximation of section 4, whose inverse is
               S^_j^{-1}(a, b) = ((tau K_p)^{-1} u2, (tau K_p)^{-1} u1),
               u1 = tau M_p z1 + (conj(d) M_p + tau L_p^T) z2,
               u2 = (d M_p + tau L_p) z1 - tau/beta M_p z2,
               z1 = (tau M_p)^{-1} b,  z2 = (tau M_p)^{-1} a.
The nonlinear Oseen preconditioner runs GMRES(G_j, P~_j^(UZ), eps).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import circulant as circ
from .krylov import gmres, minres
from .mg import ExactSolve, Levels, ScalarMG, coarse_viscosity
from .smoothers import Q1_MASS_BOUNDS, Q2_MASS_BOUNDS, chebyshev


class Settings:
    """Solver parameters of section 3.4 / section 5.

    ``tiling``: None for the multicolour SOR smoother over whole grids (the
    reading of section 3.4), or a ``smoothers.Tiling`` for the tiled variant.
    ``exact``: replace every inner approximation (multigrid, Chebyshev) by the
    exact inverse it stands for -- for pins of the block compositions."""

    def __init__(self, n_vcycles=4, n_cheb=10, n_uzawa=6, mu_uzawa=0.75,
                 inner_tol=1e-2, inner_restart=50, inner_maxit=200, tiling=None, exact=False,
                 inner_solver="gmres"):
        self.inner_solver = inner_solver
        self.tiling = tiling
        self.exact = exact
        self.n_vcycles = n_vcycles
        self.n_cheb = n_cheb
        self.n_uzawa = n_uzawa
        self.mu_uzawa = mu_uzawa
        self.inner_tol = inner_tol
        self.inner_restart = inner_restart
        self.inner_maxit = inner_maxit


def stokes_constants(d: complex, tau: float, beta: float):
    """(d_r, d_c, c1, c2) of section 3.2 (c1 with d_c squared)."""
    dr, dc = d.real, d.imag
    c2 = 1.0 / np.sqrt(1.0 / beta + dc * dc / (tau * tau))
    c1 = dr / np.sqrt(tau * tau / beta + dc * dc)
    return dr, dc, c1, c2


class _Common:
    def __init__(self, P, wind=None, settings: Settings | None = None, freqs=None):
        self.P = P
        self.s = settings or Settings()
        self.lv = Levels(P.N, wind, P.side)
        self.d = circ.d_closed_form(P.nt)
        self.freqs = range(P.nt) if freqs is None else freqs
        self.inner_its = {}

    def _mg(self, fam, alpha, gamma, eta=0.0, eta_t=0.0, gamma_levels=None):
        """Multigrid for a scalar operator of the family (or its exact inverse)."""
        if self.s.exact:
            M, K, N, _, _ = self.lv.family(fam, 0)
            A = alpha * M + gamma * K
            if eta != 0:
                A = A + eta * N
            if eta_t != 0:
                A = A + eta_t * N.T
            return ExactSolve(A, pin_node0=fam == "q1")
        return ScalarMG(self.lv, fam, alpha, gamma, eta, eta_t, gamma_levels, tiling=self.s.tiling)

    def _mass_solver(self, M, bounds):
        if self.s.exact:
            ex = ExactSolve(M)
            return lambda x: ex.solve(x)
        return lambda x: chebyshev(M, x, self.s.n_cheb, bounds)

    def _pressure_solvers(self):
        o = self.P.ops
        self.mg_Kp = self._mg("q1", 0.0, 1.0)
        self.MN = o.full["M1"].tocsr()                       # unconstrained Q1 mass
        self.cheb_MN = self._mass_solver(self.MN, Q1_MASS_BOUNDS)

    @staticmethod
    def unpin_in(r):
        """(I - e0 1^T) R^T r: extend a pinned pressure vector to all Q1 nodes,
        putting minus the sum of its entries at the pinned node 0."""
        z = np.zeros((r.shape[0] + 1,) + r.shape[1:], dtype=r.dtype)
        z[1:] = r
        z[0] = -r.sum(axis=0)
        return z

    @staticmethod
    def pin_out(y):
        """R (I - 1 e0^T) y: shift so that node 0 is zero, drop node 0."""
        return y[1:] - y[0]

    def mass_p_inv(self, r):
        """M_p^{-1} of the commutator Schur approximation on the pinned space:
        R L Cheb(M_N) L^T R^T r (Chebyshev on the unconstrained Q1 mass)."""
        return self.pin_out(self.cheb_MN(self.unpin_in(r)))

    def stiff_p_inv(self, r):
        """K_p^{-1} r = R L K_N^+ L^T R^T r by V-cycles on the unconstrained
        (singular, consistent) pressure Laplacian."""
        return self.pin_out(self.mg_Kp.solve(self.unpin_in(r), self.s.n_vcycles))

    def apply(self, r: np.ndarray, nonlinear: bool = False) -> np.ndarray:
        """z = P^{-1} r for a real all-at-once vector r (compact layout)."""
        P = self.P
        Rh = circ.time_fft(P, r)
        Yh = np.zeros_like(Rh)
        for j in self.freqs:
            r1, r2, r3, r4 = circ.split_freq(P, Rh[:, j, :])
            y = self.block_apply(j, r1, r2, r3, r4, nonlinear)
            Yh[:, j, :] = circ.join_freq(P, *y)
        return circ.time_ifft(P, Yh).real.reshape(-1)

    def freq_domain(self, r: np.ndarray, nonlinear: bool = False):
        """The per-frequency outputs y_hat[j] = (y1, y2, y3, y4) for j in freqs."""
        P = self.P
        Rh = circ.time_fft(P, r)
        out = {}
        for j in self.freqs:
            out[j] = self.block_apply(j, *circ.split_freq(P, Rh[:, j, :]), nonlinear)
        return out


class StokesPreconditioner(_Common):
    """Algorithms 1 and 2 with P~_j (section 3.2-3.4)."""

    def __init__(self, P, settings=None, freqs=None):
        super().__init__(P, None, settings, freqs)
        self._pressure_solvers()
        self.mg_W = {}

    def constants(self, j):
        return stokes_constants(self.d[j], self.P.tau, self.P.beta)

    def W_mg(self, j):
        if j not in self.mg_W:
            _, _, c1, c2 = self.constants(j)
            self.mg_W[j] = self._mg("q2", 1.0 + c1, c2 * self.P.nu)
        return self.mg_W[j]

    # --- the transforms of eq. (GJTransformation)
    def t_left_inv(self, j, r1, r2, r3, r4):
        tau = self.P.tau
        _, dc, _, c2 = self.constants(j)
        st = np.sqrt(tau)
        s1 = r1 / st
        s2 = (c2 / st) * (r2 - 1j * dc * r1 / tau)
        s3 = r3 / (st * c2)
        s4 = (r4 - 1j * dc * r3 / tau) / st
        return s1, s2, s3, s4

    def t_right_inv(self, j, x1, x2, x3, x4):
        tau = self.P.tau
        _, dc, _, c2 = self.constants(j)
        st = np.sqrt(tau)
        y2 = c2 * x2 / st
        y1 = (x1 + 1j * dc * y2 / st) / st
        y4 = x4 / st
        y3 = (x3 + 1j * dc * c2 * y4 / st) / (st * c2)
        return y1, y2, y3, y4

    def T_matrices(self, j):
        """Sparse T_l, Z_j, T_r (for checking the factorisation)."""
        o, tau = self.P.ops, self.P.tau
        _, dc, c1, c2 = self.constants(j)
        st = np.sqrt(tau)
        Iv, Ip = sp.identity(self.P.nv), sp.identity(self.P.nP)
        Tl = sp.bmat([[st * Iv, None, None, None],
                      [1j * dc / st * Iv, st / c2 * Iv, None, None],
                      [None, None, st * c2 * Ip, None],
                      [None, None, 1j * dc * c2 / st * Ip, st * Ip]], format="csr")
        Tr = sp.bmat([[st * Iv, -1j * dc / st * Iv, None, None],
                      [None, st / c2 * Iv, None, None],
                      [None, None, st * c2 * Ip, -1j * dc * c2 / st * Ip],
                      [None, None, None, st * Ip]], format="csr")
        return Tl, self.Z_matrix(j), Tr

    def Z_matrix(self, j):
        o = self.P.ops
        _, _, c1, c2 = self.constants(j)
        X = c1 * o.M + c2 * o.L
        Zp = sp.csr_matrix((self.P.nP, self.P.nP))
        return sp.bmat([[o.M, X, None, o.B.T], [X, -o.M, o.B.T, None],
                        [None, o.B, Zp, None], [o.B, None, None, Zp]], format="csr")

    # --- P~_j^{-1}
    def ptilde_inv(self, j, s1, s2, s3, s4):
        nV, nu = self.P.nV, self.P.nu
        _, _, c1, _ = self.constants(j)
        c2 = self.constants(j)[3]
        mg = self.W_mg(j)
        cyc = self.s.n_vcycles
        V = np.stack([s1[:nV], s1[nV:], s2[:nV], s2[nV:]], axis=1)    # 4 complex columns
        X = mg.solve(V, cyc)
        x1 = np.concatenate([X[:, 0], X[:, 1]])
        x2 = np.concatenate([X[:, 2], X[:, 3]])
        Z = self.unpin_in(np.stack([s3, s4], axis=1))
        Y = self.pin_out((1.0 + c1) * self.mg_Kp.solve(Z, cyc) + nu * c2 * self.cheb_MN(Z))
        return x1, x2, Y[:, 0], Y[:, 1]

    def Z_apply(self, j, x):
        return self.Z_matrix(j) @ x

    def block_apply(self, j, r1, r2, r3, r4, nonlinear=False):
        s = self.t_left_inv(j, r1, r2, r3, r4)
        if not nonlinear:
            x = self.ptilde_inv(j, *s)
        else:
            nv, nP = self.P.nv, self.P.nP
            Zj = self.Z_matrix(j)
            cut = np.cumsum([nv, nv, nP])

            def prec(v):
                return np.concatenate(self.ptilde_inv(j, *np.split(v, cut)))
            sv = np.concatenate(s)
            if self.s.inner_solver == "minres":
                # Z_j is real symmetric and P~_j Hermitian positive definite:
                # MINRES, stopping when the P~_j-norm of the residual falls
                # below inner_tol times that of s_j
                xv, its, _, _ = minres(lambda v: Zj @ v, prec, sv, self.s.inner_tol, self.s.inner_maxit)
            else:
                xv, its, _ = gmres(lambda v: Zj @ v, prec, sv, self.s.inner_tol,
                                   self.s.inner_restart, self.s.inner_maxit)
            self.inner_its[j] = its
            x = np.split(xv, cut)
        return self.t_right_inv(j, *x)


class OseenPreconditioner(_Common):
    """Algorithm 3 (P~_j^(UZ)) and its nonlinear GMRES wrapper (section 4)."""

    def __init__(self, P, wind, settings=None, freqs=None):
        super().__init__(P, wind, settings, freqs)
        self._pressure_solvers()
        o = P.ops
        self.cheb_M = self._mass_solver(o.Ms, Q2_MASS_BOUNDS)
        self.mg_Q, self.mg_QH = {}, {}

    def q_shift(self, j):
        return self.d[j] + self.P.tau / np.sqrt(self.P.beta)

    def Q_mgs(self, j):
        """Multigrid for Q_j = (d + tau/sqrt(beta)) M + tau nu K + tau N and
        Q_j^H = conj(d + tau/sqrt(beta)) M + tau nu K + tau N^T, with the
        coarse-level viscosity of ``coarse_viscosity``."""
        if j not in self.mg_Q:
            a, tau, nu = self.q_shift(j), self.P.tau, self.P.nu
            g = [tau * v for v in coarse_viscosity(nu, self.lv.wind_max, self.lv.sizes, self.P.side)]
            self.mg_Q[j] = self._mg("q2", a, tau * nu, eta=tau, gamma_levels=g)
            self.mg_QH[j] = self._mg("q2", np.conj(a), tau * nu, eta_t=tau, gamma_levels=g)
        return self.mg_Q[j], self.mg_QH[j]

    def _vec(self, f, x):
        """Apply a scalar Q2 solver to both velocity components."""
        nV = self.P.nV
        X = f(np.stack([x[:nV], x[nV:]], axis=1))
        return np.concatenate([X[:, 0], X[:, 1]])

    def G_matrix(self, j):
        return circ.G_block(self.P, self.d[j])

    def shat11_inv(self, j, y):
        """S^^{-1} y = tau Q_j^{-H} M Q_j^{-1} y with 4 V-cycles per solve."""
        o, tau = self.P.ops, self.P.tau
        mgQ, mgQH = self.Q_mgs(j)
        cyc = self.s.n_vcycles
        t = self._vec(lambda v: mgQ.solve(v, cyc), y)
        t = o.M @ t
        return tau * self._vec(lambda v: mgQH.solve(v, cyc), t)

    def uzawa(self, j, b1, b2, Minv=None, Sinv=None, mu=None, steps=None):
        """``steps`` iterations of eq. (Uzawa11) from zero on G_j^(1,1).

        Defaults: M^^{-1} = Chebyshev(M), S^^{-1} = shat11_inv, mu = 3/4, 6 steps."""
        o, tau, beta = self.P.ops, self.P.tau, self.P.beta
        d = self.d[j]
        Psi = (d * o.M + tau * o.L).tocsr()
        PsiH = (np.conj(d) * o.M + tau * o.L.T).tocsr()
        Minv = Minv or (lambda v: self._vec(self.cheb_M, v))
        Sinv = Sinv or (lambda v: self.shat11_inv(j, v))
        mu = self.s.mu_uzawa if mu is None else mu
        steps = self.s.n_uzawa if steps is None else steps
        x1 = np.zeros(self.P.nv, complex)
        x2 = np.zeros(self.P.nv, complex)
        for _ in range(steps):
            x1 = x1 + (1.0 / tau) * Minv(b1 - tau * (o.M @ x1) - PsiH @ x2)
            x2 = x2 - (1.0 / mu) * Sinv(b2 - Psi @ x1 + (tau / beta) * (o.M @ x2))
        return x1, x2

    def schur_inv(self, j, a, b):
        """S^_j^{-1}(a, b) on the pinned space: mass solves and H_p act on the
        unconstrained Q1 space (inputs extended by unpin_in), the K_p solves
        take the result with node 0 dropped."""
        o, tau, beta = self.P.ops, self.P.tau, self.P.beta
        d = self.d[j]
        cyc = self.s.n_vcycles
        MN = self.MN
        LN = (self.P.nu * o.full["K1"] + o.full["N1"]).tocsr() if "N1" in o.full else \
            (self.P.nu * o.full["K1"]).tocsr()
        Z = self.unpin_in(np.stack([b, a], axis=1))
        Zs = self.cheb_MN(Z) / tau
        z1, z2 = Zs[:, 0], Zs[:, 1]
        u1 = tau * (MN @ z1) + np.conj(d) * (MN @ z2) + tau * (LN.T @ z2)
        u2 = d * (MN @ z1) + tau * (LN @ z1) - (tau / beta) * (MN @ z2)
        U = self.stiff_p_inv(np.stack([u2[1:], u1[1:]], axis=1)) / tau
        return U[:, 0], U[:, 1]

    def puz_inv(self, j, r1, r2, r3, r4):
        o, tau = self.P.ops, self.P.tau
        y1, y2 = self.uzawa(j, r1, r2)
        a = r3 - tau * (o.B @ y2)
        b = r4 - tau * (o.B @ y1)
        y3, y4 = self.schur_inv(j, a, b)
        return y1, y2, -y3, -y4

    def block_apply(self, j, r1, r2, r3, r4, nonlinear=False):
        if not nonlinear:
            return self.puz_inv(j, r1, r2, r3, r4)
        nv, nP = self.P.nv, self.P.nP
        G = self.G_matrix(j)
        cut = np.cumsum([nv, nv, nP])

        def prec(v):
            return np.concatenate(self.puz_inv(j, *np.split(v, cut)))
        rv = np.concatenate([r1, r2, r3, r4])
        yv, its, _ = gmres(lambda v: G @ v, prec, rv, self.s.inner_tol,
                           self.s.inner_restart, self.s.inner_maxit)
        self.inner_its[j] = its
        return tuple(np.split(yv, cut))
