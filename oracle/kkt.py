"""All-at-once KKT system of the Stokes/Oseen control problem.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The problem of section 2 (eq. OseenOptimization / OseenFlow), discretised in
section 2.2 with backward Euler (tau = T/nt), gives the optimality system whose
permuted Kronecker form is eq. (FinalA):

    A = [[tau I, E^T], [E, -tau/beta I]] (x) [[M, 0], [0, 0]]
        + tau [[0, 0], [I, 0]] (x) [[L, B^T], [B, 0]]
        + tau [[0, I], [0, 0]] (x) [[L^T, B^T], [B, 0]]

with E the lower-bidiagonal backward-Euler matrix (1 on the diagonal, -1
below).  Reading used here: the identity I_t and E have size nt (one block
per backward-Euler step), the unknowns of block 0 are (v, p) at t_k = k tau,
k = 1..nt, those of block 1 are (lambda, mu) at the same times, the rows of
block 0 are the adjoint equations and those of block 1 the state equations.
With v_0 = 0, f = 0, h = 0 and lambda_{nt+1} = 0 the right-hand side is
tau M v_d(t_k) on the adjoint momentum rows and zero elsewhere (section 2.2);
``rhs_data`` forms it for a forcing f, Dirichlet data h and an initial
velocity v_0 as well (the vectors g and h of section 2.2).

Two vector layouts are used: *compact* (only free unknowns:
[b][t][v (2 n_V), p (n_P)]) and *canonical* (the library's padded layout,
``workloads`` docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import Operators


class Problem:
    """Spatial operators plus the time discretisation of one control problem."""

    def __init__(self, N: int, nt: int, T: float, nu: float, beta: float, wind=None, domain=None):
        """``domain``: (x0, y0, x1, y1) of a square, default the unit square."""
        if nt < 2:
            raise ValueError("nt must be >= 2")
        self.N, self.nt, self.T, self.nu, self.beta = N, nt, float(T), float(nu), float(beta)
        self.tau = self.T / nt
        x0, y0, x1, y1 = (0.0, 0.0, 1.0, 1.0) if domain is None else (float(v) for v in domain)
        if not (x1 > x0 and abs((y1 - y0) - (x1 - x0)) <= 1e-14 * (x1 - x0)):
            raise ValueError("domain must be a square")
        self.side = x1 - x0
        self.origin = (x0, y0)
        self.ops = Operators(N, nu, wind, self.side, self.origin)
        g = self.ops.grid
        self.nV, self.nv, self.nP = g.nV, g.nv, g.nP
        self.n = self.nv + self.nP             # unknowns per time level and block
        self.n_all = 2 * nt * self.n

    @classmethod
    def from_workload(cls, w, wind=None):
        if w.flow == 1 and wind is None:
            raise ValueError("Oseen workload needs a wind")
        return cls(w.N, w.nt, w.T, w.nu, w.beta, wind if w.flow == 1 else None)

    # ------------------------------------------------------------------ layout
    def _level_maps(self):
        g = self.ops.grid
        nq2 = g.nq2
        return np.concatenate([g.v_interior, nq2 + g.v_interior, 2 * nq2 + g.p_kept])

    def to_compact(self, xc: np.ndarray) -> np.ndarray:
        g = self.ops.grid
        lvl = 2 * g.nq2 + g.np2
        X = np.asarray(xc).reshape(2 * self.nt, lvl)
        return X[:, self._level_maps()].reshape(-1)

    def to_canonical(self, x: np.ndarray) -> np.ndarray:
        g = self.ops.grid
        lvl = 2 * g.nq2 + g.np2
        X = np.zeros((2 * self.nt, lvl), dtype=np.result_type(x, float))
        X[:, self._level_maps()] = np.asarray(x).reshape(2 * self.nt, self.n)
        return X.reshape(-1)

    # ------------------------------------------------------------ the matrix
    def E(self) -> sp.csr_matrix:
        nt = self.nt
        return sp.diags([np.ones(nt), -np.ones(nt - 1)], [0, -1], format="csr")

    def spatial_blocks(self):
        o = self.ops
        Z = sp.csr_matrix((self.nP, self.nP))
        Mb = sp.block_diag([o.M, Z]).tocsr()                                   # [[M,0],[0,0]]
        HL = sp.bmat([[o.L, o.B.T], [o.B, None]], format="csr")             # [[L,B^T],[B,0]]
        HLt = sp.bmat([[o.L.T, o.B.T], [o.B, None]], format="csr")          # [[L^T,B^T],[B,0]]
        return Mb, HL, HLt

    def kkt_matrix(self, time_matrix=None) -> sp.csr_matrix:
        """Eq. (FinalA) with the given nt x nt time-stepping matrix (default E)."""
        nt, tau, beta = self.nt, self.tau, self.beta
        E = self.E() if time_matrix is None else sp.csr_matrix(time_matrix)
        I = sp.identity(nt, format="csr")
        Mb, HL, HLt = self.spatial_blocks()
        Z = sp.csr_matrix((nt, nt))
        T1 = sp.bmat([[tau * I, E.T], [E, -(tau / beta) * I]])
        T2 = sp.bmat([[Z, Z], [I, Z]])
        T3 = sp.bmat([[Z, I], [Z, Z]])
        return (sp.kron(T1, Mb) + tau * sp.kron(T2, HL) + tau * sp.kron(T3, HLt)).tocsr()

    def kkt_apply(self, x: np.ndarray) -> np.ndarray:
        """y = A x evaluated time level by time level (same algebra as
        ``kkt_matrix`` without forming it; used at sizes where the Kronecker
        matrix would not fit in memory)."""
        o, nt, tau, beta = self.ops, self.nt, self.tau, self.beta
        nv = self.nv
        X = np.asarray(x).reshape(2, nt, self.n)
        v, p = X[0, :, :nv].T, X[0, :, nv:].T          # (nv, nt), (nP, nt)
        lam, mu = X[1, :, :nv].T, X[1, :, nv:].T
        Mv, Ml = o.M @ v, o.M @ lam
        Ml_next = np.zeros_like(Ml); Ml_next[:, :-1] = Ml[:, 1:]
        Mv_prev = np.zeros_like(Mv); Mv_prev[:, 1:] = Mv[:, :-1]
        adj_v = tau * Mv + (Ml - Ml_next) + tau * (o.L.T @ lam) + tau * (o.B.T @ mu)
        adj_p = tau * (o.B @ lam)
        st_v = (Mv - Mv_prev) + tau * (o.L @ v) + tau * (o.B.T @ p) - (tau / beta) * Ml
        st_p = tau * (o.B @ v)
        Y = np.empty((2, nt, self.n), dtype=np.result_type(x, float))
        Y[0, :, :nv], Y[0, :, nv:] = adj_v.T, adj_p.T
        Y[1, :, :nv], Y[1, :, nv:] = st_v.T, st_p.T
        return Y.reshape(-1)

    # ---------------------------------------------------------------- the rhs
    def rhs(self, vd: np.ndarray) -> np.ndarray:
        """b for v_0 = f = h = 0: tau M v_d(t_k) on adjoint momentum rows.

        ``vd`` has shape (nt, 2, (2N+1)^2) (Q2 nodal values, boundary ignored)."""
        g = self.ops.grid
        vdi = np.asarray(vd)[:, :, g.v_interior].reshape(self.nt, self.nv)   # (nt, nv)
        b = np.zeros((2, self.nt, self.n))
        b[0, :, :self.nv] = self.tau * (self.ops.M @ vdi.T).T
        return b.reshape(-1)

    def rhs_data(self, vd=None, f=None, h=None, v0=None) -> np.ndarray:
        """b of section 2.2 for general data (compact layout).

        Nodal values on the full Q2 grid, None meaning zero: ``vd`` and ``f``
        of shape (nt, 2, (2N+1)^2) at t_k = k tau, k = 1..nt; ``h`` of shape
        (nt + 1, 2, (2N+1)^2) at t_k, k = 0..nt (only its boundary entries are
        used); ``v0`` of shape (2, (2N+1)^2) (only its interior entries are
        used; its boundary values are h at t_0).

        The velocity at t_k is v_k = v_k^I + h_k^B, the unknown interior part
        plus the known boundary values.  Moving every known term of the
        discrete equations of section 2.2 to the right, with full-grid
        matrices restricted to interior rows (R):
          adjoint momentum  tau R M (v_d,k - h_k^B)
          adjoint div.      0
          state momentum    R [tau M f_k - (M + tau L) h_k^B + M w_{k-1}],
                            w_0 = v_0^I + h_0^B, w_{k-1} = h_{k-1}^B (k >= 2)
          state div.        -tau R_p B h_k^B
        """
        g, o, nt, tau = self.ops.grid, self.ops, self.nt, self.tau
        full = o.full
        nq2 = g.nq2
        bd = g.q2_boundary()
        M2 = full["M2"]
        L2 = (self.nu * full["K2"] + full["N2"]).tocsr() if "N2" in full else (self.nu * full["K2"]).tocsr()
        z = np.zeros((nt, 2, nq2))
        vd = z if vd is None else np.asarray(vd, float)
        f = z if f is None else np.asarray(f, float)
        H = np.zeros((nt + 1, 2, nq2)) if h is None else np.asarray(h, float) * bd
        v0i = np.zeros((2, nq2)) if v0 is None else np.asarray(v0, float) * ~bd
        Rv, Rp = g.Rv(), g.Rp()
        Bf = [full["Bx"], full["By"]]
        b = np.zeros((2, nt, self.n))
        for k in range(nt):
            hk = H[k + 1]
            wprev = (v0i + H[0]) if k == 0 else H[k]
            adj = [tau * (Rv @ (M2 @ (vd[k, c] - hk[c]))) for c in range(2)]
            st = [Rv @ (tau * (M2 @ f[k, c]) - (M2 @ hk[c] + tau * (L2 @ hk[c])) + M2 @ wprev[c]) for c in range(2)]
            div = -tau * (Rp @ (Bf[0] @ hk[0] + Bf[1] @ hk[1]))
            b[0, k, :self.nv] = np.concatenate(adj)
            b[1, k, :self.nv] = np.concatenate(st)
            b[1, k, self.nv:] = div
        return b.reshape(-1)

    def full_velocity(self, x: np.ndarray, h=None, v0=None) -> np.ndarray:
        """State velocity on the full Q2 grid at t_0..t_nt: (nt + 1, 2, (2N+1)^2),
        interior values from the compact solution x, boundary values from the
        Dirichlet data h (as in ``rhs_data``), t_0 from v0 and h_0."""
        g = self.ops.grid
        nq2 = g.nq2
        bd = g.q2_boundary()
        H = np.zeros((self.nt + 1, 2, nq2)) if h is None else np.asarray(h, float) * bd
        V = H.copy()
        if v0 is not None:
            V[0] += np.asarray(v0, float) * ~bd
        v, _, _, _ = self.split(x)
        for k in range(self.nt):
            V[k + 1][:, g.v_interior] = v[k].reshape(2, g.nV)
        return V

    # ----------------------------------------------------------- direct solve
    def solve_direct(self, b: np.ndarray) -> np.ndarray:
        A = self.kkt_matrix().tocsc()
        return spla.splu(A).solve(np.asarray(b, float))

    # ------------------------------------------------ sequential time stepping
    def forward(self, u: np.ndarray):
        """State equation stepped forward in time for a given control u.

        M (v_k - v_{k-1}) + tau L v_k + tau B^T p_k = tau M u_k,  tau B v_k = 0,
        k = 1..nt, v_0 = 0 (section 2.2).  u has shape (nt, n_v)."""
        o, tau = self.ops, self.tau
        K = sp.bmat([[o.M + tau * o.L, tau * o.B.T], [tau * o.B, None]], format="csc")
        lu = spla.splu(K)
        v = np.zeros((self.nt, self.nv)); p = np.zeros((self.nt, self.nP))
        vprev = np.zeros(self.nv)
        for k in range(self.nt):
            rhs = np.concatenate([o.M @ vprev + tau * (o.M @ u[k]), np.zeros(self.nP)])
            sol = lu.solve(rhs)
            v[k], p[k] = sol[:self.nv], sol[self.nv:]
            vprev = v[k]
        return v, p

    def backward(self, v: np.ndarray, vd_int: np.ndarray):
        """Adjoint equation stepped backward in time:

        M (lambda_k - lambda_{k+1}) + tau L^T lambda_k + tau B^T mu_k
            = tau M (v_d,k - v_k),  tau B lambda_k = 0,  lambda_{nt+1} = 0."""
        o, tau = self.ops, self.tau
        K = sp.bmat([[o.M + tau * o.L.T, tau * o.B.T], [tau * o.B, None]], format="csc")
        lu = spla.splu(K)
        lam = np.zeros((self.nt, self.nv)); mu = np.zeros((self.nt, self.nP))
        lnext = np.zeros(self.nv)
        for k in range(self.nt - 1, -1, -1):
            rhs = np.concatenate([o.M @ lnext + tau * (o.M @ (vd_int[k] - v[k])), np.zeros(self.nP)])
            sol = lu.solve(rhs)
            lam[k], mu[k] = sol[:self.nv], sol[self.nv:]
            lnext = lam[k]
        return lam, mu

    def vd_interior(self, vd):
        g = self.ops.grid
        return np.asarray(vd)[:, :, g.v_interior].reshape(self.nt, self.nv)

    def objective(self, u: np.ndarray, vd) -> float:
        """Discrete cost: tau/2 sum (v_k - vd_k)^T M (v_k - vd_k) + beta tau/2 sum u_k^T M u_k."""
        v, _ = self.forward(u)
        e = v - self.vd_interior(vd)
        M = self.ops.M
        return 0.5 * self.tau * np.einsum("ki,ki->", e, (M @ e.T).T) + \
            0.5 * self.beta * self.tau * np.einsum("ki,ki->", u, (M @ u.T).T)

    def reduced_gradient(self, u: np.ndarray, vd) -> np.ndarray:
        """g(u) = tau beta M u - tau M lambda(u) (gradient equation, section 2.1)."""
        v, _ = self.forward(u)
        lam, _ = self.backward(v, self.vd_interior(vd))
        M = self.ops.M
        return self.tau * self.beta * (M @ u.T).T - self.tau * (M @ lam.T).T

    def split(self, x: np.ndarray):
        """(v, p, lambda, mu) with time as the leading axis."""
        X = np.asarray(x).reshape(2, self.nt, self.n)
        return X[0, :, :self.nv], X[0, :, self.nv:], X[1, :, :self.nv], X[1, :, self.nv:]
