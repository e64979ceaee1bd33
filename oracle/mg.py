"""Geometric multigrid on the nested uniform grids N, N/2, ..., 2.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section 3.4 applies "4 V-cycles" of a geometric multigrid method with SOR
smoothing to W_j and K_p (Stokes) and to Q_j, Q_j^H and K_p (Oseen).  Readings
used (the paper leaves these unstated):

* V(1,1) cycle: one forward sweep of multicolour Gauss-Seidel (SOR with
  relaxation factor 1 over the whole grid, ``smoothers.ColouredSOR``) before
  the coarse correction, one backward sweep after it (so the cycle is
  symmetric for symmetric operators); coarsest grid N = 2 solved exactly by
  dense LU.  ``tiling`` (a ``smoothers.Tiling``) selects instead the tiled
  block-Jacobi/Gauss-Seidel variant a GPU may run, with the caller's tiles.
* Coarse operators are rediscretised with the same coefficients on the coarse
  grid; for nested conforming spaces with exact quadrature this equals the
  Galerkin product P^T A P.  The coarse-grid wind is the fine nodal wind
  injected at the coarse nodes.
* Prolongation P is finite-element interpolation: Q2 one-dimensional weights
  are 1 at coincident nodes and (3/8, 3/4, -1/8) / (-1/8, 3/4, 3/8) at the
  quarter points of a coarse element; Q1 uses (1/2, 1/2) at midpoints.
  Restriction is P^T.  Dirichlet (Q2) nodes are excluded on every level.
* Pressure-space (Q1) operators act on the *unconstrained* node set with
  natural boundary conditions.  The pressure Laplacian K_N is then singular
  with the constants as kernel, and V-cycles are applied to consistent
  right-hand sides only; the coarsest singular system is solved with node
  (0,0) held at zero (any solution is acceptable, the caller removes the
  constant).  This is how the pinned K_p^{-1} is applied, through the exact
  identity  K_p^{-1} = R L K_N^+ L^T R^T,  L = I - 1 e_0^T, R = drop node 0,
  which multigrid approximates far better than V-cycles on the pinned matrix
  (the pin leaves a mode with an O(h^2) eigenvalue that coarse grids cannot
  represent).
* ``cycles`` V-cycles start from x = 0; each later cycle starts its
  pre-smoothing from the current iterate.

A scalar operator on a level is  alpha M + gamma K + eta N + eta_t N^T  with
M, K, N the mass, stiffness and convection matrices of the family (Q2
interior or pinned Q1) and complex-allowed scalar coefficients.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .fem import Operators
from .smoothers import ColouredSOR, TiledSOR, colours_q2, tiles_of


def prolong_1d_q2(Nc: int) -> np.ndarray:
    """(2Nf+1) x (2Nc+1) 1-D Q2 interpolation, Nf = 2 Nc."""
    Nf = 2 * Nc
    P = np.zeros((2 * Nf + 1, 2 * Nc + 1))
    for i in range(2 * Nf + 1):
        e, r = divmod(i, 4)
        if r == 0:
            P[i, 2 * e] = 1.0
        elif r == 2:
            P[i, 2 * e + 1] = 1.0
        elif r == 1:
            P[i, 2 * e: 2 * e + 3] = [3 / 8, 3 / 4, -1 / 8]
        else:
            P[i, 2 * e: 2 * e + 3] = [-1 / 8, 3 / 4, 3 / 8]
    return P


def prolong_1d_q1(Nc: int) -> np.ndarray:
    Nf = 2 * Nc
    P = np.zeros((Nf + 1, Nc + 1))
    for i in range(Nf + 1):
        if i % 2 == 0:
            P[i, i // 2] = 1.0
        else:
            P[i, (i - 1) // 2] = 0.5
            P[i, (i + 1) // 2] = 0.5
    return P


def inject_wind(wind, Nf: int):
    """Fine Q2 nodal wind -> coarse (Nf/2) Q2 nodal wind by injection."""
    if wind is None:
        return None
    nqf = 2 * Nf + 1
    W = np.asarray(wind).reshape(2, nqf, nqf)
    return W[:, ::2, ::2].reshape(2, -1)


class Levels:
    """Level matrices and transfer operators of one hierarchy (one wind)."""

    def __init__(self, N: int, wind=None, side: float = 1.0):
        if N < 2 or (N & (N - 1)):
            raise ValueError("N must be a power of two >= 2")
        self.sizes = []
        self.side = float(side)
        n = N
        while n >= 2:
            self.sizes.append(n)
            n //= 2
        self.ops = []
        w = None if wind is None else np.asarray(wind)
        # largest nodal wind speed of the finest grid (0 without wind)
        self.wind_max = 0.0 if w is None else float(np.sqrt((w.reshape(2, -1) ** 2).sum(axis=0)).max())
        for l, n in enumerate(self.sizes):
            self.ops.append(Operators(n, 1.0, w, side))
            if l + 1 < len(self.sizes):
                w = inject_wind(w, n)
        self.P2, self.P1 = [], []
        for l in range(len(self.sizes) - 1):
            f, c = self.ops[l].grid, self.ops[l + 1].grid
            p = prolong_1d_q2(self.sizes[l + 1])
            P = sp.csr_matrix(np.kron(p, p))
            self.P2.append((f.Rv() @ P @ c.Rv().T).tocsr())
            p = prolong_1d_q1(self.sizes[l + 1])
            self.P1.append(sp.csr_matrix(np.kron(p, p)))      # unconstrained Q1

    def family(self, fam: str, l: int):
        """(M, K, N, colours, (ix, iy, nodes per side)) of a level's node set."""
        o = self.ops[l]
        g = o.grid
        if fam == "q2":
            iy, ix = np.divmod(g.v_interior, g.nq)
            return o.Ms, o.Ks, o.Ns, colours_q2(g), (ix, iy, g.nq)
        if fam == "q1":
            f = o.full
            Nn = f["N1"] if "N1" in f else sp.csr_matrix(f["M1"].shape)
            iy, ix = np.divmod(np.arange(g.np2), g.np1)
            return f["M1"], f["K1"], Nn, 2 * (iy % 2) + (ix % 2), (ix, iy, g.np1)
        raise ValueError(fam)

    def prolong(self, fam: str, l: int):
        return self.P2[l] if fam == "q2" else self.P1[l]


def coarse_viscosity(nu: float, wind_max: float, sizes, side: float = 1.0) -> list:
    """Viscosity of the multigrid level operators of a convection-diffusion
    operator: the true nu on the finest level; on a coarser level of n x n
    elements (side h = side/n) at least wind_max h / 4, so that its mesh Peclet
    number wind_max h / (2 nu_l) stays at most 2.  Rediscretising at the true
    nu makes the V-cycle diverge once the coarse levels are convection
    dominated (the Gauss-Seidel smoother and the coarse correction both
    amplify there); the finest level, where the residual is formed, keeps the
    true operator, so the cycle stays a preconditioner for it."""
    return [nu if l == 0 else max(nu, wind_max * side / (4.0 * n)) for l, n in enumerate(sizes)]


class ScalarMG:
    """V(1,1) multigrid for  alpha M + gamma K + eta N + eta_t N^T.

    ``gamma_levels`` (optional, one value per level) replaces gamma on each
    level's operator (the finest included).  ``tiling`` (optional
    ``smoothers.Tiling``) replaces the global multicolour sweep by the tiled
    variant."""

    def __init__(self, levels: Levels, fam: str, alpha, gamma, eta=0.0, eta_t=0.0, gamma_levels=None,
                 tiling=None):
        self.lv, self.fam = levels, fam
        self.A, self.sor = [], []
        for l in range(len(levels.sizes)):
            M, K, N, col, (ix, iy, side) = levels.family(fam, l)
            A = alpha * M + (gamma if gamma_levels is None else gamma_levels[l]) * K
            if eta != 0:
                A = A + eta * N
            if eta_t != 0:
                A = A + eta_t * N.T
            A = sp.csr_matrix(A)
            self.A.append(A)
            if tiling is None:
                self.sor.append(ColouredSOR(A, col))
            else:
                T = tiling.q2 if fam == "q2" else tiling.q1
                self.sor.append(TiledSOR(A, col, tiles_of(ix, iy, side, T)))
        Ac = self.A[-1].toarray()
        self.pin_coarse = fam == "q1"
        self.coarse = sla.lu_factor(Ac[1:, 1:] if self.pin_coarse else Ac)

    def coarse_solve(self, b):
        if not self.pin_coarse:
            return sla.lu_solve(self.coarse, b)
        x = np.zeros_like(b)
        x[1:] = sla.lu_solve(self.coarse, b[1:])
        return x

    def vcycle(self, l: int, b: np.ndarray, x: np.ndarray) -> np.ndarray:
        if l == len(self.A) - 1:
            return self.coarse_solve(b)
        x = self.sor[l].forward(b, x)
        r = b - self.A[l] @ x
        P = self.lv.prolong(self.fam, l)
        rc = P.T @ r
        ec = self.vcycle(l + 1, rc, np.zeros_like(rc))
        x = x + P @ ec
        return self.sor[l].backward(b, x)

    def solve(self, b: np.ndarray, cycles: int = 4) -> np.ndarray:
        dt = np.result_type(b, self.A[0].dtype)
        x = np.zeros(b.shape, dtype=dt)
        b = b.astype(dt)
        for _ in range(cycles):
            x = self.vcycle(0, b, x)
        return x


class ExactSolve:
    """Drop-in for ``ScalarMG`` that solves the level-0 operator exactly
    (sparse LU), for pins that replace the paper's inner approximations by the
    inverses they approximate.  Q1 operators act on the unconstrained node set
    and may be singular (the pressure Laplacian): node 0 is then held at zero,
    which solves every consistent system."""

    def __init__(self, A, pin_node0: bool = False):
        import scipy.sparse.linalg as spla
        A = sp.csc_matrix(A)
        self.pin = pin_node0
        self.real = not np.iscomplexobj(A.data)
        self.lu = spla.splu(A[1:, 1:].tocsc() if pin_node0 else A)

    def _lu(self, b):
        if self.real and np.iscomplexobj(b):
            return self.lu.solve(np.ascontiguousarray(b.real)) + 1j * self.lu.solve(np.ascontiguousarray(b.imag))
        return self.lu.solve(b)

    def _one(self, b):
        if not self.pin:
            return self._lu(b)
        x = np.zeros(b.shape, dtype=np.result_type(b, 1.0))
        x[1:] = self._lu(np.ascontiguousarray(b[1:]))
        return x

    def solve(self, b: np.ndarray, cycles: int = 0) -> np.ndarray:
        if b.ndim == 1:
            return self._one(b)
        return np.stack([self._one(np.ascontiguousarray(b[:, k])) for k in range(b.shape[1])], axis=1)
