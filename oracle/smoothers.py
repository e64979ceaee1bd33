"""Stationary building blocks: multicolour SOR sweeps and Chebyshev semi-iteration.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section 3.4 approximates mass-matrix inverses by the Chebyshev semi-iteration
(10 steps) and smooths the multigrid levels with successive over-relaxation.
The paper states neither the SOR ordering, the relaxation factor nor the
Chebyshev spectrum bounds; the readings used here are:

* SOR: relaxation factor 1 (Gauss-Seidel) in a multicolour ordering.  Q2 nodes
  couple only with nodes at most 2 grid indices away in each direction, so the
  9 classes (ix mod 3, iy mod 3) are independent sets; Q1 nodes couple within
  1 index, so (ix mod 2, iy mod 2) gives 4.  Colour number = 3*(iy%3) + ix%3
  (Q2) or 2*(iy%2) + ix%2 (Q1) with (ix, iy) the padded-grid node indices.
  A forward sweep visits colours 0..C-1, a backward sweep C-1..0.
* Tiled variant (not the paper's method).  A GPU may run the sweep inside
  square tiles held in fast on-chip memory: the grid is cut into tiles of T
  node indices per side, tile (ix // T, iy // T); the colour sweep runs inside
  every tile while couplings to other tiles use the values the sweep started
  from (block Jacobi between tiles, Gauss-Seidel inside).  ``TiledSOR`` states
  that sweep for a tile size the caller passes in; this module fixes none.
  Grids of at most T nodes per side form a single tile, where the tiled sweep
  is plain multicolour Gauss-Seidel.
* Chebyshev: Jacobi-preconditioned semi-iteration of Golub and Varga with the
  element-wise spectrum bounds of diag(M)^{-1} M: the 1-D P2 element gives
  [1/2, 5/4] and P1 gives [1/2, 3/2]; tensor products give [1/4, 25/16] for
  Q2 and [1/4, 9/4] for Q1.  ``k`` steps from x_0 = 0 return x_k.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

Q2_MASS_BOUNDS = (0.25, 25.0 / 16.0)
Q1_MASS_BOUNDS = (0.25, 9.0 / 4.0)


def colours_q2(grid) -> np.ndarray:
    """Colour of every interior Q2 node (compact order)."""
    iy, ix = np.divmod(grid.v_interior, grid.nq)
    return 3 * (iy % 3) + (ix % 3)


def colours_q1(grid) -> np.ndarray:
    """Colour of every kept (non-pinned) Q1 node (compact order)."""
    iy, ix = np.divmod(grid.p_kept, grid.np1)
    return 2 * (iy % 2) + (ix % 2)


def tiles_of(ix, iy, nside, T) -> np.ndarray:
    """Tile number of nodes (ix, iy) on a grid of nside nodes per side."""
    ntx = (nside + T - 1) // T
    return (iy // T) * ntx + ix // T


class ColouredSOR:
    """Gauss-Seidel sweeps over independent colour classes of a sparse matrix."""

    def __init__(self, A: sp.spmatrix, colours: np.ndarray, omega: float = 1.0):
        A = sp.csr_matrix(A)
        self.A = A
        self.diag = A.diagonal()
        self.omega = omega
        self.ncol = int(colours.max()) + 1 if colours.size else 0
        self.idx = [np.flatnonzero(colours == c) for c in range(self.ncol)]
        self.rows = [A[i, :] for i in self.idx]
        for c, R in enumerate(self.rows):        # independence of each class
            sub = R[:, self.idx[c]].tocoo()
            assert np.all(sub.row == sub.col), "colour class is not an independent set"

    def _update(self, c, b, x):
        i = self.idx[c]
        d = self.diag[i] if x.ndim == 1 else self.diag[i][:, None]
        x[i] += self.omega * (b[i] - self.rows[c] @ x) / d

    def forward(self, b, x):
        for c in range(self.ncol):
            self._update(c, b, x)
        return x

    def backward(self, b, x):
        for c in range(self.ncol - 1, -1, -1):
            self._update(c, b, x)
        return x


class Tiling:
    """Tile sizes (node indices per side) of the tiled smoother variant on Q2
    and Q1 grids.  Passed in by whoever compares against a tiled sweep."""

    def __init__(self, q2: int, q1: int):
        if q2 < 1 or q1 < 1:
            raise ValueError("tile sizes must be positive")
        self.q2, self.q1 = int(q2), int(q1)


class TiledSOR:
    """Multicolour Gauss-Seidel inside tiles, block Jacobi between tiles.

    Split A = A_in + A_out with A_in the couplings between nodes of the same
    tile.  A sweep from x computes b' = b - A_out x once (neighbour tiles seen
    at the start of the sweep) and then runs the colour sweep of A_in on b'.
    Forward and backward sweeps are transposes of each other for symmetric A."""

    def __init__(self, A: sp.spmatrix, colours: np.ndarray, tiles: np.ndarray):
        C = sp.csr_matrix(A).tocoo()
        same = tiles[C.row] == tiles[C.col]
        n = A.shape[0]
        self.A = sp.csr_matrix(A)
        A_in = sp.csr_matrix((C.data[same], (C.row[same], C.col[same])), shape=(n, n))
        self.A_out = sp.csr_matrix((C.data[~same], (C.row[~same], C.col[~same])), shape=(n, n))
        self.inner = ColouredSOR(A_in, colours)
        self.ncol = self.inner.ncol
        self.diag = self.inner.diag

    def forward(self, b, x):
        return self.inner.forward(b - self.A_out @ x, x)

    def backward(self, b, x):
        return self.inner.backward(b - self.A_out @ x, x)


def chebyshev(A: sp.spmatrix, b: np.ndarray, steps: int, bounds) -> np.ndarray:
    """Jacobi-preconditioned Chebyshev semi-iteration, ``steps`` steps from 0.

    With D = diag(A) and spectrum(D^{-1} A) in [lo, hi]:
        gamma = 2 / (lo + hi),  sigma = (hi - lo) / (hi + lo)
        x_1 = gamma D^{-1} b
        x_{k+1} = omega_{k+1} (x_k - x_{k-1} + gamma D^{-1}(b - A x_k)) + x_{k-1}
        omega_2 = 1 / (1 - sigma^2 / 2),  omega_{k+1} = 1 / (1 - sigma^2 omega_k / 4).
    """
    lo, hi = bounds
    D = A.diagonal()
    if b.ndim > 1:
        D = D[:, None]
    gamma = 2.0 / (lo + hi)
    sigma = (hi - lo) / (hi + lo)
    if steps <= 0:
        return np.zeros_like(b)
    x_prev = np.zeros_like(b)
    x = gamma * b / D
    omega = 1.0
    for k in range(1, steps):
        omega = 1.0 / (1.0 - 0.5 * sigma * sigma) if k == 1 else 1.0 / (1.0 - 0.25 * sigma * sigma * omega)
        x_new = omega * (x - x_prev + gamma * (b - A @ x) / D) + x_prev
        x_prev, x = x, x_new
    return x


def chebyshev_error_bound(steps: int, bounds) -> float:
    """1 / T_k(1/sigma): the energy-norm error reduction guaranteed after k steps."""
    lo, hi = bounds
    sigma = (hi - lo) / (hi + lo)
    return 1.0 / np.cosh(steps * np.arccosh(1.0 / sigma))
