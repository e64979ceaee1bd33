"""Q2-Q1 Taylor-Hood matrices on N x N uniform quadrilaterals of a square.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section 2.2 of the paper discretises velocity with Q2 and pressure with Q1
(Taylor-Hood) elements and names the matrices used throughout:

* ``M``  velocity mass matrix,
* ``L``  the weak form of  -nu Laplace + w . grad  (per velocity component),
* ``B``  the discretised *negative* divergence,
* ``M_p, K_p, L_p`` their pressure-space counterparts (section 2.3 and 4).

The square is [x0, x0 + side] x [y0, y0 + side] (default: the unit square;
the paper's own experiments use [-1, 1]^2, section 5).

Node numbering (both here and at the library boundary): a Q2 grid has
``nq = 2N+1`` nodes per side with spacing h/2, numbered ``iy*nq + ix`` (x
fastest); a Q1 grid has ``N+1`` nodes per side numbered ``iy*(N+1) + ix``.
Homogeneous Dirichlet velocity data is imposed by eliminating boundary Q2
nodes; the pressure is fixed at the Q1 node (0,0) (section 2.2) by removing
that node.  All integrals use the 3x3 Gauss-Legendre rule per element, which
is exact for M, K, B, M_p, K_p and for the convection term whenever the wind
has degree <= 1 in the variable it is *not* differentiated against (true for
the wind used in the Oseen workload).  The wind is represented by its Q2
nodal interpolant.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from numpy.polynomial import Polynomial as Poly

# 3-point Gauss-Legendre rule on [0, 1]
GAUSS_X = np.array([0.5 - np.sqrt(15.0) / 10.0, 0.5, 0.5 + np.sqrt(15.0) / 10.0])
GAUSS_W = np.array([5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0])


def p2_basis(s):
    """1-D quadratic Lagrange basis on [0,1] with nodes 0, 1/2, 1: values, d/ds."""
    s = np.asarray(s, dtype=float)
    val = np.array([(1 - s) * (1 - 2 * s), 4 * s * (1 - s), s * (2 * s - 1)])
    der = np.array([4 * s - 3, 4 - 8 * s, 4 * s - 1])
    return val, der


def p1_basis(s):
    """1-D linear Lagrange basis on [0,1] with nodes 0, 1: values, d/ds."""
    s = np.asarray(s, dtype=float)
    val = np.array([1 - s, s])
    der = np.array([-np.ones_like(s), np.ones_like(s)])
    return val, der


class Grid:
    """Index bookkeeping for the Q2 velocity and Q1 pressure grids."""

    def __init__(self, N: int, side: float = 1.0, origin=(0.0, 0.0)):
        if N < 1:
            raise ValueError("N must be >= 1")
        if side <= 0:
            raise ValueError("side must be positive")
        self.N = N
        self.side = float(side)
        self.x0, self.y0 = float(origin[0]), float(origin[1])
        self.h = self.side / N
        self.nq = 2 * N + 1          # Q2 nodes per side
        self.np1 = N + 1             # Q1 nodes per side
        self.nq2 = self.nq * self.nq
        self.np2 = self.np1 * self.np1
        iy, ix = np.divmod(np.arange(self.nq2), self.nq)
        inner = (ix > 0) & (ix < self.nq - 1) & (iy > 0) & (iy < self.nq - 1)
        self.v_interior = np.flatnonzero(inner)          # kept Q2 nodes
        self.p_kept = np.arange(1, self.np2)             # Q1 node 0 is pinned
        self.nV = self.v_interior.size                   # (2N-1)^2
        self.nP = self.p_kept.size                       # (N+1)^2 - 1
        self.nv = 2 * self.nV

    # node coordinates
    def q2_xy(self):
        iy, ix = np.divmod(np.arange(self.nq2), self.nq)
        return self.x0 + ix * (self.h / 2), self.y0 + iy * (self.h / 2)

    def q1_xy(self):
        iy, ix = np.divmod(np.arange(self.np2), self.np1)
        return self.x0 + ix * self.h, self.y0 + iy * self.h

    def q2_boundary(self):
        """Mask of the Q2 nodes on the boundary (Dirichlet velocity nodes)."""
        iy, ix = np.divmod(np.arange(self.nq2), self.nq)
        return (ix == 0) | (iy == 0) | (ix == self.nq - 1) | (iy == self.nq - 1)

    # restriction operators (rows select kept nodes)
    def Rv(self):
        return sp.csr_matrix((np.ones(self.nV), (np.arange(self.nV), self.v_interior)),
                             shape=(self.nV, self.nq2))

    def Rp(self):
        return sp.csr_matrix((np.ones(self.nP), (np.arange(self.nP), self.p_kept)),
                             shape=(self.nP, self.np2))

    # element -> global node maps
    def q2_elem_nodes(self):
        ey, ex = np.divmod(np.arange(self.N * self.N), self.N)
        loc = [(a, b) for b in range(3) for a in range(3)]        # l = 3b + a
        return np.stack([(2 * ey + b) * self.nq + (2 * ex + a) for a, b in loc], axis=1)

    def q1_elem_nodes(self):
        ey, ex = np.divmod(np.arange(self.N * self.N), self.N)
        loc = [(a, b) for b in range(2) for a in range(2)]        # l = 2b + a
        return np.stack([(ey + b) * self.np1 + (ex + a) for a, b in loc], axis=1)


def _tabulate(h):
    """Basis values/gradients at the 9 Gauss points of one h x h element."""
    v2, d2 = p2_basis(GAUSS_X)
    v1, d1 = p1_basis(GAUSS_X)
    qa = [(qx, qy) for qy in range(3) for qx in range(3)]         # q = 3qy + qx
    wq = np.array([GAUSS_W[qx] * GAUSS_W[qy] for qx, qy in qa]) * h * h
    PHI = np.array([[v2[a, qx] * v2[b, qy] for qx, qy in qa] for b in range(3) for a in range(3)])
    DX = np.array([[d2[a, qx] / h * v2[b, qy] for qx, qy in qa] for b in range(3) for a in range(3)])
    DY = np.array([[v2[a, qx] * d2[b, qy] / h for qx, qy in qa] for b in range(3) for a in range(3)])
    PSI = np.array([[v1[a, qx] * v1[b, qy] for qx, qy in qa] for b in range(2) for a in range(2)])
    PDX = np.array([[d1[a, qx] / h * v1[b, qy] for qx, qy in qa] for b in range(2) for a in range(2)])
    PDY = np.array([[v1[a, qx] * d1[b, qy] / h for qx, qy in qa] for b in range(2) for a in range(2)])
    return wq, PHI, DX, DY, PSI, PDX, PDY


def _assemble(rows_map, cols_map, elem_mats, shape):
    """Scatter-add element matrices elem_mats[e, i, j] into a global CSR matrix."""
    ne, ni = rows_map.shape
    nj = cols_map.shape[1]
    R = np.repeat(rows_map[:, :, None], nj, axis=2)
    C = np.repeat(cols_map[:, None, :], ni, axis=1)
    em = np.broadcast_to(elem_mats, (ne, ni, nj))
    return sp.coo_matrix((em.ravel(), (R.ravel(), C.ravel())), shape=shape).tocsr()


def assemble_full(N: int, wind=None, side: float = 1.0):
    """Element-by-element assembly on the full (unconstrained) node sets.

    Returns a dict with Q2 scalar matrices ``M2, K2`` (and ``N2`` if a wind is
    given), Q1 matrices ``M1, K1`` (and ``N1``), and the negative-divergence
    blocks ``Bx, By`` of shape ((N+1)^2, (2N+1)^2):
        Bx[i, j] = - int psi_i d/dx phi_j ,   By[i, j] = - int psi_i d/dy phi_j.
    ``wind`` is a pair of Q2 nodal arrays (wx, wy) of length (2N+1)^2.
    Convection: N2[i, j] = int (w . grad phi_j) phi_i, N1 likewise with psi.
    ``side``: side length of the square (elements of side side / N).
    """
    g = Grid(N, side)
    wq, PHI, DX, DY, PSI, PDX, PDY = _tabulate(g.h)
    e2 = g.q2_elem_nodes()
    e1 = g.q1_elem_nodes()
    out = {}
    Me = np.einsum("q,iq,jq->ij", wq, PHI, PHI)
    Ke = np.einsum("q,iq,jq->ij", wq, DX, DX) + np.einsum("q,iq,jq->ij", wq, DY, DY)
    out["M2"] = _assemble(e2, e2, Me[None], (g.nq2, g.nq2))
    out["K2"] = _assemble(e2, e2, Ke[None], (g.nq2, g.nq2))
    Mpe = np.einsum("q,iq,jq->ij", wq, PSI, PSI)
    Kpe = np.einsum("q,iq,jq->ij", wq, PDX, PDX) + np.einsum("q,iq,jq->ij", wq, PDY, PDY)
    out["M1"] = _assemble(e1, e1, Mpe[None], (g.np2, g.np2))
    out["K1"] = _assemble(e1, e1, Kpe[None], (g.np2, g.np2))
    Bxe = -np.einsum("q,iq,jq->ij", wq, PSI, DX)
    Bye = -np.einsum("q,iq,jq->ij", wq, PSI, DY)
    out["Bx"] = _assemble(e1, e2, Bxe[None], (g.np2, g.nq2))
    out["By"] = _assemble(e1, e2, Bye[None], (g.np2, g.nq2))
    if wind is not None:
        wx = np.asarray(wind[0], float)[e2]            # (ne, 9) nodal wind per element
        wy = np.asarray(wind[1], float)[e2]
        wxq = wx @ PHI                                  # (ne, 9 quad points)
        wyq = wy @ PHI
        Ne = np.einsum("q,iq,eq,jq->eij", wq, PHI, wxq, DX) + np.einsum("q,iq,eq,jq->eij", wq, PHI, wyq, DY)
        out["N2"] = _assemble(e2, e2, Ne, (g.nq2, g.nq2))
        Npe = np.einsum("q,iq,eq,jq->eij", wq, PSI, wxq, PDX) + np.einsum("q,iq,eq,jq->eij", wq, PSI, wyq, PDY)
        out["N1"] = _assemble(e1, e1, Npe, (g.np2, g.np2))
    return out


class Operators:
    """The constrained spatial matrices of section 2.2 for one problem.

    Velocity unknowns are (v_x, v_y) on interior Q2 nodes (length n_v = 2 n_V);
    pressure unknowns are Q1 nodes except the pinned node (0,0) (length n_P).

    * ``Ms``  scalar Q2 mass,  ``Ks`` scalar Q2 stiffness, ``Ns`` scalar convection
    * ``M  = diag(Ms, Ms)``,  ``L = diag(Ls, Ls)`` with ``Ls = nu Ks + Ns``
    * ``B  = [Bx By]``  (negative divergence, n_P x n_v)
    * ``Mp, Kp, Np``, ``Lp = nu Kp + Np`` (pressure space, natural BCs, pinned)
    """

    def __init__(self, N: int, nu: float, wind=None, side: float = 1.0, origin=(0.0, 0.0)):
        self.grid = g = Grid(N, side, origin)
        self.nu = float(nu)
        full = assemble_full(N, wind, side)
        Rv, Rp = g.Rv(), g.Rp()
        r = lambda A, R1, R2: (R1 @ A @ R2.T).tocsr()
        self.Ms = r(full["M2"], Rv, Rv)
        self.Ks = r(full["K2"], Rv, Rv)
        self.Ns = r(full["N2"], Rv, Rv) if wind is not None else sp.csr_matrix((g.nV, g.nV))
        self.Mp = r(full["M1"], Rp, Rp)
        self.Kp = r(full["K1"], Rp, Rp)
        self.Np = r(full["N1"], Rp, Rp) if wind is not None else sp.csr_matrix((g.nP, g.nP))
        self.Bx = r(full["Bx"], Rp, Rv)
        self.By = r(full["By"], Rp, Rv)
        self.Ls = (self.nu * self.Ks + self.Ns).tocsr()
        self.Lp = (self.nu * self.Kp + self.Np).tocsr()
        self.M = sp.block_diag([self.Ms, self.Ms]).tocsr()
        self.L = sp.block_diag([self.Ls, self.Ls]).tocsr()
        self.B = sp.hstack([self.Bx, self.By]).tocsr()
        self.full = full


# ---------------------------------------------------------------------------
# Independent route: exact 1-D integrals of polynomials and Kronecker products.
# Used only to pin the element-by-element assembly above.
# ---------------------------------------------------------------------------

def _element_polys_1d(h, kind):
    """Lagrange basis polynomials of one element [0, h] (physical coordinate)."""
    if kind == 2:
        nodes = [0.0, h / 2, h]
    else:
        nodes = [0.0, h]
    polys = []
    for i, xi in enumerate(nodes):
        p = Poly([1.0])
        for j, xj in enumerate(nodes):
            if j != i:
                p = p * Poly([-xj, 1.0]) / (xi - xj)
        polys.append(p)
    return polys


def _integral(p: Poly, a: float, b: float) -> float:
    P = p.integ()
    return P(b) - P(a)


def kron_1d(N: int, f_weight=None):
    """Global 1-D matrices on [0,1] with N elements, exact polynomial integration.

    Returns Q2-Q2 mass ``m2``, stiffness ``k2``, Q1-Q1 ``m1, k1``, mixed Q1-Q2
    ``mix`` (int psi_i phi_j) and ``gmix`` (int psi_i phi_j').  If ``f_weight``
    (a Polynomial in x on [0,1]) is given, also ``cw`` with
    cw[i, j] = int f phi_j' phi_i and ``mw`` with mw[i, j] = int f phi_j phi_i
    (Q2-Q2), and their Q1 versions ``cw1``, ``mw1``.
    """
    h = 1.0 / N
    n2, n1 = 2 * N + 1, N + 1
    P2 = _element_polys_1d(h, 2)
    P1 = _element_polys_1d(h, 1)
    m2 = np.zeros((n2, n2)); k2 = np.zeros((n2, n2))
    m1 = np.zeros((n1, n1)); k1 = np.zeros((n1, n1))
    mix = np.zeros((n1, n2)); gmix = np.zeros((n1, n2))
    cw = np.zeros((n2, n2)); mw = np.zeros((n2, n2))
    cw1 = np.zeros((n1, n1)); mw1 = np.zeros((n1, n1))
    for e in range(N):
        x0 = e * h
        # integrate in the element-local coordinate s = x - x0 (no cancellation)
        q2, q1 = P2, P1
        a, b = 0.0, h
        fw = None if f_weight is None else f_weight(Poly([x0, 1.0]))
        for i in range(3):
            for j in range(3):
                I, J = 2 * e + i, 2 * e + j
                m2[I, J] += _integral(q2[i] * q2[j], a, b)
                k2[I, J] += _integral(q2[i].deriv() * q2[j].deriv(), a, b)
                if f_weight is not None:
                    cw[I, J] += _integral(fw * q2[j].deriv() * q2[i], a, b)
                    mw[I, J] += _integral(fw * q2[j] * q2[i], a, b)
        for i in range(2):
            for j in range(2):
                I, J = e + i, e + j
                m1[I, J] += _integral(q1[i] * q1[j], a, b)
                k1[I, J] += _integral(q1[i].deriv() * q1[j].deriv(), a, b)
                if f_weight is not None:
                    cw1[I, J] += _integral(fw * q1[j].deriv() * q1[i], a, b)
                    mw1[I, J] += _integral(fw * q1[j] * q1[i], a, b)
            for j in range(3):
                I, J = e + i, 2 * e + j
                mix[I, J] += _integral(q1[i] * q2[j], a, b)
                gmix[I, J] += _integral(q1[i] * q2[j].deriv(), a, b)
    out = dict(m2=m2, k2=k2, m1=m1, k1=k1, mix=mix, gmix=gmix)
    if f_weight is not None:
        out.update(cw=cw, mw=mw, cw1=cw1, mw1=mw1)
    return out
