"""Pins of the oracle's finite-element assembly (section 2.2) against closed
forms, invariants and an independent Kronecker-product assembly."""
import os

import numpy as np
import pytest
import scipy.sparse as sp
from numpy.polynomial import Polynomial as Poly

import workloads as W
from oracle.fem import Grid, Operators, assemble_full, kron_1d
from oracle.smoothers import Q1_MASS_BOUNDS, Q2_MASS_BOUNDS

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden_element():
    out = {}
    for line in open(os.path.join(GOLD, "p2_element.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, *vals = line.split()
        v = np.array([float(x) for x in vals])
        n = int(round(np.sqrt(v.size)))
        out[name] = v.reshape(n, n)
    return out


@pytest.mark.parametrize("N", [1, 2])
def test_element_matrices_closed_form(N):
    """On one element the assembled 1-D tensor factors are the textbook ones."""
    g = _golden_element()
    k = kron_1d(1)
    assert np.allclose(k["m2"], g["mass2"] / 30, atol=1e-15)
    assert np.allclose(k["k2"], g["stiff2"] / 3, atol=1e-14)
    assert np.allclose(k["m1"], g["mass1"] / 6, atol=1e-15)
    assert np.allclose(k["k1"], g["stiff1"], atol=1e-15)
    # 2-D element: tensor products of the 1-D ones
    full = assemble_full(1)
    m2, k2 = g["mass2"] / 30, g["stiff2"] / 3
    assert np.allclose(full["M2"].toarray(), np.kron(m2, m2), atol=1e-15)
    assert np.allclose(full["K2"].toarray(), np.kron(k2, m2) + np.kron(m2, k2), atol=1e-14)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_elementwise_equals_kronecker(N):
    """P1: 3x3-Gauss element assembly equals exact 1-D integrals combined by
    Kronecker products (x fastest, so 2-D = kron(y-factor, x-factor))."""
    full = assemble_full(N)
    k = kron_1d(N)
    kr = lambda a, b: np.kron(a, b)
    assert np.allclose(full["M2"].toarray(), kr(k["m2"], k["m2"]), atol=1e-15)
    assert np.allclose(full["K2"].toarray(), kr(k["k2"], k["m2"]) + kr(k["m2"], k["k2"]), atol=1e-13)
    assert np.allclose(full["M1"].toarray(), kr(k["m1"], k["m1"]), atol=1e-15)
    assert np.allclose(full["K1"].toarray(), kr(k["k1"], k["m1"]) + kr(k["m1"], k["k1"]), atol=1e-13)
    # B_x = -int psi d/dx phi = -(mix_y (x) gmix_x); B_y = -(gmix_y (x) mix_x)
    assert np.allclose(full["Bx"].toarray(), -kr(k["mix"], k["gmix"]), atol=1e-14)
    assert np.allclose(full["By"].toarray(), -kr(k["gmix"], k["mix"]), atol=1e-14)


@pytest.mark.parametrize("N", [2, 4])
def test_convection_separable_wind(N):
    """P1 for N(w): the Oseen wind (2y(1-x^2), -2x(1-y^2)) is a sum of
    separable terms, so N(w) is a sum of Kronecker products of exact 1-D
    integrals: int w_x d/dx phi_j phi_i = [int y phi phi]_y (x) [int 2(1-x^2) phi' phi]_x."""
    wind = W.wind_nodal(N)
    full = assemble_full(N, wind)
    fx = kron_1d(N, Poly([2.0, 0.0, -2.0]))          # 2(1 - x^2)
    fy = kron_1d(N, Poly([0.0, 1.0]))                # y
    gx = kron_1d(N, Poly([0.0, -2.0]))               # -2x
    gy = kron_1d(N, Poly([1.0, 0.0, -1.0]))          # 1 - y^2
    # x-term: w_x = (2(1-x^2)) * y ; y-term: w_y = (-2x) * (1-y^2)
    Nx = np.kron(fy["mw"], fx["cw"])
    Ny = np.kron(gy["cw"], gx["mw"])
    assert np.allclose(full["N2"].toarray(), Nx + Ny, atol=1e-13)
    Nx1 = np.kron(fy["mw1"], fx["cw1"])
    Ny1 = np.kron(gy["cw1"], gx["mw1"])
    assert np.allclose(full["N1"].toarray(), Nx1 + Ny1, atol=1e-13)


@pytest.mark.parametrize("N", [2, 5])
def test_invariants(N):
    """P2: total mass = area, stiffness kills constants, B of the interpolant
    of v = (x, 0) equals -M_p 1, constants are in ker B^T on interior
    velocity columns, N is skew on interior nodes for a solenoidal wind."""
    g = Grid(N)
    full = assemble_full(N, W.wind_nodal(N))
    one2, one1 = np.ones(g.nq2), np.ones(g.np2)
    assert abs(full["M2"].sum() - 1.0) < 1e-13
    assert abs(full["M1"].sum() - 1.0) < 1e-13
    assert np.abs(full["K2"] @ one2).max() < 1e-12
    assert np.abs(full["K1"] @ one1).max() < 1e-12
    x, _ = g.q2_xy()
    assert np.allclose(full["Bx"] @ x, -(full["M1"] @ one1), atol=1e-14)
    ops = Operators(N, 1.0, W.wind_nodal(N))
    assert np.abs(g.Rv() @ (full["Bx"].T @ one1)).max() < 1e-13
    assert np.abs(g.Rv() @ (full["By"].T @ one1)).max() < 1e-13
    assert np.abs((ops.Ns + ops.Ns.T).toarray()).max() < 1e-13


def test_mass_jacobi_bounds():
    """The Chebyshev intervals: spectrum of diag(M)^{-1} M inside
    [1/4, 25/16] (Q2) and [1/4, 9/4] (Q1), constrained and unconstrained."""
    for N in (2, 4, 6):
        o = Operators(N, 1.0)
        for A, (lo, hi) in ((o.Ms, Q2_MASS_BOUNDS), (o.Mp, Q1_MASS_BOUNDS),
                            (o.full["M2"], Q2_MASS_BOUNDS), (o.full["M1"], Q1_MASS_BOUNDS)):
            A = A.toarray()
            d = np.diag(A)
            ev = np.linalg.eigvalsh(A / np.sqrt(np.outer(d, d)))
            assert ev.min() >= lo - 1e-12 and ev.max() <= hi + 1e-12


def test_dof_counts_match_tables():
    """P17: the #DOFs columns of Tables 1-5 equal 2 n_t (2(2N+1)^2 + (N+1)^2)."""
    for line in open(os.path.join(GOLD, "dof_counts.txt")):
        if line.startswith("#") or not line.strip():
            continue
        N, nt, val = line.split()
        N, nt, val = int(N), int(nt), float(val)
        w = W.Workload(0, N, nt, 1.0, 1.0, 1.0, 0, 1.0)
        assert float(f"{w.n_all:.2e}") == val


def test_restriction_sizes():
    g = Grid(4)
    assert g.nV == 49 and g.nP == 24 and g.nv == 98
    assert sp.issparse(g.Rv()) and g.Rv().shape == (49, 81)
