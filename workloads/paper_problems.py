"""Data of the paper's own test problems (section 5), sampled at the nodes.

Input generation only: the analytic fields of section 5.1 (Stokes, with a
known exact solution of the optimality system) and section 5.2 (Oseen,
lid-driven cavity) evaluated at the Q2 / Q1 nodes of an N x N grid of the
square [-1, 1]^2 at the backward-Euler time levels t_k = k tau.  Nothing
here discretises or solves anything; the oracle and the library both take
these arrays as inputs (forcing f, Dirichlet data h, initial velocity v_0,
desired state v_d and, for the cavity, the wind).

Array shapes (x component first, grids row-major with x fastest):
  vd, f        (nt, 2, (2N+1)^2)     at t_1 .. t_nt
  h            (nt + 1, 2, (2N+1)^2) at t_0 .. t_nt (boundary values matter)
  v0           (2, (2N+1)^2)
  wind         (2, (2N+1)^2)
"""
from __future__ import annotations

import dataclasses

import numpy as np

DOMAIN = (-1.0, -1.0, 1.0, 1.0)


@dataclasses.dataclass
class PaperProblem:
    name: str
    flow: int          # 0 Stokes, 1 Oseen
    N: int
    nt: int
    T: float
    nu: float
    beta: float
    domain: tuple
    vd: np.ndarray
    f: np.ndarray
    h: np.ndarray
    v0: np.ndarray
    wind: np.ndarray | None = None
    exact: dict | None = None       # analytic state/adjoint at the nodes, when known


def q2_nodes(N: int, domain=DOMAIN):
    x0, y0, x1, _ = domain
    nq = 2 * N + 1
    iy, ix = np.divmod(np.arange(nq * nq), nq)
    hh = (x1 - x0) / (2 * N)
    return x0 + ix * hh, y0 + iy * hh


def q1_nodes(N: int, domain=DOMAIN):
    x0, y0, x1, _ = domain
    np1 = N + 1
    iy, ix = np.divmod(np.arange(np1 * np1), np1)
    hh = (x1 - x0) / N
    return x0 + ix * hh, y0 + iy * hh


def stokes_exact_fields(x, y, t, T: float = 1.0, beta: float = 1e-2) -> dict:
    """Section 5.1 at points (x, y) (arrays of one shape) and a time t:
    the printed desired state v_d and forcing f, the printed state
    v = e^{T-t} (20 x y^3, 5 x^4 - 5 y^4) and pressure
    p = e^{T-t} (60 x^2 y - 20 y^3), and the adjoint pair they imply (nu = 1):
    substituting v, p into the state equation leaves
    lambda / beta = (e^{T-t} - 1) psi with the divergence-free
    psi = (2 y (x^2-1)^2 (y^2-1), -2 x (x^2-1) (y^2-1)^2); the adjoint
    equation then holds with mu = 4 beta e^{T-t} x y.  Vector fields have a
    leading axis of length 2 (x component first)."""
    x, y = np.asarray(x, float), np.asarray(y, float)
    e = np.exp(T - t)
    v = e * np.stack([20 * x * y ** 3, 5 * x ** 4 - 5 * y ** 4])
    p = e * (60 * x ** 2 * y - 20 * y ** 3)
    psi = np.stack([2 * y * (x ** 2 - 1) ** 2 * (y ** 2 - 1), -2 * x * (x ** 2 - 1) * (y ** 2 - 1) ** 2])
    lam = beta * (e - 1.0) * psi
    mu = 4 * beta * e * x * y
    c = 4 * beta * np.stack([y * (2 * (3 * x ** 2 - 1) * (y ** 2 - 1) + 3 * (x ** 2 - 1) ** 2),
                             -x * (3 * (y ** 2 - 1) ** 2 + 2 * (x ** 2 - 1) * (3 * y ** 2 - 1))])
    g = np.stack([20 * x * y ** 3 + 2 * beta * y * ((x ** 2 - 1) ** 2 * (y ** 2 - 7)
                                                    - 4 * (3 * x ** 2 - 1) * (y ** 2 - 1) + 2),
                  5 * (x ** 4 - y ** 4) - 2 * beta * x * ((y ** 2 - 1) ** 2 * (x ** 2 - 7)
                                                          - 4 * (x ** 2 - 1) * (3 * y ** 2 - 1) - 2)])
    fa = np.stack([-20 * x * y ** 3 - 2 * y * (x ** 2 - 1) ** 2 * (y ** 2 - 1),
                   5 * (y ** 4 - x ** 4) + 2 * x * (x ** 2 - 1) * (y ** 2 - 1) ** 2])
    fb = np.stack([2 * y * (x ** 2 - 1) ** 2 * (y ** 2 - 1), -2 * x * (x ** 2 - 1) * (y ** 2 - 1) ** 2])
    return {"v": v, "p": p, "lambda": lam, "mu": mu, "vd": c + e * g, "f": e * fa + fb}


def stokes_exact(N: int, nt: int, T: float = 1.0, beta: float = 1e-2) -> PaperProblem:
    """Section 5.1 on the nodes (nu = 1; initial and boundary values are those
    of the known state v); ``exact`` carries v, p, lambda and mu at the nodes
    for t_0 .. t_nt (see ``stokes_exact_fields``)."""
    x, y = q2_nodes(N)
    xp, yp = q1_nodes(N)
    tk = np.arange(nt + 1) * (T / nt)
    F = [stokes_exact_fields(x, y, t, T, beta) for t in tk]
    Fp = [stokes_exact_fields(xp, yp, t, T, beta) for t in tk]
    v = np.stack([F[k]["v"] for k in range(nt + 1)])
    vd = np.stack([F[k]["vd"] for k in range(1, nt + 1)])
    f = np.stack([F[k]["f"] for k in range(1, nt + 1)])
    exact = {"v": v, "lambda": np.stack([F[k]["lambda"] for k in range(nt + 1)]),
             "p": np.stack([Fp[k]["p"] for k in range(nt + 1)]), "mu": np.stack([Fp[k]["mu"] for k in range(nt + 1)])}
    return PaperProblem("stokes_exact", 0, N, nt, T, 1.0, beta, DOMAIN, vd, f, v.copy(), v[0].copy(), exact=exact)


def cavity_wind(N: int) -> np.ndarray:
    """Section 5.2's two-vortex wind at the Q2 nodes.  Reading: the first
    vortex c1 ((100/99)^2 y, -(100/49)^2 (x - 1/2)) as printed; in the second
    the printed x component (-100/99)^2 y is read as -(100/99)^2 y, the sign
    that makes it divergence-free like the first (as printed its divergence
    is nonzero wherever x y != 0 inside its support)."""
    x, y = q2_nodes(N)
    a, b = (100.0 / 49.0), (100.0 / 99.0)
    c1 = 1.0 - np.sqrt((a * (x - 0.5)) ** 2 + (b * y) ** 2)
    c2 = 1.0 - np.sqrt((a * (x + 0.5)) ** 2 + (b * y) ** 2)
    wx = np.where(c1 >= 0, c1 * b * b * y, 0.0) + np.where(c2 >= 0, -c2 * b * b * y, 0.0)
    wy = np.where(c1 >= 0, -c1 * a * a * (x - 0.5), 0.0) + np.where(c2 >= 0, c2 * a * a * (x + 0.5), 0.0)
    return np.stack([wx, wy])


def cavity(N: int, nt: int, T: float = 1.0, beta: float = 1e-2, nu: float = 1e-2) -> PaperProblem:
    """Section 5.2: lid-driven cavity Oseen problem (time-independent v_d and
    f, the lid h = (1, 0) on the top edge y = 1, v_0 = (1, 0) in the wedge
    -y < x < y, the two-vortex wind of ``cavity_wind``); nu = 1e-2 as in every
    experiment of section 5."""
    x, y = q2_nodes(N)
    q = (1 - x ** 4) * (1 - y ** 4)
    vd1 = np.stack([2 * y * q, -2 * x * q]) + np.stack([np.where(y >= 0.8, 5 * y - 4, 0.0), np.zeros_like(x)])
    f1 = np.stack([-20 * x * y ** 3 - 2 * y * (x ** 2 - 1) ** 2 * (y ** 2 - 1),
                   5 * (y ** 4 - x ** 4) + 2 * x * (x ** 2 - 1) * (y ** 2 - 1) ** 2])
    v0 = np.stack([np.where((x > -y) & (x < y), 1.0, 0.0), np.zeros_like(x)])
    lid = np.stack([np.where(np.isclose(y, 1.0), 1.0, 0.0), np.zeros_like(x)])
    vd = np.broadcast_to(vd1, (nt, 2, x.size)).copy()
    f = np.broadcast_to(f1, (nt, 2, x.size)).copy()
    h = np.broadcast_to(lid, (nt + 1, 2, x.size)).copy()
    return PaperProblem("cavity", 1, N, nt, T, nu, beta, DOMAIN, vd, f, h, v0, wind=cavity_wind(N))
