"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws and samples data: problem parameters, the desired
velocity state, the Oseen wind and random test vectors in the library's
canonical layout.  It contains none of the solver's arithmetic, so the oracle
and the HIP path can both consume it without sharing method code.

Canonical all-at-once layout (real FP64), length 2*nt*(2*(2N+1)^2 + (N+1)^2):
``[b in {0,1}][t = 1..nt][v_x (2N+1)^2, v_y (2N+1)^2, p (N+1)^2]`` where block 0
holds (v, p) unknowns / adjoint-equation rows and block 1 holds (lambda, mu)
unknowns / state-equation rows.  Grids are row-major with x fastest.  Entries
on the Dirichlet boundary of the velocity grids and the pinned pressure node
(0,0) are zero.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

STOKES, OSEEN = 0, 1


@dataclasses.dataclass
class Workload:
    """One control problem: unit square, Q2-Q1 on N x N quads, backward Euler."""
    flow: int
    N: int
    nt: int
    T: float
    nu: float
    beta: float
    seed: int
    amplitude: float
    noise_sigma: float = 1e-3

    @property
    def tau(self) -> float:
        return self.T / self.nt

    @property
    def level_size(self) -> int:
        nq = 2 * self.N + 1
        return 2 * nq * nq + (self.N + 1) ** 2

    @property
    def n_all(self) -> int:
        return 2 * self.nt * self.level_size

    @property
    def name(self) -> str:
        f = "stokes" if self.flow == STOKES else "oseen"
        return f"{f}_N{self.N}_nt{self.nt}_beta{self.beta:g}_nu{self.nu:g}"


def config(idx: int, seed: int | None = None) -> Workload:
    """The three single-problem workloads.

    1: Stokes N=8, nt=16, T=1, nu=1, beta=1e-2, amplitude 1.
    2: Stokes N=128, nt=256, T=1, nu=1, beta=1e-4, amplitude ~ U[0.5, 2].
    3: Oseen N=128, nt=128, T=1, nu=1/100, beta=1e-4, amplitude ~ U[0.5, 2],
       wind w = (2y(1-x^2), -2x(1-y^2)).
    """
    seed = idx if seed is None else seed
    rng = np.random.default_rng(seed)
    if idx == 1:
        return Workload(STOKES, 8, 16, 1.0, 1.0, 1e-2, seed, 1.0)
    if idx == 2:
        return Workload(STOKES, 128, 256, 1.0, 1.0, 1e-4, seed, float(rng.uniform(0.5, 2.0)))
    if idx == 3:
        return Workload(OSEEN, 128, 128, 1.0, 0.01, 1e-4, seed, float(rng.uniform(0.5, 2.0)))
    raise ValueError(f"unknown config {idx}")


def batch_mix(count: int = 64, seed: int = 4) -> list:
    """The batched workload: ``count`` independent control problems.

    N ~ U{32, 64, 128}, nt ~ U{32, 64, 128, 256}, log10(beta) ~ U[-6, -2],
    nu ~ U{1, 1/50, 1/100}, Stokes or Oseen with probability 1/2 each (Oseen
    with the wind of ``wind_nodal``), T = 1, amplitude ~ U[0.5, 2].  Draw order
    from ``default_rng(seed)``: every problem parameter array, then the
    amplitudes; problem k's noise comes from its own stream (its Workload seed
    is 1000 * seed + k)."""
    rng = np.random.default_rng(seed)
    Ns = rng.choice([32, 64, 128], size=count)
    nts = rng.choice([32, 64, 128, 256], size=count)
    lbeta = rng.uniform(-6.0, -2.0, size=count)
    nus = rng.choice([1.0, 1.0 / 50.0, 1.0 / 100.0], size=count)
    flows = rng.integers(0, 2, size=count)
    amps = rng.uniform(0.5, 2.0, size=count)
    return [Workload(int(flows[k]), int(Ns[k]), int(nts[k]), 1.0, float(nus[k]), float(10.0 ** lbeta[k]),
                     1000 * seed + k, float(amps[k])) for k in range(count)]


def serve_stream(count: int = 256, seed: int = 5, max_N: int = 256) -> list:
    """The served workload: ``count`` requests with parameters drawn as in
    ``batch_mix`` except N ~ U{32, 64, 128, 256} (capped at ``max_N``).
    Returns (workload, unit-rate arrival time) pairs: the arrivals of a Poisson
    process of rate 1 (cumulative sums of Exp(1) gaps from
    ``default_rng((seed, 2))``); divide by a rate lambda for that rate."""
    rng = np.random.default_rng(seed)
    Ns = rng.choice([n for n in (32, 64, 128, 256) if n <= max_N], size=count)
    nts = rng.choice([32, 64, 128, 256], size=count)
    lbeta = rng.uniform(-6.0, -2.0, size=count)
    nus = rng.choice([1.0, 1.0 / 50.0, 1.0 / 100.0], size=count)
    flows = rng.integers(0, 2, size=count)
    amps = rng.uniform(0.5, 2.0, size=count)
    arrivals = np.cumsum(np.random.default_rng((seed, 2)).exponential(1.0, size=count))
    return [(Workload(int(flows[k]), int(Ns[k]), int(nts[k]), 1.0, float(nus[k]), float(10.0 ** lbeta[k]),
                      1000 * seed + k, float(amps[k])), float(arrivals[k])) for k in range(count)]


def small(flow: int, N: int, nt: int, beta: float = 1e-2, nu: float = 1.0,
          T: float = 1.0, seed: int = 0, amplitude: float = 1.0) -> Workload:
    """A small workload of the same family, for parity tests."""
    return Workload(flow, N, nt, T, nu, beta, seed, amplitude)


def q2_coords(N: int):
    nq = 2 * N + 1
    iy, ix = np.divmod(np.arange(nq * nq), nq)
    return ix / (2 * N), iy / (2 * N)


def wind_nodal(N: int):
    """Oseen wind w = (2y(1-x^2), -2x(1-y^2)) sampled at the Q2 nodes.

    Returns a (2, (2N+1)^2) float64 array (x component first)."""
    x, y = q2_coords(N)
    return np.stack([2 * y * (1 - x * x), -2 * x * (1 - y * y)])


def _boundary_mask_q2(N: int):
    nq = 2 * N + 1
    iy, ix = np.divmod(np.arange(nq * nq), nq)
    return (ix == 0) | (iy == 0) | (ix == nq - 1) | (iy == nq - 1)


def desired_state(w: Workload) -> np.ndarray:
    """v_d at t_k = k tau, k = 1..nt, on Q2 nodes: shape (nt, 2, (2N+1)^2).

    v_d(x, t) = a t s(x) + eta_k(x) with the divergence-free swirl
    s = (sin^2(pi x) sin(2 pi y), -sin(2 pi x) sin^2(pi y)) and i.i.d.
    N(0, sigma^2) nodal noise eta (sigma = 1e-3).  Boundary entries are zero.
    The noise comes from its own stream, ``default_rng((seed, 1))``, so it does
    not depend on how the problem parameters were drawn.
    """
    rng = np.random.default_rng((w.seed, 1))
    x, y = q2_coords(w.N)
    s = np.stack([np.sin(np.pi * x) ** 2 * np.sin(2 * np.pi * y),
                  -np.sin(2 * np.pi * x) * np.sin(np.pi * y) ** 2])
    nq2 = (2 * w.N + 1) ** 2
    noise = rng.normal(0.0, w.noise_sigma, size=(w.nt, 2, nq2))
    t = w.tau * np.arange(1, w.nt + 1)
    vd = w.amplitude * t[:, None, None] * s[None] + noise
    vd[:, :, _boundary_mask_q2(w.N)] = 0.0
    return vd


def canonical_mask(N: int, nt: int) -> np.ndarray:
    """Boolean mask of the free entries of a canonical vector."""
    nq2 = (2 * N + 1) ** 2
    bnd = _boundary_mask_q2(N)
    pmask = np.ones((N + 1) ** 2, bool)
    pmask[0] = False
    level = np.concatenate([~bnd, ~bnd, pmask])
    return np.tile(level, 2 * nt)


def random_canonical(N: int, nt: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Standard-normal entries on the free positions of a canonical vector."""
    rng = np.random.default_rng(seed)
    m = canonical_mask(N, nt)
    x = np.zeros(m.size)
    x[m] = scale * rng.standard_normal(int(m.sum()))
    return x


def single_frequency_canonical(N: int, nt: int, j: int, seed: int) -> np.ndarray:
    """A canonical vector whose time dependence is one Fourier mode j:
    r(t) = a cos(2 pi j t / nt) + b sin(2 pi j t / nt), t = 0..nt-1, with
    random spatial fields a, b on the free positions."""
    rng = np.random.default_rng(seed)
    m = canonical_mask(N, nt).reshape(2, nt, -1)[:, 0, :]
    a = np.where(m, rng.standard_normal(m.shape), 0.0)
    b = np.where(m, rng.standard_normal(m.shape), 0.0)
    t = np.arange(nt)
    c = np.cos(2 * math.pi * j * t / nt)
    s = np.sin(2 * math.pi * j * t / nt)
    x = a[:, None, :] * c[None, :, None] + b[:, None, :] * s[None, :, None]
    return x.reshape(-1)
