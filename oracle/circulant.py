"""Circulant perturbation of the all-at-once matrix and its FFT diagonalisation.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section 3.1: replacing the backward-Euler matrix E by the circulant C (first
column c_1 = (1, -1, 0, ..., 0)^T) gives P_C, which the block Fourier transform
in time diagonalises: C = F^{-1} D F with D = diag(F c_1).  With the forward
DFT F[j, t] = exp(-2 pi i j t / nt) (unnormalised; inverse carries 1/nt) the
diagonal is d_j = 1 - exp(-2 pi i j / nt), and C^T = F^{-1} conj(D) F.

After the transform, P_C is block diagonal with the blocks of eq. (SubBlockG),
written in the unknown order (v, lambda, p, mu) and the row order
(adjoint momentum, state momentum, adjoint divergence, state divergence):

    G_j = [[tau M,          conj(d_j) M + tau L^T, 0,       tau B^T],
           [d_j M + tau L,  -tau/beta M,           tau B^T, 0      ],
           [0,              tau B,                 0,       0      ],
           [tau B,          0,                     0,       0      ]]

Mapping from the transformed residual r_hat[b][j] (b = 0: adjoint rows,
b = 1: state rows; each split into velocity and pressure parts):
r1 = r_hat[0] velocity, r2 = r_hat[1] velocity, r3 = r_hat[0] pressure,
r4 = r_hat[1] pressure; and back: y1 -> v, y2 -> lambda, y3 -> p, y4 -> mu.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def d_closed_form(nt: int) -> np.ndarray:
    """Eigenvalues of the circulant C: d_j = 1 - exp(-2 pi i j / nt)."""
    j = np.arange(nt)
    return 1.0 - np.exp(-2j * np.pi * j / nt)


def circulant_C(nt: int) -> sp.csr_matrix:
    """C: E with the extra -1 in the top-right corner (section 3.1)."""
    C = sp.lil_matrix((nt, nt))
    for k in range(nt):
        C[k, k] = 1.0
        C[k, k - 1] = -1.0            # k = 0 wraps to the corner entry
    return C.tocsr()


def time_fft(P, x: np.ndarray) -> np.ndarray:
    """Forward block Fourier transform: (2, nt, n) real -> (2, nt, n) complex."""
    X = np.asarray(x).reshape(2, P.nt, P.n)
    return np.fft.fft(X, axis=1)


def time_ifft(P, Xh: np.ndarray) -> np.ndarray:
    return np.fft.ifft(Xh, axis=1)


def split_freq(P, Xh_j):
    """(2, n) transformed block at one frequency -> (r1, r2, r3, r4)."""
    nv = P.nv
    return Xh_j[0, :nv], Xh_j[1, :nv], Xh_j[0, nv:], Xh_j[1, nv:]


def join_freq(P, y1, y2, y3, y4):
    nv = P.nv
    out = np.empty((2, P.n), dtype=complex)
    out[0, :nv], out[1, :nv], out[0, nv:], out[1, nv:] = y1, y2, y3, y4
    return out


def G_block(P, d: complex) -> sp.csr_matrix:
    """G_j of eq. (SubBlockG) in the (v, lambda, p, mu) ordering."""
    o, tau, beta = P.ops, P.tau, P.beta
    M, L, B = o.M.astype(complex), o.L.astype(complex), o.B.astype(complex)
    return sp.bmat([
        [tau * M, np.conj(d) * M + tau * L.T, None, tau * B.T],
        [d * M + tau * L, -(tau / beta) * M, tau * B.T, None],
        [None, tau * B, sp.csr_matrix((P.nP, P.nP)), None],
        [tau * B, None, None, sp.csr_matrix((P.nP, P.nP))],
    ], format="csc")


def pc_apply_fft(P, r: np.ndarray) -> np.ndarray:
    """P_C^{-1} r through the FFT route: one sparse LU per frequency."""
    Rh = time_fft(P, r)
    d = d_closed_form(P.nt)
    Yh = np.empty_like(Rh)
    for j in range(P.nt):
        r1, r2, r3, r4 = split_freq(P, Rh[:, j, :])
        rhs = np.concatenate([r1, r2, r3, r4])
        y = spla.splu(G_block(P, d[j])).solve(rhs)
        nv, nP = P.nv, P.nP
        Yh[:, j, :] = join_freq(P, y[:nv], y[nv:2 * nv], y[2 * nv:2 * nv + nP], y[2 * nv + nP:])
    return time_ifft(P, Yh).real.reshape(-1)


def pc_apply_direct(P, r: np.ndarray) -> np.ndarray:
    """P_C^{-1} r by a sparse LU of the assembled P_C (E replaced by C)."""
    A = P.kkt_matrix(time_matrix=circulant_C(P.nt)).tocsc()
    return spla.splu(A).solve(np.asarray(r, float))


def freq_domain_apply(P, Xh: np.ndarray) -> np.ndarray:
    """A^ X^ = (F A F^{-1}) X^ for a transformed vector X^ of shape (2, nt, n)
    (all nt frequencies), written as Theorem 1's split A = P_C + U (section
    3.1): the diagonal blocks G_j of P_C act frequency by frequency, and the
    corner term U, which is all that E and C differ by (E - C has its one entry
    1 at row 0, column nt - 1), adds M v_{nt-1} to the state momentum rows of
    time step 0 and M lambda_0 to the adjoint momentum rows of step nt - 1
    (E^T - C^T).  In the Fourier basis those rows become all frequencies: the
    state rows of frequency j get M v_{nt-1} (the DFT of e_0 is all ones), the
    adjoint rows exp(2 pi i j / nt) M lambda_0 (the DFT of e_{nt-1}), where
    v_{nt-1} and lambda_0 are time samples of the inverse transform."""
    nt, nv = P.nt, P.nv
    d = d_closed_form(nt)
    Yh = np.empty_like(Xh, dtype=complex)
    for j in range(nt):
        x1, x2, x3, x4 = split_freq(P, Xh[:, j, :])
        y = G_block(P, d[j]) @ np.concatenate([x1, x2, x3, x4])
        Yh[:, j, :] = join_freq(P, y[:nv], y[nv:2 * nv], y[2 * nv:2 * nv + P.nP], y[2 * nv + P.nP:])
    x_t = np.fft.ifft(Xh, axis=1)                   # time samples
    v_last = x_t[0, nt - 1, :nv]                    # v at the last step
    lam_first = x_t[1, 0, :nv]                      # lambda at the first step
    Mv, Ml = P.ops.M @ v_last, P.ops.M @ lam_first
    ph = np.exp(2j * np.pi * np.arange(nt) / nt)
    Yh[1, :, :nv] += Mv[None, :]
    Yh[0, :, :nv] += ph[:, None] * Ml[None, :]
    return Yh
