"""Krylov solvers: right-preconditioned GMRES and flexible GMRES.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

GMRES (Saad & Schultz) solves the per-frequency blocks in the nonlinear
preconditioners (Algorithm 2 and its Oseen analogue); flexible GMRES (Saad)
is the outer iteration, since a preconditioner that contains an inner Krylov
solve changes from one application to the next (section 3.4).  Both use
modified Gram-Schmidt Arnoldi with Givens rotations, work for complex data
with the Hermitian inner product, and start from x_0 = 0 unless told
otherwise.
"""
from __future__ import annotations

import numpy as np


def _givens(a, b):
    """Rotation (c, s) with [c, s; -conj(s), c] [a; b] = [r; 0], c real."""
    if b == 0:
        return 1.0, 0.0
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    t = np.hypot(abs(a), abs(b))
    c = abs(a) / t
    s = (a / abs(a)) * np.conj(b) / t
    return c, s


def _arnoldi_cycle(matvec, precond, r0, beta0, m, stop_abs, flexible):
    """One restart cycle.  Returns (update, its, residual estimate, breakdown)."""
    n = r0.shape[0]
    dt = np.result_type(r0, complex) if np.iscomplexobj(r0) else float
    V = np.zeros((m + 1, n), dtype=dt)
    Z = np.zeros((m, n), dtype=dt) if flexible else None
    H = np.zeros((m + 1, m), dtype=dt)
    cs = np.zeros(m); sn = np.zeros(m, dtype=dt)
    g = np.zeros(m + 1, dtype=dt)
    g[0] = beta0
    V[0] = r0 / beta0
    k = 0
    for k in range(m):
        z = precond(V[k])
        if flexible:
            Z[k] = z
        w = matvec(z)
        for i in range(k + 1):                          # modified Gram-Schmidt
            H[i, k] = np.vdot(V[i], w)
            w = w - H[i, k] * V[i]
        H[k + 1, k] = np.linalg.norm(w)
        breakdown = H[k + 1, k] == 0
        if not breakdown:
            V[k + 1] = w / H[k + 1, k]
        for i in range(k):                              # apply earlier rotations
            hi, hj = H[i, k], H[i + 1, k]
            H[i, k] = cs[i] * hi + sn[i] * hj
            H[i + 1, k] = -np.conj(sn[i]) * hi + cs[i] * hj
        cs[k], sn[k] = _givens(H[k, k], H[k + 1, k])
        H[k, k] = cs[k] * H[k, k] + sn[k] * H[k + 1, k]
        H[k + 1, k] = 0.0
        g[k + 1] = -np.conj(sn[k]) * g[k]
        g[k] = cs[k] * g[k]
        if abs(g[k + 1]) <= stop_abs or breakdown:
            k += 1
            break
    else:
        k = m
    y = np.linalg.solve(np.triu(H[:k, :k]), g[:k]) if k > 0 else np.zeros(0)
    basis = Z[:k] if flexible else V[:k]
    upd = y @ basis
    if not flexible:
        upd = precond(upd)
    return upd, k, abs(g[k]), breakdown


def gmres(matvec, precond, b, tol, restart=50, maxit=200, x0=None):
    """Right-preconditioned restarted GMRES; stops when the Arnoldi residual
    estimate satisfies ||r_k|| <= tol ||b||.  Returns (x, iterations, history)."""
    precond = precond or (lambda v: v)
    x = np.zeros_like(b) if x0 is None else x0.astype(np.result_type(b, x0))
    bnorm = np.linalg.norm(b)
    if bnorm == 0:
        return x, 0, [0.0]
    hist, its = [], 0
    r = b - matvec(x) if x0 is not None else b.copy()
    while its < maxit:
        beta0 = np.linalg.norm(r)
        hist.append(beta0 / bnorm)
        if beta0 <= tol * bnorm:
            break
        m = min(restart, maxit - its)
        upd, k, est, brk = _arnoldi_cycle(matvec, precond, r, beta0, m, tol * bnorm, False)
        x = x + upd
        its += k
        r = b - matvec(x)
        if est <= tol * bnorm or brk:
            hist.append(np.linalg.norm(r) / bnorm)
            break
    return x, its, hist


def fgmres(matvec, precond, b, tol, restart=10, maxit=200, x0=None):
    """Restarted flexible GMRES.  The cycle stops on the Arnoldi estimate; the
    outer loop stops on the true residual ||b - A x|| <= tol ||b||.
    Returns (x, iterations, history of true relative residuals)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0:
        return x, 0, [0.0]
    r = b - matvec(x) if x0 is not None else b.copy()
    hist, its = [np.linalg.norm(r) / bnorm], 0
    while its < maxit and hist[-1] > tol:
        beta0 = np.linalg.norm(r)
        m = min(restart, maxit - its)
        upd, k, est, brk = _arnoldi_cycle(matvec, precond, r, beta0, m, tol * bnorm, True)
        x = x + upd
        its += k
        r = b - matvec(x)
        hist.append(np.linalg.norm(r) / bnorm)
        if brk and hist[-1] > tol:
            break
    return x, its, hist
