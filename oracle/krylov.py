"""Krylov solvers: right-preconditioned GMRES, flexible GMRES and
preconditioned MINRES.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

GMRES (Saad & Schultz) solves the per-frequency blocks in the nonlinear
preconditioners (Algorithm 2 and its Oseen analogue); flexible GMRES (Saad)
is the outer iteration, since a preconditioner that contains an inner Krylov
solve changes from one application to the next (section 3.4).  Both use
modified Gram-Schmidt Arnoldi with Givens rotations, work for complex data
with the Hermitian inner product, and start from x_0 = 0 unless told
otherwise.  MINRES (Paige & Saunders) applies to the symmetric Stokes system
with the symmetric positive definite linear preconditioner of section 3.3,
and to the real symmetric Stokes blocks Z_j with P~_j (section 3.2) as an
inner solver.
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


def minres(matvec, precond, b, tol, maxit=500, x0=None, check_every=0):
    """Preconditioned MINRES (Paige & Saunders) for a Hermitian matrix and a
    Hermitian positive definite preconditioner ``precond`` ~ A^{-1} (real
    symmetric data, or complex vectors with a real symmetric matrix such as
    the Stokes blocks Z_j of section 3.2): the Lanczos coefficients are real,
    inner products take the conjugate of their first argument.

    Lanczos in the inner product of the preconditioner: v_j are the Lanczos
    vectors, z_j = precond(v_j) / gamma_j with gamma_j^2 = <z_j, v_j>; the
    tridiagonal T_j (diagonal delta_j, off-diagonal gamma_j) is reduced by
    Givens rotations and the iterate is advanced along the search directions
    w_j.  |eta_j| equals the residual norm ||r_j||_{precond} of the j-th
    iterate, which minimises it over the preconditioned Krylov space.

    check_every = 0: stop when |eta_j| <= tol gamma_1.  check_every = c > 0:
    stop on the true residual ||b - A x_j||_2 <= tol ||b||_2, tested every c
    steps once |eta_j| <= 100 tol gamma_1 and at every step where
    |eta_j| <= tol gamma_1.  Returns (x, iterations, history of
    |eta_j| / gamma_1, converged on the true residual (check_every > 0))."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    v = b - matvec(x) if x0 is not None else b.copy()
    bnorm = np.linalg.norm(b)
    z = precond(v)
    g = np.sqrt(max(float(np.vdot(v, z).real), 0.0))
    if g == 0.0:
        return x, 0, [0.0], True
    g1, eta = g, g
    v_old = np.zeros_like(b)
    w_old = np.zeros_like(b)
    w = np.zeros_like(b)
    g_old = 1.0
    c_old, c, s_old, s = 1.0, 1.0, 0.0, 0.0
    hist, its, done = [1.0], 0, False
    while its < maxit:
        z = z / g
        Az = matvec(z)
        delta = float(np.vdot(z, Az).real)
        v_new = Az - (delta / g) * v - (g / g_old) * v_old
        z_new = precond(v_new)
        g2 = float(np.vdot(v_new, z_new).real)
        g_new = np.sqrt(max(g2, 0.0))
        a0 = c * delta - c_old * s * g
        a1 = np.hypot(a0, g_new)
        a2 = s * delta + c_old * c * g
        a3 = s_old * g
        if not a1 > 0:
            break
        c_old, s_old = c, s
        c, s = a0 / a1, g_new / a1
        w_new = (z - a3 * w_old - a2 * w) / a1
        x = x + (c * eta) * w_new
        eta = -s * eta
        its += 1
        hist.append(abs(eta) / g1)
        if check_every:
            if abs(eta) <= tol * g1 or (abs(eta) <= 100 * tol * g1 and its % check_every == 0):
                if np.linalg.norm(b - matvec(x)) <= tol * bnorm:
                    done = True
                    break
        elif abs(eta) <= tol * g1:
            break
        if not g2 > 0:
            break
        v_old, v, z, g_old, g = v, v_new, z_new, g, g_new
        w_old, w = w, w_new
    return x, its, hist, done


def minres_restarted(matvec, precond, b, tol, maxit=500, check_every=5):
    """MINRES stopping on the true residual ||b - A x||_2 <= tol ||b||_2
    (``minres`` with check_every), started again from the iterate only if the
    recurrence breaks down first.  Returns (x, iterations, true relative
    residual at the end of every run)."""
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bnorm == 0:
        return x, 0, [0.0]
    its, hist = 0, []
    while its < maxit:
        x, k, _, done = minres(matvec, precond, b, tol, maxit - its, x0=x if its else None, check_every=check_every)
        its += k
        hist.append(np.linalg.norm(b - matvec(x)) / bnorm)
        if done or hist[-1] <= tol or k == 0:
            break
    return x, its, hist
