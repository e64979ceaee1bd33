"""Pins of the oracle's all-at-once system (eq. FinalA) and of the circulant
preconditioner (section 3.1) against the mathematics they must satisfy."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import circulant as circ
from oracle.fem import Operators, assemble_full
from oracle.kkt import Problem


@pytest.fixture(scope="module")
def small_stokes():
    w = W.small(W.STOKES, 2, 4, beta=1e-2)
    return w, Problem.from_workload(w)


@pytest.fixture(scope="module")
def small_oseen():
    w = W.small(W.OSEEN, 2, 4, beta=1e-2, nu=0.1)
    return w, Problem.from_workload(w, W.wind_nodal(2))


def test_kkt_symmetric_and_blockwise(small_stokes, small_oseen):
    """A is the Hessian-plus-constraint matrix of a quadratic program, hence
    symmetric; the time-level evaluation equals the Kronecker matrix."""
    for _, P in (small_stokes, small_oseen):
        A = P.kkt_matrix()
        assert abs(A - A.T).max() < 1e-15
        x = np.random.default_rng(1).standard_normal(P.n_all)
        assert np.allclose(A @ x, P.kkt_apply(x), atol=1e-14)


def test_layout_roundtrip(small_stokes):
    w, P = small_stokes
    x = np.random.default_rng(0).standard_normal(P.n_all)
    xc = P.to_canonical(x)
    assert xc.size == w.n_all
    assert np.array_equal(P.to_compact(xc), x)
    assert np.all(xc[~W.canonical_mask(w.N, w.nt)] == 0)


def test_unpinned_system_singular():
    """P3: without fixing the pressure, a constant pressure (in both blocks)
    is annihilated, because constants are in the kernel of B^T on interior
    velocity columns (section 2.2)."""
    N = 2
    full = assemble_full(N)
    o = Operators(N, 1.0)
    Bfull = sp.hstack([full["Bx"] @ o.grid.Rv().T, full["By"] @ o.grid.Rv().T])   # (N+1)^2 x n_v
    one = np.ones(o.grid.np2)
    assert np.abs(Bfull.T @ one).max() < 1e-14


def test_pinned_system_nonsingular(small_stokes):
    """P3: with the pin, A is non-singular (smallest singular value > 0)."""
    _, P = small_stokes
    s = np.linalg.svd(P.kkt_matrix().toarray(), compute_uv=False)
    assert s.min() > 1e-8 * s.max()


@pytest.mark.parametrize("which", ["stokes", "oseen"])
def test_optimality_against_time_stepping(which, small_stokes, small_oseen):
    """P4: the direct solve satisfies A x = b to 1e-13; with u = lambda/beta
    the sequentially time-stepped state equals the KKT state and the reduced
    gradient g(u) = tau beta M u - tau M lambda(u) vanishes; perturbing u
    raises the discrete cost by a positive quadratic amount."""
    w, P = small_stokes if which == "stokes" else small_oseen
    vd = W.desired_state(w)
    b = P.rhs(vd)
    x = P.solve_direct(b)
    A = P.kkt_matrix()
    assert np.linalg.norm(b - A @ x) <= 1e-13 * np.linalg.norm(b)
    v, p, lam, mu = P.split(x)
    u = lam / P.beta
    vs, ps = P.forward(u)
    assert np.abs(vs - v).max() <= 1e-10 * np.abs(v).max()
    g = P.reduced_gradient(u, vd)
    scale = np.linalg.norm(P.tau * P.beta * (P.ops.M @ u.T).T)
    assert np.linalg.norm(g) <= 1e-10 * scale
    J0 = P.objective(u, vd)
    rng = np.random.default_rng(3)
    dlt = rng.standard_normal(u.shape)
    d1 = P.objective(u + 1e-3 * dlt, vd) - J0
    d2 = P.objective(u + 2e-3 * dlt, vd) - J0
    assert d1 > 0 and abs(d2 / d1 - 4.0) < 1e-6          # exactly quadratic growth


def test_manufactured_solution(small_stokes):
    """P5: b = A x* for a random x* with discretely divergence-free velocity
    fields; the direct solve recovers x*."""
    _, P = small_stokes
    rng = np.random.default_rng(5)
    B = P.ops.B.toarray()
    proj = np.eye(P.nv) - B.T @ np.linalg.solve(B @ B.T, B)
    X = rng.standard_normal((2, P.nt, P.n))
    X[:, :, :P.nv] = X[:, :, :P.nv] @ proj.T
    assert np.abs(X[:, :, :P.nv] @ B.T).max() < 1e-12
    xs = X.reshape(-1)
    x = P.solve_direct(P.kkt_matrix() @ xs)
    assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)


@pytest.mark.parametrize("nt", [4, 6, 16])
def test_dft_and_circulant_eigenvalues(nt):
    """P6/P7: the FFT used for the time transform equals an explicit DFT sum;
    d_j = 1 - exp(-2 pi i j/nt) equals the DFT of c_1 = (1, -1, 0, ...), and
    F^{-1} diag(d) F = C, F^{-1} diag(conj d) F = C^T."""
    rng = np.random.default_rng(nt)
    x = rng.standard_normal(nt)
    F = np.exp(-2j * np.pi * np.outer(np.arange(nt), np.arange(nt)) / nt)
    assert np.allclose(np.fft.fft(x), F @ x, atol=1e-13)
    c1 = np.zeros(nt); c1[0], c1[1] = 1.0, -1.0
    d = circ.d_closed_form(nt)
    assert np.allclose(d, F @ c1, atol=1e-14)
    C = circ.circulant_C(nt).toarray()
    Fi = np.conj(F) / nt
    assert np.allclose(Fi @ np.diag(d) @ F, C, atol=1e-14)
    assert np.allclose(Fi @ np.diag(np.conj(d)) @ F, C.T, atol=1e-14)


@pytest.mark.parametrize("which", ["stokes", "oseen"])
def test_pc_fft_route_equals_direct(which, small_stokes, small_oseen):
    """P7: P_C^{-1} r through the FFT and the blocks G_j (eq. SubBlockG)
    equals a sparse LU of the assembled P_C."""
    _, P = small_stokes if which == "stokes" else small_oseen
    r = np.random.default_rng(2).standard_normal(P.n_all)
    z1 = circ.pc_apply_fft(P, r)
    z2 = circ.pc_apply_direct(P, r)
    assert np.linalg.norm(z1 - z2) <= 1e-12 * np.linalg.norm(z2)


def test_theorem1_low_rank_and_unit_eigenvalues(small_stokes):
    """P8 (Theorem 1): A - P_C has rank n_v, i.e. at most 2 n_v, and
    P_C^{-1} A has at least 2 nt (n_v + n_p) - 2 n_v unit eigenvalues."""
    _, P = small_stokes
    A = P.kkt_matrix().toarray()
    PC = P.kkt_matrix(time_matrix=circ.circulant_C(P.nt)).toarray()
    rk = np.linalg.matrix_rank(A - PC, tol=1e-12)
    assert rk <= 2 * P.nv
    ev = np.linalg.eigvals(np.linalg.solve(PC, A))
    n_unit = int(np.sum(np.abs(ev - 1.0) < 1e-8))
    assert n_unit >= 2 * P.nt * (P.nv + P.nP) - 2 * P.nv


@pytest.mark.parametrize("flow", [0, 1])
def test_frequency_domain_operator_is_blocks_plus_corner(flow):
    """Theorem 1 in the Fourier basis: F A F^{-1} equals the block-diagonal
    G_j plus the corner term (two time samples spread over all frequencies),
    checked against the assembled all-at-once matrix on random complex
    spectra (not only Hermitian-symmetric ones), with planted mistakes (no
    corner term, the corner phase conjugated) failing."""
    import workloads as W
    from oracle import circulant as circ
    from oracle.kkt import Problem
    N, nt = 4, 8
    wind = W.wind_nodal(N) if flow else None
    P = Problem(N, nt, 1.0, 0.1, 1e-2, wind)
    A = P.kkt_matrix()
    rng = np.random.default_rng(3)
    Xh = rng.standard_normal((2, nt, P.n)) + 1j * rng.standard_normal((2, nt, P.n))
    x = np.fft.ifft(Xh, axis=1).reshape(-1)
    ref = np.fft.fft((A @ x).reshape(2, nt, P.n), axis=1)
    got = circ.freq_domain_apply(P, Xh)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # planted mistakes: the corner term left out / its phase conjugated
    no_corner = np.empty_like(ref)
    d = circ.d_closed_form(nt)
    for j in range(nt):
        v = circ.G_block(P, d[j]) @ np.concatenate(circ.split_freq(P, Xh[:, j, :]))
        no_corner[:, j, :] = circ.join_freq(P, v[:P.nv], v[P.nv:2 * P.nv], v[2 * P.nv:2 * P.nv + P.nP],
                                            v[2 * P.nv + P.nP:])
    assert np.abs(no_corner - ref).max() > 1e-3 * np.abs(ref).max()
    x_t = np.fft.ifft(Xh, axis=1)
    bad = no_corner.copy()
    bad[1, :, :P.nv] += (P.ops.M @ x_t[0, nt - 1, :P.nv])[None, :]
    bad[0, :, :P.nv] += np.exp(-2j * np.pi * np.arange(nt) / nt)[:, None] * (P.ops.M @ x_t[1, 0, :P.nv])[None, :]
    assert np.abs(bad - ref).max() > 1e-3 * np.abs(ref).max()
