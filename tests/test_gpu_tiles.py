"""GPU parity where the multigrid tile kernels run (grids above 16 elements per
side), for both smoothers, against the oracle.

Below 32 elements per side every V-cycle runs in the one-work-group small-grid
kernels; these cases exercise the tiled sweeps, the fused residual/restriction
with its side-buffer fix-up, the Q1 tile sweeps and residual/restriction, and
(GMRES mode) their masked launches.  N = 32 and 64 give 65 and 129 Q2 nodes
per side: two and three 48-node tiles, the last one ragged, and a ragged
32-node Q1 tile.

* smoother GLOBAL (multicolour SOR over whole grids) against the oracle's
  plain smoother (the reading of section 3.4);
* smoother TILED against the oracle's tiled variant with the library's tile
  sizes (48 Q2 / 32 Q1 node indices, stated in include/pintoc.h);
* FP64: elementwise within 1e-10 of the largest entry and 1e-10 in the
  2-norm; FP32 inner solves against the same FP64 oracle within 2e-5 (the
  FP32 unit roundoff 6e-8 times the growth of rounding errors through 4
  V-cycles, 10 Chebyshev steps and 6 Uzawa steps; measured values print);
* full-size single-mode checks (a residual with one temporal Fourier mode
  excites only frequencies j and nt - j) at j = 0 (d_j = 0, the block the
  paper singles out as hardest) and j = nt/2 (d_j = 2), both smoothers;
* the smallest configuration driven to a true residual of 1e-13 and
  compared with the oracle's sparse direct solve.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

Q2_TILE, Q1_TILE = 48, 32           # the library's tiled smoother (include/pintoc.h)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def lib():
    import paper_2405_18964_amd as P
    P.library()
    return P


def _settings(smoother, **kw):
    from oracle.precond import Settings
    from oracle.smoothers import Tiling
    return Settings(tiling=Tiling(Q2_TILE, Q1_TILE) if smoother == "tiled" else None, **kw)


def _problem(lib, flow, N, nt, smoother, **opts):
    from oracle.kkt import Problem as OP
    if flow == W.STOKES:
        w = W.small(W.STOKES, N, nt, beta=1e-4)
        wind = None
    else:
        w = W.Workload(W.OSEEN, N, nt, 1.0, 0.01, 1e-4, 0, 1.0)
        wind = W.wind_nodal(N)
    sm = lib.SMOOTHER_TILED if smoother == "tiled" else lib.SMOOTHER_GLOBAL
    return w, wind, OP.from_workload(w, wind), lib.Problem.from_workload(w, smoother=sm, **opts)


def _oracle_pc(op, wind, flow, settings, freqs=None):
    from oracle.precond import OseenPreconditioner, StokesPreconditioner
    if flow == W.STOKES:
        return StokesPreconditioner(op, settings, freqs=freqs)
    return OseenPreconditioner(op, wind, settings, freqs=freqs)


CASES = [(f, N, nt) for f in (W.STOKES, W.OSEEN) for N in (32, 64) for nt in (8, 16)]


def _ids(c):
    return f"{'stokes' if c[0] == W.STOKES else 'oseen'}-N{c[1]}-nt{c[2]}"


@pytest.mark.parametrize("smoother", ["tiled", "global"])
@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_precond_linear_tile_levels(lib, case, smoother):
    flow, N, nt = case
    print(f"tile-level precond {_ids(case)} smoother={smoother}", flush=True)
    w, wind, op, gp = _problem(lib, flow, N, nt, smoother)
    r = W.random_canonical(N, nt, seed=21)
    z = _host(gp.precond_apply(_dev(r)))
    ref = op.to_canonical(_oracle_pc(op, wind, flow, _settings(smoother)).apply(op.to_compact(r)))
    err2 = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    errm = np.abs(z - ref).max() / np.abs(ref).max()
    print(f"  rel 2-norm {err2:.2e}, max {errm:.2e}", flush=True)
    assert err2 <= 1e-10 and errm <= 1e-10
    assert np.all(z[~W.canonical_mask(N, nt)] == 0)


def test_smoothers_differ_above_one_tile(lib):
    """The two smoothers are different operators once a grid spans several
    tiles (guards against a test that compares one sweep with itself)."""
    _, _, _, gt = _problem(lib, W.STOKES, 32, 8, "tiled")
    _, _, _, gg = _problem(lib, W.STOKES, 32, 8, "global")
    r = _dev(W.random_canonical(32, 8, seed=21))
    zt, zg = _host(gt.precond_apply(r)), _host(gg.precond_apply(r))
    assert np.linalg.norm(zt - zg) > 1e-8 * np.linalg.norm(zg)


GMRES_CASES = [(W.STOKES, 32, 8, "tiled"), (W.STOKES, 32, 8, "global"), (W.STOKES, 64, 8, "tiled"),
               (W.OSEEN, 32, 8, "tiled"), (W.OSEEN, 32, 8, "global")]


@pytest.mark.parametrize("flow,N,nt,smoother", GMRES_CASES)
def test_precond_gmres_tile_levels(lib, flow, N, nt, smoother):
    """Algorithm 2 / its Oseen analogue with masked launches at tile-kernel
    sizes: the inner counts equal the oracle's and the outputs agree."""
    print(f"tile-level gmres flow={flow} N={N} nt={nt} smoother={smoother}", flush=True)
    w, wind, op, gp = _problem(lib, flow, N, nt, smoother, inner=lib.INNER_GMRES)
    r = op.to_canonical(op.rhs(W.desired_state(w)))
    z = _host(gp.precond_apply(_dev(r)))
    pc = _oracle_pc(op, wind, flow, _settings(smoother))
    ref = op.to_canonical(pc.apply(op.to_compact(r), nonlinear=True))
    counts = gp.last_inner_iterations()
    print(f"  counts {counts}", flush=True)
    assert counts == [pc.inner_its[j] for j in range(nt // 2 + 1)]
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("smoother", ["tiled", "global"])
@pytest.mark.parametrize("flow,N,nt", [(W.STOKES, 32, 8), (W.STOKES, 64, 16), (W.OSEEN, 32, 8), (W.OSEEN, 64, 8)])
def test_precond_fp32_tile_levels(lib, flow, N, nt, smoother):
    """FP32 inner solves (storage and tile arithmetic in FP32) against the
    FP64 oracle."""
    print(f"tile-level fp32 flow={flow} N={N} nt={nt} smoother={smoother}", flush=True)
    w, wind, op, gp = _problem(lib, flow, N, nt, smoother, precision=lib.PREC_FP32_INNER)
    r = W.random_canonical(N, nt, seed=22)
    z = _host(gp.precond_apply(_dev(r)))
    ref = op.to_canonical(_oracle_pc(op, wind, flow, _settings(smoother)).apply(op.to_compact(r)))
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    print(f"  fp32 rel error {err:.2e}", flush=True)
    assert err <= 2e-5


def _single_mode(lib, flow, j, smoother):
    w = W.config(2) if flow == W.STOKES else W.config(3)
    print(f"full-size single mode {w.name} j={j} smoother={smoother}", flush=True)
    sm = lib.SMOOTHER_TILED if smoother == "tiled" else lib.SMOOTHER_GLOBAL
    gp = lib.Problem.from_workload(w, smoother=sm)
    r = W.single_frequency_canonical(w.N, w.nt, j, seed=3)
    z = _host(gp.precond_apply(_dev(r)))
    del gp
    torch.cuda.empty_cache()
    from oracle.kkt import Problem as OP
    wind = W.wind_nodal(w.N) if flow == W.OSEEN else None
    op = OP.from_workload(w, wind)
    freqs = sorted({j, (w.nt - j) % w.nt})
    ref = op.to_canonical(_oracle_pc(op, wind, flow, _settings(smoother), freqs=freqs).apply(op.to_compact(r)))
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    print(f"  rel error {err:.2e}", flush=True)
    assert err <= 1e-10


@pytest.mark.parametrize("smoother", ["tiled", "global"])
@pytest.mark.parametrize("j", [0, 128])
def test_precond_full_size_stokes_extreme_modes(lib, j, smoother):
    """Stokes N=128, nt=256 workload, frequency j = 0 and j = nt/2."""
    _single_mode(lib, W.STOKES, j, smoother)


@pytest.mark.parametrize("smoother", ["tiled", "global"])
@pytest.mark.parametrize("j", [0, 64])
def test_precond_full_size_oseen_extreme_modes(lib, j, smoother):
    """Oseen N=128, nt=128 workload, frequency j = 0 and j = nt/2."""
    _single_mode(lib, W.OSEEN, j, smoother)


@pytest.mark.parametrize("smoother", ["tiled", "global"])
def test_solve_config1_tight(lib, smoother):
    """The N=8, nt=16 Stokes configuration driven to a true residual of 1e-13
    in FP64: the solution agrees with the oracle's sparse direct solve within
    1e-10 (relative, 2-norm), and the residual the oracle recomputes is at
    most 1e-13 as well."""
    from oracle.kkt import Problem as OP
    w = W.config(1)
    sm = lib.SMOOTHER_TILED if smoother == "tiled" else lib.SMOOTHER_GLOBAL
    gp = lib.Problem.from_workload(w, restart=30, max_outer=900, tol=1e-13, smoother=sm)
    b = gp.assemble_rhs(_dev(W.desired_state(w)))
    x, st, ok = gp.solve(b)
    print(f"tight solve: {st['outer_iterations']} its, residual {st['rel_residual']:.2e}", flush=True)
    assert ok and st["rel_residual"] <= 1e-13
    op = OP.from_workload(w)
    bh, xh = _host(b), _host(x)
    res = np.linalg.norm(bh - op.to_canonical(op.kkt_apply(op.to_compact(xh)))) / np.linalg.norm(bh)
    xs = op.to_canonical(op.solve_direct(op.to_compact(bh)))
    err = np.linalg.norm(xh - xs) / np.linalg.norm(xs)
    print(f"  oracle residual {res:.2e}, error against sparse LU {err:.2e}", flush=True)
    assert res <= 1e-13
    assert err <= 1e-10
