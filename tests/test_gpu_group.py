"""Fused batched form (pintoc_group_*): several problems of one grid and
flow in one handle, their kept frequencies in one batch of every
per-frequency kernel, their FGMRES iterations in lockstep.

* the fused linear preconditioner equals each member's lone application bit
  for bit (Stokes members with different nt, beta and nu; Oseen members with
  different tau, beta and nu, which exercises the per-frequency parameters of
  the Uzawa and Schur steps) and the oracle within 1e-10;
* a member left out of an application (r = NULL) leaves its output alone and
  does not change the others;
* group solves (inner GMRES, FP64 and FP32 inner) equal the lone solves bit
  for bit, member by member, with the same iteration counts; the oracle
  recomputes each member's true residual (at most 1e-8), also for members that
  converge at different outer iterations.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

STOKES_MIX = [W.small(W.STOKES, 16, 8, beta=1e-2, seed=31),
              W.Workload(W.STOKES, 16, 32, 2.0, 0.02, 1e-4, 32, 1.5),
              W.small(W.STOKES, 16, 16, beta=1e-6, nu=0.01, seed=33)]
OSEEN_MIX = [W.Workload(W.OSEEN, 16, 16, 1.0, 0.02, 1e-2, 41, 1.0),
             W.Workload(W.OSEEN, 16, 8, 1.0, 0.1, 1e-3, 42, 1.0),
             W.Workload(W.OSEEN, 16, 32, 2.0, 0.05, 1e-4, 43, 0.7)]


@pytest.fixture(scope="module")
def lib():
    import paper_2405_18964_amd as P
    P.library()
    return P


def _member(w):
    return {"N": w.N, "nt": w.nt, "T": w.T, "nu": w.nu, "beta": w.beta, "flow": w.flow,
            "wind": W.wind_nodal(w.N) if w.flow == W.OSEEN else None}


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("mix", ["stokes", "oseen"])
def test_fused_linear_preconditioner(lib, mix):
    from oracle.kkt import Problem as OP
    from oracle.precond import OseenPreconditioner, Settings, StokesPreconditioner
    from oracle.smoothers import Tiling
    ws = STOKES_MIX if mix == "stokes" else OSEEN_MIX
    print(f"fused linear preconditioner, {mix} group of {len(ws)}", flush=True)
    g = lib.Group([_member(w) for w in ws])
    rs = [torch.from_numpy(W.random_canonical(w.N, w.nt, seed=50 + k)).cuda() for k, w in enumerate(ws)]
    zs = [_host(z) for z in g.precond_apply(rs)]
    for k, w in enumerate(ws):
        lone = lib.Problem.from_workload(w)
        zl = _host(lone.precond_apply(rs[k]))
        print(f"  member {k} ({w.name}): equal to lone {np.array_equal(zs[k], zl)}", flush=True)
        assert np.array_equal(zs[k], zl)
    # one member against the oracle
    w = ws[1]
    wind = W.wind_nodal(w.N) if w.flow == W.OSEEN else None
    op = OP.from_workload(w, wind)
    st = Settings(tiling=Tiling(48, 32))
    pc = StokesPreconditioner(op, st) if w.flow == W.STOKES else OseenPreconditioner(op, wind, st)
    ref = op.to_canonical(pc.apply(op.to_compact(_host(rs[1]))))
    err = np.linalg.norm(zs[1] - ref) / np.linalg.norm(ref)
    print(f"  member 1 against the oracle: {err:.2e}", flush=True)
    assert err <= 1e-10
    # leave member 0 out: its output stays, the others do not change
    marker = torch.full_like(rs[0], 7.0)
    outs = g.precond_apply([None, rs[1], rs[2]], [marker, g.empty(1), g.empty(2)])
    assert torch.all(outs[0] == 7.0)
    assert np.array_equal(_host(outs[1]), zs[1]) and np.array_equal(_host(outs[2]), zs[2])


@pytest.mark.parametrize("mix,precision", [("stokes", "fp64"), ("oseen", "fp64"), ("stokes", "fp32"),
                                           ("oseen", "fp32")])
def test_group_solve_equals_lone_solves(lib, mix, precision):
    from oracle.kkt import Problem as OP
    ws = STOKES_MIX if mix == "stokes" else OSEEN_MIX
    prec = lib.PREC_FP64 if precision == "fp64" else lib.PREC_FP32_INNER
    opts = dict(inner=lib.INNER_GMRES, precision=prec, max_outer=100)
    print(f"group solve, {mix} x{len(ws)}, {precision}", flush=True)
    g = lib.Group([_member(w) for w in ws], **opts)
    vds = [torch.from_numpy(W.desired_state(w)).cuda() for w in ws]
    bs = [g.assemble_rhs(k, vds[k]) for k in range(len(ws))]
    xs, sts, oks = g.solve(bs)
    its = [st["outer_iterations"] for st in sts]
    print(f"  outer iterations {its}, converged {oks}", flush=True)
    for k, w in enumerate(ws):
        lone = lib.Problem.from_workload(w, **opts)
        bl = lone.assemble_rhs(vds[k])
        assert torch.equal(bl, bs[k])
        xl, stl, okl = lone.solve(bl)
        same = torch.equal(xl, xs[k])
        print(f"  member {k} ({w.name}): {sts[k]['outer_iterations']} its (lone {stl['outer_iterations']}), "
              f"inner mean {sts[k]['inner_iterations_mean']:.1f} (lone {stl['inner_iterations_mean']:.1f}), "
              f"bitwise equal {same}", flush=True)
        assert oks[k] and okl and same
        assert sts[k]["outer_iterations"] == stl["outer_iterations"]
        assert sts[k]["inner_counts"] == stl["inner_counts"]
        op = OP.from_workload(w, W.wind_nodal(w.N) if w.flow == W.OSEEN else None)
        bh, xh = _host(bs[k]), _host(xs[k])
        res = np.linalg.norm(bh - op.to_canonical(op.kkt_apply(op.to_compact(xh)))) / np.linalg.norm(bh)
        print(f"    oracle residual {res:.2e}", flush=True)
        assert res <= 1e-8


def test_fused_runner_and_autotuner(lib):
    """batch.autotune picks a group size and smoother per (N, flow) class by
    timing fused applications; batch.run_fused then solves the jobs in those
    groups.  With the tiled smoother forced, every fused result equals the
    concurrent runner's (one problem per stream) bit for bit."""
    from paper_2405_18964_amd.batch import autotune, run, run_fused
    mix = STOKES_MIX + OSEEN_MIX + [W.small(W.STOKES, 8, 16, beta=1e-3, seed=61)]
    jobs = [dict(_member(w), vd=W.desired_state(w)) for w in mix]
    opts = dict(inner=lib.INNER_GMRES, precision=lib.PREC_FP32_INNER, max_outer=100)
    plan = autotune(jobs, sizes=(1, 2, 3), **opts)
    print(f"plan { {k: (v['size'], v['smoother']) for k, v in plan.items()} }", flush=True)
    assert set(plan) == {(16, 0), (16, 1), (8, 0)}
    assert all(v["trials"] and v["size"] >= 1 for v in plan.values())
    tiled = {k: dict(v, smoother=lib.SMOOTHER_TILED) for k, v in plan.items()}
    fused = run_fused(jobs, tiled, workers=2, checksum=True, **opts)
    conc = run(jobs, workers=2, checksum=True, **opts)
    for k, (a, b) in enumerate(zip(fused, conc)):
        print(f"  job {k}: group {a['group']} of {a['group_size']}, same as concurrent {a['digest'] == b['digest']}",
              flush=True)
        assert a["converged"] and a["digest"] == b["digest"]
