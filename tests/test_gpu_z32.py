"""FP32 outer basis (options.z_fp32): the preconditioned vectors of the
outer FGMRES (section 3.4) stored in FP32 with FP32 inner solves.

The vectors come out of FP32 block solves, so FP32 storage drops nothing
they carry beyond their own rounding (unit 6e-8); the solution update reads
them and the true residual of every restart corrects the rest.  Checks: the
solve reaches the true residual 1e-8 (recomputed by the oracle), within two
outer iterations of the FP64-basis solve and within 1e-6 of its solution
(two solves to 1e-8 of a system whose condition number is ~1e2 differ by
about that much); a fused group with the FP32 basis equals its lone solves
bit for bit.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


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


CASES = [W.small(W.STOKES, 32, 16, beta=1e-4), W.Workload(W.OSEEN, 16, 16, 1.0, 0.02, 1e-3, 0, 1.0)]


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_fp32_basis_solve(lib, w):
    from oracle.kkt import Problem as OP
    print(f"z_fp32 solve {w.name}", flush=True)
    wind = W.wind_nodal(w.N) if w.flow == W.OSEEN else None
    out = {}
    for z in (0, 1):
        gp = lib.Problem.from_workload(w, inner=lib.INNER_GMRES, precision=lib.PREC_FP32_INNER, z_fp32=z)
        b = gp.assemble_rhs(_dev(W.desired_state(w)))
        x, st, ok = gp.solve(b)
        assert ok and st["rel_residual"] <= 1e-8
        out[z] = (_host(x), _host(b), st, gp.workspace_bytes)
    (x0, b0, s0, w0), (x1, b1, s1, w1) = out[0], out[1]
    assert np.array_equal(b0, b1) and w1 < w0
    op = OP.from_workload(w, wind)
    res = np.linalg.norm(b1 - op.to_canonical(op.kkt_apply(op.to_compact(x1)))) / np.linalg.norm(b1)
    diff = np.linalg.norm(x1 - x0) / np.linalg.norm(x0)
    print(f"  its {s1['outer_iterations']} (FP64 basis {s0['outer_iterations']}), oracle residual {res:.2e}, "
          f"difference {diff:.2e}, workspace {w1 / 2**20:.1f} MiB (FP64 basis {w0 / 2**20:.1f} MiB)")
    assert res <= 1e-8
    assert abs(s1["outer_iterations"] - s0["outer_iterations"]) <= 2
    assert diff <= 1e-6


def test_fp32_basis_group_equals_lone(lib):
    print("z_fp32 group", flush=True)
    ws = [W.small(W.STOKES, 16, 16, beta=1e-3), W.small(W.STOKES, 16, 32, beta=1e-2)]
    opts = dict(inner=lib.INNER_GMRES, precision=lib.PREC_FP32_INNER, z_fp32=1)
    members = [{"N": w.N, "nt": w.nt, "T": w.T, "nu": w.nu, "beta": w.beta, "flow": w.flow} for w in ws]
    g = lib.Group(members, **opts)
    bs = [g.assemble_rhs(i, _dev(W.desired_state(w))) for i, w in enumerate(ws)]
    xs, sts, oks = g.solve(bs)
    for i, w in enumerate(ws):
        gp = lib.Problem.from_workload(w, **opts)
        b = gp.assemble_rhs(_dev(W.desired_state(w)))
        x, st, ok = gp.solve(b)
        assert oks[i] and ok
        assert sts[i]["outer_iterations"] == st["outer_iterations"]
        assert np.array_equal(_host(xs[i]), _host(x))
