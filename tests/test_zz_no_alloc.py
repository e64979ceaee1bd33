"""The allocation-free binding (pintoc_bind_scratch) through the C ABI.

Two problems in a row share the library's static scratch array: the first
(Stokes N=16, nt=16, GMRES inner solves) and then a smaller one (Oseen N=8,
nt=8, linear preconditioner).  Each result computed on the scratch array is
compared with the same call on a problem bound to a caller workspace
(pintoc_bind_workspace): preconditioner application and full solve, FP64,
within 1e-12 relative (the same kernels run on the same data, so the results
agree to rounding order; they are in fact expected to be identical).  The
first problem loses the array to the second and must then refuse to run."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _handle(lib, L, w, wind, **opts):
    wp = wind.ctypes.data_as(C.POINTER(C.c_double)) if wind is not None else None
    d = L.Desc(w.N, w.nt, w.T, w.nu, w.beta, w.flow, wp, 0.0, 0.0, 0.0, 0.0)
    o = L.default_options(**opts)
    h = C.c_void_p()
    assert lib.pintoc_problem_create(C.byref(d), C.byref(o), C.byref(h)) == 0, lib.pintoc_last_error()
    return h


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _case(lib, L, w, opts):
    wind = np.ascontiguousarray(W.wind_nodal(w.N).reshape(-1)) if w.flow == W.OSEEN else None
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ref = _handle(lib, L, w, wind, **opts)
    nbytes = lib.pintoc_workspace_bytes(ref)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    assert lib.pintoc_bind_workspace(ref, _ptr(ws), nbytes, stream) == 0, lib.pintoc_last_error()
    h = _handle(lib, L, w, wind, **opts)
    assert lib.pintoc_bind_scratch(h, stream) == 0, lib.pintoc_last_error()
    n = lib.pintoc_vector_length(h)
    r = torch.from_numpy(W.random_canonical(w.N, w.nt, seed=5)).cuda()
    outs = {}
    for name, hd in (("ref", ref), ("scratch", h)):
        z = torch.zeros(n, dtype=torch.float64, device="cuda")
        assert lib.pintoc_precond_apply(hd, _ptr(r), _ptr(z), stream) == 0, lib.pintoc_last_error()
        vd = torch.from_numpy(W.desired_state(w)).cuda()
        b = torch.zeros(n, dtype=torch.float64, device="cuda")
        assert lib.pintoc_assemble_rhs(hd, _ptr(vd), _ptr(b), stream) == 0
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        st = L.SolveStats()
        rc = lib.pintoc_solve(hd, _ptr(b), _ptr(x), C.byref(st), stream)
        assert rc == 0, (rc, lib.pintoc_last_error(), st.outer_iterations, st.rel_residual)
        torch.cuda.synchronize()
        outs[name] = (z.cpu().numpy(), x.cpu().numpy(), st.outer_iterations, st.rel_residual)
    (zr, xr, itr, rr), (zs, xs, its, rs) = outs["ref"], outs["scratch"]
    ez = np.linalg.norm(zs - zr) / np.linalg.norm(zr)
    ex = np.linalg.norm(xs - xr) / np.linalg.norm(xr)
    print(f"  {w.name}: precond rel diff {ez:.2e}, solve rel diff {ex:.2e}, its {its}/{itr}, res {rs:.2e}",
          flush=True)
    assert ez <= 1e-12 and ex <= 1e-12 and its == itr and rs <= 1e-8
    lib.pintoc_problem_destroy(ref)
    del ws
    return h


def test_bind_scratch_two_problems_in_a_row():
    from paper_2405_18964_amd import _lib as L
    lib = L.library()
    print("no-alloc: Stokes N=16 nt=16 GMRES", flush=True)
    h1 = _case(lib, L, W.small(W.STOKES, 16, 16, beta=1e-2), dict(inner=L.INNER_GMRES, max_outer=60))
    print("no-alloc: Oseen N=8 nt=8 linear (smaller, takes the array over)", flush=True)
    wo = W.Workload(W.OSEEN, 8, 8, 1.0, 0.1, 1e-2, 3, 1.0)
    h2 = _case(lib, L, wo, dict(inner=L.INNER_LINEAR, restart=30, max_outer=300))
    # the first problem lost its device memory to the second
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    n1 = lib.pintoc_vector_length(h1)
    a = torch.zeros(n1, dtype=torch.float64, device="cuda")
    bvec = torch.zeros(n1, dtype=torch.float64, device="cuda")
    assert lib.pintoc_precond_apply(h1, _ptr(a), _ptr(bvec), stream) == L.ESTATE
    lib.pintoc_problem_destroy(h1)
    lib.pintoc_problem_destroy(h2)


def test_bind_scratch_too_large():
    from paper_2405_18964_amd import _lib as L
    lib = L.library()
    w = W.small(W.STOKES, 32, 32)
    h = _handle(lib, L, w, None, inner=L.INNER_GMRES)
    assert lib.pintoc_workspace_bytes(h) > (128 << 20)
    assert lib.pintoc_bind_scratch(h, None) == L.ENOMEM
    assert b"static scratch" in lib.pintoc_last_error()
    lib.pintoc_problem_destroy(h)
