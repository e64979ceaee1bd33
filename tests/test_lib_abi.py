"""The C-ABI library loads on the CPU and exports every symbol that
include/pintoc.h declares; host-side validation works without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pintoc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pintoc_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    import paper_2405_18964_amd as P
    try:
        return P.library()
    except P.LibraryMissing:
        from paper_2405_18964_amd.build import build
        build()
        P._lib._lib = None
        return P.library()


def test_every_declared_symbol_exported(lib):
    names = _declared()
    assert "pintoc_solve" in names and "pintoc_precond_apply" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_2405_18964_amd._lib import SIGNATURES
    assert set(_declared()) <= set(SIGNATURES)


def test_host_validation(lib):
    from paper_2405_18964_amd._lib import Desc, default_options
    o = default_options()
    h = ctypes.c_void_p()
    for bad in [Desc(3, 8, 1.0, 1.0, 1e-2, 0, None), Desc(4, 3, 1.0, 1.0, 1e-2, 0, None),
                Desc(4, 8, 0.0, 1.0, 1e-2, 0, None), Desc(4, 8, 1.0, 1.0, 0.0, 0, None)]:
        assert lib.pintoc_problem_create(ctypes.byref(bad), ctypes.byref(o), ctypes.byref(h)) == -1
        assert lib.pintoc_last_error()
    good = Desc(8, 16, 1.0, 1.0, 1e-2, 0, None)
    assert o.stall_guard == 1
    bad_opt = default_options(stall_guard=2)
    assert lib.pintoc_problem_create(ctypes.byref(good), ctypes.byref(bad_opt), ctypes.byref(h)) == -1
    # MINRES: outer method 1 needs the Stokes flow, the linear preconditioner and restart >= 4
    assert o.outer == 0
    for bad_opt in (default_options(outer=3), default_options(outer=1, inner=1), default_options(outer=1, restart=3)):
        assert lib.pintoc_problem_create(ctypes.byref(good), ctypes.byref(bad_opt), ctypes.byref(h)) == -1
    # FP32 outer basis: FP32 inner solves and the time-domain FGMRES only; it
    # shrinks the workspace by half the restart length of canonical vectors
    assert o.z_fp32 == 0
    for bad_opt in (default_options(z_fp32=1), default_options(z_fp32=1, precision=1, outer=2),
                    default_options(z_fp32=2, precision=1)):
        assert lib.pintoc_problem_create(ctypes.byref(good), ctypes.byref(bad_opt), ctypes.byref(h)) == -1
        assert b"z_fp32" in lib.pintoc_last_error()
    sizes = []
    for z in (0, 1):
        assert lib.pintoc_problem_create(ctypes.byref(good), ctypes.byref(default_options(precision=1, z_fp32=z)),
                                         ctypes.byref(h)) == 0
        sizes.append((lib.pintoc_workspace_bytes(h), lib.pintoc_vector_length(h)))
        lib.pintoc_problem_destroy(h)
    (w0, n_all), (w1, _) = sizes
    assert w0 - w1 == pytest.approx(o.restart * 4 * n_all, abs=4096 * (o.restart + 2))
    # smoother option and domain validation
    assert o.smoother == 0
    assert lib.pintoc_problem_create(ctypes.byref(good), ctypes.byref(default_options(smoother=2)),
                                     ctypes.byref(h)) == -1
    assert b"smoother" in lib.pintoc_last_error()
    assert lib.pintoc_problem_create(ctypes.byref(good), ctypes.byref(default_options(smoother=1)),
                                     ctypes.byref(h)) == 0
    lib.pintoc_problem_destroy(h)
    for dom in [(0.0, 0.0, 1.0, 2.0), (1.0, 0.0, 1.0, 0.0), (0.0, 0.0, -1.0, -1.0)]:
        bad = Desc(8, 16, 1.0, 1.0, 1e-2, 0, None, *dom)
        assert lib.pintoc_problem_create(ctypes.byref(bad), ctypes.byref(o), ctypes.byref(h)) == -1
        assert b"square" in lib.pintoc_last_error()
    wind = (ctypes.c_double * (2 * 17 * 17))()
    oseen = Desc(8, 16, 1.0, 1.0, 1e-2, 1, ctypes.cast(wind, ctypes.POINTER(ctypes.c_double)))
    assert lib.pintoc_problem_create(ctypes.byref(oseen), ctypes.byref(default_options(outer=1)), ctypes.byref(h)) == -1
    assert lib.pintoc_problem_create(ctypes.byref(oseen), ctypes.byref(default_options(inner=2)), ctypes.byref(h)) == -1
    assert b"MINRES" in lib.pintoc_last_error()
    assert lib.pintoc_problem_create(ctypes.byref(good), ctypes.byref(default_options(outer=1)), ctypes.byref(h)) == 0
    lib.pintoc_problem_destroy(h)
    assert lib.pintoc_problem_create(ctypes.byref(good), ctypes.byref(o), ctypes.byref(h)) == 0
    assert lib.pintoc_vector_length(h) == 2 * 16 * (2 * 17 ** 2 + 9 ** 2)
    assert lib.pintoc_workspace_bytes(h) > 0
    assert lib.pintoc_bind_workspace(h, None, 0, None) == -1
    assert lib.pintoc_kkt_apply(h, None, None, None) < 0          # unbound: refused before any GPU call
    lib.pintoc_problem_destroy(h)


def test_solve_batch_validation(lib):
    """pintoc_solve_batch rejects bad arguments before any GPU work."""
    from paper_2405_18964_amd._lib import Desc, SolveStats, default_options
    V = ctypes.c_void_p
    assert lib.pintoc_solve_batch(None, None, None, None, None, 0) == 0
    assert lib.pintoc_solve_batch(None, None, None, None, None, -1) == -1
    assert lib.pintoc_solve_batch(None, None, None, None, None, 1) == -1
    o = default_options()
    h = ctypes.c_void_p()
    d = Desc(8, 16, 1.0, 1.0, 1e-2, 0, None)
    assert lib.pintoc_problem_create(ctypes.byref(d), ctypes.byref(o), ctypes.byref(h)) == 0
    P = (V * 1)(h.value)
    vecs = (V * 1)(16)                     # never dereferenced: refused first
    st = (SolveStats * 1)()
    assert lib.pintoc_solve_batch(P, vecs, (V * 1)(32), st, (V * 1)(None), 1) == -1    # NULL stream
    assert lib.pintoc_solve_batch(P, vecs, (V * 1)(32), st, (V * 1)(64), 1) == -4      # no workspace bound
    assert b"problem 0" in lib.pintoc_last_error()
    lib.pintoc_problem_destroy(h)


def test_batch_job_bytes_and_mix():
    """Memory accounting of the batch runner and the batched workload draw."""
    import workloads as W
    from paper_2405_18964_amd.batch import job_bytes
    mix = W.batch_mix()
    assert len(mix) == 64 and mix == W.batch_mix()
    assert {w.N for w in mix} <= {32, 64, 128} and {w.nt for w in mix} <= {32, 64, 128, 256}
    assert all(1e-6 <= w.beta <= 1e-2 for w in mix)
    small = {"N": 8, "nt": 16, "nu": 1.0, "beta": 1e-2, "flow": 0}
    big = dict(small, nt=32)
    assert 0 < job_bytes(small) < job_bytes(big)
    assert job_bytes(small, precision=1) < job_bytes(small, precision=0)
    # a job's own options override the run's (here: the inner MINRES of a Stokes job)
    assert job_bytes(dict(small, options={"inner": 2}), inner=1) < job_bytes(small, inner=1)
    assert job_bytes(dict(small, options={"inner": 1}), inner=2) == job_bytes(small, inner=1)


def test_batch_arena_first_fit():
    """The batch runner's arena: first fit, exhaustion, and freed ranges that
    coalesce so a job as large as the whole arena fits again (host logic on a
    CPU buffer)."""
    import random
    from paper_2405_18964_amd.batch import _Arena
    a = _Arena(1000, "cpu")
    assert a.alloc(400) == 0 and a.alloc(300) == 400 and a.alloc(400) is None
    assert a.alloc(300) == 700 and a.largest() == 0
    a.release(400, 300)
    assert a.alloc(301) is None and a.alloc(200) == 400 and a.largest() == 100
    a.release(0, 400)
    a.release(700, 300)
    assert a.free == [(0, 400), (600, 400)]
    a.release(400, 200)
    assert a.free == [(0, 1000)] and a.alloc(1000) == 0
    a.release(0, 1000)
    rng = random.Random(3)
    held = []
    for _ in range(2000):                       # random traffic never overlaps ranges
        if held and rng.random() < 0.5:
            held.remove(r := rng.choice(held))
            a.release(*r)
        else:
            n = rng.randint(1, 300)
            o = a.alloc(n)
            if o is not None:
                assert all(o + n <= q or q + m <= o for q, m in held)
                held.append((o, n))
    for r in held:
        a.release(*r)
    assert a.free == [(0, 1000)]


def test_serve_stream_draw():
    """Served workload: seeded Poisson arrivals (increasing, mean gap 1 at unit
    rate) and request parameters drawn like the batched mix."""
    import numpy as np
    import workloads as W
    s = W.serve_stream(256)
    assert len(s) == 256 and [a for _, a in s] == [a for _, a in W.serve_stream(256)]
    arr = np.array([a for _, a in s])
    assert np.all(np.diff(arr) > 0) and 0.8 < arr[-1] / 256 < 1.2
    assert {w.N for w, _ in s} <= {32, 64, 128, 256} and 256 in {w.N for w, _ in s}
    assert max(w.N for w, _ in W.serve_stream(64, max_N=128)) <= 128


def test_struct_layout_matches_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's field
    offsets and sizes (the header compiled by gcc on the host)."""
    import subprocess
    from paper_2405_18964_amd._lib import Desc, KernelTiming, Options, SolveStats
    structs = {"pintoc_problem_desc": Desc, "pintoc_options": Options, "pintoc_solve_stats": SolveStats,
               "pintoc_kernel_timing": KernelTiming}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pintoc.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_bind_scratch_rejects_before_gpu_work():
    """pintoc_bind_scratch refuses a NULL handle and a problem whose workspace
    exceeds the static array before touching the device."""
    from paper_2405_18964_amd._lib import ENOMEM, EINVAL, Desc, default_options, library
    lib = library()
    assert lib.pintoc_bind_scratch(None, None) == EINVAL
    d = Desc(32, 32, 1.0, 1.0, 1e-2, 0, None, 0.0, 0.0, 0.0, 0.0)
    h = ctypes.c_void_p()
    assert lib.pintoc_problem_create(ctypes.byref(d), ctypes.byref(default_options(inner=1)), ctypes.byref(h)) == 0
    assert lib.pintoc_workspace_bytes(h) > (128 << 20)
    assert lib.pintoc_bind_scratch(h, None) == ENOMEM
    assert b"static scratch" in lib.pintoc_last_error()
    lib.pintoc_problem_destroy(h)


def test_group_create_validation():
    """pintoc_group_create accepts members that differ in nt, T, nu and beta
    and refuses members of other grids, flows, domains or winds (host only)."""
    import numpy as np

    import workloads as W
    from paper_2405_18964_amd._lib import EINVAL, Desc, default_options, library
    lib = library()
    o = default_options(inner=1)

    def grp(descs, opts=o):
        arr = (Desc * len(descs))(*descs)
        h = ctypes.c_void_p()
        rc = lib.pintoc_group_create(arr, len(descs), ctypes.byref(opts), ctypes.byref(h))
        return rc, h

    a = Desc(8, 16, 1.0, 1.0, 1e-2, 0, None, 0.0, 0.0, 0.0, 0.0)
    b = Desc(8, 32, 2.0, 0.5, 1e-4, 0, None, 0.0, 0.0, 0.0, 0.0)
    rc, h = grp([a, b])
    assert rc == 0
    assert lib.pintoc_group_size(h) == 2
    assert lib.pintoc_group_vector_length(h, 1) == 2 * 32 * (2 * 17 ** 2 + 81)
    assert lib.pintoc_group_vector_length(h, 2) == 0
    assert lib.pintoc_kkt_apply(h, None, None, None) < 0     # unbound, and a group takes the group calls
    lib.pintoc_problem_destroy(h)
    assert grp([a, Desc(16, 16, 1.0, 1.0, 1e-2, 0, None, 0.0, 0.0, 0.0, 0.0)])[0] == EINVAL
    w1 = np.ascontiguousarray(W.wind_nodal(8).reshape(-1))
    w2 = 0.5 * w1
    o1 = Desc(8, 16, 1.0, 0.01, 1e-2, 1, w1.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0.0, 0.0, 0.0, 0.0)
    o2 = Desc(8, 8, 1.0, 0.02, 1e-3, 1, w2.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0.0, 0.0, 0.0, 0.0)
    assert grp([a, o1])[0] == EINVAL                          # flows differ
    assert grp([o1, o2])[0] == EINVAL                         # winds differ
    assert b"wind" in lib.pintoc_last_error()
    o3 = Desc(8, 8, 1.0, 0.02, 1e-3, 1, w1.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0.0, 0.0, 0.0, 0.0)
    rc, h = grp([o1, o3])
    assert rc == 0
    lib.pintoc_problem_destroy(h)
    sq = Desc(8, 16, 1.0, 1.0, 1e-2, 0, None, -1.0, -1.0, 1.0, 1.0)
    assert grp([sq, sq])[0] == EINVAL                         # groups on the unit square only
    assert grp([a, b], default_options(outer=1, restart=10))[0] == EINVAL
    h = ctypes.c_void_p()
    assert lib.pintoc_group_create((Desc * 1)(a), 0, ctypes.byref(o), ctypes.byref(h)) == EINVAL


def test_frequency_domain_outer_validation():
    """The frequency-domain FGMRES takes single problems on the unit square
    (Oseen in FP64 only)."""
    import numpy as np

    import workloads as W
    from paper_2405_18964_amd._lib import EINVAL, Desc, default_options, library
    lib = library()
    h = ctypes.c_void_p()
    st = Desc(8, 16, 1.0, 1.0, 1e-2, 0, None, 0.0, 0.0, 0.0, 0.0)
    for prec in (0, 1):
        assert lib.pintoc_problem_create(ctypes.byref(st), ctypes.byref(default_options(outer=2, precision=prec)),
                                         ctypes.byref(h)) == 0
        lib.pintoc_problem_destroy(h)
    w = np.ascontiguousarray(W.wind_nodal(8).reshape(-1))
    os_ = Desc(8, 16, 1.0, 0.1, 1e-2, 1, w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0.0, 0.0, 0.0, 0.0)
    assert lib.pintoc_problem_create(ctypes.byref(os_), ctypes.byref(default_options(outer=2)), ctypes.byref(h)) == 0
    lib.pintoc_problem_destroy(h)
    assert lib.pintoc_problem_create(ctypes.byref(os_), ctypes.byref(default_options(outer=2, precision=1)),
                                     ctypes.byref(h)) == EINVAL
    sq = Desc(8, 16, 1.0, 1.0, 1e-2, 0, None, -1.0, -1.0, 1.0, 1.0)
    assert lib.pintoc_problem_create(ctypes.byref(sq), ctypes.byref(default_options(outer=2)), ctypes.byref(h)) == EINVAL
    assert lib.pintoc_problem_create(ctypes.byref(st), ctypes.byref(default_options(outer=3)), ctypes.byref(h)) == EINVAL
