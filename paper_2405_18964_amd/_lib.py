"""ctypes binding of libpintoc.so (names follow include/pintoc.h)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libpintoc.so")

STOKES, OSEEN = 0, 1
INNER_LINEAR, INNER_GMRES, INNER_MINRES = 0, 1, 2
PREC_FP64, PREC_FP32_INNER = 0, 1
OUTER_FGMRES, OUTER_MINRES, OUTER_FGMRES_FREQ = 0, 1, 2
SMOOTHER_TILED, SMOOTHER_GLOBAL = 0, 1
OK, NOT_CONVERGED, PAUSED = 0, 1, 2
EINVAL, ENOMEM, EHIP, ESTATE = -1, -2, -3, -4


class LibraryMissing(RuntimeError):
    pass


class Desc(C.Structure):
    _fields_ = [("N", C.c_int32), ("nt", C.c_int32), ("T", C.c_double), ("nu", C.c_double),
                ("beta", C.c_double), ("flow", C.c_int32), ("wind", C.POINTER(C.c_double)),
                ("x0", C.c_double), ("y0", C.c_double), ("x1", C.c_double), ("y1", C.c_double)]


class Options(C.Structure):
    _fields_ = [("inner", C.c_int32), ("precision", C.c_int32), ("restart", C.c_int32),
                ("max_outer", C.c_int32), ("tol", C.c_double), ("inner_tol", C.c_double),
                ("inner_restart", C.c_int32), ("inner_maxit", C.c_int32), ("n_vcycles", C.c_int32),
                ("n_cheb", C.c_int32), ("n_uzawa", C.c_int32), ("mu_uzawa", C.c_double),
                ("stall_guard", C.c_int32), ("outer", C.c_int32), ("smoother", C.c_int32),
                ("pressure_stream", C.c_int32), ("graphs", C.c_int32), ("z_fp32", C.c_int32)]


NPHASES = 5
PHASES = ("fft", "blocks", "ifft", "matvec", "orth")


class SolveStats(C.Structure):
    _fields_ = [("outer_iterations", C.c_int32), ("converged", C.c_int32), ("rel_residual", C.c_double),
                ("inner_iterations_mean", C.c_double), ("inner_iterations_max", C.c_int32),
                ("precond_applications", C.c_int32), ("seconds", C.c_double), ("model_bytes", C.c_double),
                ("precond_model_bytes", C.c_double), ("phase_seconds", C.c_double * NPHASES),
                ("residual_history", C.POINTER(C.c_double)), ("history_capacity", C.c_int32),
                ("history_length", C.c_int32), ("inner_counts", C.POINTER(C.c_int32)),
                ("inner_counts_capacity", C.c_int32), ("cycle_budget", C.c_int32), ("resume", C.c_int32)]

    def as_dict(self):
        out = {}
        for k, _ in self._fields_:
            if k in ("residual_history", "inner_counts", "history_capacity", "inner_counts_capacity",
                     "cycle_budget", "resume"):
                continue
            v = getattr(self, k)
            out[k] = dict(zip(PHASES, list(v))) if k == "phase_seconds" else v
        return out


class KernelTiming(C.Structure):
    _fields_ = [("avg_ms", C.c_double), ("launches", C.c_int64), ("algorithmic_bytes", C.c_double),
                ("post_avg_ms", C.c_double), ("post_launches", C.c_int64), ("post_algorithmic_bytes", C.c_double)]


_lib = None

# exported symbols and their signatures (restype, argtypes)
SIGNATURES = {
    "pintoc_default_options": (C.c_int, [C.POINTER(Options)]),
    "pintoc_problem_create": (C.c_int, [C.POINTER(Desc), C.POINTER(Options), C.POINTER(C.c_void_p)]),
    "pintoc_workspace_bytes": (C.c_size_t, [C.c_void_p]),
    "pintoc_bind_workspace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "pintoc_bind_scratch": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pintoc_assemble_rhs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pintoc_assemble_rhs_data": (C.c_int, [C.c_void_p] * 7),
    "pintoc_kkt_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pintoc_precond_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pintoc_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(SolveStats), C.c_void_p]),
    "pintoc_solve_batch": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                      C.POINTER(SolveStats), C.POINTER(C.c_void_p), C.c_int32]),
    "pintoc_problem_destroy": (None, [C.c_void_p]),
    "pintoc_group_create": (C.c_int, [C.POINTER(Desc), C.c_int32, C.POINTER(Options), C.POINTER(C.c_void_p)]),
    "pintoc_group_size": (C.c_int32, [C.c_void_p]),
    "pintoc_group_vector_length": (C.c_int64, [C.c_void_p, C.c_int32]),
    "pintoc_group_assemble_rhs": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pintoc_group_kkt_apply": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pintoc_group_precond_apply": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_void_p]),
    "pintoc_group_solve": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                      C.POINTER(SolveStats), C.c_void_p]),
    "pintoc_last_error": (C.c_char_p, []),
    "pintoc_vector_length": (C.c_int64, [C.c_void_p]),
    "pintoc_last_inner_iterations": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.c_int32]),
    "pintoc_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "pintoc_profile_read": (C.c_int, [C.c_void_p, C.POINTER(KernelTiming)]),
}


def library_path() -> str:
    return _LIB_PATH


def library():
    """Load libpintoc.so (once).  Raises LibraryMissing if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise LibraryMissing(f"{_LIB_PATH} not found: run paper_2405_18964_amd.build.build() first")
        lib = C.CDLL(_LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int, what: str):
    if rc < 0:
        msg = library().pintoc_last_error().decode()
        raise RuntimeError(f"{what} failed ({rc}): {msg}")
    return rc


def default_options(**kw) -> Options:
    o = Options()
    library().pintoc_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


class Problem:
    """One control problem bound to device memory.

    Vectors are torch float64 CUDA tensors in the canonical layout of
    include/pintoc.h (length :attr:`n_all`)."""

    def __init__(self, N, nt, T, nu, beta, flow=STOKES, wind=None, device="cuda", domain=None, workspace=None,
                 **options):
        """``workspace``: optional caller-provided uint8 CUDA tensor (at least
        ``workspace_bytes``, 256-byte aligned) to bind instead of a new one."""
        import numpy as np
        import torch
        lib = library()
        self._torch = torch
        self.N, self.nt, self.T, self.nu, self.beta, self.flow = N, nt, T, nu, beta, flow
        self._wind = None
        wptr = None
        if wind is not None:
            self._wind = np.ascontiguousarray(np.asarray(wind, dtype=np.float64).reshape(-1))
            wptr = self._wind.ctypes.data_as(C.POINTER(C.c_double))
        x0, y0, x1, y1 = (0.0, 0.0, 0.0, 0.0) if domain is None else tuple(float(v) for v in domain)
        d = Desc(N, nt, T, nu, beta, flow, wptr, x0, y0, x1, y1)
        self.options = default_options(**options)
        h = C.c_void_p()
        _check(lib.pintoc_problem_create(C.byref(d), C.byref(self.options), C.byref(h)), "pintoc_problem_create")
        self._h = h
        self.n_all = int(lib.pintoc_vector_length(h))
        self.workspace_bytes = int(lib.pintoc_workspace_bytes(h))
        self.device = torch.device(device)
        if workspace is None:
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        else:
            if not (isinstance(workspace, torch.Tensor) and workspace.is_cuda and workspace.dtype == torch.uint8
                    and workspace.numel() >= self.workspace_bytes):
                raise ValueError(f"workspace must be a uint8 CUDA tensor of at least {self.workspace_bytes} bytes")
            self._ws = workspace
        _check(lib.pintoc_bind_workspace(h, C.c_void_p(self._ws.data_ptr()), self.workspace_bytes,
                                         self._stream()), "pintoc_bind_workspace")

    @classmethod
    def from_workload(cls, w, **options):
        import workloads as W
        wind = W.wind_nodal(w.N) if w.flow == OSEEN else None
        return cls(w.N, w.nt, w.T, w.nu, w.beta, w.flow, wind, **options)

    def _stream(self):
        return C.c_void_p(self._torch.cuda.current_stream(self.device).cuda_stream)

    def _vec(self, v, name):
        t = self._torch
        if not (isinstance(v, t.Tensor) and v.is_cuda and v.dtype == t.float64 and v.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
        if v.numel() != self.n_all:
            raise ValueError(f"{name} has {v.numel()} entries, expected {self.n_all}")
        return C.c_void_p(v.data_ptr())

    def empty(self):
        return self._torch.zeros(self.n_all, dtype=self._torch.float64, device=self.device)

    def assemble_rhs(self, vd, out=None):
        t = self._torch
        nq2 = (2 * self.N + 1) ** 2
        if not (isinstance(vd, t.Tensor) and vd.is_cuda and vd.dtype == t.float64 and vd.is_contiguous()
                and vd.numel() == self.nt * 2 * nq2):
            raise TypeError("vd must be a contiguous float64 CUDA tensor of shape [nt, 2, (2N+1)^2]")
        out = self.empty() if out is None else out
        _check(library().pintoc_assemble_rhs(self._h, C.c_void_p(vd.data_ptr()), self._vec(out, "out"),
                                             self._stream()), "pintoc_assemble_rhs")
        return out

    def assemble_rhs_data(self, vd=None, f=None, h=None, v0=None, out=None):
        """Right-hand side for a desired state, forcing, Dirichlet data and an
        initial velocity (float64 CUDA tensors of Q2 nodal values, None = 0):
        vd, f [nt, 2, (2N+1)^2], h [nt + 1, 2, (2N+1)^2], v0 [2, (2N+1)^2]."""
        t = self._torch
        nq2 = (2 * self.N + 1) ** 2
        ptrs = []
        for name, a, n in (("vd", vd, self.nt * 2 * nq2), ("f", f, self.nt * 2 * nq2),
                           ("h", h, (self.nt + 1) * 2 * nq2), ("v0", v0, 2 * nq2)):
            if a is None:
                ptrs.append(None)
                continue
            if not (isinstance(a, t.Tensor) and a.is_cuda and a.dtype == t.float64 and a.is_contiguous()
                    and a.numel() == n):
                raise TypeError(f"{name} must be a contiguous float64 CUDA tensor with {n} entries")
            ptrs.append(C.c_void_p(a.data_ptr()))
        out = self.empty() if out is None else out
        _check(library().pintoc_assemble_rhs_data(self._h, *ptrs, self._vec(out, "out"), self._stream()),
               "pintoc_assemble_rhs_data")
        return out

    def kkt_apply(self, x, out=None):
        out = self.empty() if out is None else out
        _check(library().pintoc_kkt_apply(self._h, self._vec(x, "x"), self._vec(out, "out"), self._stream()),
               "pintoc_kkt_apply")
        return out

    def precond_apply(self, r, out=None):
        out = self.empty() if out is None else out
        _check(library().pintoc_precond_apply(self._h, self._vec(r, "r"), self._vec(out, "out"),
                                              self._stream()), "pintoc_precond_apply")
        return out

    def solve(self, b, x=None, history=0, cycle_budget=0, resume=False):
        """Returns (x, stats dict, converged flag).  The stats carry the
        per-frequency inner GMRES counts of the solve and, with ``history``
        > 0, up to that many per-iteration residual estimates.  With
        ``cycle_budget`` > 0 the call returns after that many FGMRES restart
        cycles (stats "paused" true if not converged); ``resume`` continues
        the paused solve (same b and x)."""
        x = self.empty() if x is None else x
        st = SolveStats()
        st.cycle_budget = int(cycle_budget)
        st.resume = 1 if resume else 0
        nf = self.nt // 2 + 1
        counts = (C.c_int32 * nf)()
        st.inner_counts = C.cast(counts, C.POINTER(C.c_int32))
        st.inner_counts_capacity = nf
        hist = (C.c_double * max(int(history), 1))()
        if history > 0:
            st.residual_history = C.cast(hist, C.POINTER(C.c_double))
            st.history_capacity = int(history)
        rc = _check(library().pintoc_solve(self._h, self._vec(b, "b"), self._vec(x, "x"), C.byref(st),
                                           self._stream()), "pintoc_solve")
        out = st.as_dict()
        out["inner_counts"] = [int(counts[j]) for j in range(nf)]
        out["residual_history"] = [float(hist[k]) for k in range(st.history_length)]
        out["paused"] = rc == PAUSED
        return x, out, rc == OK

    def last_inner_iterations(self):
        """Inner GMRES counts per kept frequency of the last application."""
        nf = self.nt // 2 + 1
        arr = (C.c_int32 * nf)()
        k = _check(library().pintoc_last_inner_iterations(self._h, arr, nf), "pintoc_last_inner_iterations")
        return [int(arr[i]) for i in range(k)]

    def profile_enable(self, on=True):
        """Start (or stop) timing the finest-level velocity smoother launches
        (pre- and post-smoothing sweeps)."""
        _check(library().pintoc_profile_enable(self._h, 1 if on else 0), "pintoc_profile_enable")

    def profile_read(self):
        kt = KernelTiming()
        _check(library().pintoc_profile_read(self._h, C.byref(kt)), "pintoc_profile_read")
        return {"avg_ms": kt.avg_ms, "launches": kt.launches, "algorithmic_bytes": kt.algorithmic_bytes,
                "post": {"avg_ms": kt.post_avg_ms, "launches": kt.post_launches,
                         "algorithmic_bytes": kt.post_algorithmic_bytes}}

    def close(self):
        if getattr(self, "_h", None):
            library().pintoc_problem_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Group:
    """Several problems of the same N and flow (and wind, for Oseen) as one
    handle (``pintoc_group_create``): their kept frequencies run as one batch
    in every per-frequency kernel, their FGMRES iterations in lockstep.
    ``members`` is a list of dicts with N, nt, T, nu, beta, flow and wind (the
    keys of :class:`Problem`).  Vectors of member k are float64 CUDA tensors
    of ``n_all[k]`` entries."""

    def __init__(self, members, device="cuda", **options):
        import numpy as np
        import torch
        lib = library()
        self._torch = torch
        self.members = [dict(m) for m in members]
        n = len(members)
        descs = (Desc * n)()
        self._winds = []
        for k, m in enumerate(members):
            wptr = None
            if m.get("wind") is not None:
                w = np.ascontiguousarray(np.asarray(m["wind"], dtype=np.float64).reshape(-1))
                self._winds.append(w)
                wptr = w.ctypes.data_as(C.POINTER(C.c_double))
            descs[k] = Desc(m["N"], m["nt"], m.get("T", 1.0), m["nu"], m["beta"], m.get("flow", STOKES), wptr,
                            0.0, 0.0, 0.0, 0.0)
        self.options = default_options(**options)
        h = C.c_void_p()
        _check(lib.pintoc_group_create(descs, n, C.byref(self.options), C.byref(h)), "pintoc_group_create")
        self._h = h
        self.size = int(lib.pintoc_group_size(h))
        self.n_all = [int(lib.pintoc_group_vector_length(h, k)) for k in range(n)]
        self.workspace_bytes = int(lib.pintoc_workspace_bytes(h))
        self.device = torch.device(device)
        self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        _check(lib.pintoc_bind_workspace(h, C.c_void_p(self._ws.data_ptr()), self.workspace_bytes,
                                         self._stream()), "pintoc_bind_workspace")

    def _stream(self):
        return C.c_void_p(self._torch.cuda.current_stream(self.device).cuda_stream)

    def _vec(self, v, k, name):
        t = self._torch
        if not (isinstance(v, t.Tensor) and v.is_cuda and v.dtype == t.float64 and v.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
        if v.numel() != self.n_all[k]:
            raise ValueError(f"{name} of member {k} has {v.numel()} entries, expected {self.n_all[k]}")
        return v.data_ptr()

    def empty(self, k):
        return self._torch.zeros(self.n_all[k], dtype=self._torch.float64, device=self.device)

    def assemble_rhs(self, k, vd, out=None):
        out = self.empty(k) if out is None else out
        _check(library().pintoc_group_assemble_rhs(self._h, k, C.c_void_p(vd.data_ptr()),
                                                   C.c_void_p(self._vec(out, k, "out")), self._stream()),
               "pintoc_group_assemble_rhs")
        return out

    def kkt_apply(self, k, x, out=None):
        out = self.empty(k) if out is None else out
        _check(library().pintoc_group_kkt_apply(self._h, k, C.c_void_p(self._vec(x, k, "x")),
                                                C.c_void_p(self._vec(out, k, "out")), self._stream()),
               "pintoc_group_kkt_apply")
        return out

    def precond_apply(self, rs, outs=None):
        """z[k] = P_k^{-1} r[k] for the members with r[k] not None (one fused application)."""
        n = self.size
        outs = [None if r is None else self.empty(k) for k, r in enumerate(rs)] if outs is None else list(outs)
        R = (C.c_void_p * n)(*[None if r is None else self._vec(r, k, "r") for k, r in enumerate(rs)])
        Z = (C.c_void_p * n)(*[None if z is None else self._vec(z, k, "z") for k, z in enumerate(outs)])
        _check(library().pintoc_group_precond_apply(self._h, R, Z, self._stream()), "pintoc_group_precond_apply")
        return outs

    def solve(self, bs, xs=None, history=0):
        """Returns (list of x, list of stats dicts, list of converged flags)."""
        n = self.size
        xs = [self.empty(k) for k in range(n)] if xs is None else list(xs)
        st = (SolveStats * n)()
        counts = [(C.c_int32 * (m["nt"] // 2 + 1))() for m in self.members]
        hists = [(C.c_double * max(int(history), 1))() for _ in range(n)]
        for k in range(n):
            st[k].inner_counts = C.cast(counts[k], C.POINTER(C.c_int32))
            st[k].inner_counts_capacity = self.members[k]["nt"] // 2 + 1
            if history > 0:
                st[k].residual_history = C.cast(hists[k], C.POINTER(C.c_double))
                st[k].history_capacity = int(history)
        B = (C.c_void_p * n)(*[self._vec(b, k, "b") for k, b in enumerate(bs)])
        X = (C.c_void_p * n)(*[self._vec(x, k, "x") for k, x in enumerate(xs)])
        _check(library().pintoc_group_solve(self._h, B, X, st, self._stream()), "pintoc_group_solve")
        out = []
        for k in range(n):
            d = st[k].as_dict()
            d["inner_counts"] = [int(counts[k][j]) for j in range(self.members[k]["nt"] // 2 + 1)]
            d["residual_history"] = [float(hists[k][i]) for i in range(st[k].history_length)]
            out.append(d)
        return xs, out, [bool(d["converged"]) for d in out]

    def close(self):
        if getattr(self, "_h", None):
            library().pintoc_problem_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def group_bytes(members, **options) -> int:
    """Device bytes of a group's workspace (host-side set-up only)."""
    import numpy as np
    lib = library()
    n = len(members)
    descs = (Desc * n)()
    keep = []
    for k, m in enumerate(members):
        wptr = None
        if m.get("wind") is not None:
            w = np.ascontiguousarray(np.asarray(m["wind"], dtype=np.float64).reshape(-1))
            keep.append(w)
            wptr = w.ctypes.data_as(C.POINTER(C.c_double))
        descs[k] = Desc(m["N"], m["nt"], m.get("T", 1.0), m["nu"], m["beta"], m.get("flow", STOKES), wptr,
                        0.0, 0.0, 0.0, 0.0)
    o = default_options(**options)
    h = C.c_void_p()
    _check(lib.pintoc_group_create(descs, n, C.byref(o), C.byref(h)), "pintoc_group_create")
    try:
        return int(lib.pintoc_workspace_bytes(h))
    finally:
        lib.pintoc_problem_destroy(h)


def solve_batch(problems, bs, xs=None):
    """Solve several bound problems concurrently (``pintoc_solve_batch``):
    problem k on its own HIP stream, driven by its own host thread inside the
    library.  ``bs``/``xs`` are the problems' canonical vectors (``xs[k]`` is
    the initial guess and receives the solution; zeros when None).  Returns a
    list of (x, stats dict, converged flag).  Each result equals that of a
    separate :meth:`Problem.solve` call."""
    n = len(problems)
    if len(bs) != n or (xs is not None and len(xs) != n):
        raise ValueError("one right-hand side (and initial guess) per problem")
    if n == 0:
        return []
    torch = problems[0]._torch
    xs = [p.empty() for p in problems] if xs is None else list(xs)
    cur = torch.cuda.current_stream(problems[0].device)
    streams = [torch.cuda.Stream(device=p.device) for p in problems]    # default priority
    for s in streams:
        s.wait_stream(cur)                      # inputs were produced on the current stream
    for k in range(n):
        if bs[k].data_ptr() == xs[k].data_ptr():
            raise ValueError("b and x alias")
    P = (C.c_void_p * n)(*[p._h.value for p in problems])
    B = (C.c_void_p * n)(*[p._vec(b, "b").value for p, b in zip(problems, bs)])
    X = (C.c_void_p * n)(*[p._vec(x, "x").value for p, x in zip(problems, xs)])
    S = (C.c_void_p * n)(*[s.cuda_stream for s in streams])
    st = (SolveStats * n)()
    _check(library().pintoc_solve_batch(P, B, X, st, S, n), "pintoc_solve_batch")
    for s in streams:
        cur.wait_stream(s)
    return [(xs[k], st[k].as_dict(), st[k].converged == 1) for k in range(n)]