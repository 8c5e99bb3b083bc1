"""Python binding of libkkt.so (include/kkt.h): argument marshalling only.

Every step of the solver runs in the library (host analysis in C++, refactorization,
triangular solves and FGMRES-IR in HIP kernels).  PyTorch supplies device memory and the
stream; arrays cross the boundary as raw pointers.  If the library is missing this module
raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import pathlib

import numpy as np

_LIB_PATH = pathlib.Path(__file__).resolve().parent / "libkkt.so"
_lib = None

KKT_OK, KKT_EINVAL, KKT_ENOMEM, KKT_ESINGULAR, KKT_ENOCONV, KKT_EDEVICE, KKT_ESTATE = range(7)
PREC_FP64, PREC_MIXED = 0, 1
GUARD_PERTURB, GUARD_FAIL = 0, 1
STOP_PAPER, STOP_NRBE = 0, 1
ORDER_MD, ORDER_ND = 0, 1
IR_FGMRES, IR_RICHARDSON, IR_ERROR_FGMRES = 0, 1, 2
RESID_FP64, RESID_DD = 0, 1
GS_CGS2, GS_DCGS2 = 0, 1

#: every entry point declared in include/kkt.h
EXPORTS = ["kkt_opts_default", "kkt_analyze", "kkt_get_analysis_info", "kkt_get_permutations",
           "kkt_get_factor_pattern", "kkt_get_analysis_values", "kkt_workspace_size",
           "kkt_bind_workspace", "kkt_refactor", "kkt_refactor_batch", "kkt_refactor_batch_graph",
           "kkt_graph_launches", "kkt_solve", "kkt_direct_solve", "kkt_direct_solve_noalloc",
           "kkt_residual",
           "kkt_get_factor_values", "kkt_set_profiling", "kkt_set_profiling_mask", "kkt_get_kernel_times",
           "kkt_release",
           "kkt_last_error",
           "kkt_clone", "kkt_server_create", "kkt_server_add_pattern", "kkt_server_submit",
           "kkt_server_wait", "kkt_server_poll", "kkt_server_stats", "kkt_server_configure",
           "kkt_server_batch_stats", "kkt_server_destroy",
           "kkt_hykkt_opts_default", "kkt_hykkt_analyze", "kkt_hykkt_workspace_size", "kkt_hykkt_bind_workspace",
           "kkt_hykkt_refactor", "kkt_hykkt_solve", "kkt_hykkt_get_hgamma", "kkt_hykkt_sizes",
           "kkt_hykkt_factor_handle", "kkt_hykkt_last_error", "kkt_hykkt_release"]

KERNEL_CLASSES = ["ingest", "refactor", "trsv_l", "trsv_u", "spmv", "cgs", "resid", "other"]


class Opts(C.Structure):
    _fields_ = [("ordering", C.c_int32), ("nd_leaf", C.c_int32), ("pivot_tau", C.c_double), ("restart", C.c_int32),
                ("max_restarts", C.c_int32), ("delta_tol", C.c_double), ("nrbe_target", C.c_double),
                ("precision", C.c_int32), ("guard_policy", C.c_int32), ("stop_mode", C.c_int32),
                ("mixed_fallback", C.c_int32), ("mixed_max_cycles", C.c_int32), ("ir_method", C.c_int32),
                ("richardson_max_it", C.c_int32), ("ratio_stop", C.c_double), ("inner_tol", C.c_double),
                ("residual", C.c_int32), ("repivot_cycles", C.c_int32), ("gram_schmidt", C.c_int32),
                ("tile_lds_kib", C.c_int32), ("narrow_columns", C.c_int32), ("deterministic", C.c_int32)]


class AnalysisInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("nnz_l", C.c_int64), ("nnz_u", C.c_int64),
                ("offdiag_pivots", C.c_int64), ("levels_refactor", C.c_int64),
                ("levels_l", C.c_int64), ("levels_u", C.c_int64), ("updates", C.c_int64),
                ("analysis_seconds", C.c_double), ("max_column", C.c_int64), ("tiles_l", C.c_int64),
                ("tiles_u", C.c_int64), ("unstaged_l", C.c_int64), ("unstaged_u", C.c_int64)]


class RequestTimes(C.Structure):
    _fields_ = [("queued_ms", C.c_double), ("service_ms", C.c_double), ("latency_ms", C.c_double),
                ("slot", C.c_int32), ("new_slot", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveInfo(C.Structure):
    _fields_ = [("converged", C.c_int32), ("iterations", C.c_int32), ("cycles", C.c_int32),
                ("refined", C.c_int32), ("precision", C.c_int32), ("fallback", C.c_int32),
                ("pivots_perturbed", C.c_int64), ("nrbe", C.c_double), ("nrbe0", C.c_double),
                ("rel_resid", C.c_double), ("rr", C.c_double), ("est_resid", C.c_double),
                ("true_resid", C.c_double), ("knorm_inf", C.c_double), ("nsr", C.c_double),
                ("precond_applications", C.c_int64), ("repivoted", C.c_int32), ("restored_best", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class HyOpts(C.Structure):
    _fields_ = [("gamma", C.c_double), ("gamma_scale", C.c_double), ("cg_tol", C.c_double),
                ("cg_max_iter", C.c_int32), ("reserved", C.c_int32), ("lu", Opts)]


class HyInfo(C.Structure):
    _fields_ = [("converged", C.c_int32), ("cg_iterations", C.c_int32), ("gamma", C.c_double),
                ("cg_rel_resid", C.c_double), ("nrbe", C.c_double), ("rel_resid", C.c_double),
                ("true_resid", C.c_double), ("knorm_inf", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelTimes(C.Structure):
    _fields_ = [("launches", C.c_int64 * 8), ("ms", C.c_double * 8)]


class KKTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("kkt status %d: %s" % (code, msg))
        self.code = code


def lib():
    """Load libkkt.so (built by paper_2401_13926_amd.build); raises if it is absent."""
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            raise ImportError("libkkt.so is not built: run __graft_entry__.build() or "
                              "python -m paper_2401_13926_amd.build")
        L = C.CDLL(str(_LIB_PATH))
        vp, i64, i64p, i32p, f64p = C.c_void_p, C.c_int64, C.POINTER(C.c_int64), \
            C.POINTER(C.c_int32), C.POINTER(C.c_double)
        L.kkt_opts_default.argtypes = [C.POINTER(Opts)]
        L.kkt_opts_default.restype = None
        L.kkt_analyze.argtypes = [C.POINTER(Opts), i64, i64p, i32p, f64p, C.POINTER(vp)]
        L.kkt_get_analysis_info.argtypes = [vp, C.POINTER(AnalysisInfo)]
        L.kkt_get_permutations.argtypes = [vp, i32p, i32p]
        L.kkt_get_factor_pattern.argtypes = [vp, i64p, i32p, i64p, i32p]
        L.kkt_get_analysis_values.argtypes = [vp, f64p, f64p]
        L.kkt_workspace_size.argtypes = [vp, C.c_int32, C.POINTER(C.c_size_t)]
        L.kkt_refactor_batch.argtypes = [C.POINTER(vp), C.POINTER(vp), C.c_int32, vp]
        L.kkt_refactor_batch_graph.argtypes = [C.POINTER(vp), C.POINTER(vp), C.c_int32, vp]
        L.kkt_graph_launches.argtypes = [vp, C.POINTER(C.c_int64)]
        L.kkt_bind_workspace.argtypes = [vp, vp, C.c_size_t, vp]
        L.kkt_refactor.argtypes = [vp, vp, vp]
        L.kkt_solve.argtypes = [vp, vp, vp, C.c_double, C.POINTER(SolveInfo), vp]
        L.kkt_direct_solve.argtypes = [vp, vp, vp, vp]
        L.kkt_direct_solve_noalloc.argtypes = [vp, vp, vp, vp]
        L.kkt_residual.argtypes = [vp, vp, vp, vp, vp]
        L.kkt_get_factor_values.argtypes = [vp, C.c_int32, f64p, f64p, vp]
        L.kkt_set_profiling.argtypes = [vp, C.c_int32]
        L.kkt_set_profiling_mask.argtypes = [vp, C.c_uint32]
        L.kkt_get_kernel_times.argtypes = [vp, C.POINTER(KernelTimes), vp]
        L.kkt_release.argtypes = [vp]
        L.kkt_clone.argtypes = [vp, C.POINTER(vp)]
        L.kkt_server_create.argtypes = [vp, C.c_size_t, C.c_int32, C.POINTER(vp)]
        L.kkt_server_add_pattern.argtypes = [vp, C.POINTER(Opts), i64, i64p, i32p, f64p, i32p]
        L.kkt_server_submit.argtypes = [vp, C.c_int32, vp, vp, vp, C.c_double, i64p]
        L.kkt_server_wait.argtypes = [vp, i64, C.POINTER(SolveInfo), C.POINTER(RequestTimes)]
        L.kkt_server_poll.argtypes = [vp, i64, i32p]
        L.kkt_server_stats.argtypes = [vp, i64p, i64p, i64p, i64p]
        L.kkt_server_destroy.argtypes = [vp]
        L.kkt_server_configure.argtypes = [vp, C.c_int32, C.c_int32]
        L.kkt_hykkt_opts_default.argtypes = [C.POINTER(HyOpts)]
        L.kkt_hykkt_opts_default.restype = None
        L.kkt_hykkt_analyze.argtypes = [C.POINTER(HyOpts), i64, i64, i64p, i32p, f64p, C.POINTER(vp)]
        L.kkt_hykkt_workspace_size.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.kkt_hykkt_bind_workspace.argtypes = [vp, vp, C.c_size_t, vp]
        L.kkt_hykkt_refactor.argtypes = [vp, vp, vp]
        L.kkt_hykkt_solve.argtypes = [vp, vp, vp, C.POINTER(HyInfo), vp]
        L.kkt_hykkt_get_hgamma.argtypes = [vp, i64p, i32p, f64p, f64p, vp]
        L.kkt_hykkt_sizes.argtypes = [vp, i64p, i64p]
        L.kkt_hykkt_factor_handle.argtypes = [vp, C.POINTER(vp)]
        L.kkt_hykkt_last_error.argtypes = [vp]
        L.kkt_hykkt_last_error.restype = C.c_char_p
        L.kkt_hykkt_release.argtypes = [vp]
        L.kkt_server_batch_stats.argtypes = [vp, i64p, i64p, i64p]
        L.kkt_last_error.argtypes = [vp]
        L.kkt_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("kkt_opts_default", "kkt_last_error", "kkt_hykkt_opts_default", "kkt_hykkt_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().kkt_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Solver:
    """A handle: analysis of one pattern plus (after bind) its device workspace."""

    def __init__(self, rowptr, colidx, values_first, **opts):
        self._h = None
        rp = np.ascontiguousarray(rowptr, np.int64)
        ci = np.ascontiguousarray(colidx, np.int32)
        v = np.ascontiguousarray(values_first, np.float64)
        self.n = rp.size - 1
        self.opts = default_opts(**opts)
        h = C.c_void_p()
        rc = lib().kkt_analyze(C.byref(self.opts), self.n, _p(rp, C.c_int64), _p(ci, C.c_int32),
                               _p(v, C.c_double), C.byref(h))
        if rc != KKT_OK:
            raise KKTError(rc, lib().kkt_last_error(None).decode())
        self._h = h
        self.workspace = None

    def graph_launches(self) -> int:
        n = C.c_int64()
        self._check(lib().kkt_graph_launches(self._h, C.byref(n)))
        return n.value

    def clone(self):
        """kkt_clone: a new unbound Solver on the same analysis (for kkt_refactor_batch)."""
        h = C.c_void_p()
        self._check(lib().kkt_clone(self._h, C.byref(h)))
        c = Solver.__new__(Solver)
        c._h = h
        c.n = self.n
        c.opts = self.opts
        c.workspace = None
        return c

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.kkt_release(self._h)
            self._h = None

    def _check(self, rc, allow=()):
        if rc != KKT_OK and rc not in allow:
            raise KKTError(rc, lib().kkt_last_error(self._h).decode())
        return rc

    # --- host-side queries -------------------------------------------------------------
    def info(self) -> dict:
        ai = AnalysisInfo()
        self._check(lib().kkt_get_analysis_info(self._h, C.byref(ai)))
        return {k: getattr(ai, k) for k, _ in ai._fields_}

    def permutations(self):
        prow = np.empty(self.n, np.int32)
        q = np.empty(self.n, np.int32)
        self._check(lib().kkt_get_permutations(self._h, _p(prow, C.c_int32), _p(q, C.c_int32)))
        return prow, q

    def pattern(self):
        inf = self.info()
        lp = np.empty(self.n + 1, np.int64)
        up = np.empty(self.n + 1, np.int64)
        li = np.empty(inf["nnz_l"], np.int32)
        ui = np.empty(inf["nnz_u"], np.int32)
        self._check(lib().kkt_get_factor_pattern(self._h, _p(lp, C.c_int64), _p(li, C.c_int32),
                                                 _p(up, C.c_int64), _p(ui, C.c_int32)))
        return lp, li, up, ui

    def analysis_values(self):
        inf = self.info()
        lx = np.empty(inf["nnz_l"])
        ux = np.empty(inf["nnz_u"])
        self._check(lib().kkt_get_analysis_values(self._h, _p(lx, C.c_double), _p(ux, C.c_double)))
        return lx, ux

    def workspace_size(self, batch: int = 1) -> int:
        s = C.c_size_t()
        self._check(lib().kkt_workspace_size(self._h, int(batch), C.byref(s)))
        return s.value

    # --- device -------------------------------------------------------------------------
    def bind(self, device=None, stream=None, slack: float = 1.5):
        """Allocate the workspace as a torch uint8 tensor and bind it.  `slack` times the
        current size leaves room for a re-pivoted factorization with more fill
        (opts.repivot_cycles)."""
        import torch
        dev = torch.device("cuda" if device is None else device)
        nbytes = int(self.workspace_size() * max(1.0, slack)) + (1 << 20)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = ws.data_ptr()
        off = (-base) % 256
        self._check(lib().kkt_bind_workspace(self._h, C.c_void_p(base + off), nbytes, _stream_ptr(stream)))
        self.workspace = ws
        return self

    def refactor(self, values, stream=None):
        """values: float64 CUDA tensor (nnz) in the CSR order of the analysed pattern."""
        assert values.is_cuda and values.dtype.is_floating_point and values.element_size() == 8
        assert values.is_contiguous()
        self._check(lib().kkt_refactor(self._h, C.c_void_p(values.data_ptr()), _stream_ptr(stream)))
        self._values_ref = values
        return self

    def solve(self, b, x=None, tol: float = 0.0, stream=None, allow_noconv=False):
        """Solve with FGMRES-IR; returns (x, info dict).  b: float64 CUDA tensor (n)."""
        import torch
        assert b.is_cuda and b.dtype == torch.float64 and b.is_contiguous() and b.numel() == self.n
        if x is None:
            x = torch.empty_like(b)
        info = SolveInfo()
        rc = lib().kkt_solve(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), float(tol),
                             C.byref(info), _stream_ptr(stream))
        self._check(rc, allow=(KKT_ENOCONV,) if allow_noconv else ())
        d = info.as_dict()
        d["status"] = rc
        return x, d

    def direct_solve(self, b, x=None, stream=None):
        import torch
        assert b.is_cuda and b.dtype == torch.float64 and b.numel() == self.n
        if x is None:
            x = torch.empty_like(b)
        self._check(lib().kkt_direct_solve(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                           _stream_ptr(stream)))
        return x

    def direct_solve_noalloc(self, b, x, stream=None):
        """kkt_direct_solve_noalloc: x = Q U^-1 L^-1 P b with the library's static scratch; x is
        the caller's output tensor (nothing is allocated)."""
        import torch
        for t in (b, x):
            assert t.is_cuda and t.dtype == torch.float64 and t.numel() == self.n
        self._check(lib().kkt_direct_solve_noalloc(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                                   _stream_ptr(stream)))
        return x

    def residual(self, b, x, r=None, stream=None):
        """r = b - K x for the last refactored K (kkt_residual; precision per opts.residual)."""
        import torch
        for t in (b, x):
            assert t.is_cuda and t.dtype == torch.float64 and t.numel() == self.n
        if r is None:
            r = torch.empty_like(b)
        self._check(lib().kkt_residual(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                       C.c_void_p(r.data_ptr()), _stream_ptr(stream)))
        return r

    def factor_values(self, precision=0, stream=None):
        inf = self.info()
        lx = np.empty(inf["nnz_l"])
        ux = np.empty(inf["nnz_u"])
        self._check(lib().kkt_get_factor_values(self._h, int(precision), _p(lx, C.c_double),
                                                _p(ux, C.c_double), _stream_ptr(stream)))
        return lx, ux

    # --- per-kernel timing ------------------------------------------------------------
    def set_profiling(self, on=True, classes=None):
        """Per-launch event timing: all kernel classes, or only those named in `classes`
        (names of KERNEL_CLASSES)."""
        if classes is None:
            self._check(lib().kkt_set_profiling(self._h, 1 if on else 0))
            return
        mask = 0
        for c in classes:
            mask |= 1 << KERNEL_CLASSES.index(c)
        self._check(lib().kkt_set_profiling_mask(self._h, mask if on else 0))

    def kernel_times(self, stream=None) -> dict:
        """{class: (launches, total ms)} since profiling was enabled (syncs the stream)."""
        t = KernelTimes()
        self._check(lib().kkt_get_kernel_times(self._h, C.byref(t), _stream_ptr(stream)))
        return {name: (int(t.launches[i]), float(t.ms[i])) for i, name in enumerate(KERNEL_CLASSES)}


def refactor_batch(solvers, values, stream=None, graph=False):
    """kkt_refactor_batch (graph=True: kkt_refactor_batch_graph): one refactorization launch for
    several bound Solvers of one analysis (clones of one Solver); values: float64 CUDA tensors
    (nnz each), one per solver."""
    solvers, values = list(solvers), list(values)
    if len(solvers) != len(values) or not solvers:
        raise ValueError("one value tensor per solver")
    for v in values:
        assert v.is_cuda and v.element_size() == 8 and v.is_contiguous()
    hs = (C.c_void_p * len(solvers))(*[s_._h for s_ in solvers])
    vs = (C.c_void_p * len(values))(*[v.data_ptr() for v in values])
    fn = lib().kkt_refactor_batch_graph if graph else lib().kkt_refactor_batch
    rc = fn(hs, vs, len(solvers), _stream_ptr(stream))
    if rc != KKT_OK:
        raise KKTError(rc, lib().kkt_last_error(solvers[0]._h).decode(errors="replace"))
    for s_, v in zip(solvers, values):
        s_._values_ref = v


class Server:
    """Serving loop (kkt_server_*): patterns are registered once; requests (device values, b,
    x) are queued and solved by `workers` concurrent host threads on their own streams, with
    solver slots carved from one device pool (a torch tensor of pool_bytes)."""

    def __init__(self, pool_bytes: int, workers: int = 4, device=None, max_batch: int = 4, graphs: bool = True):
        import torch
        dev = torch.device("cuda" if device is None else device)
        self.pool = torch.empty(int(pool_bytes) + 256, dtype=torch.uint8, device=dev)
        base = self.pool.data_ptr()
        off = (-base) % 256
        h = C.c_void_p()
        rc = lib().kkt_server_create(C.c_void_p(base + off), int(pool_bytes), int(workers), C.byref(h))
        if rc != KKT_OK:
            raise KKTError(rc, "kkt_server_create failed")
        self._h = h
        self._keep = {}  # ticket -> tensors that must outlive the request
        rc = lib().kkt_server_configure(h, int(max_batch), 1 if graphs else 0)
        if rc != KKT_OK:
            self.close()
            raise KKTError(rc, "kkt_server_configure: max_batch must be 1..8")

    def add_pattern(self, rowptr, colidx, values_first, **opts) -> int:
        o = default_opts(**opts)
        rp = np.ascontiguousarray(rowptr, np.int64)
        ci = np.ascontiguousarray(colidx, np.int32)
        v = np.ascontiguousarray(values_first, np.float64)
        pid = C.c_int32()
        rc = lib().kkt_server_add_pattern(self._h, C.byref(o), rp.size - 1, _p(rp, C.c_int64), _p(ci, C.c_int32),
                                          _p(v, C.c_double), C.byref(pid))
        if rc != KKT_OK:
            raise KKTError(rc, lib().kkt_last_error(None).decode())
        return pid.value

    def submit(self, pattern_id: int, values, b, x, tol: float = 0.0) -> int:
        for t in (values, b, x):
            assert t.is_cuda and t.element_size() == 8 and t.is_contiguous()
        tk = C.c_int64()
        rc = lib().kkt_server_submit(self._h, int(pattern_id), C.c_void_p(values.data_ptr()),
                                     C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), float(tol), C.byref(tk))
        if rc != KKT_OK:
            raise KKTError(rc, "kkt_server_submit failed")
        self._keep[tk.value] = (values, b, x)
        return tk.value

    def poll(self, ticket: int) -> bool:
        d = C.c_int32()
        rc = lib().kkt_server_poll(self._h, int(ticket), C.byref(d))
        if rc != KKT_OK:
            raise KKTError(rc, "kkt_server_poll: unknown ticket")
        return bool(d.value)

    def wait(self, ticket: int):
        """(status, info dict, times dict); the request's tensors are released."""
        info = SolveInfo()
        times = RequestTimes()
        rc = lib().kkt_server_wait(self._h, int(ticket), C.byref(info), C.byref(times))
        if rc == KKT_EINVAL and int(ticket) not in self._keep:
            raise KKTError(rc, "kkt_server_wait: unknown ticket")
        self._keep.pop(int(ticket), None)
        return rc, info.as_dict(), times.as_dict()

    def stats(self) -> dict:
        v = [C.c_int64() for _ in range(4)]
        lib().kkt_server_stats(self._h, *[C.byref(x) for x in v])
        w = [C.c_int64() for _ in range(3)]
        lib().kkt_server_batch_stats(self._h, *[C.byref(x) for x in w])
        return dict(completed=v[0].value, slots_created=v[1].value, slots_evicted=v[2].value,
                    pool_in_use=v[3].value, batches=w[0].value, batched_requests=w[1].value,
                    graph_launches=w[2].value)

    def close(self):
        if getattr(self, "_h", None):
            lib().kkt_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HyKKT:
    """HyKKT handle (kkt_hykkt_*): KKT systems with a zero (2,2) block solved through
    H_gamma = H + D + gamma J^T J and CG on the Schur complement; n_primal primal rows."""

    def __init__(self, rowptr, colidx, values_first, n_primal, gamma=0.0, gamma_scale=1e4, cg_tol=1e-12,
                 cg_max_iter=1000, **lu_opts):
        self._h = None
        rp = np.ascontiguousarray(rowptr, np.int64)
        ci = np.ascontiguousarray(colidx, np.int32)
        v = np.ascontiguousarray(values_first, np.float64)
        self.n = rp.size - 1
        self.n_primal = int(n_primal)
        o = HyOpts()
        lib().kkt_hykkt_opts_default(C.byref(o))
        o.gamma, o.gamma_scale, o.cg_tol, o.cg_max_iter = float(gamma), float(gamma_scale), float(cg_tol), int(cg_max_iter)
        o.lu = default_opts(**lu_opts)
        h = C.c_void_p()
        rc = lib().kkt_hykkt_analyze(C.byref(o), self.n, self.n_primal, _p(rp, C.c_int64), _p(ci, C.c_int32),
                                     _p(v, C.c_double), C.byref(h))
        if rc != KKT_OK:
            raise KKTError(rc, lib().kkt_hykkt_last_error(None).decode())
        self._h = h
        self.workspace = None

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.kkt_hykkt_release(self._h)
            self._h = None

    def _check(self, rc, allow=()):
        if rc != KKT_OK and rc not in allow:
            raise KKTError(rc, lib().kkt_hykkt_last_error(self._h).decode())
        return rc

    def sizes(self):
        a, b = C.c_int64(), C.c_int64()
        self._check(lib().kkt_hykkt_sizes(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def bind(self, device=None, stream=None):
        import torch
        dev = torch.device("cuda" if device is None else device)
        nb = C.c_size_t()
        self._check(lib().kkt_hykkt_workspace_size(self._h, C.byref(nb)))
        ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=dev)
        base = ws.data_ptr()
        off = (-base) % 256
        self._check(lib().kkt_hykkt_bind_workspace(self._h, C.c_void_p(base + off), nb.value, _stream_ptr(stream)))
        self.workspace = ws
        return self

    def refactor(self, values, stream=None):
        assert values.is_cuda and values.element_size() == 8 and values.is_contiguous()
        self._check(lib().kkt_hykkt_refactor(self._h, C.c_void_p(values.data_ptr()), _stream_ptr(stream)))
        self._values_ref = values
        return self

    def solve(self, b, x=None, stream=None, allow_noconv=False):
        import torch
        assert b.is_cuda and b.dtype == torch.float64 and b.is_contiguous() and b.numel() == self.n
        if x is None:
            x = torch.empty_like(b)
        info = HyInfo()
        rc = lib().kkt_hykkt_solve(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), C.byref(info),
                                   _stream_ptr(stream))
        self._check(rc, allow=(KKT_ENOCONV,) if allow_noconv else ())
        d = info.as_dict()
        d["status"] = rc
        return x, d

    def hgamma(self, with_values=True, stream=None):
        """(rowptr, colidx, values or None, gamma) of H_gamma."""
        nh, _ = self.sizes()
        rp = np.empty(self.n_primal + 1, np.int64)
        ci = np.empty(nh, np.int32)
        vals = np.empty(nh) if with_values else None
        g = C.c_double()
        self._check(lib().kkt_hykkt_get_hgamma(self._h, _p(rp, C.c_int64), _p(ci, C.c_int32),
                                               _p(vals, C.c_double) if with_values else None, C.byref(g),
                                               _stream_ptr(stream) if with_values else None))
        return rp, ci, vals, g.value

    def factor_values(self, stream=None):
        """(L, U) of H_gamma in the layout of kkt_get_factor_pattern."""
        h = C.c_void_p()
        self._check(lib().kkt_hykkt_factor_handle(self._h, C.byref(h)))
        inner = Solver.__new__(Solver)
        inner._h = h
        inner.n = self.n_primal
        try:
            return inner.factor_values(0, stream)
        finally:
            inner._h = None  # owned by the HyKKT handle
