"""CPU oracle: a plain, slow, independent reference for the KKT refactorization solver.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the benchmark's
CPU-baseline leg, never by the GPU library.  It shares no code with the GPU path.

Layers:
  * liboracle.so (oracle.c, plain C, -ffp-contract=off): ordering, pivoted sparse LU,
    static-pivot refactorization (FP64/FP32), triangular solves, residual/NRBE/NSR,
    condition estimate, FGMRES-IR.  Each C function cites the passage it follows.
  * dense.py: pure-Python/numpy dense brute force used to pin the C code.
"""
from __future__ import annotations

import ctypes as C
import os
import pathlib
import subprocess

import numpy as np

_HERE = pathlib.Path(__file__).resolve().parent
_SRC = _HERE / "oracle.c"
_LIB = _HERE / "liboracle.so"
_lib = None

OK, EINVAL, ENOMEM, ESINGULAR = 0, 1, 2, 3


def build(force: bool = False) -> pathlib.Path:
    """Compile liboracle.so with gcc (IEEE arithmetic, no contraction)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-msse2",
                        "-mfpmath=sse", "-fPIC", "-shared", "-o", str(tmp), str(_SRC), "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(str(_LIB))
        i64, i32p, i64p, f64p, f32p = C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_int64), \
            C.POINTER(C.c_double), C.POINTER(C.c_float)
        L.or_check_csr.argtypes = [i64, i64p, i32p]
        L.or_order.argtypes = [i64, i64p, i32p, i32p]
        L.or_order_leaf.argtypes = [i64, i64p, i32p, i64, i32p]
        L.or_order_md.argtypes = [i64, i64p, i32p, i32p]
        L.or_factor.restype = C.c_void_p
        L.or_factor.argtypes = [i64, i64p, i32p, f64p, i32p, C.c_double, C.POINTER(C.c_int), i64p]
        L.or_free.argtypes = [C.c_void_p]
        L.or_lu_sizes.argtypes = [C.c_void_p, i64p, i64p]
        L.or_lu_export.argtypes = [C.c_void_p, i64p, i32p, f64p, i64p, i32p, f64p, i32p, i32p]
        L.or_refactor64.argtypes = [C.c_void_p, i64p, i32p, f64p, C.c_int, f64p, f64p, i64p, i64p]
        L.or_refactor32.argtypes = [C.c_void_p, i64p, i32p, f64p, C.c_int, f32p, f32p, i64p, i64p]
        L.or_solve_with.argtypes = [C.c_void_p, f64p, f64p, f64p, f64p]
        L.or_arnoldi.argtypes = [C.c_void_p, f64p, f64p, f32p, f32p, C.c_int, i64p, i32p, f64p, f64p,
                                 C.c_int, C.c_int, f64p, f64p, f64p]
        L.or_solve_with32.argtypes = [C.c_void_p, f32p, f32p, f64p, f64p]
        L.or_residual.argtypes = [i64, i64p, i32p, f64p, f64p, f64p, f64p]
        L.or_residual_dd.argtypes = [i64, i64p, i32p, f64p, f64p, f64p, f64p]
        L.or_metrics.argtypes = [i64, i64p, i32p, f64p, f64p, f64p, f64p]
        L.or_norm_inf_mat.restype = C.c_double
        L.or_norm_inf_mat.argtypes = [i64, i64p, f64p]
        L.or_condest.restype = C.c_double
        L.or_condest.argtypes = [C.c_void_p, i64p, f64p]
        L.or_fgmres_ir.argtypes = [C.c_void_p, f64p, f64p, f32p, f32p, C.c_int, i64p, i32p, f64p,
                                   f64p, f64p, C.c_int, C.c_int, C.c_double, C.c_int, f64p, f64p,
                                   i64]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _csr(rowptr, colidx, values=None):
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(colidx, dtype=np.int32)
    v = None if values is None else np.ascontiguousarray(values, dtype=np.float64)
    return rp, ci, v


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


def check_csr(rowptr, colidx) -> bool:
    rp, ci, _ = _csr(rowptr, colidx)
    return lib().or_check_csr(rp.size - 1, _p(rp, C.c_int64), _p(ci, C.c_int32)) == OK


def order(rowptr, colidx, method: str = "md", leaf: int = 64) -> np.ndarray:
    """Fill-reducing ordering Q (Q[j] = original column eliminated at step j):
    method "md" = exact minimum degree (default), "nd" = BFS nested dissection."""
    rp, ci, _ = _csr(rowptr, colidx)
    n = rp.size - 1
    Q = np.empty(n, dtype=np.int32)
    if method == "md":
        rc = lib().or_order_md(n, _p(rp, C.c_int64), _p(ci, C.c_int32), _p(Q, C.c_int32))
    elif method == "nd":
        rc = lib().or_order_leaf(n, _p(rp, C.c_int64), _p(ci, C.c_int32), int(leaf), _p(Q, C.c_int32))
    else:
        raise ValueError(method)
    if rc != OK:
        raise OracleError(rc, "or_order failed: %d" % rc)
    return Q


class LU:
    """Pivoted factors of K(:,Q): P K Q = L U (see or_factor in oracle.c)."""

    def __init__(self, rowptr, colidx, values, Q=None, tau=1e-10):
        rp, ci, v = _csr(rowptr, colidx, values)
        n = rp.size - 1
        if Q is None:
            Q = order(rp, ci)
        Q = np.ascontiguousarray(Q, dtype=np.int32)
        st = C.c_int(0)
        bad = C.c_int64(-1)
        h = lib().or_factor(n, _p(rp, C.c_int64), _p(ci, C.c_int32), _p(v, C.c_double),
                            _p(Q, C.c_int32), float(tau), C.byref(st), C.byref(bad))
        if not h:
            raise OracleError(st.value, "or_factor failed: status %d at column %d" % (st.value, bad.value))
        self._h = h
        self.n = n
        lnz, unz = C.c_int64(), C.c_int64()
        lib().or_lu_sizes(h, C.byref(lnz), C.byref(unz))
        self.Lp = np.empty(n + 1, np.int64)
        self.Li = np.empty(lnz.value, np.int32)
        self.Lx = np.empty(lnz.value, np.float64)
        self.Up = np.empty(n + 1, np.int64)
        self.Ui = np.empty(unz.value, np.int32)
        self.Ux = np.empty(unz.value, np.float64)
        self.prow = np.empty(n, np.int32)
        self.Q = np.empty(n, np.int32)
        lib().or_lu_export(h, _p(self.Lp, C.c_int64), _p(self.Li, C.c_int32), _p(self.Lx, C.c_double),
                           _p(self.Up, C.c_int64), _p(self.Ui, C.c_int32), _p(self.Ux, C.c_double),
                           _p(self.prow, C.c_int32), _p(self.Q, C.c_int32))
        self.pinv = np.empty(n, np.int32)
        self.pinv[self.prow] = np.arange(n, dtype=np.int32)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.or_free(h)
            self._h = None

    @property
    def lnz(self):
        return int(self.Lp[-1])

    @property
    def unz(self):
        return int(self.Up[-1])

    def refactor64(self, rowptr, colidx, values, guard_policy=0):
        rp, ci, v = _csr(rowptr, colidx, values)
        Lx = np.empty(self.lnz, np.float64)
        Ux = np.empty(self.unz, np.float64)
        ng, bad = C.c_int64(), C.c_int64()
        rc = lib().or_refactor64(self._h, _p(rp, C.c_int64), _p(ci, C.c_int32), _p(v, C.c_double),
                                 int(guard_policy), _p(Lx, C.c_double), _p(Ux, C.c_double),
                                 C.byref(ng), C.byref(bad))
        if rc != OK:
            raise OracleError(rc, "or_refactor64 failed: %d at column %d" % (rc, bad.value))
        return Lx, Ux, ng.value

    def refactor32(self, rowptr, colidx, values, guard_policy=0):
        rp, ci, v = _csr(rowptr, colidx, values)
        Lx = np.empty(self.lnz, np.float32)
        Ux = np.empty(self.unz, np.float32)
        ng, bad = C.c_int64(), C.c_int64()
        rc = lib().or_refactor32(self._h, _p(rp, C.c_int64), _p(ci, C.c_int32), _p(v, C.c_double),
                                 int(guard_policy), _p(Lx, C.c_float), _p(Ux, C.c_float),
                                 C.byref(ng), C.byref(bad))
        if rc != OK:
            raise OracleError(rc, "or_refactor32 failed: %d at column %d" % (rc, bad.value))
        return Lx, Ux, ng.value

    def solve(self, b, Lx=None, Ux=None):
        """x = Q U^-1 L^-1 P b with the given (default: own) FP64 factor values."""
        b = np.ascontiguousarray(b, np.float64)
        Lx = self.Lx if Lx is None else np.ascontiguousarray(Lx, np.float64)
        Ux = self.Ux if Ux is None else np.ascontiguousarray(Ux, np.float64)
        x = np.empty(self.n)
        lib().or_solve_with(self._h, _p(Lx, C.c_double), _p(Ux, C.c_double), _p(b, C.c_double),
                            _p(x, C.c_double))
        return x

    def solve32(self, b, Lx32, Ux32):
        b = np.ascontiguousarray(b, np.float64)
        Lx32 = np.ascontiguousarray(Lx32, np.float32)
        Ux32 = np.ascontiguousarray(Ux32, np.float32)
        x = np.empty(self.n)
        lib().or_solve_with32(self._h, _p(Lx32, C.c_float), _p(Ux32, C.c_float), _p(b, C.c_double),
                              _p(x, C.c_double))
        return x

    def condest(self, rowptr, values):
        rp = np.ascontiguousarray(rowptr, np.int64)
        v = np.ascontiguousarray(values, np.float64)
        return lib().or_condest(self._h, _p(rp, C.c_int64), _p(v, C.c_double))

    def fgmres_ir(self, rowptr, colidx, values, b, Lx=None, Ux=None, Lx32=None, Ux32=None,
                  restart=10, max_restarts=20, eta=1e-12, mode=0, hist_cap=4096, residual="fp64",
                  gs="cgs2", keep_best=True):
        """FGMRES-IR with these factors as right preconditioner (see or_fgmres_ir);
        residual="dd" forms every residual in extended precision (or_residual_dd);
        gs="dcgs2" runs the Arnoldi steps with delayed CGS2 (one reduction per step);
        keep_best=False returns the last iterate of a refinement that does not converge
        instead of the one with the lowest true residual."""
        if residual not in ("fp64", "dd"):
            raise ValueError("residual must be 'fp64' or 'dd'")
        if residual == "dd":
            mode = int(mode) | 2
        if gs not in ("cgs2", "dcgs2"):
            raise ValueError("gs must be 'cgs2' or 'dcgs2'")
        if gs == "dcgs2":
            mode = int(mode) | 4
        if not keep_best:
            mode = int(mode) | 8
        rp, ci, v = _csr(rowptr, colidx, values)
        b = np.ascontiguousarray(b, np.float64)
        prec = 1 if Lx32 is not None else 0
        Lx = self.Lx if Lx is None else np.ascontiguousarray(Lx, np.float64)
        Ux = self.Ux if Ux is None else np.ascontiguousarray(Ux, np.float64)
        l32 = np.zeros(1, np.float32) if Lx32 is None else np.ascontiguousarray(Lx32, np.float32)
        u32 = np.zeros(1, np.float32) if Ux32 is None else np.ascontiguousarray(Ux32, np.float32)
        x = np.empty(self.n)
        info = np.zeros(9)
        hist = np.zeros(hist_cap)
        lib().or_fgmres_ir(self._h, _p(Lx, C.c_double), _p(Ux, C.c_double), _p(l32, C.c_float),
                           _p(u32, C.c_float), prec, _p(rp, C.c_int64), _p(ci, C.c_int32),
                           _p(v, C.c_double), _p(b, C.c_double), _p(x, C.c_double), int(restart),
                           int(max_restarts), float(eta), int(mode), _p(info, C.c_double),
                           _p(hist, C.c_double), hist_cap)
        it = int(info[0])
        return x, dict(iters=it, cycles=int(info[1]), nrbe=info[2], rr=info[3],
                       converged=bool(info[4]), nrbe0=info[5], est=info[6], true_resid=info[7],
                       applications=int(info[8]), hist=hist[:min(it, hist_cap)].copy())

    def arnoldi(self, rowptr, colidx, values, r0, restart, gs="cgs2", Lx=None, Ux=None, Lx32=None, Ux32=None):
        """One FGMRES Arnoldi cycle from r0 run to `restart` steps (see or_arnoldi); with
        Lx32/Ux32 the preconditioner is the binary32 solve with those FP32 factors.
        Returns (V, Z, Hbar, k): columns of V and Z are basis vectors, Hbar is unrotated."""
        if gs not in ("cgs2", "dcgs2"):
            raise ValueError("gs must be 'cgs2' or 'dcgs2'")
        rp, ci, v = _csr(rowptr, colidx, values)
        Lx = self.Lx if Lx is None else np.ascontiguousarray(Lx, np.float64)
        Ux = self.Ux if Ux is None else np.ascontiguousarray(Ux, np.float64)
        prec = 1 if Lx32 is not None else 0
        l32 = np.zeros(1, np.float32) if Lx32 is None else np.ascontiguousarray(Lx32, np.float32)
        u32 = np.zeros(1, np.float32) if Ux32 is None else np.ascontiguousarray(Ux32, np.float32)
        r0 = np.ascontiguousarray(r0, np.float64)
        R = int(restart)
        V = np.zeros((R + 1, self.n))
        Z = np.zeros((R, self.n))
        H = np.zeros((R, R + 1))
        k = lib().or_arnoldi(self._h, _p(Lx, C.c_double), _p(Ux, C.c_double), _p(l32, C.c_float),
                             _p(u32, C.c_float), prec, _p(rp, C.c_int64),
                             _p(ci, C.c_int32), _p(v, C.c_double), _p(r0, C.c_double), R,
                             1 if gs == "dcgs2" else 0, _p(V, C.c_double), _p(Z, C.c_double),
                             _p(H, C.c_double))
        if k < 0:
            raise MemoryError("or_arnoldi failed")
        return V.T, Z.T, H.T, k

    # step-indexed views (rows of P K Q), used to compare layouts
    def L_step_csc(self):
        """L as CSC with row indices converted to pivot steps (strictly lower)."""
        return self.Lp, self.pinv[self.Li], self.Lx


def residual(rowptr, colidx, values, x, b, precision="fp64"):
    """rho = b - K x; precision "dd" carries each row in double-double (or_residual_dd)."""
    rp, ci, v = _csr(rowptr, colidx, values)
    x = np.ascontiguousarray(x, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    r = np.empty(rp.size - 1)
    if precision not in ("fp64", "dd"):
        raise ValueError("precision must be 'fp64' or 'dd'")
    fn = lib().or_residual_dd if precision == "dd" else lib().or_residual
    fn(rp.size - 1, _p(rp, C.c_int64), _p(ci, C.c_int32), _p(v, C.c_double),
       _p(x, C.c_double), _p(b, C.c_double), _p(r, C.c_double))
    return r


def metrics(rowptr, colidx, values, x, b) -> dict:
    """NRBE (eq. (nbre)), NSR, norms and ||rho||/||b|| of a candidate solution."""
    rp, ci, v = _csr(rowptr, colidx, values)
    x = np.ascontiguousarray(x, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    out = np.zeros(7)
    lib().or_metrics(rp.size - 1, _p(rp, C.c_int64), _p(ci, C.c_int32), _p(v, C.c_double),
                     _p(x, C.c_double), _p(b, C.c_double), _p(out, C.c_double))
    return dict(nrbe=out[0], nsr=out[1], resid=out[2], knorm=out[3], xnorm=out[4], bnorm=out[5],
                rel_resid=out[6])


def norm_inf(rowptr, values) -> float:
    rp = np.ascontiguousarray(rowptr, np.int64)
    v = np.ascontiguousarray(values, np.float64)
    return lib().or_norm_inf_mat(rp.size - 1, _p(rp, C.c_int64), _p(v, C.c_double))


def direct_solve(rowptr, colidx, values, b, Q, tau=1e-10):
    """Plain direct method (fresh pivoting with threshold tau, ordering reused): the CPU
    baseline solve.  The default tau = 1e-10 keeps the diagonal pivots of a quasi-definite
    K (the library's default); tau = 0.1 is textbook threshold partial pivoting."""
    f = LU(rowptr, colidx, values, Q=Q, tau=tau)
    return f.solve(b), f


def _richardson_bind():
    L = lib()
    if not getattr(L, "_rich_bound", False):
        i64, i32p, i64p, f64p = C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_double)
        L.or_richardson.argtypes = [C.c_void_p, f64p, f64p, i64p, i32p, f64p, f64p, f64p, C.c_int, C.c_double,
                                    C.c_double, C.c_int, C.c_double, f64p, f64p, i64]
        L._rich_bound = True
    return L


def richardson(f: LU, rowptr, colidx, values, b, Lx=None, Ux=None, max_it=50, tol=1e-14, ratio=0.5,
               inner_restart=0, inner_tol=1e-2, hist_cap=256):
    """Richardson iterative refinement with these factors (or_richardson in oracle.c);
    inner_restart > 0 solves each correction with FGMRES on the error system."""
    L = _richardson_bind()
    rp, ci, v = _csr(rowptr, colidx, values)
    b = np.ascontiguousarray(b, np.float64)
    Lx = f.Lx if Lx is None else np.ascontiguousarray(Lx, np.float64)
    Ux = f.Ux if Ux is None else np.ascontiguousarray(Ux, np.float64)
    x = np.empty(f.n)
    info = np.zeros(6)
    hist = np.zeros(hist_cap)
    L.or_richardson(f._h, _p(Lx, C.c_double), _p(Ux, C.c_double), _p(rp, C.c_int64), _p(ci, C.c_int32),
                    _p(v, C.c_double), _p(b, C.c_double), _p(x, C.c_double), int(max_it), float(tol),
                    float(ratio), int(inner_restart), float(inner_tol), _p(info, C.c_double),
                    _p(hist, C.c_double), hist_cap)
    it = int(info[0])
    return x, dict(corrections=it, applications=int(info[1]), nsr=info[2], nrbe=info[3],
                   converged=bool(info[4]), rr=info[5], hist=hist[:min(it, hist_cap)].copy())
