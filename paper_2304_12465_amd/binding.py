"""ctypes binding of libkrr.so (the C ABI declared in include/krr.h).

Argument marshalling only: torch tensors provide device memory (their
``data_ptr``) and the current HIP stream; every step of the method runs in
the library's kernels.  The library must be built (``__graft_entry__.build``
or ``python paper_2304_12465_amd/_build.py``); loading fails loudly otherwise.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkrr.so")

GAUSSIAN, LAPLACE = 0, 1
FP64, FP32, MIXED = 0, 1, 2
PIVOT_RPCHOL, PIVOT_UNIFORM, PIVOT_GREEDY = 0, 1, 2
NOT_CONVERGED = 1
ERRORS = {-1: "EINVAL", -2: "EWORKSPACE", -3: "ENOTSPD", -4: "ENAN", -5: "EHIP"}

_lib = None
_c = ctypes
_i32, _i64, _u64, _dbl, _vp, _sz = _c.c_int32, _c.c_int64, _c.c_uint64, _c.c_double, _c.c_void_p, _c.c_size_t
_szp = _c.POINTER(_c.c_size_t)

class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged_cols", ctypes.c_int32),
                ("relres_recursive", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("build_seconds", ctypes.c_double), ("solve_seconds", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int32),
                ("history_len", ctypes.c_int32), ("products", ctypes.c_int32)]


_pp = ctypes.POINTER(ctypes.c_void_p)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)

_SIGS = {
    "krr_last_error": ([], _c.c_char_p),
    "krr_timing_enable": ([_i32], _i32),
    "krr_timing_read": ([ctypes.POINTER(ctypes.c_double), _i64p], _i32),
    "krr_timing_read_vectors": ([_i32, ctypes.POINTER(ctypes.c_double), _i64p,
                                 ctypes.POINTER(ctypes.c_double), _i64p], _i32),
    "krr_rpchol_ws": ([_i32, _i32, _i64, _i32, _i32, _i32, _i32, _szp], _i32),
    "krr_rpchol_build": ([_i32, _dbl, _i32, _vp, _i64, _i32, _dbl, _i32, _i32, _u64, _i32, _vp,
                          _sz, _pp, _vp], _i32),
    "krr_nystrom_build": ([_i32, _dbl, _i32, _vp, _i64, _i32, _dbl, _i32, _i32, _u64, _i32, _i32,
                           _vp, _sz, _pp, _vp], _i32),
    "krr_restricted_direct_ws": ([_i32, _i64, _i32, _i32, _i32, _szp], _i32),
    "krr_restricted_direct": ([_i32, _dbl, _vp, _i64, _i32, _dbl, _vp, _i32, _vp, _i32, _vp, _vp,
                               _sz, _vp], _i32),
    "krr_rpchol_factor": ([_vp, _vp, _vp], _i32),
    "krr_krill_ws": ([_i32, _i32, _i64, _i32, _i32, _i32, _i32, _i32, _szp], _i32),
    "krr_krill_build": ([_i32, _dbl, _i32, _vp, _i64, _i32, _dbl, _vp, _i32, _i32, _i32, _u64,
                         _i32, _vp, _sz, _pp, _vp], _i32),
    "krr_krill_stored_ws": ([_i32, _i32, _i64, _i32, _i32, _i32, _i32, _i32, _szp], _i32),
    "krr_krill_build_stored": ([_i32, _dbl, _i32, _vp, _i64, _i32, _dbl, _vp, _i32, _i32, _i32,
                                _u64, _i32, _vp, _sz, _pp, _vp], _i32),
    "krr_krill_export": ([_vp, _i32, _vp, _sz, _vp], _i32),
    "krr_precond_dims": ([_vp, _i32p, _i64p], _i32),
    "krr_precond_pivots": ([_vp, _i64p, _i32, _i32p], _i32),
    "krr_precond_apply": ([_vp, _vp, _i32, _vp, _vp], _i32),
    "krr_precond_operator": ([_vp, _vp, _i32, _vp, _vp], _i32),
    "krr_precond_free": ([_vp], None),
    "krr_solve_begin": ([_vp, _vp, _i32, _dbl, _i32, _pp, _vp], _i32),
    "krr_solve_step": ([_pp, _i32, _i32p, _vp], _i32),
    "krr_solve_end": ([_vp, _vp, ctypes.POINTER(SolveInfo), _vp], _i32),
    "krr_solve_free": ([_vp], None),
    "krr_pcg_solve": ([_vp, _vp, _i32, _dbl, _i32, _vp, ctypes.POINTER(SolveInfo), _vp], _i32),
    "krr_predict_ws": ([_vp, _i32, _i64, _i32, _szp], _i32),
    "krr_predict": ([_vp, _i32, _vp, _vp, _i64, _vp, _i32, _vp, _vp, _sz, _vp], _i32),
    "krr_kernel_matvec_ws": ([_i32, _i64, _i64, _i32, _i32, _szp], _i32),
    "krr_kernel_matvec": ([_i32, _dbl, _i32, _vp, _i64, _vp, _i64, _i32, _vp, _i32, _dbl, _vp,
                           _vp, _sz, _vp], _i32),
    "krr_kernel_matvec_noalloc": ([_i32, _dbl, _i32, _vp, _i64, _vp, _i64, _i32, _vp, _i32,
                                   _dbl, _vp, _vp], _i32),
}


class KrrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"krr error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


def lib():
    """Loads libkrr.so once; raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def declared_symbols():
    return list(_SIGS)


def check(rc):
    if rc < 0:
        raise KrrError(rc, lib().krr_last_error().decode())
    return rc


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def workspace(nbytes, device):
    """A caller-owned workspace buffer (256-byte aligned torch storage)."""
    ws = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + max(int(nbytes), 256)]


def _f64(t):
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return t


def kernel_matvec_ws(prec, nr, nc, d, m):
    b = ctypes.c_size_t(0)
    check(lib().krr_kernel_matvec_ws(prec, nr, nc, d, m, ctypes.byref(b)))
    return b.value


def kernel_matvec(kind, sigma, prec, Xr, Xc, V, shift=0.0, out=None, ws=None):
    """W = K(Xr, Xc) V + shift V on the GPU (all float64 device tensors)."""
    _f64(Xr), _f64(Xc), _f64(V)
    squeeze = V.dim() == 1
    V2 = V.reshape(-1, 1) if squeeze else V
    nr, d = Xr.shape
    nc = Xc.shape[0]
    m = V2.shape[1]
    W = out if out is not None else torch.empty((nr, m), dtype=torch.float64, device=Xr.device)
    if ws is None:
        ws = workspace(kernel_matvec_ws(prec, nr, nc, d, m), Xr.device)
    check(lib().krr_kernel_matvec(kind, float(sigma), prec, _ptr(Xr), nr, _ptr(Xc), nc, d,
                                  _ptr(V2), m, float(shift), _ptr(W), _ptr(ws), ws.numel(),
                                  _stream(Xr.device)))
    return W.reshape(-1) if squeeze else W


def kernel_matvec_noalloc(kind, sigma, prec, Xr, Xc, V, shift=0.0, out=None):
    """W = K(Xr, Xc) V + shift V through the allocation-free entry point (the
    library's fixed device scratch; `out` may be preallocated)."""
    _f64(Xr), _f64(Xc), _f64(V)
    squeeze = V.dim() == 1
    V2 = V.reshape(-1, 1) if squeeze else V
    nr, d = Xr.shape
    nc = Xc.shape[0]
    m = V2.shape[1]
    W = out if out is not None else torch.empty((nr, m), dtype=torch.float64, device=Xr.device)
    check(lib().krr_kernel_matvec_noalloc(kind, float(sigma), prec, _ptr(Xr), nr, _ptr(Xc), nc,
                                          d, _ptr(V2), m, float(shift), _ptr(W),
                                          _stream(Xr.device)))
    return W.reshape(-1) if squeeze else W


class Precond:
    """A built preconditioner: owns its workspace tensor and keeps X alive."""

    def __init__(self, handle, ws, X, m_max, kind):
        self.h = handle
        self.ws = ws
        self.X = X
        self.m_max = m_max
        self.kind = kind
        self.device = X.device

    def __del__(self):
        try:
            if self.h:
                lib().krr_precond_free(self.h)
                self.h = None
        except Exception:
            pass

    def dims(self):
        r = ctypes.c_int32(0)
        n = ctypes.c_int64(0)
        check(lib().krr_precond_dims(self.h, ctypes.byref(r), ctypes.byref(n)))
        return r.value, n.value

    def pivots(self):
        cnt = ctypes.c_int32(0)
        check(lib().krr_precond_pivots(self.h, None, 0, ctypes.byref(cnt)))
        buf = (ctypes.c_int64 * max(cnt.value, 1))()
        check(lib().krr_precond_pivots(self.h, buf, cnt.value, ctypes.byref(cnt)))
        return [int(buf[i]) for i in range(cnt.value)]

    def _block(self, Z):
        _f64(Z)
        return Z.reshape(-1, 1) if Z.dim() == 1 else Z

    def apply(self, Z):
        """P^{-1} Z (n x m)."""
        Z2 = self._block(Z)
        out = torch.empty_like(Z2)
        check(lib().krr_precond_apply(self.h, _ptr(Z2), Z2.shape[1], _ptr(out), _stream(self.device)))
        return out.reshape(Z.shape)

    def operator(self, V):
        """M V with the system operator (n x m)."""
        V2 = self._block(V)
        out = torch.empty_like(V2)
        check(lib().krr_precond_operator(self.h, _ptr(V2), V2.shape[1], _ptr(out),
                                         _stream(self.device)))
        return out.reshape(V.shape)

    def factor(self):
        """F^T (rank x N) of an RPCholesky preconditioner."""
        r, _ = self.dims()
        FT = torch.empty((r, self.X.shape[0]), dtype=torch.float64, device=self.device)
        check(lib().krr_rpchol_factor(self.h, _ptr(FT), _stream(self.device)))
        return FT

    def predict(self, Xtest, beta, prec=0, ws=None):
        """f(Xtest) of the solved model: K(Xtest, X) beta (full data) or
        K(Xtest, X(S,:)) beta (restricted), ntest x m."""
        _f64(Xtest)
        B2 = self._block(beta)
        nt, m = Xtest.shape[0], B2.shape[1]
        # the C call reads ntest x d and n x m: check the tensors hold that
        if Xtest.dim() != 2 or Xtest.shape[1] != self.X.shape[1]:
            raise ValueError(f"Xtest must be ntest x {self.X.shape[1]}")
        if B2.shape[0] != self.dims()[1]:
            raise ValueError(f"beta must have {self.dims()[1]} rows")
        if ws is None:
            b = ctypes.c_size_t(0)
            check(lib().krr_predict_ws(self.h, int(prec), nt, m, ctypes.byref(b)))
            ws = workspace(b.value, self.device)
        out = torch.empty((nt, m), dtype=torch.float64, device=self.device)
        check(lib().krr_predict(self.h, int(prec), _ptr(self.X), _ptr(Xtest), nt, _ptr(B2), m,
                                _ptr(out), _ptr(ws), ws.numel(), _stream(self.device)))
        return out.reshape(-1) if beta.dim() == 1 else out

    def solve(self, Y, tol, max_iter=1000, history=0):
        """PCG; returns (beta, info dict).  Y: N x m targets."""
        Y2 = self._block(Y)
        r, n = self.dims()
        beta = torch.empty((n, Y2.shape[1]), dtype=torch.float64, device=self.device)
        info = SolveInfo()
        hist = None
        if history:
            hist = (ctypes.c_double * history)()
            info.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
            info.history_cap = history
        rc = check(lib().krr_pcg_solve(self.h, _ptr(Y2), Y2.shape[1], float(tol), int(max_iter),
                                       _ptr(beta), ctypes.byref(info), _stream(self.device)))
        d = dict(iters=info.iters, converged_cols=info.converged_cols,
                 relres_recursive=info.relres_recursive, relres_true=info.relres_true,
                 build_seconds=info.build_seconds, solve_seconds=info.solve_seconds,
                 products=info.products, converged=(rc == 0))
        if hist is not None:
            d["history"] = [hist[i] for i in range(info.history_len)]
        return (beta.reshape(-1) if Y.dim() == 1 else beta), d


def rpchol_ws(kind, prec, N, d, r, B=0, m_max=1):
    b = ctypes.c_size_t(0)
    check(lib().krr_rpchol_ws(kind, prec, N, d, r, B, m_max, ctypes.byref(b)))
    return b.value


def rpchol_build(kind, sigma, prec, X, mu, r, B=0, seed=0, m_max=1, ws=None):
    """Blocked RPCholesky preconditioner for (A + mu I) beta = y."""
    _f64(X)
    N, d = X.shape
    if ws is None:
        ws = workspace(rpchol_ws(kind, prec, N, d, r, B, m_max), X.device)
    h = ctypes.c_void_p(0)
    check(lib().krr_rpchol_build(kind, float(sigma), prec, _ptr(X), N, d, float(mu), int(r),
                                 int(B), ctypes.c_uint64(seed & (2 ** 64 - 1)), int(m_max), _ptr(ws),
                                 ws.numel(), ctypes.byref(h), _stream(X.device)))
    return Precond(h, ws, X, m_max, kind)


def nystrom_build(kind, sigma, prec, X, mu, r, rule, B=0, seed=0, m_max=1, ws=None):
    """Nystrom preconditioner with pivot rule PIVOT_RPCHOL, PIVOT_UNIFORM or
    PIVOT_GREEDY (same workspace as rpchol_build)."""
    _f64(X)
    N, d = X.shape
    if ws is None:
        ws = workspace(rpchol_ws(kind, prec, N, d, r, B, m_max), X.device)
    h = ctypes.c_void_p(0)
    check(lib().krr_nystrom_build(kind, float(sigma), prec, _ptr(X), N, d, float(mu), int(r),
                                  int(B), ctypes.c_uint64(seed & (2 ** 64 - 1)), int(rule),
                                  int(m_max), _ptr(ws), ws.numel(), ctypes.byref(h),
                                  _stream(X.device)))
    return Precond(h, ws, X, m_max, kind)


def restricted_direct(kind, sigma, X, mu, centers, Y, ws=None):
    """beta (k x m) of the restricted system by forming and factoring
    A(S,:)A(:,S) + H in FP64; `centers` is a device int64 tensor."""
    _f64(X)
    _f64(Y)
    if centers.dtype != torch.int64 or not centers.is_contiguous():
        raise TypeError("centers must be a contiguous int64 tensor")
    N, d = X.shape
    Y2 = Y.reshape(-1, 1) if Y.dim() == 1 else Y
    k, m = centers.numel(), Y2.shape[1]
    if ws is None:
        b = ctypes.c_size_t(0)
        check(lib().krr_restricted_direct_ws(kind, N, d, k, m, ctypes.byref(b)))
        ws = workspace(b.value, X.device)
    beta = torch.empty(k, m, dtype=torch.float64, device=X.device)
    check(lib().krr_restricted_direct(kind, float(sigma), _ptr(X), N, d, float(mu), _ptr(centers),
                                      k, _ptr(Y2), m, _ptr(beta), _ptr(ws), ws.numel(),
                                      _stream(X.device)))
    return beta


def timing_enable(on=True):
    check(lib().krr_timing_enable(1 if on else 0))


def timing_read():
    """(total ms, launches) of product tiles since the last read."""
    ms = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    check(lib().krr_timing_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def timing_read_vectors(vectors):
    """(total ms, launches) of product tiles since the last read, and the
    same for the Gaussian matrix-core tiles carrying `vectors` vectors."""
    ms, n = ctypes.c_double(0), ctypes.c_int64(0)
    mms, mn = ctypes.c_double(0), ctypes.c_int64(0)
    check(lib().krr_timing_read_vectors(int(vectors), ctypes.byref(ms), ctypes.byref(n),
                                        ctypes.byref(mms), ctypes.byref(mn)))
    return ms.value, n.value, mms.value, mn.value


def krill_ws(kind, prec, N, d, k, sketch_rows=0, zeta=0, m_max=1):
    b = ctypes.c_size_t(0)
    check(lib().krr_krill_ws(kind, prec, N, d, k, sketch_rows, zeta, m_max, ctypes.byref(b)))
    return b.value


def krill_stored_ws(kind, prec, N, d, k, sketch_rows=0, zeta=0, m_max=1):
    b = ctypes.c_size_t(0)
    check(lib().krr_krill_stored_ws(kind, prec, N, d, k, sketch_rows, zeta, m_max,
                                    ctypes.byref(b)))
    return b.value


def krill_build(kind, sigma, prec, X, mu, k, centers=None, sketch_rows=0, zeta=0, seed=0,
                m_max=1, ws=None, stored=False):
    """KRILL preconditioner for restricted KRR (centres sampled if None);
    stored=True keeps A(:,S) in the workspace (krr_krill_build_stored)."""
    _f64(X)
    N, d = X.shape
    if ws is None:
        q = krill_stored_ws if stored else krill_ws
        ws = workspace(q(kind, prec, N, d, k, sketch_rows, zeta, m_max), X.device)
    if centers is not None and (centers.dtype != torch.int64 or not centers.is_cuda):
        raise ValueError("centers must be an int64 CUDA tensor")
    h = ctypes.c_void_p(0)
    fn = lib().krr_krill_build_stored if stored else lib().krr_krill_build
    check(fn(kind, float(sigma), prec, _ptr(X), N, d, float(mu), _ptr(centers),
             int(k), int(sketch_rows), int(zeta), ctypes.c_uint64(seed & (2 ** 64 - 1)),
             int(m_max), _ptr(ws), ws.numel(), ctypes.byref(h), _stream(X.device)))
    P = Precond(h, ws, X, m_max, kind)
    P.centers_arg = centers
    return P


def krill_export(P, what, shape, dtype):
    out = torch.empty(shape, dtype=dtype, device=P.device)
    check(lib().krr_krill_export(P.h, int(what), _ptr(out), out.numel() * out.element_size(),
                                 _stream(P.device)))
    return out


class Solve:
    """An in-flight stepped PCG solve on a Precond (one per precond)."""

    def __init__(self, P, Y, tol, max_iter=1000):
        self.P = P
        self.Y = P._block(Y)
        self.m = self.Y.shape[1]
        h = ctypes.c_void_p(0)
        check(lib().krr_solve_begin(P.h, _ptr(self.Y), self.m, float(tol), int(max_iter),
                                    ctypes.byref(h), _stream(P.device)))
        self.h = h
        self.state = 0

    def end(self, history=0):
        r, n = self.P.dims()
        beta = torch.empty((n, self.m), dtype=torch.float64, device=self.P.device)
        info = SolveInfo()
        hist = None
        if history:
            hist = (ctypes.c_double * history)()
            info.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
            info.history_cap = history
        h, self.h = self.h, None
        rc = check(lib().krr_solve_end(h, _ptr(beta), ctypes.byref(info), _stream(self.P.device)))
        d = dict(iters=info.iters, converged_cols=info.converged_cols,
                 relres_recursive=info.relres_recursive, relres_true=info.relres_true,
                 build_seconds=info.build_seconds, solve_seconds=info.solve_seconds,
                 products=info.products, converged=(rc == 0))
        if hist is not None:
            d["history"] = [hist[i] for i in range(info.history_len)]
        return beta, d

    def free(self):
        """Abandons the solve (its precond is free for other calls again)."""
        if self.h:
            lib().krr_solve_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def solve_step(solves, device=None):
    """One PCG step for every solve in the list; returns their states."""
    n = len(solves)
    if n == 0:
        return []
    arr = (ctypes.c_void_p * n)(*[s.h.value for s in solves])
    st = (ctypes.c_int32 * n)()
    dev = device or solves[0].P.device
    check(lib().krr_solve_step(ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)), n, st,
                               _stream(dev)))
    out = [int(st[i]) for i in range(n)]
    for s_, v in zip(solves, out):
        s_.state = v
    return out
