"""Thin Python binding of the C ABI in include/rqrcp.h.

Argument marshalling only: every step runs in the gfx950 kernels of
``librqrcp.so``.  PyTorch provides device memory (inputs, outputs and the
workspace) and the current HIP stream.  Matrices are float64 CUDA tensors;
the library works on column-major storage, so inputs are converted to a
column-major (Fortran-ordered) tensor ``X`` of the same shape, i.e. with
``X.stride() == (1, ld)``.

If the shared library has not been built the import of any entry point
raises: there is no CPU fallback.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librqrcp.so")

(RQ_OP_RQRCP, RQ_OP_TRQRCP, RQ_OP_TUXV, RQ_OP_QR, RQ_OP_SAMPLE_QRCP, RQ_OP_SVD, RQ_OP_RSRQRCP,
 RQ_OP_TUXV_MIXED, RQ_OP_TRQRCP_MIXED) = range(9)
RQ_TUXV_MAX_ITER = 64

_c_i32, _c_i64, _c_u64, _c_sz, _c_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_void_p

_SIGS = {
    "rq_version": ([], ctypes.c_char_p),
    "rq_set_lookahead": ([_c_i32], ctypes.c_int),
    "rq_workspace_bytes": ([_c_i32, _c_i64, _c_i64, _c_i64, _c_i32, _c_i32, ctypes.POINTER(_c_sz)], ctypes.c_int),
    "rq_rqrcp": ([_c_p, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_u64, _c_p, _c_p, _c_p, _c_sz, _c_p],
                 ctypes.c_int),
    "rq_rqrcp_omega": ([_c_p, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_p, _c_i64, _c_p, _c_p, _c_p, _c_sz,
                        _c_p], ctypes.c_int),
    "rq_rsrqrcp": ([_c_p, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_u64, _c_p, _c_p, _c_p, _c_sz, _c_p],
                   ctypes.c_int),
    "rq_tuxv_mixed": ([_c_p, _c_i64, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_u64, _c_p, _c_i64, _c_p, _c_p,
                       _c_i64, _c_p, _c_sz, _c_p], ctypes.c_int),
    "rq_tuxv_iter": ([_c_p, _c_i64, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_u64, _c_i32, _c_p, _c_i64, _c_p,
                      _c_p, _c_i64, _c_p, _c_sz, _c_p], ctypes.c_int),
    "rq_trqrcp": ([_c_p, _c_i64, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_u64, _c_p, _c_p, _c_p, _c_sz,
                   _c_p], ctypes.c_int),
    "rq_trqrcp_mixed": ([_c_p, _c_i64, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_u64, _c_p, _c_p, _c_p,
                         _c_sz, _c_p], ctypes.c_int),
    "rq_trqrcp_omega": ([_c_p, _c_i64, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_p, _c_i64, _c_p, _c_p, _c_p,
                         _c_sz, _c_p], ctypes.c_int),
    "rq_tuxv": ([_c_p, _c_i64, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_u64, _c_p, _c_i64, _c_p, _c_p,
                 _c_i64, _c_p, _c_sz, _c_p], ctypes.c_int),
    "rq_tuxv_omega": ([_c_p, _c_i64, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_p, _c_i64, _c_p, _c_i64,
                       _c_p, _c_p, _c_i64, _c_p, _c_sz, _c_p], ctypes.c_int),
    "rq_unpivoted_qr": ([_c_p, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_p, _c_p, _c_sz, _c_p], ctypes.c_int),
    "rq_omega": ([_c_p, _c_u64, _c_i64, _c_i64, _c_p, _c_i64], ctypes.c_int),
    "rq_sketch": ([_c_p, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_u64, _c_p, _c_i64, _c_p, _c_sz], ctypes.c_int),
    "rq_sample_qrcp": ([_c_p, _c_i32, _c_i64, _c_i32, _c_p, _c_i64, _c_p, _c_p, _c_sz, _c_p], ctypes.c_int),
    "rq_small_svd": ([_c_p, _c_i32, _c_p, _c_i64, _c_p, _c_i64, _c_p, _c_p, _c_i64, _c_p, _c_sz], ctypes.c_int),
    "rq_profile_start": ([], ctypes.c_int),
    "rq_profile_stop": ([], ctypes.c_int),
    "rq_profile_select": ([ctypes.c_uint32], ctypes.c_int),
    "rq_profile_get": ([_c_i32, ctypes.POINTER(_c_i64), ctypes.POINTER(ctypes.c_double),
                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "rq_profile_name": ([_c_i32], ctypes.c_char_p),
    "rq_profile_classes": ([], ctypes.c_int32),
}

_lib = None


def load():
    """Load librqrcp.so (raises if it is missing) and declare the signatures."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1509_06820_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


class RQError(RuntimeError):
    pass


def _check(rc, name):
    if rc != 0:
        raise RQError(f"{name} returned {rc}")


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def fortran(A):
    """Column-major float64 CUDA copy (or A itself if it already is one)."""
    if A.dtype != torch.float64 or not A.is_cuda:
        raise TypeError("expected a float64 CUDA tensor")
    if A.dim() != 2:
        raise ValueError("expected a matrix")
    m, n = A.shape
    if A.stride(0) == 1 and (n <= 1 or A.stride(1) >= max(1, m)):
        return A
    return A.t().contiguous().t()


def _ld(X):
    m, n = X.shape
    return max(1, X.stride(1)) if n > 1 else max(1, m)


def rq_workspace_bytes(op, m, n, k, b, p):
    out = _c_sz(0)
    _check(load().rq_workspace_bytes(op, m, n, k, b, p, ctypes.byref(out)), "rq_workspace_bytes")
    return out.value


def workspace(op, m, n, k, b, p, device):
    nbytes = rq_workspace_bytes(op, m, n, k, b, p)
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def rq_rqrcp(A, b, p, seed=0, Omega=None, work=None, stream=None):
    """Alg. 4.  Returns (F, tau, jpvt, info): F = R above/on the diagonal and
    reflectors below (column-major m x n); A is not modified."""
    F = fortran(A).clone()
    m, n = F.shape
    k = min(m, n)
    dev = F.device
    jpvt = torch.empty(n, dtype=torch.int64, device=dev)
    tau = torch.empty(k, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    if work is None:
        work = workspace(RQ_OP_RQRCP, m, n, k, b, p, dev)
    L = load()
    if Omega is None:
        rc = L.rq_rqrcp(_stream(stream), m, n, _ptr(F), _ld(F), b, p, seed, _ptr(jpvt), _ptr(tau), _ptr(work),
                        work.numel(), _ptr(info))
        _check(rc, "rq_rqrcp")
    else:
        Om = fortran(Omega)
        rc = L.rq_rqrcp_omega(_stream(stream), m, n, _ptr(F), _ld(F), b, p, _ptr(Om), _ld(Om), _ptr(jpvt), _ptr(tau),
                              _ptr(work), work.numel(), _ptr(info))
        _check(rc, "rq_rqrcp_omega")
    return F, tau, jpvt, info


def rq_rsrqrcp(A, b, p, seed=0, work=None, stream=None):
    """Alg. 5 (a new compression matrix and sample per block).  Returns
    (F, tau, jpvt, info) in the layout of rq_rqrcp; A is not modified."""
    F = fortran(A).clone()
    m, n = F.shape
    k = min(m, n)
    dev = F.device
    jpvt = torch.empty(n, dtype=torch.int64, device=dev)
    tau = torch.empty(k, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    if work is None:
        work = workspace(RQ_OP_RSRQRCP, m, n, k, b, p, dev)
    rc = load().rq_rsrqrcp(_stream(stream), m, n, _ptr(F), _ld(F), b, p, seed, _ptr(jpvt), _ptr(tau), _ptr(work),
                           work.numel(), _ptr(info))
    _check(rc, "rq_rsrqrcp")
    return F, tau, jpvt, info


def rq_trqrcp(A, k, b, p, seed=0, Omega=None, work=None, stream=None, mixed=False):
    """Alg. 6.  Returns (F, tau, jpvt, info) (layout as in include/rqrcp.h).
    mixed: rq_trqrcp_mixed (FP32 sketch and Y2^T A; no Omega argument)."""
    F = fortran(A).clone()
    m, n = F.shape
    dev = F.device
    jpvt = torch.empty(n, dtype=torch.int64, device=dev)
    tau = torch.empty(k, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    if work is None:
        work = workspace(RQ_OP_TRQRCP_MIXED if mixed else RQ_OP_TRQRCP, m, n, k, b, p, dev)
    L = load()
    if mixed:
        if Omega is not None:
            raise ValueError("the mixed-precision TRQRCP draws its own Omega")
        rc = L.rq_trqrcp_mixed(_stream(stream), m, n, k, _ptr(F), _ld(F), b, p, seed, _ptr(jpvt), _ptr(tau),
                               _ptr(work), work.numel(), _ptr(info))
        _check(rc, "rq_trqrcp_mixed")
    elif Omega is None:
        rc = L.rq_trqrcp(_stream(stream), m, n, k, _ptr(F), _ld(F), b, p, seed, _ptr(jpvt), _ptr(tau), _ptr(work),
                         work.numel(), _ptr(info))
        _check(rc, "rq_trqrcp")
    else:
        Om = fortran(Omega)
        rc = L.rq_trqrcp_omega(_stream(stream), m, n, k, _ptr(F), _ld(F), b, p, _ptr(Om), _ld(Om), _ptr(jpvt),
                               _ptr(tau), _ptr(work), work.numel(), _ptr(info))
        _check(rc, "rq_trqrcp_omega")
    return F, tau, jpvt, info


def rq_tuxv(A, k, b, p, seed=0, Omega=None, work=None, stream=None, jmax=1, mixed=False):
    """Alg. 7 + SVD of X.  Returns (U, sigma, VT, info).  jmax > 1 (seeded
    Omega only) runs the further LQ/QR steps through rq_tuxv_iter; mixed=True
    (j_max = 1, seeded Omega) the mixed-precision path rq_tuxv_mixed."""
    Af = fortran(A)
    m, n = Af.shape
    dev = Af.device
    U = torch.empty((k, m), dtype=torch.float64, device=dev).t()  # column-major m x k
    VT = torch.empty((n, k), dtype=torch.float64, device=dev).t()  # column-major k x n
    sigma = torch.empty(k, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    if work is None:
        work = workspace(RQ_OP_TUXV_MIXED if mixed else RQ_OP_TUXV, m, n, k, b, p, dev)
    L = load()
    if mixed:
        if Omega is not None or jmax != 1:
            raise ValueError("the mixed-precision path takes j_max = 1 and the seeded compression matrix")
        rc = L.rq_tuxv_mixed(_stream(stream), m, n, k, _ptr(Af), _ld(Af), b, p, seed, _ptr(U), m, _ptr(sigma),
                             _ptr(VT), k, _ptr(work), work.numel(), _ptr(info))
        _check(rc, "rq_tuxv_mixed")
    elif jmax != 1:
        if Omega is not None:
            raise ValueError("jmax > 1 takes the seeded compression matrix")
        rc = L.rq_tuxv_iter(_stream(stream), m, n, k, _ptr(Af), _ld(Af), b, p, seed, jmax, _ptr(U), m, _ptr(sigma),
                            _ptr(VT), k, _ptr(work), work.numel(), _ptr(info))
        _check(rc, "rq_tuxv_iter")
    elif Omega is None:
        rc = L.rq_tuxv(_stream(stream), m, n, k, _ptr(Af), _ld(Af), b, p, seed, _ptr(U), m, _ptr(sigma), _ptr(VT), k,
                       _ptr(work), work.numel(), _ptr(info))
        _check(rc, "rq_tuxv")
    else:
        Om = fortran(Omega)
        rc = L.rq_tuxv_omega(_stream(stream), m, n, k, _ptr(Af), _ld(Af), b, p, _ptr(Om), _ld(Om), _ptr(U), m,
                             _ptr(sigma), _ptr(VT), k, _ptr(work), work.numel(), _ptr(info))
        _check(rc, "rq_tuxv_omega")
    return U, sigma, VT, info


def rq_unpivoted_qr(A, b, work=None, stream=None):
    """Unpivoted blocked Householder QR.  Returns (F, tau, info)."""
    F = fortran(A).clone()
    m, n = F.shape
    k = min(m, n)
    dev = F.device
    tau = torch.empty(k, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    if work is None:
        work = workspace(RQ_OP_QR, m, n, k, b, 0, dev)
    rc = load().rq_unpivoted_qr(_stream(stream), m, n, _ptr(F), _ld(F), b, _ptr(tau), _ptr(work), work.numel(),
                                _ptr(info))
    _check(rc, "rq_unpivoted_qr")
    return F, tau, info


def rq_omega(seed, l, m, device="cuda", stream=None):
    Om = torch.empty((m, l), dtype=torch.float64, device=device).t()  # column-major l x m
    _check(load().rq_omega(_stream(stream), seed, l, m, _ptr(Om), l), "rq_omega")
    return Om


def rq_sketch(A, l, seed, work=None, stream=None):
    Af = fortran(A)
    m, n = Af.shape
    B = torch.empty((n, l), dtype=torch.float64, device=Af.device).t()
    if work is None:
        work = workspace(RQ_OP_RQRCP, m, n, min(m, n), l, 0, Af.device)
    _check(load().rq_sketch(_stream(stream), m, n, _ptr(Af), _ld(Af), l, seed, _ptr(B), l, _ptr(work), work.numel()),
           "rq_sketch")
    return B


def rq_sample_qrcp(B, bsteps, work=None, stream=None):
    """Partial QRCP of a sample.  Returns (S, piv, info); piv are sequential swaps."""
    S = fortran(B).clone()
    l, n = S.shape
    piv = torch.empty(bsteps, dtype=torch.int32, device=S.device)
    info = torch.zeros(1, dtype=torch.int32, device=S.device)
    if work is None:
        work = workspace(RQ_OP_SAMPLE_QRCP, l, n, 0, bsteps, 0, S.device)
    _check(load().rq_sample_qrcp(_stream(stream), l, n, bsteps, _ptr(S), _ld(S), _ptr(piv), _ptr(work), work.numel(),
                                 _ptr(info)), "rq_sample_qrcp")
    return S, piv, info


def rq_small_svd(X, work=None, stream=None):
    """One-sided Jacobi SVD of a square matrix.  Returns (U, sigma, V)."""
    Xw = fortran(X).clone()
    k = Xw.shape[0]
    U = torch.empty((k, k), dtype=torch.float64, device=Xw.device).t()
    V = torch.empty((k, k), dtype=torch.float64, device=Xw.device).t()
    sig = torch.empty(k, dtype=torch.float64, device=Xw.device)
    if work is None:
        work = workspace(RQ_OP_SVD, k, k, k, 1, 0, Xw.device)
    _check(load().rq_small_svd(_stream(stream), k, _ptr(Xw), _ld(Xw), _ptr(U), k, _ptr(sig), _ptr(V), k, _ptr(work),
                               work.numel()), "rq_small_svd")
    return U, sig, V


def rq_set_lookahead(on):
    """Turn RQRCP's look-ahead trailing update on or off; returns the previous setting."""
    return bool(load().rq_set_lookahead(1 if on else 0))


def rq_profile_start(stages=None):
    """Start stage timing; `stages` (names) limits the events to those stages."""
    L = load()
    mask = 0xFFFFFFFF
    if stages is not None:
        names = [L.rq_profile_name(c).decode() for c in range(L.rq_profile_classes())]
        mask = 0
        for nm in stages:
            mask |= 1 << names.index(nm)
    _check(L.rq_profile_select(mask), "rq_profile_select")
    _check(L.rq_profile_start(), "rq_profile_start")


def rq_profile_stop():
    """Stop stage timing; returns {name: dict(count, ms, bytes, flops)}."""
    L = load()
    _check(L.rq_profile_stop(), "rq_profile_stop")
    out = {}
    for c in range(L.rq_profile_classes()):
        cnt, ms, by, fl = _c_i64(0), ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
        _check(L.rq_profile_get(c, ctypes.byref(cnt), ctypes.byref(ms), ctypes.byref(by), ctypes.byref(fl)),
               "rq_profile_get")
        if cnt.value:
            out[L.rq_profile_name(c).decode()] = dict(count=cnt.value, ms=ms.value, bytes=by.value, flops=fl.value)
    return out


# short aliases
rqrcp = rq_rqrcp
rsrqrcp = rq_rsrqrcp
trqrcp = rq_trqrcp
tuxv = rq_tuxv
unpivoted_qr = rq_unpivoted_qr
