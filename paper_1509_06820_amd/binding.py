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
# RQRCP_LIB selects another build of the same ABI (the host-sanitized one)
LIB_PATH = os.environ.get("RQRCP_LIB") or os.path.join(_HERE, "librqrcp.so")

(RQ_OP_RQRCP, RQ_OP_TRQRCP, RQ_OP_TUXV, RQ_OP_QR, RQ_OP_SAMPLE_QRCP, RQ_OP_SVD, RQ_OP_RSRQRCP) = range(7)
RQ_FP64, RQ_MIXED, RQ_MIXED_BF16 = 0, 1, 2
PRECISIONS = {"fp64": RQ_FP64, "mixed": RQ_MIXED, "mixed_bf16": RQ_MIXED_BF16}
RQ_TUXV_MAX_ITER = 64

_c_i32, _c_i64, _c_u64, _c_sz, _c_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_void_p

_SIGS = {
    "rq_version": ([], ctypes.c_char_p),
    "rq_set_lookahead": ([_c_i32], ctypes.c_int),
    "rq_set_panel_path": ([_c_i32], ctypes.c_int),
    "rq_set_block_dump": ([_c_p, _c_i64], ctypes.c_int),
    "rq_workspace_bytes": ([_c_i32, _c_i64, _c_i64, _c_i64, _c_i32, _c_i32, _c_i32, ctypes.POINTER(_c_sz)],
                           ctypes.c_int),
    "rq_rqrcp": ([_c_p, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_u64, _c_i32, _c_p, _c_p, _c_p, _c_sz, _c_p],
                 ctypes.c_int),
    "rq_rqrcp_noalloc": ([_c_p, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_u64, _c_i32, _c_p, _c_p, _c_p],
                         ctypes.c_int),
    "rq_rqrcp_omega": ([_c_p, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_p, _c_i64, _c_p, _c_p, _c_p, _c_sz,
                        _c_p], ctypes.c_int),
    "rq_rsrqrcp": ([_c_p, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_u64, _c_p, _c_p, _c_p, _c_sz, _c_p],
                   ctypes.c_int),
    "rq_tuxv_iter": ([_c_p, _c_i64, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_u64, _c_i32, _c_p, _c_i64, _c_p,
                      _c_p, _c_i64, _c_p, _c_sz, _c_p], ctypes.c_int),
    "rq_trqrcp": ([_c_p, _c_i64, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_u64, _c_i32, _c_p, _c_p, _c_p,
                   _c_sz, _c_p], ctypes.c_int),
    "rq_trqrcp_omega": ([_c_p, _c_i64, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_p, _c_i64, _c_p, _c_p, _c_p,
                         _c_sz, _c_p], ctypes.c_int),
    "rq_tuxv": ([_c_p, _c_i64, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_u64, _c_i32, _c_p, _c_i64, _c_p,
                 _c_p, _c_i64, _c_p, _c_sz, _c_p], ctypes.c_int),
    "rq_tuxv_omega": ([_c_p, _c_i64, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_p, _c_i64, _c_p, _c_i64,
                       _c_p, _c_p, _c_i64, _c_p, _c_sz, _c_p], ctypes.c_int),
    "rq_unpivoted_qr": ([_c_p, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_p, _c_p, _c_sz, _c_p], ctypes.c_int),
    "rq_omega": ([_c_p, _c_u64, _c_i64, _c_i64, _c_p, _c_i64], ctypes.c_int),
    "rq_sketch": ([_c_p, _c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_u64, _c_i32, _c_p, _c_i64, _c_p, _c_sz],
                  ctypes.c_int),
    "rq_sample_qrcp": ([_c_p, _c_i32, _c_i64, _c_i32, _c_p, _c_i64, _c_p, _c_p, _c_sz, _c_p], ctypes.c_int),
    "rq_small_svd": ([_c_p, _c_i32, _c_p, _c_i64, _c_p, _c_i64, _c_p, _c_p, _c_i64, _c_p, _c_sz], ctypes.c_int),
    "rq_batch_workspace_bytes": ([_c_p, _c_i32, _c_i64, _c_i32, _c_i32, _c_i32, ctypes.POINTER(_c_sz)],
                                 ctypes.c_int),
    "rq_batch_plan_create": ([_c_p, _c_i32, _c_i64, _c_i32, _c_i32, _c_i32, _c_i32, _c_p, _c_sz,
                              ctypes.POINTER(_c_p)], ctypes.c_int),
    "rq_tuxv_batched": ([_c_p, _c_p], ctypes.c_int),
    "rq_batch_plan_destroy": ([_c_p], ctypes.c_int),
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


def _prec(precision):
    return PRECISIONS[precision] if isinstance(precision, str) else int(precision)


def rq_workspace_bytes(op, m, n, k, b, p, precision=RQ_FP64):
    out = _c_sz(0)
    _check(load().rq_workspace_bytes(op, m, n, k, b, p, _prec(precision), ctypes.byref(out)), "rq_workspace_bytes")
    return out.value


def workspace(op, m, n, k, b, p, device, precision=RQ_FP64):
    nbytes = rq_workspace_bytes(op, m, n, k, b, p, precision)
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def rq_rqrcp(A, b, p, seed=0, Omega=None, work=None, stream=None, precision=RQ_FP64):
    """Alg. 4.  Returns (F, tau, jpvt, info): F = R above/on the diagonal and
    reflectors below (column-major m x n); A is not modified.  precision:
    RQ_FP64, RQ_MIXED or RQ_MIXED_BF16 (or "fp64", "mixed", "mixed_bf16")."""
    F = fortran(A).clone()
    m, n = F.shape
    k = min(m, n)
    dev = F.device
    jpvt = torch.empty(n, dtype=torch.int64, device=dev)
    tau = torch.empty(k, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    prec = _prec(precision)
    if work is None:
        work = workspace(RQ_OP_RQRCP, m, n, k, b, p, dev, prec)
    L = load()
    if Omega is None:
        rc = L.rq_rqrcp(_stream(stream), m, n, _ptr(F), _ld(F), b, p, seed, prec, _ptr(jpvt), _ptr(tau), _ptr(work),
                        work.numel(), _ptr(info))
        _check(rc, "rq_rqrcp")
    else:
        if prec != RQ_FP64:
            raise ValueError("a caller-supplied Omega takes the FP64 path")
        Om = fortran(Omega)
        rc = L.rq_rqrcp_omega(_stream(stream), m, n, _ptr(F), _ld(F), b, p, _ptr(Om), _ld(Om), _ptr(jpvt), _ptr(tau),
                              _ptr(work), work.numel(), _ptr(info))
        _check(rc, "rq_rqrcp_omega")
    return F, tau, jpvt, info


RQ_NOALLOC_SCRATCH_BYTES = 96 << 20
RQ_ERR_SCRATCH_TOO_SMALL = 2002


def rq_rqrcp_noalloc(A, b, p, seed=0, stream=None, precision=RQ_FP64):
    """rq_rqrcp without a workspace (the library's static per-device scratch).
    Returns (F, tau, jpvt, info); A is not modified."""
    F = fortran(A).clone()
    m, n = F.shape
    dev = F.device
    jpvt = torch.empty(n, dtype=torch.int64, device=dev)
    tau = torch.empty(min(m, n), dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    rc = load().rq_rqrcp_noalloc(_stream(stream), m, n, _ptr(F), _ld(F), b, p, seed, _prec(precision), _ptr(jpvt),
                                 _ptr(tau), _ptr(info))
    _check(rc, "rq_rqrcp_noalloc")
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


def rq_trqrcp(A, k, b, p, seed=0, Omega=None, work=None, stream=None, precision=RQ_FP64):
    """Alg. 6.  Returns (F, tau, jpvt, info) (layout as in include/rqrcp.h).
    precision RQ_MIXED / RQ_MIXED_BF16: lower-precision sketch and Y2^T A
    (seeded Omega only)."""
    F = fortran(A).clone()
    m, n = F.shape
    dev = F.device
    jpvt = torch.empty(n, dtype=torch.int64, device=dev)
    tau = torch.empty(k, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    prec = _prec(precision)
    if work is None:
        work = workspace(RQ_OP_TRQRCP, m, n, k, b, p, dev, prec)
    L = load()
    if Omega is None:
        rc = L.rq_trqrcp(_stream(stream), m, n, k, _ptr(F), _ld(F), b, p, seed, prec, _ptr(jpvt), _ptr(tau),
                         _ptr(work), work.numel(), _ptr(info))
        _check(rc, "rq_trqrcp")
    else:
        if prec != RQ_FP64:
            raise ValueError("a caller-supplied Omega takes the FP64 path")
        Om = fortran(Omega)
        rc = L.rq_trqrcp_omega(_stream(stream), m, n, k, _ptr(F), _ld(F), b, p, _ptr(Om), _ld(Om), _ptr(jpvt),
                               _ptr(tau), _ptr(work), work.numel(), _ptr(info))
        _check(rc, "rq_trqrcp_omega")
    return F, tau, jpvt, info


def rq_tuxv(A, k, b, p, seed=0, Omega=None, work=None, stream=None, jmax=1, precision=RQ_FP64):
    """Alg. 7 + SVD of X.  Returns (U, sigma, VT, info).  jmax > 1 (seeded
    Omega, FP64) runs the further LQ/QR steps through rq_tuxv_iter;
    precision RQ_MIXED / RQ_MIXED_BF16 (j_max = 1, seeded Omega) the
    lower-precision products."""
    Af = fortran(A)
    m, n = Af.shape
    dev = Af.device
    U = torch.empty((k, m), dtype=torch.float64, device=dev).t()  # column-major m x k
    VT = torch.empty((n, k), dtype=torch.float64, device=dev).t()  # column-major k x n
    sigma = torch.empty(k, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    prec = _prec(precision)
    if prec != RQ_FP64 and (Omega is not None or jmax != 1):
        raise ValueError("the mixed-precision path takes j_max = 1 and the seeded compression matrix")
    if work is None:
        work = workspace(RQ_OP_TUXV, m, n, k, b, p, dev, prec)
    L = load()
    if jmax != 1:
        if Omega is not None:
            raise ValueError("jmax > 1 takes the seeded compression matrix")
        rc = L.rq_tuxv_iter(_stream(stream), m, n, k, _ptr(Af), _ld(Af), b, p, seed, jmax, _ptr(U), m, _ptr(sigma),
                            _ptr(VT), k, _ptr(work), work.numel(), _ptr(info))
        _check(rc, "rq_tuxv_iter")
    elif Omega is None:
        rc = L.rq_tuxv(_stream(stream), m, n, k, _ptr(Af), _ld(Af), b, p, seed, prec, _ptr(U), m, _ptr(sigma),
                       _ptr(VT), k, _ptr(work), work.numel(), _ptr(info))
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


def rq_sketch(A, l, seed, work=None, stream=None, precision=RQ_FP64):
    Af = fortran(A)
    m, n = Af.shape
    B = torch.empty((n, l), dtype=torch.float64, device=Af.device).t()
    if work is None:  # the RQRCP workspace of b + p = l holds Omega and the sample
        work = workspace(RQ_OP_RQRCP, m, n, min(m, n), min(l, 64), l - min(l, 64), Af.device)
    _check(load().rq_sketch(_stream(stream), m, n, _ptr(Af), _ld(Af), l, seed, _prec(precision), _ptr(B), l,
                            _ptr(work), work.numel()), "rq_sketch")
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


def rq_set_panel_path(mode):
    """Test hook: 0 = CholeskyQR2 panel with fallback, 1 = column-by-column
    Householder panel for every block.  Returns the previous mode."""
    rc = load().rq_set_panel_path(int(mode))
    if rc < 0:
        raise RQError(f"rq_set_panel_path returned {rc}")
    return rc


def rq_set_block_dump(buf):
    """Test hook: dump each block's sample into the float64 CUDA tensor
    `buf` (None turns the dump off); see include/rqrcp.h for the layout."""
    if buf is None:
        _check(load().rq_set_block_dump(ctypes.c_void_p(0), 0), "rq_set_block_dump")
        return
    if buf.dtype != torch.float64 or not buf.is_cuda or not buf.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    _check(load().rq_set_block_dump(_ptr(buf), buf.numel()), "rq_set_block_dump")


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


class RQBatchMatrix(ctypes.Structure):
    """rq_batch_matrix of include/rqrcp.h."""
    _fields_ = [("m", _c_i64), ("n", _c_i64), ("A", _c_p), ("lda", _c_i64), ("U", _c_p), ("ldu", _c_i64),
                ("sigma", _c_p), ("VT", _c_p), ("ldvt", _c_i64), ("jpvt", _c_p), ("info", _c_p), ("seed", _c_u64)]


RQ_TILE_64x64, RQ_TILE_32x32, RQ_TILE_128x64 = 0, 1, 2


class BatchTUXV:
    """A planned batch of rq_tuxv solves (rq_batch_plan_create): the inputs
    are float64 CUDA matrices (kept referenced; they must not change shape),
    the outputs U[i] (m_i x k), sigma[i] (k), VT[i] (k x n_i), jpvt[i] (k)
    and info (count) are allocated here.  run() enqueues the whole batch on
    the stream (capturable in a CUDA/HIP graph)."""

    def __init__(self, mats, k, b, p, seeds, precision=RQ_FP64, tile=RQ_TILE_64x64, device=None):
        L = load()
        self.mats = [fortran(A) for A in mats]
        count = len(self.mats)
        dev = self.mats[0].device if count else torch.device("cuda")
        self.k, self.b, self.p, self.precision, self.tile = k, b, p, _prec(precision), tile
        self.U = [torch.empty((k, A.shape[0]), dtype=torch.float64, device=dev).t() for A in self.mats]
        self.sigma = [torch.empty(k, dtype=torch.float64, device=dev) for _ in self.mats]
        self.VT = [torch.empty((A.shape[1], k), dtype=torch.float64, device=dev).t() for A in self.mats]
        self.jpvt = [torch.empty(k, dtype=torch.int64, device=dev) for _ in self.mats]
        self.info = torch.zeros(max(count, 1), dtype=torch.int32, device=dev)
        items = (RQBatchMatrix * max(count, 1))()
        for i, A in enumerate(self.mats):
            m, n = A.shape
            items[i] = RQBatchMatrix(m, n, A.data_ptr(), _ld(A), self.U[i].data_ptr(), m, self.sigma[i].data_ptr(),
                                     self.VT[i].data_ptr(), k, self.jpvt[i].data_ptr(),
                                     self.info.data_ptr() + 4 * i, int(seeds[i]))
        self._items = items
        nbytes = _c_sz(0)
        _check(L.rq_batch_workspace_bytes(ctypes.byref(items), count, k, b, p, self.precision, ctypes.byref(nbytes)),
               "rq_batch_workspace_bytes")
        self.work = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=dev)
        plan = _c_p(0)
        torch.cuda.synchronize()
        _check(L.rq_batch_plan_create(ctypes.byref(items), count, k, b, p, self.precision, tile, _ptr(self.work),
                                      self.work.numel(), ctypes.byref(plan)), "rq_batch_plan_create")
        self._plan = plan

    def run(self, stream=None):
        _check(load().rq_tuxv_batched(_stream(stream), self._plan), "rq_tuxv_batched")

    def close(self):
        if self._plan is not None and self._plan.value:
            load().rq_batch_plan_destroy(self._plan)
        self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # pragma: no cover
            pass


def batch_workspace_bytes(shapes, k, b, p, precision=RQ_FP64):
    """rq_batch_workspace_bytes for matrices of the given (m, n) shapes (host only)."""
    items = (RQBatchMatrix * max(len(shapes), 1))()
    for i, (m, n) in enumerate(shapes):
        items[i] = RQBatchMatrix(m, n, 1, m, 1, m, 1, 1, k, 0, 0, 0)
    out = _c_sz(0)
    _check(load().rq_batch_workspace_bytes(ctypes.byref(items), len(shapes), k, b, p, _prec(precision),
                                           ctypes.byref(out)), "rq_batch_workspace_bytes")
    return out.value


# short aliases
rqrcp = rq_rqrcp
rsrqrcp = rq_rsrqrcp
trqrcp = rq_trqrcp
tuxv = rq_tuxv
unpivoted_qr = rq_unpivoted_qr
