"""C ABI checks that need no GPU: the library loads, exports every entry
point declared in include/rqrcp.h, answers workspace queries, and rejects
invalid arguments (LAPACK-style -i) before enqueueing anything."""

import ctypes
import os
import re

import pytest

from paper_1509_06820_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rqrcp.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_1509_06820_amd import build
        build.build()
    return binding.load()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rq_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_symbols()
    for must in ["rq_rqrcp", "rq_trqrcp", "rq_tuxv", "rq_unpivoted_qr", "rq_workspace_bytes", "rq_omega",
                 "rq_sketch", "rq_sample_qrcp", "rq_small_svd", "rq_rqrcp_omega", "rq_trqrcp_omega",
                 "rq_tuxv_omega", "rq_version"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(binding.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(raw, name), name
    assert b"rqrcp" in lib.rq_version()


def test_binding_covers_every_symbol():
    for name in declared_symbols():
        assert name in binding._SIGS, name


@pytest.mark.parametrize("op,m,n,k,b,p", [
    (binding.RQ_OP_RQRCP, 512, 512, 0, 32, 8),
    (binding.RQ_OP_RQRCP, 8192, 8192, 0, 64, 8),
    (binding.RQ_OP_QR, 8192, 8192, 0, 64, 0),
    (binding.RQ_OP_TRQRCP, 20000, 10000, 256, 64, 8),
    (binding.RQ_OP_TUXV, 20000, 10000, 256, 64, 8),
    (binding.RQ_OP_SAMPLE_QRCP, 72, 8192, 0, 64, 0),
    (binding.RQ_OP_SVD, 256, 256, 256, 1, 0),
    (binding.RQ_OP_RSRQRCP, 8192, 8192, 0, 64, 8),
])
def test_workspace_query(lib, op, m, n, k, b, p):
    nbytes = binding.rq_workspace_bytes(op, m, n, k, b, p)
    assert nbytes > 0
    # the workspace of the full factorization stays a small fraction of A
    if op == binding.RQ_OP_RQRCP and m == 8192:
        assert nbytes < 0.25 * m * n * 8


def test_workspace_query_rejects_bad_arguments(lib):
    out = ctypes.c_size_t(0)
    assert lib.rq_workspace_bytes(0, -1, 5, 0, 8, 0, 0, ctypes.byref(out)) == -2
    assert lib.rq_workspace_bytes(0, 5, -1, 0, 8, 0, 0, ctypes.byref(out)) == -3
    assert lib.rq_workspace_bytes(0, 5, 5, 0, 0, 0, 0, ctypes.byref(out)) == -5
    assert lib.rq_workspace_bytes(0, 5, 5, 0, 65, 0, 0, ctypes.byref(out)) == -5
    assert lib.rq_workspace_bytes(0, 5, 5, 0, 64, 65, 0, ctypes.byref(out)) == -6
    assert lib.rq_workspace_bytes(1, 5, 5, 6, 4, 0, 0, ctypes.byref(out)) == -4
    assert lib.rq_workspace_bytes(99, 5, 5, 1, 4, 0, 0, ctypes.byref(out)) == -1
    # precision: one of the three levels, and only for RQRCP, TRQRCP and TUXV
    assert lib.rq_workspace_bytes(0, 5, 5, 0, 4, 0, 3, ctypes.byref(out)) == -7
    assert lib.rq_workspace_bytes(0, 5, 5, 0, 4, 0, -1, ctypes.byref(out)) == -7
    assert lib.rq_workspace_bytes(binding.RQ_OP_QR, 5, 5, 0, 4, 0, 1, ctypes.byref(out)) == -7
    assert lib.rq_workspace_bytes(0, 5, 5, 0, 4, 0, 0, None) == -8


def test_entry_points_reject_bad_arguments_before_any_launch(lib):
    null = ctypes.c_void_p(0)
    # m < 0, n < 0, lda < m, b out of range, p out of range, precision out of range
    assert lib.rq_rqrcp(null, -1, 4, null, 1, 8, 0, 1, 0, null, null, null, 0, null) == -2
    assert lib.rq_rqrcp(null, 4, -1, null, 4, 8, 0, 1, 0, null, null, null, 0, null) == -3
    assert lib.rq_rqrcp(null, 4, 4, null, 3, 8, 0, 1, 0, null, null, null, 0, null) == -5
    assert lib.rq_rqrcp(null, 4, 4, null, 4, 0, 0, 1, 0, null, null, null, 0, null) == -6
    assert lib.rq_rqrcp(null, 4, 4, null, 4, 8, -1, 1, 0, null, null, null, 0, null) == -7
    assert lib.rq_rqrcp(null, 4, 4, null, 4, 8, 0, 1, 3, null, null, null, 0, null) == -9
    assert lib.rq_trqrcp(null, 10, 10, 11, null, 10, 4, 4, 1, 0, null, null, null, 0, null) == -4
    assert lib.rq_trqrcp(null, 10, 10, 3, null, 10, 4, 4, 1, 7, null, null, null, 0, null) == -10
    assert lib.rq_tuxv(null, 10, 10, 0, null, 10, 4, 4, 1, 0, null, 10, null, null, 1, null, 0, null) == -4
    assert lib.rq_tuxv(null, 10, 10, 3, null, 10, 4, 4, 1, 5, null, 10, null, null, 3, null, 0, null) == -10
    assert lib.rq_tuxv(null, 10, 10, 3, null, 10, 4, 4, 1, 0, null, 9, null, null, 3, null, 0, null) == -12
    assert lib.rq_tuxv(null, 10, 10, 3, null, 10, 4, 4, 1, 1, null, 10, null, null, 2, null, 0, null) == -15
    assert lib.rq_rqrcp_omega(null, 4, 4, null, 4, 2, 2, null, 4, null, null, null, 0, null) == -8
    assert lib.rq_unpivoted_qr(null, 4, 4, null, 2, 2, null, null, 0, null) == -5
    assert lib.rq_sample_qrcp(null, 0, 4, 1, null, 1, null, null, 0, null) == -2
    assert lib.rq_sample_qrcp(null, 8, 4, 9, null, 8, null, null, 0, null) == -4
    assert lib.rq_small_svd(null, 0, null, 1, null, 1, null, null, 1, null, 0) == -2
    assert lib.rq_rsrqrcp(null, 4, 4, null, 3, 8, 0, 1, null, null, null, 0, null) == -5
    assert lib.rq_rsrqrcp(null, 4, 4, null, 4, 8, -1, 1, null, null, null, 0, null) == -7
    assert lib.rq_sketch(null, 4, 4, null, 4, 2, 1, 9, null, 2, null, 0) == -8
    assert lib.rq_sketch(null, 4, 4, null, 4, 2, 1, 0, null, 1, null, 0) == -10
    # j_max outside [1, RQ_TUXV_MAX_ITER], then ldu < m and ldvt < k
    for jmax in (0, -3, binding.RQ_TUXV_MAX_ITER + 1):
        assert lib.rq_tuxv_iter(null, 10, 10, 3, null, 10, 4, 4, 1, jmax, null, 10, null, null, 3, null, 0,
                                null) == -10
    assert lib.rq_tuxv_iter(null, 10, 10, 3, null, 10, 4, 4, 1, 2, null, 9, null, null, 3, null, 0, null) == -12
    assert lib.rq_tuxv_iter(null, 10, 10, 3, null, 10, 4, 4, 1, 2, null, 10, null, null, 2, null, 0, null) == -15
    assert lib.rq_tuxv_iter(null, 10, 10, 11, null, 10, 4, 4, 1, 2, null, 10, null, null, 11, null, 0, null) == -4
    # empty matrices are valid and enqueue nothing
    assert lib.rq_rsrqrcp(null, 0, 4, null, 1, 8, 0, 1, null, null, null, 0, null) == 0
    assert lib.rq_rqrcp(null, 0, 4, null, 1, 8, 0, 1, 0, null, null, null, 0, null) == 0
    # a workspace below the size query makes the size argument invalid
    assert lib.rq_rqrcp(null, 40, 40, null, 40, 8, 0, 1, 0, null, null, null, 16, null) == -13
    assert lib.rq_rqrcp_omega(null, 40, 40, null, 40, 8, 0, ctypes.c_void_p(256), 8, null, null, null, 16,
                              null) == -13
    assert lib.rq_rsrqrcp(null, 40, 40, null, 40, 8, 0, 1, null, null, null, 16, null) == -12
    assert lib.rq_unpivoted_qr(null, 40, 40, null, 40, 8, null, null, 16, null) == -9
    assert lib.rq_trqrcp(null, 40, 40, 8, null, 40, 8, 0, 1, 1, null, null, null, 16, null) == -14
    assert lib.rq_tuxv(null, 40, 40, 8, null, 40, 8, 0, 1, 2, null, 40, null, null, 8, null, 16, null) == -17
    assert lib.rq_tuxv_iter(null, 40, 40, 8, null, 40, 8, 0, 1, 3, null, 40, null, null, 8, null, 16, null) == -17
    assert lib.rq_sample_qrcp(null, 8, 40, 4, null, 8, null, null, 16, null) == -9
    assert lib.rq_small_svd(null, 40, null, 40, null, 40, null, null, 40, null, 16) == -11
    assert lib.rq_sketch(null, 40, 40, null, 40, 8, 1, 0, null, 8, null, 16) == -12


@pytest.mark.parametrize("op,k", [(binding.RQ_OP_TUXV, 256), (binding.RQ_OP_TRQRCP, 256), (binding.RQ_OP_RQRCP, 0)])
def test_mixed_workspace(lib, op, k):
    """The mixed levels of TRQRCP and TUXV add the FP32 copy of A (4 m n
    bytes; TUXV also the permuted V, 8 n k bytes); the mixed RQRCP updates A
    in place and needs nothing more.  Both mixed levels need the same space."""
    m, n, b, p = 20000, 10000, 64, 8
    base = binding.rq_workspace_bytes(op, m, n, k, b, p, binding.RQ_FP64)
    for prec in (binding.RQ_MIXED, binding.RQ_MIXED_BF16):
        extra = binding.rq_workspace_bytes(op, m, n, k, b, p, prec) - base
        if op == binding.RQ_OP_TUXV:
            assert 4 * m * n + 8 * n * k <= extra <= 4 * m * n + 8 * n * k + 1024
        elif op == binding.RQ_OP_TRQRCP:
            assert 4 * m * n <= extra <= 4 * m * n + 512
        else:
            assert extra == 0


def test_rsrqrcp_workspace_matches_rqrcp(lib):
    """Alg. 5 needs the buffers of Alg. 4: one sample and one Omega of the
    first block's size, reused by every block."""
    for m, n, b, p in [(8192, 8192, 64, 8), (300, 200, 32, 8)]:
        assert (binding.rq_workspace_bytes(binding.RQ_OP_RSRQRCP, m, n, 0, b, p)
                == binding.rq_workspace_bytes(binding.RQ_OP_RQRCP, m, n, 0, b, p))


def test_host_switches_are_host_only(lib):
    """The look-ahead, panel-path and block-dump switches touch no GPU and
    report the previous setting (or reject an invalid one)."""
    prev = lib.rq_set_lookahead(0)
    assert prev in (0, 1)
    assert lib.rq_set_lookahead(1) == 0
    assert lib.rq_set_lookahead(prev) == 1
    assert lib.rq_set_panel_path(1) == 0
    assert lib.rq_set_panel_path(0) == 1
    assert lib.rq_set_panel_path(2) == -1
    assert lib.rq_set_block_dump(ctypes.c_void_p(0), -1) == -2
    assert lib.rq_set_block_dump(ctypes.c_void_p(0), 0) == 0


def test_batch_workspace_query_and_argument_checks(lib):
    """rq_batch_workspace_bytes: grows with the matrices and rejects what the
    batched engine cannot take (k > 64, b not dividing k, b + p > 64, an item
    with k > min(m, n) or n > 8192, the BF16 level)."""
    small = binding.batch_workspace_bytes([(100, 80)], 16, 8, 8)
    two = binding.batch_workspace_bytes([(100, 80), (300, 200)], 16, 8, 8)
    assert 0 < small < two
    for args in [([(100, 80)], 65, 8, 8), ([(100, 80)], 16, 6, 8), ([(100, 80)], 16, 8, 57),
                 ([(10, 80)], 16, 8, 8), ([(9000, 8500)], 16, 8, 8)]:
        with pytest.raises(binding.RQError):
            binding.batch_workspace_bytes(*args)
    with pytest.raises(binding.RQError):
        binding.batch_workspace_bytes([(100, 80)], 16, 8, 8, precision=binding.RQ_MIXED_BF16)
    assert binding.batch_workspace_bytes([], 16, 8, 8) > 0


def test_autotune_host_logic(tmp_path):
    """Block candidates divide k and keep b + p <= 64; the size signature
    groups matrices by (log2 m, log2 n); a cached choice is found again."""
    import json

    from paper_1509_06820_amd import autotune
    assert autotune.block_candidates(32, 8) == [8, 16, 32]
    assert autotune.block_candidates(32, 40) == [8, 16]
    assert autotune.block_candidates(24, 8) == [8]
    assert autotune.signature([(100, 80), (120, 70), (1000, 900)]) == "6x6:2;9x9:1"
    shapes = [(100, 80), (300, 200)]
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({autotune.key(shapes, 16, 8, 0): {"b": 8, "tile": 1, "ms": 1.0}}))
    assert autotune.lookup(shapes, 16, 8, 0, str(path))["tile"] == 1
    assert autotune.lookup(shapes, 32, 8, 0, str(path)) is None


def test_noalloc_rejects_oversize_before_any_launch(lib):
    """rq_rqrcp_noalloc checks its arguments and the size of its static
    scratch on the host: a factorization that needs more than
    RQ_NOALLOC_SCRATCH_BYTES is rejected with RQ_ERR_SCRATCH_TOO_SMALL, bad
    arguments with -i, neither touching a GPU."""
    null = ctypes.c_void_p(0)
    m, n, b, p = 30000, 20000, 64, 64
    assert binding.rq_workspace_bytes(binding.RQ_OP_RQRCP, m, n, 0, b, p) > binding.RQ_NOALLOC_SCRATCH_BYTES
    assert lib.rq_rqrcp_noalloc(null, m, n, null, m, b, p, 1, 0, null, null, null) == binding.RQ_ERR_SCRATCH_TOO_SMALL
    assert lib.rq_rqrcp_noalloc(null, -1, 4, null, 1, 8, 0, 1, 0, null, null, null) == -2
    assert lib.rq_rqrcp_noalloc(null, 4, 4, null, 4, 8, 0, 1, 7, null, null, null) == -9


# sizes spanning the valid range, the limits and far past them (2^62)
_SIZES = [0, 1, 7, 64, 65, 4096, 65536, 65537, 2 ** 31, 2 ** 40, 2 ** 40 + 1, 2 ** 62, -1]


def test_workspace_queries_never_wrap(lib):
    """Random and extreme arguments to rq_workspace_bytes: either a documented
    argument error (-1 .. -8) or a size that holds at least the buffers every
    path needs -- Omega (l x m) and the sample (l x n) for the sampled
    factorizations, the FP32 copy of A (m x n) for mixed TRQRCP and TUXV, the
    rotations (k x k) for the SVD -- so that no size query wraps round to a
    small number (overflowed sizes once came back as a few MB)."""
    import random
    rng = random.Random(1509)
    out = ctypes.c_size_t(0)
    for _ in range(4000):
        op = rng.choice([0, 1, 2, 3, 4, 5, 6, 7, -1])
        m, n, k = (rng.choice(_SIZES) for _ in range(3))
        b, p = rng.choice([0, 1, 8, 32, 64, 65]), rng.choice([0, 4, 8, 64, 100])
        prec = rng.choice([0, 1, 2, 3])
        out.value = 0
        rc = lib.rq_workspace_bytes(op, m, n, k, b, p, prec, ctypes.byref(out))
        if rc:
            assert -8 <= rc <= -1, (op, m, n, k, b, p, prec, rc)
            continue
        nbytes, l = out.value, b + p
        assert 0 < nbytes < 2 ** 62
        if op in (binding.RQ_OP_RQRCP, binding.RQ_OP_RSRQRCP):
            assert nbytes >= 8 * l * (m + n), (op, m, n, b, p)
        elif op == binding.RQ_OP_TRQRCP or op == binding.RQ_OP_TUXV:
            assert nbytes >= 8 * l * (m + n) + (4 * m * n if prec else 0), (op, m, n, k, b, p, prec)
        elif op == binding.RQ_OP_SAMPLE_QRCP:
            assert 1 <= m <= 128 and nbytes >= 8 * m * n
        elif op == binding.RQ_OP_SVD:
            assert nbytes >= 8 * k * k
        elif op == binding.RQ_OP_QR:
            assert m <= 2 ** 40 and n <= 65536


def test_batch_workspace_query_never_wraps(lib):
    """rq_batch_workspace_bytes over batches with huge or many matrices:
    an error on the items, or a size covering every matrix's Omega (l x m)
    and its Q, P, P2 (m x k each)."""
    import random
    rng = random.Random(6820)
    for _ in range(300):
        count = rng.choice([1, 2, 5, 40])
        k, b, p = 32, 16, 8
        shapes = [(rng.choice([32, 1000, 2 ** 20, 2 ** 40, 2 ** 40 + 1, 2 ** 62]),
                   rng.choice([32, 500, 8192, 8193])) for _ in range(count)]
        try:
            nbytes = binding.batch_workspace_bytes(shapes, k, b, p)
        except binding.RQError as e:
            assert "returned -1" in str(e)
            assert any(m > 2 ** 40 or n > 8192 for m, n in shapes) or nbytes_would_exceed(shapes, k)
            continue
        need = sum(8 * (b + p) * m + 3 * 8 * m * k for m, _ in shapes)
        assert need <= nbytes < 2 ** 64


def nbytes_would_exceed(shapes, k):
    """More output tiles than 32-bit tile indices can address."""
    return sum(((m + 31) // 32) * ((k + 31) // 32) for m, _ in shapes) > 2 ** 24


def test_sample_register_tiles_in_the_size_query(lib):
    """The sample is stored in register tiles of 32, 40, 48, 64, 72, 80 or
    128 rows: the sample QRCP's workspace grows with the tile, not with l,
    so every l of one tile asks for the same bytes and the next l for more."""
    out = ctypes.c_size_t(0)
    n = 4096

    def q(l):
        assert lib.rq_workspace_bytes(binding.RQ_OP_SAMPLE_QRCP, l, n, 0, 1, 0, 0, ctypes.byref(out)) == 0
        return out.value

    tiles = [32, 40, 48, 64, 72, 80, 128]
    lo = 1
    for t in tiles:
        sizes = {q(l) for l in range(lo, t + 1)}
        assert len(sizes) == 1, (lo, t)
        lo = t + 1
    per_tile = [q(t) for t in tiles]
    assert per_tile == sorted(per_tile) and len(set(per_tile)) == len(tiles)
    # the sample itself (n columns of the tile's rows) is part of it
    assert q(41) - q(40) >= 8 * n * (48 - 40)
