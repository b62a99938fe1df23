"""rq_rqrcp_noalloc (the RQRCP entry point that allocates nothing and uses
the library's static per-device scratch) against rq_rqrcp with a caller
workspace: bit for bit on two calls in a row, the second smaller than the
first (the scratch keeps the first call's contents, which the second must
not depend on), and an oversized problem rejected before any launch."""

import numpy as np
import pytest
import torch

from paper_1509_06820_amd import binding, inputs

pytestmark = pytest.mark.gpu


def dev(A):
    return torch.from_numpy(np.asfortranarray(A)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_noalloc_matches_workspace_entry_point_on_two_calls():
    binding.load()
    cases = [(2100, 1300, 32, 8, 9), (512, 512, 32, 8, 1)]   # second call smaller than the first
    outs = []
    for m, n, b, p, seed in cases:
        print(f"[case] rqrcp_noalloc {m}x{n} b={b} p={p} seed={seed}", flush=True)
        A = dev(inputs.with_spectrum(seed, m, n, inputs.sigma_decade(min(m, n), 8)))
        # the allocation-free entry point runs the blocks in the sequential
        # order (no look-ahead); compare with rq_rqrcp in that same order
        prev = binding.rq_set_lookahead(False)
        try:
            ref = [host(x) for x in binding.rq_rqrcp(A, b, p, seed)]
        finally:
            binding.rq_set_lookahead(prev)
        got = [host(x) for x in binding.rq_rqrcp_noalloc(A, b, p, seed)]
        assert got[3][0] == 0 and ref[3][0] == 0
        for x, y in zip(got, ref):
            assert np.array_equal(x, y)
        outs.append(got)
    # a third call at the first size again: still identical (nothing left over from the second)
    m, n, b, p, seed = cases[0]
    A = dev(inputs.with_spectrum(seed, m, n, inputs.sigma_decade(min(m, n), 8)))
    again = [host(x) for x in binding.rq_rqrcp_noalloc(A, b, p, seed)]
    for x, y in zip(again, outs[0]):
        assert np.array_equal(x, y)


def test_noalloc_mixed_level_matches_workspace_entry_point():
    print("[case] rqrcp_noalloc mixed 1000x700", flush=True)
    A = dev(inputs.with_spectrum(8, 1000, 700, inputs.sigma_decade(700, 2)))
    ref = [host(x) for x in binding.rq_rqrcp(A, 64, 8, 8, precision="mixed")]
    got = [host(x) for x in binding.rq_rqrcp_noalloc(A, 64, 8, 8, precision="mixed")]
    for x, y in zip(got, ref):
        assert np.array_equal(x, y)


def test_noalloc_rejects_sizes_beyond_its_scratch():
    print("[case] rqrcp_noalloc oversize rejection", flush=True)
    m, n, b, p = 30000, 20000, 64, 64
    assert binding.rq_workspace_bytes(binding.RQ_OP_RQRCP, m, n, 0, b, p) > binding.RQ_NOALLOC_SCRATCH_BYTES
    null = None
    rc = binding.load().rq_rqrcp_noalloc(null, m, n, null, m, b, p, 1, 0, null, null, null)
    assert rc == binding.RQ_ERR_SCRATCH_TOO_SMALL
