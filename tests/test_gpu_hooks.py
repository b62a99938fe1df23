"""GPU checks through the test hooks of the C ABI.

* rq_set_block_dump: every block's sample (the initial sketch for the first
  block, the sample refreshed by eq. (update1) of Section 4 for the later
  ones) against the oracle's block-by-block trace, at the 512 x 512
  configuration and a ragged shape, normalised by ||Omega||_F ||A||_F (the
  refreshed rows are formed by cancellation, so their own norm is no
  yardstick).
* rq_set_panel_path(1): the column-by-column Householder panel and the
  forward T recurrence for every block (the fallback of the CholeskyQR2
  panel), against the oracle: pivots, R, tau, residual and orthogonality.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1509_06820_amd import binding, inputs
from test_gpu_parity import compare_rqrcp, dev, host, qr_checks, say, trusted_prefix

pytestmark = pytest.mark.gpu


def dumped_samples(l, n, b, k, buf):
    out, off, i0 = [], 0, 0
    while i0 < k:
        nJ = n - i0
        out.append(buf[off:off + l * nJ].reshape(nJ, l).T)
        off += l * nJ
        i0 += min(b, k - i0)
    return out


@pytest.mark.parametrize("m,n,b,p,seed", [(512, 512, 32, 8, 1), (300, 230, 24, 8, 4)])
def test_block_dump_matches_oracle_trace(m, n, b, p, seed):
    say(f"block dump rqrcp {m}x{n} b={b} p={p}")
    if (m, n) == (512, 512):
        A, _ = inputs.config_matrix("c1", seed)
    else:
        A = inputs.with_spectrum(seed, m, n, inputs.sigma_decade(min(m, n), 8))
    k = min(m, n)
    l = b + p
    ref = oracle.rqrcp(A, b, p, seed=seed, trace=True)
    t = trusted_prefix(ref["gaps"], k)
    total = sum(l * (n - i0) for i0 in range(0, k, b))
    buf = torch.full((total,), np.nan, dtype=torch.float64, device="cuda")
    binding.rq_set_block_dump(buf)
    try:
        F, tau, jpvt, info = [host(x) for x in binding.rq_rqrcp(dev(A), b, p, seed)]
    finally:
        binding.rq_set_block_dump(None)
    assert info[0] == 0
    blocks = dumped_samples(l, n, b, k, host(buf))
    assert len(blocks) == len(ref["trace"])
    scale = np.linalg.norm(ref["Omega"]) * np.linalg.norm(A)
    for J, (Bg, rec) in enumerate(zip(blocks, ref["trace"])):
        if rec["i0"] > t:   # a near tie before this block may legitimately change it
            break
        err = np.linalg.norm(Bg - rec["B"]) / scale
        assert err <= 1e-12, (J, err)
    # the first block's sample is the sketch itself
    assert np.linalg.norm(blocks[0] - ref["Omega"] @ A) <= 1e-13 * scale


def test_block_dump_trqrcp_equals_rqrcp_samples():
    """TRQRCP (Alg. 6) refreshes the sample with the same eq. (update1) from
    rows of R it forms on demand: its per-block samples equal RQRCP's."""
    m, n, k, b, p, seed = 600, 500, 160, 32, 8, 7
    say(f"block dump trqrcp vs rqrcp {m}x{n} k={k}")
    A = inputs.with_spectrum(seed, m, n, inputs.sigma_decade(min(m, n), 8))
    l = b + p
    total = sum(l * (n - i0) for i0 in range(0, k, b))
    bufs = []
    for fn in ("rqrcp", "trqrcp"):
        buf = torch.zeros(total, dtype=torch.float64, device="cuda")
        binding.rq_set_block_dump(buf)
        try:
            if fn == "rqrcp":
                _, _, jp_r, _ = binding.rq_rqrcp(dev(A), b, p, seed)
            else:
                _, _, jp_t, _ = binding.rq_trqrcp(dev(A), k, b, p, seed)
        finally:
            binding.rq_set_block_dump(None)
        bufs.append(host(buf))
    assert np.array_equal(host(jp_r)[:k], host(jp_t)[:k])
    scale = np.linalg.norm(oracle.omega(seed, l, m)) * np.linalg.norm(A)
    assert np.linalg.norm(bufs[0] - bufs[1]) <= 1e-12 * scale


def test_block_dump_capacity_stops_at_a_block_boundary():
    """A buffer too small for every block holds the blocks that fit and
    leaves the rest untouched."""
    m, n, b, p, seed = 200, 150, 32, 8, 3
    say("block dump capacity")
    A = inputs.gaussian(seed, m, n)
    l = b + p
    first_two = l * n + l * (n - b)
    buf = torch.full((first_two + 100,), -5.0, dtype=torch.float64, device="cuda")
    binding.rq_set_block_dump(buf)
    try:
        binding.rq_rqrcp(dev(A), b, p, seed)
    finally:
        binding.rq_set_block_dump(None)
    h = host(buf)
    assert np.all(h[first_two:] == -5.0)
    assert np.all(np.isfinite(h[:first_two])) and not np.any(h[:first_two] == -5.0)


class ForcedColumnPanel:
    def __enter__(self):
        self.prev = binding.rq_set_panel_path(1)

    def __exit__(self, *exc):
        binding.rq_set_panel_path(self.prev)


@pytest.mark.parametrize("m,n,b,p,seed", [
    (512, 512, 32, 8, 1),      # the 512 x 512 configuration
    (2100, 1300, 32, 8, 9),    # nine panel workgroups exchanging partial sums
    (97, 97, 64, 3, 6),        # ragged last block
    (600, 500, 64, 64, 10),    # l = 128
])
def test_forced_column_panel_rqrcp_matches_oracle(m, n, b, p, seed):
    say(f"forced column panel rqrcp {m}x{n} b={b}")
    if (m, n) == (512, 512):
        A, _ = inputs.config_matrix("c1", seed)
    else:
        A = inputs.with_spectrum(seed, m, n, inputs.sigma_decade(min(m, n), 8))
    with ForcedColumnPanel():
        F, tau, jpvt, ref = compare_rqrcp(A, b, p, seed)
    # tau where every pivot agrees.  tau_j depends on the direction of the
    # column it reflects, |R_jj| long, which rounding of size eps ||A|| turns
    # by up to eps ||A|| / |R_jj|: the bar scales with ||A||_F / |R_jj| (on
    # the graded 512 x 512 matrix |R_jj| falls to 1e-10 ||A||).
    k = min(m, n)
    t = trusted_prefix(ref["gaps"], k)
    if t == k:
        rjj = np.maximum(np.abs(np.diag(ref["F"][:k, :k])), 1e-300)
        bar = 1e-12 * np.maximum(1.0, np.linalg.norm(A) / rjj)
        assert np.all(np.abs(tau - ref["tau"]) <= bar)


def test_forced_column_panel_qr_trqrcp_tuxv():
    say("forced column panel: unpivoted qr 700x500, trqrcp 600x500 k=100, tuxv 400x300 k=40")
    with ForcedColumnPanel():
        A = inputs.gaussian(1200, 700, 500)
        F, tau, info = [host(x) for x in binding.rq_unpivoted_qr(dev(A), 32)]
        Fr, tr = oracle.unpivoted_qr(A, 32)
        nrm = np.linalg.norm(A)
        assert info[0] == 0
        assert np.abs(np.triu(F) - np.triu(Fr)).max() <= 1e-12 * nrm
        assert np.abs(tau - tr).max() <= 1e-12
        res, orth = qr_checks(A, F, tau, np.arange(500), 500)
        assert res <= 1e-12 and orth <= 1e-13

        A = inputs.with_spectrum(1, 600, 500, inputs.sigma_decade(500, 8))
        ref = oracle.trqrcp(A, 100, 32, 8, seed=1)
        F, tau, jpvt, info = [host(x) for x in binding.rq_trqrcp(dev(A), 100, 32, 8, 1)]
        t = trusted_prefix(ref["gaps"], 100)
        assert info[0] == 0 and np.array_equal(jpvt[:t], ref["jpvt"][:t])
        if t == 100:
            assert np.abs(np.triu(F[:100]) - np.triu(ref["F"][:100])).max() <= 1e-12 * np.linalg.norm(A)

        sig = inputs.sigma_decade(300, 6)
        A = inputs.with_spectrum(1, 400, 300, sig)
        ref = oracle.tuxv(A, 40, 16, 8, seed=1)
        U, s, VT, info = [host(x) for x in binding.rq_tuxv(dev(A), 40, 16, 8, 1)]
        assert info[0] == 0
        assert np.abs(s - ref["s"]).max() <= 1e-12 * ref["s"][0]
