"""Pins for the oracle's compression-matrix generator (Section 3: Omega has
i.i.d. unit-variance Gaussian entries; E||Omega a||^2 = l||a||^2 and
Var||Omega a||^2 = 2 l ||a||^4)."""

import numpy as np
import pytest
from scipy import stats

from oracle import philox


@pytest.mark.parametrize("seed", [0, 1, 2, 12345, 2**63 + 17, 2**64 - 1])
def test_raw_words_match_numpy_philox(seed):
    # numpy's Philox is an independent implementation of the same SC'11
    # generator; block q of its stream is counter q + 1 with key (seed, 0).
    ours = philox.raw_words(seed, 64)
    ref = np.random.Philox(key=seed).random_raw(256).reshape(64, 4)
    assert np.array_equal(ours, ref)


def test_counter_carry_and_key_high_word():
    # explicit counter words beyond the low word and a nonzero high key word
    ctr = np.array([[2**64 - 1, 5, 7, 9]], dtype=np.uint64)
    key = (0xDEADBEEF, 0x1234)
    g = np.random.Philox(key=(0x1234 << 64) | 0xDEADBEEF,
                         counter=(9 << 192) | (7 << 128) | (5 << 64) | (2**64 - 2))
    ref = g.random_raw(4)
    assert np.array_equal(philox.philox4x64_10(ctr, key)[0], ref)


def test_uniform_map_endpoints():
    x = np.array([0, 2**64 - 1, 2**63], dtype=np.uint64)
    u = philox.uniform52(x)
    assert u[0] == 2.0 ** -53
    assert u[1] == 1.0 - 2.0 ** -53
    assert u[2] == 0.5 + 2.0 ** -53
    assert np.all((u > 0) & (u < 1))


def test_box_muller_pairs_words_and_lanes():
    # Each normal pair lies on the circle of radius sqrt(-2 ln u_even) at
    # angle 2 pi u_odd: checks that word 0 (resp. 2) sets the radius and
    # word 1 (resp. 3) the angle, and that cos/sin sit in even/odd lanes.
    w = philox.raw_words(7, 1000)
    z = philox.box_muller(w)
    u = philox.uniform52(w)
    for a, c in ((0, 1), (2, 3)):
        r2 = z[:, a] ** 2 + z[:, c] ** 2
        assert np.allclose(r2, -2 * np.log(u[:, a]), rtol=1e-13, atol=1e-13)
        ang = np.mod(np.arctan2(z[:, c], z[:, a]), 2 * np.pi)
        d = np.abs(ang - 2 * np.pi * u[:, c])
        d = np.minimum(d, 2 * np.pi - d)
        assert d.max() < 1e-9


def test_omega_layout_row_major_stream():
    l, m = 5, 7
    Om = philox.omega(3, l, m)
    flat = philox.box_muller(philox.raw_words(3, (l * m + 3) // 4)).reshape(-1)
    for r in range(l):
        for c in range(m):
            assert Om[r, c] == flat[r * m + c]
    # rows do not depend on l
    assert np.array_equal(philox.omega(3, l + 4, m)[:l], Om)


def test_omega_is_standard_normal():
    Om = philox.omega(11, 64, 4096).ravel()
    assert abs(Om.mean()) < 5 / np.sqrt(Om.size)
    assert abs(Om.var() - 1) < 5 * np.sqrt(2 / Om.size)
    assert stats.kstest(Om, "norm").pvalue > 1e-4
    # pairs within a block are independent (no correlation between lanes)
    z = philox.box_muller(philox.raw_words(5, 50000))
    c = np.corrcoef(z.T)
    assert np.abs(c - np.eye(4)).max() < 0.03


def test_sample_norm_law():
    # Section 3: ||Omega a||^2 = x ||a||^2 with x ~ chi^2_l:
    # mean l ||a||^2, variance 2 l ||a||^4.
    rng = np.random.default_rng(0)
    m, l = 200, 12
    a = rng.standard_normal(m)
    a2 = a @ a
    vals = np.array([np.sum((philox.omega(s, l, m) @ a) ** 2) for s in range(3000)])
    x = vals / a2
    assert abs(x.mean() - l) < 5 * np.sqrt(2 * l / len(x))
    assert abs(x.var() - 2 * l) < 0.2 * 2 * l
    assert stats.kstest(x, stats.chi2(l).cdf).pvalue > 1e-4
