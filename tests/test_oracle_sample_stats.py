"""Pins for the sample statistics of Section 3 (oracle/sample_stats.py):
the selection expectation of Fig. selectExpect and the truncated Chi-squared
law of the trailing sample norms (Section 3.3, its theorem and expectation).
Each quantity is checked against a route that shares nothing with it: the
incomplete-beta law of a ratio of Chi-squared variables, brute-force draws,
the Chi-squared moment identity, direct quadrature, limits, and the oracle's
own sample QRCP run on Gaussian samples."""

import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle
from oracle import sample_stats as ss
from paper_1509_06820_amd import inputs


# ---------------------------------------------------------------- selection (Section 3.2)

@pytest.mark.parametrize("phi,l", [(0.3, 4), (0.7, 8), (0.9, 4), (0.95, 16), (0.99, 32)])
def test_select_two_columns_matches_beta_law(phi, l):
    """n = 2: column 1 wins when phi^2 x1 > x0, i.e. x0 / (x0 + x1) <
    phi^2 / (1 + phi^2); x0 / (x0 + x1) is Beta(l/2, l/2)."""
    p1 = special.betainc(l / 2, l / 2, phi ** 2 / (1 + phi ** 2))
    assert abs(ss.select_expectation(phi, l, 2) - ((1 - p1) + phi * p1)) <= 1e-12


@pytest.mark.parametrize("phi,l,n", [(0.9, 8, 200), (0.99, 4, 300), (0.8, 2, 60)])
def test_select_matches_brute_force(phi, l, n):
    e = ss.select_expectation(phi, l, n)
    mean, se = ss.select_monte_carlo(phi, l, n, 3000, np.random.default_rng(int(phi * 1000) + l))
    assert abs(mean - e) <= 4 * se


def test_select_limits_and_monotonicity():
    """More sample rows select better (the figure's message); a fast decay
    selects nearly optimally, and so do nearly equal norms (phi -> 1), with
    the worst case in between (phi about 0.9-0.95).  From l = 8 up that worst
    case stays above 0.9 of the optimum 1, as the figure's caption reports; at
    l = 4 it dips to about 0.88."""
    for phi in (0.8, 0.95, 0.99):
        es = [ss.select_expectation(phi, l, 400) for l in (2, 4, 8, 16, 32)]
        assert all(b > a for a, b in zip(es, es[1:]))
    down = [ss.select_expectation(phi, 8, 500) for phi in (0.3, 0.5, 0.8, 0.9)]
    up = [ss.select_expectation(phi, 8, 500) for phi in (0.95, 0.99, 0.999, 0.9999)]
    assert all(b < a for a, b in zip(down, down[1:]))
    assert all(b > a for a, b in zip(up, up[1:]))
    assert ss.select_expectation(1e-3, 4, 50) > 1 - 1e-5
    grid = (0.8, 0.85, 0.9, 0.93, 0.95, 0.97, 0.99)
    assert min(ss.select_expectation(phi, 8, 500) for phi in grid) > 0.9
    assert min(ss.select_expectation(phi, 4, 500) for phi in grid) < 0.89


# ---------------------------------------------------------------- truncated Chi-squared (Section 3.3)

@pytest.mark.parametrize("d", [1, 2, 5, 10, 40])
def test_truncated_mean_identity_and_quadrature(d):
    """x g_d(x) = d g_{d+2}(x) for Chi-squared densities, so the truncated
    mean is d G_{d+2}(tau) / G_d(tau); also direct quadrature of x g_d(x).
    The paper's form d (1 - e^(-z) / f) cancels when tau << d, so the bar is
    absolute, in units of the untruncated mean d."""
    for tau in (1e-3, 0.5, 2.0, float(d), 3.0 * d + 5):
        ref = d * stats.chi2.cdf(tau, d + 2) / stats.chi2.cdf(tau, d)
        num, _ = integrate.quad(lambda x: x * stats.chi2.pdf(x, d), 0, tau, epsabs=0, epsrel=1e-12)
        quad_mean = num / stats.chi2.cdf(tau, d)
        got = float(ss.truncated_chi2_mean(d, tau))
        assert abs(got - ref) <= 1e-12 * d
        assert abs(got - quad_mean) <= 1e-11 * d


def test_truncated_mean_limits_and_monotone():
    """Zero at tau = 0 (leading term tau d / (d + 2)), d for large tau,
    increasing in between."""
    for d in (1, 4, 16):
        small = 1e-4
        assert abs(float(ss.truncated_chi2_mean(d, small)) - small * d / (d + 2)) <= 1e-3 * small
        assert abs(float(ss.truncated_chi2_mean(d, 1e3)) - d) <= 1e-12 * d
        taus = np.linspace(0.01, 5 * d, 200)
        assert np.all(np.diff(ss.truncated_chi2_mean(d, taus)) > 0)


def _orthogonal_columns(seed, m, n, phi):
    Q = inputs.haar_columns(np.random.default_rng(seed), m, n)
    norms = phi ** np.arange(n)
    return Q * norms, norms ** 2


def _truncation_samples(trials, l, J, m, n, phi, seed):
    A, norms2 = _orthogonal_columns(seed, m, n, phi)
    rng = np.random.default_rng(seed + 1)
    xs, taus = [], []
    for _ in range(trials):
        B = rng.standard_normal((l, m)) @ A
        out = oracle.sample_qrcp(B, J)
        perm = ss.permutation_from_swaps(out["piv"], n)
        x, tau = ss.trailing_statistics(out["S"], J, norms2[perm])
        xs.append(x)
        taus.append(tau)
    return np.concatenate(xs), np.concatenate(taus)


def test_trailing_norms_follow_truncated_chi2():
    """The theorem on the oracle's sample QRCP: every remaining column obeys
    x <= tau (the earlier pivot decisions), and u = G(x) / G(tau) with l - J
    degrees of freedom is uniform (Kolmogorov-Smirnov) with the mean of the
    theorem's expectation.  One degree of freedom more or less is rejected,
    so the check has power."""
    l, J = 12, 4
    x, tau = _truncation_samples(400, l, J, 80, 64, 0.97, 5)
    assert np.all(x <= tau * (1 + 1e-12))
    d = l - J
    u = ss.truncated_chi2_cdf(d, tau, x)
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    r = x - ss.truncated_chi2_mean(d, tau)
    assert abs(r.mean()) <= 4 * r.std(ddof=1) / np.sqrt(len(r))
    for dd in (d - 1, d + 1):
        assert stats.kstest(ss.truncated_chi2_cdf(dd, tau, x), "uniform").pvalue < 1e-6


def test_trailing_statistics_small_case_by_hand():
    """Two steps on a 3 x 3 sample: tau and x from the definitions written
    out element by element."""
    S = np.array([[5.0, 1.0, 2.0], [0.0, 4.0, 1.5], [0.0, 0.0, 0.5]])
    x, tau = ss.trailing_statistics(S, 2, np.array([9.0, 9.0, 4.0]))
    assert np.allclose(x, [0.25 / 4.0])
    # i = 0: 25 - (2^2 + 1.5^2); i = 1: 16 - 1.5^2
    assert np.allclose(tau, [min(25 - 4 - 2.25, 16 - 2.25) / 4.0])
    assert list(ss.permutation_from_swaps([2, 2], 4)) == [2, 0, 1, 3]
