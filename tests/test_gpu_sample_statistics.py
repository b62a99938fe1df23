"""GPU replay of the sample statistics of Section 3 through the C ABI: the
sketch (rq_sketch, Philox Omega) and the sample QRCP (rq_sample_qrcp) of the
product path run on matrices with mutually orthogonal columns of norms phi^j,
and their outcomes are compared with the oracle's exact laws:

* Fig. selectExpect (Section 3.2): the first pivot of the sample, i.e. the
  column of largest sample norm; the mean of ||a_jmax|| over seeded trials
  against the exact expectation (within 4 standard errors);
* Section 3.3: after J sample-QRCP steps, the trailing sample norms follow the
  theorem's truncated Chi-squared law with l - J degrees of freedom (every
  x <= tau, Kolmogorov-Smirnov on G(x) / G(tau), the mean of the paper's
  expectation, one degree of freedom more or less rejected).

Seeds are fixed, so each check has one fixed outcome."""

import time

import numpy as np
import pytest
import torch
from scipy import stats

from oracle import sample_stats as ss
from paper_1509_06820_amd import binding, inputs
from test_gpu_parity import dev, say

pytestmark = pytest.mark.gpu


def _orthogonal_columns(seed, n, phi):
    Q = inputs.haar_columns(np.random.default_rng(seed), n, n)
    norms = phi ** np.arange(n)
    return dev(Q * norms), norms ** 2


def _run_trials(A, l, bsteps, seeds):
    """Sketch + sample QRCP per seed; returns the stacked samples S and swaps."""
    m, n = A.shape
    wk = binding.workspace(binding.RQ_OP_RQRCP, m, n, min(m, n), l, 0, A.device)
    ws = binding.workspace(binding.RQ_OP_SAMPLE_QRCP, l, n, 0, bsteps, 0, A.device)
    Ss, pivs, infos = [], [], []
    for sd in seeds:
        B = binding.rq_sketch(A, l, int(sd), work=wk)
        S, piv, info = binding.rq_sample_qrcp(B, bsteps, work=ws)
        Ss.append(S)
        pivs.append(piv)
        infos.append(info)
    torch.cuda.synchronize()
    assert int(torch.stack(infos).abs().sum().item()) == 0
    return torch.stack(Ss).cpu().numpy(), torch.stack(pivs).cpu().numpy()


@pytest.mark.parametrize("phi,l", [(0.5, 8), (0.9, 8), (0.95, 16), (0.99, 4), (0.99, 32)])
def test_select_expectation_replay(phi, l):
    n, trials = 512, 1500
    say(f"selectExpect replay phi={phi} l={l} n={n} trials={trials}")
    A, _ = _orthogonal_columns(int(phi * 1000) + l, n, phi)
    t0 = time.time()
    _, piv = _run_trials(A, l, 1, 7_000_000 + 10_000 * l + np.arange(trials))
    dt = time.time() - t0
    vals = phi ** piv[:, 0].astype(np.float64)
    mean, se = vals.mean(), vals.std(ddof=1) / np.sqrt(trials)
    exact = ss.select_expectation(phi, l, n)
    say(f"  E(||a_jmax||) GPU {mean:.4f} +- {se:.4f}, exact {exact:.4f}, {trials / dt:.0f} trials/s")
    assert abs(mean - exact) <= 4 * se


def test_truncated_chi2_replay():
    l, J, n, phi, trials = 16, 6, 256, 0.98, 600
    say(f"truncated chi-squared replay l={l} J={J} n={n} phi={phi} trials={trials}")
    A, norms2 = _orthogonal_columns(99, n, phi)
    S, piv = _run_trials(A, l, J, 8_000_000 + np.arange(trials))
    xs, taus = [], []
    for t in range(trials):
        perm = ss.permutation_from_swaps(piv[t], n)
        x, tau = ss.trailing_statistics(S[t], J, norms2[perm])
        xs.append(x)
        taus.append(tau)
    x, tau = np.concatenate(xs), np.concatenate(taus)
    # the pivot decisions: no remaining column beats an earlier pivot
    # (downdated norms decide near ties, hence the small margin)
    assert np.all(x <= tau * (1 + 1e-9))
    d = l - J
    p = stats.kstest(ss.truncated_chi2_cdf(d, tau, x), "uniform").pvalue
    r = x - ss.truncated_chi2_mean(d, tau)
    z = r.mean() / (r.std(ddof=1) / np.sqrt(len(r)))
    say(f"  {len(x)} trailing norms: KS p = {p:.3f}, mean residual {z:.2f} standard errors")
    assert p > 1e-3
    assert abs(z) <= 4
    for dd in (d - 1, d + 1):
        assert stats.kstest(ss.truncated_chi2_cdf(dd, tau, x), "uniform").pvalue < 1e-6
