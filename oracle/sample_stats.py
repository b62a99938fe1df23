"""Sample statistics of Section 3: how well the sample's column norms steer
the pivot choice (the selection experiment of Fig. selectExpect, Section 3.2)
and the truncated Chi-squared law of the trailing sample norms after a partial
QRCP of the sample (Section 3.3, its theorem and the expectation that follows
it).  Test infrastructure like the rest of the oracle.

Setting of both experiments: A has mutually orthogonal columns, column j
(0-based) of 2-norm phi^j, so that for a GIID Omega the sample columns
b_j = Omega a_j are independent, ||b_j||^2 = phi^(2j) x_j with x_j
Chi-squared with l degrees of freedom (Section 3.1).

Readings of points the paper leaves open:
* Fig. selectExpect plots E(||a_jmax||) for A with n columns; n is not
  stated.  Here n is an argument; phi^n is meant to be negligible.
* Section 3.3 indexes completed rows 1..j; here the first J steps are rows
  0..J-1 and the trailing sample of a remaining column j' is rows J..l-1.
"""

import numpy as np
from scipy import integrate, special, stats


# ---------------------------------------------------------------- Section 3.2

def select_expectation(phi, l, n):
    """E(||a_jmax||) where jmax maximizes ||b_j||, column norms phi^j, j < n.

    With y_j = ||b_j||^2 = phi^(2j) x_j (independent, x_j Chi-squared(l)),
    y_j has density g_j(y) = g(y / c_j) / c_j and distribution function
    G_j(y) = G(y / c_j), c_j = phi^(2j).  Column j wins when y_j = y and every
    other y_i < y:  P(jmax = j) = integral of g_j(y) prod_{i != j} G_i(y) dy.
    So E = sum_j phi^j P(jmax = j) = integral of
    prod_i G_i(y) sum_j phi^j g_j(y) / G_j(y) dy, one quadrature in y (the
    products in logarithms, so that no factor underflows).  Columns with
    phi^j < 1e-17 are left out: they add less than that to E, and their
    factors G_i are 1 wherever the integrand is not negligible.
    """
    if phi == 0.0 or phi == 1.0:
        return 1.0
    chi = stats.chi2(l)
    j = np.arange(n)
    j = j[phi ** j >= 1e-17]
    c = phi ** (2.0 * j)
    w = phi ** j

    def integrand(y):
        if y <= 0.0:
            return 0.0
        u = y / c
        logG = chi.logcdf(u)
        logg = chi.logpdf(u) - np.log(c)
        return float(np.sum(w * np.exp(np.sum(logG) - logG + logg)))

    top = chi.isf(1e-18)   # P(max_j y_j > top) <= n 1e-18
    val, _ = integrate.quad(integrand, 0.0, top, limit=500, epsabs=1e-14, epsrel=1e-12)
    return val


def select_monte_carlo(phi, l, n, trials, rng):
    """Brute-force draw of the same experiment: GIID Omega (l x n) applied to
    the column norms, the column of largest sample norm taken (first on
    ties).  Returns (mean of phi^jmax, its standard error)."""
    norms = phi ** np.arange(n)
    vals = np.empty(trials)
    for t in range(trials):
        W = rng.standard_normal((l, n))
        s = np.sum(W * W, axis=0) * norms ** 2
        vals[t] = norms[int(np.argmax(s))]
    return vals.mean(), vals.std(ddof=1) / np.sqrt(trials)


# ---------------------------------------------------------------- Section 3.3

def truncated_chi2_mean(d, tau):
    """Expectation of a Chi-squared(d) variable conditioned on x <= tau, in
    the form the paper gives after its theorem: d (1 - e^(-tau/2) / f(d/2,
    tau/2)) with f(s, z) = s gamma(s, z) / z^s (gamma the lower incomplete
    gamma function), and f -> 1 as z -> 0."""
    s, z = 0.5 * d, 0.5 * np.asarray(tau, dtype=np.float64)
    lower = special.gammainc(s, z) * special.gamma(s)      # gamma(s, z)
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(z > 0, s * lower / np.power(z, s, where=z > 0, out=np.ones_like(z)), 1.0)
        return d * (1.0 - np.exp(-z) / f)


def truncated_chi2_cdf(d, tau, x):
    """P(X <= x | X <= tau) for X Chi-squared(d): the theorem's truncated
    density integrated, gamma(d/2, x/2) / gamma(d/2, tau/2)."""
    return special.gammainc(0.5 * d, 0.5 * x) / special.gammainc(0.5 * d, 0.5 * tau)


def trailing_statistics(S, J, col_norms2):
    """The quantities of the theorem after J steps of QRCP on the sample.

    S: the l x n sample after J steps (rows 0..J-1 of S11 | S12 and the
    trailing sample S22 in rows J..l-1, columns in pivoted order);
    col_norms2: the true trailing squared norms ||a_j'||^2 of A's columns in
    the same order (for mutually orthogonal columns, their squared norms).
    For every remaining column j' >= J:
      x_j'   = ||S(J:, j')||^2 / ||a_j'||^2,
      tau_j' = min over i < J of (S(i, i)^2 - sum_{k=i}^{J-1} S(k, j')^2) / ||a_j'||^2
    (each earlier pivot i beat column j', so its squared trailing norm bounds
    j''s trailing sample norm from above).  Returns (x, tau)."""
    S = np.asarray(S, dtype=np.float64)
    l, n = S.shape
    rest = np.arange(J, n)
    a2 = np.asarray(col_norms2, dtype=np.float64)[rest]
    x = np.sum(S[J:, rest] ** 2, axis=0) / a2
    tau = np.full(len(rest), np.inf)
    for i in range(J):
        bound = S[i, i] ** 2 - np.sum(S[i:J, rest] ** 2, axis=0)
        tau = np.minimum(tau, bound / a2)
    return x, tau


def permutation_from_swaps(piv, n):
    """Column order after sequential swaps (step t exchanges t and piv[t])."""
    perm = np.arange(n)
    for t, p in enumerate(piv):
        perm[[t, p]] = perm[[p, t]]
    return perm
