"""Seeded synthetic test matrices shaped like the paper's workloads.

This module only draws inputs.  It holds none of the factorization's
arithmetic, imports neither the GPU library nor the oracle, and is used by
both sides (and by the benchmark) to get identical inputs from a seed.

All generators use numpy's PCG64 ``default_rng(seed)`` and return float64,
Fortran-ordered (column-major) arrays.

* ``gaussian``          i.i.d. N(0, 1) entries: the GIID timing matrices of
                        the paper's experiments (Section 7).
* ``low_rank_plus_noise``  G1 (m x r) @ G2 (r x n) + eps * E, drawn in that
                        order.
* ``with_spectrum``     U diag(sigma) V^T with Haar-random orthonormal
                        factors (QR of a Gaussian with the R-diagonal sign
                        fix), U drawn before V.
* ``sigma_decade``, ``sigma_power`` give the singular value profiles of the
                        configurations (sigma_i = 10^(-10 i/n), 0.9^(i/10)),
                        index i starting at 0.
* ``batch_c4``          the batched workload (512 uneven matrices,
                        sigma_j = 10^(-6 j/n)).
* ``serving_c5``, ``serving_matrix``  the served request stream
                        (sigma_i = 0.95^i).
"""

import numpy as np


def _rng(seed):
    return np.random.default_rng(seed)


def haar_columns(rng, m, r):
    """m x r matrix with orthonormal, Haar-distributed columns (r <= m)."""
    G = rng.standard_normal((m, r))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def gaussian(seed, m, n):
    return np.asfortranarray(_rng(seed).standard_normal((m, n)))


def low_rank_plus_noise(seed, m, n, r, eps):
    rng = _rng(seed)
    G1 = rng.standard_normal((m, r))
    G2 = rng.standard_normal((r, n))
    A = G1 @ G2
    if eps:
        A += eps * rng.standard_normal((m, n))
    return np.asfortranarray(A)


def rank_r(seed, m, n, r):
    """Exactly rank-r product of Gaussian factors (no noise)."""
    return low_rank_plus_noise(seed, m, n, r, 0.0)


def with_spectrum(seed, m, n, sigma, rank=None):
    """U diag(sigma) V^T; U (m x q), V (n x q) Haar, q = min(m, n).

    ``rank`` keeps only the leading singular triplets (use it when the
    remaining sigma are below double-precision resolution of sigma_0; the
    factors are then the leading columns of Haar matrices, which are
    themselves Haar distributed)."""
    rng = _rng(seed)
    q = min(m, n)
    sigma = np.asarray(sigma, dtype=np.float64)
    assert sigma.shape == (q,)
    r = q if rank is None else min(rank, q)
    U = haar_columns(rng, m, r)
    V = haar_columns(rng, n, r)
    return np.asfortranarray((U * sigma[:r]) @ V.T)


def sigma_decade(n, decades=10.0):
    """sigma_i = 10^(-decades * i / n), i = 0..n-1."""
    return 10.0 ** (-decades * np.arange(n) / n)


def sigma_power(n, base, scale=1.0):
    """sigma_i = base^(i / scale), i = 0..n-1."""
    return base ** (np.arange(n) / scale)


def optimal_truncation_error(sigma, k):
    """Eckart-Young: relative Frobenius error of the best rank-k approximation
    of a matrix with singular values sigma (a closed form, not the method)."""
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    return float(np.sqrt(s2[k:].sum() / s2.sum()))


def batch_c4(count=512, seed=4000):
    """The batched workload: matrix i draws from default_rng(seed + i)
    m = round(exp(U(ln 64, ln 2048))), n = round(U(64, m)) (uniform on
    [64, m]), then U diag(sigma) V^T with sigma_j = 10^(-6 j / n) and Haar
    factors (U before V).  Returns a list of (A, params) with k = 32, p = 8."""
    out = []
    for i in range(count):
        rng = _rng(seed + i)
        m = int(round(np.exp(rng.uniform(np.log(64), np.log(2048)))))
        n = int(round(rng.uniform(64, m)))
        q = min(m, n)
        sig = 10.0 ** (-6.0 * np.arange(q) / n)
        U = haar_columns(rng, m, q)
        V = haar_columns(rng, n, q)
        out.append((np.asfortranarray((U * sig) @ V.T), dict(m=m, n=n, k=min(n, 32), p=8, seed=seed + i)))
    return out


def serving_c5(count=2000, seed=5, smin=256, smax=8192):
    """The served request stream: request i (rng = default_rng(seed), drawn in
    order) has m, n = max and min of two log-uniform draws on [smin, smax],
    k uniform in {16, 32, 64, 128, 256} (at most n), precision FP64 or mixed
    with probability 1/2, and an inter-arrival gap drawn as Exp(1) (scaled
    to the arrival rate by the caller).  The matrix itself is drawn by
    serving_matrix(i, m, n), sigma_i = 0.95^i, Haar factors."""
    rng = _rng(seed)
    reqs = []
    for i in range(count):
        a, b = np.exp(rng.uniform(np.log(smin), np.log(smax), size=2))
        m, n = int(round(max(a, b))), int(round(min(a, b)))
        k = int(min(n, rng.choice([16, 32, 64, 128, 256])))
        mixed = bool(rng.uniform() < 0.5)
        gap = float(rng.exponential(1.0))
        reqs.append(dict(i=i, m=m, n=n, k=k, mixed=mixed, gap=gap))
    return reqs


def serving_matrix(i, m, n, seed=5):
    """The matrix of served request i: U diag(0.95^j) V^T, Haar factors from
    default_rng(seed * 100003 + i); triplets below 1e-17 sigma_0 dropped."""
    rng = _rng(seed * 100003 + i)
    q = min(m, n)
    r = min(q, int(np.ceil(np.log(1e-17) / np.log(0.95))))
    sig = 0.95 ** np.arange(r)
    U = haar_columns(rng, m, r)
    V = haar_columns(rng, n, r)
    return np.asfortranarray((U * sig) @ V.T)


# The configurations of the benchmark plan, by name.
def config_matrix(name, seed=None):
    """Return (A, params) for a named configuration.

    c1     512 x 512, sigma_i = 10^(-10 i / 512), b = 32, p = 8, seed 1.
    c2_iid 8192 x 8192 i.i.d. N(0, 1), b = 64, p = 8, seed 2.
    c2_lr  8192 x 8192 rank-512 product of Gaussians + 1e-8 N(0, 1), seed 2.
    c3     20000 x 10000, sigma_i = 0.9^(i/10), k = 256, b = 64, p = 8, seed 3
           (singular triplets below 1e-17 relative are dropped, see with_spectrum).
    """
    if name == "c1":
        s = 1 if seed is None else seed
        return with_spectrum(s, 512, 512, sigma_decade(512)), dict(b=32, p=8, seed=s)
    if name == "c2_iid":
        s = 2 if seed is None else seed
        return gaussian(s, 8192, 8192), dict(b=64, p=8, seed=s)
    if name == "c2_lr":
        s = 2 if seed is None else seed
        return low_rank_plus_noise(s, 8192, 8192, 512, 1e-8), dict(b=64, p=8, seed=s)
    if name == "c3":
        s = 3 if seed is None else seed
        sig = sigma_power(10000, 0.9, 10.0)
        r = int(np.searchsorted(-sig, -1e-17 * sig[0]))
        return with_spectrum(s, 20000, 10000, sig, rank=r), dict(b=64, p=8, seed=s, k=256)
    raise KeyError(name)
