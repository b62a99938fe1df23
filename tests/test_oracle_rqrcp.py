"""Pins for the oracle's sample QRCP and RQRCP (Alg. 1 on the sample, Alg. 4,
eq. sample, eq. sampleR and eq. update1)."""

import itertools

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.linalg.lapack as lapack
from hypothesis import given, settings, strategies as st

import oracle
from oracle import qrcp as rq
from paper_1509_06820_amd import inputs


# ---------------------------------------------------------------- helpers
def selected_columns(piv, n):
    """Original column indices in selection order from sequential swaps."""
    perm = list(range(n))
    for t, pt in enumerate(piv):
        perm[t], perm[pt] = perm[pt], perm[t]
    return perm


def greedy_qrcp_bruteforce(B, steps):
    """Greedy QRCP by the determinant-growth view (Section 2.1): the next
    pivot maximises det(G_{S+c}) / det(G_S), G = B^T B.  Returns (order, gaps)."""
    G = B.T @ B
    S, gaps = [], []
    for _ in range(steps):
        d0 = np.linalg.det(G[np.ix_(S, S)]) if S else 1.0
        res = {}
        for c in range(B.shape[1]):
            if c in S:
                continue
            idx = S + [c]
            res[c] = np.linalg.det(G[np.ix_(idx, idx)]) / d0
        best = sorted(res.items(), key=lambda kv: (-kv[1], kv[0]))
        S.append(best[0][0])
        gaps.append((best[0][1] - best[1][1]) / best[0][1] if len(best) > 1 else 1.0)
    return S, gaps


def q_from(F, tau):
    Q, _, info = lapack.dorgqr(F.copy(), tau)
    assert info == 0
    return Q


def residuals(A, out):
    F, tau, jpvt = out["F"], out["tau"], out["jpvt"]
    m, n = A.shape
    k = len(tau)
    Q = q_from(np.asfortranarray(F[:, :k]), tau)
    R = np.triu(F[:k, :])
    res = np.linalg.norm(A[:, jpvt] - Q @ R) / np.linalg.norm(A)
    orth = np.linalg.norm(Q.T @ Q - np.eye(k))
    return res, orth


def product_of_reflectors(nrows, reflectors):
    """Explicit H_0 H_1 ... for a list of (t, y, tau) acting on rows t.."""
    Q = np.eye(nrows)
    for t, y, tau in reflectors:
        H = np.eye(nrows)
        H[t:, t:] -= tau * np.outer(y, y)
        Q = Q @ H
    return Q


# ---------------------------------------------------------------- sample QRCP
@pytest.mark.parametrize("seed", range(12))
def test_sample_qrcp_matches_bruteforce_greedy(seed):
    rng = np.random.default_rng(1000 + seed)
    for _ in range(200):  # rejection-sample well separated inputs
        l, n, b = 8, int(rng.integers(4, 9)), int(rng.integers(1, 5))
        B = rng.standard_normal((l, n)) * rng.uniform(0.2, 3.0, size=n)
        order, gaps = greedy_qrcp_bruteforce(B, b)
        if min(gaps) > 0.1:
            break
    else:
        pytest.skip("no separated input drawn")
    sq = rq.sample_qrcp(B, b)
    assert selected_columns(sq["piv"], n)[:b] == order


@pytest.mark.parametrize("seed", range(6))
def test_sample_qrcp_factorization_and_dgeqp3(seed):
    rng = np.random.default_rng(seed)
    l, n, b = 40, 300, 32
    B = rng.standard_normal((l, n)) @ np.diag(rng.uniform(0.5, 2, n))
    sq = rq.sample_qrcp(B, b)
    perm = selected_columns(sq["piv"], n)
    Qb = product_of_reflectors(l, sq["refl"])
    S = sq["S"]
    # B P = Q_b S with S zero below the diagonal in the first b columns
    assert np.allclose(Qb @ S, B[:, perm], atol=1e-13 * np.linalg.norm(B))
    assert np.allclose(np.tril(S[:, :b], -1), 0)
    # LAPACK dgeqp3 (norm downdating) picks the same first b pivots on
    # inputs whose pivot gaps are not tiny
    if min(sq["gaps"]) > 1e-6:
        _, _, P = sl.qr(B, pivoting=True, mode="economic")
        assert list(P[:b]) == perm[:b]


def test_sample_qrcp_ties_and_nan():
    B = np.array([[1.0, 2.0, 2.0, 0.5], [0.0, 0.0, 0.0, 0.1]])
    sq = rq.sample_qrcp(B, 1)
    assert sq["piv"] == [1]  # tie between columns 1 and 2: lowest position
    B = np.array([[np.nan, 1.0, 3.0], [1.0, 0.0, 0.0]])
    sq = rq.sample_qrcp(B, 1)
    assert sq["piv"] == [2] and sq["info"] == 1
    Z = np.zeros((3, 4))
    sq = rq.sample_qrcp(Z, 3)
    assert sq["piv"] == [0, 1, 2] and np.all(sq["S"] == 0)


# ---------------------------------------------------------------- RQRCP
@pytest.mark.parametrize("m,n,b,p,seed", [
    (512, 512, 32, 8, 1),     # the 512 x 512 configuration
    (300, 200, 24, 8, 4),     # tall, b does not divide k
    (150, 260, 16, 5, 5),     # wide
    (97, 97, 97, 3, 6),       # a single block
    (64, 40, 1, 4, 7),        # b = 1
])
def test_rqrcp_ap_equals_qr(m, n, b, p, seed):
    if (m, n) == (512, 512):
        A, _ = inputs.config_matrix("c1", seed)
    else:
        A = inputs.with_spectrum(seed, m, n, inputs.sigma_decade(min(m, n), 8))
    out = oracle.rqrcp(A, b, p, seed=seed)
    assert sorted(out["jpvt"]) == list(range(n))
    res, orth = residuals(A, out)
    assert res <= 1e-13
    assert orth <= 1e-13
    assert out["info"] == 0


def test_sketch_is_omega_times_a():
    A = inputs.gaussian(9, 13, 11)
    out = oracle.rqrcp(A, 3, 2, seed=9, trace=True)
    Om = oracle.omega(9, 5, 13)
    B0 = out["trace"][0]["B"]
    for r, c in itertools.product(range(5), range(11)):
        s = 0.0
        for i in range(13):
            s += Om[r, i] * A[i, c]
        assert abs(B0[r, c] - s) <= 1e-14 * (1 + abs(s))


@pytest.mark.parametrize("m,n,b,p,seed", [(64, 64, 8, 8, 1), (120, 90, 16, 6, 2), (80, 150, 12, 4, 3)])
def test_sample_update_tracks_explicit_omega(m, n, b, p, seed):
    """eq. sample / eq. sampleR / eq. update1: with Omega carried explicitly
    through Q_b^T Omega Q^[J], W21 R11 = 0, W11 R11 = S11, and the updated
    sample equals the new compression matrix times the trailing matrix."""
    A = inputs.with_spectrum(seed, m, n, inputs.sigma_decade(min(m, n), 10))
    out = oracle.rqrcp(A, b, p, seed=seed, trace=True)
    Om = out["Omega"]
    scale = np.linalg.norm(Om) * np.linalg.norm(A)
    Omega_cur = Om.copy()
    prev = A
    for J, rec in enumerate(out["trace"]):
        i0, bJ = rec["i0"], rec["bJ"]
        A_trail = prev[i0:, i0:]
        assert np.linalg.norm(rec["B"] - Omega_cur @ A_trail) <= 1e-12 * scale
        Qb = product_of_reflectors(b + p, rec["refl"])
        mJ = m - i0
        panel = rec["panel"]
        QJ = product_of_reflectors(mJ, [(j, np.concatenate(([1.0], panel[j + 1:, j])), rec["tau"][j])
                                        for j in range(bJ)])
        Wt = Qb.T @ Omega_cur @ QJ
        R11 = np.triu(panel[:bJ, :bJ])
        S11 = np.triu(rec["S"][:bJ, :bJ])
        assert np.linalg.norm(Wt[bJ:, :bJ] @ R11) <= 1e-14 * scale
        assert np.linalg.norm(Wt[:bJ, :bJ] @ R11 - S11) <= 1e-14 * scale
        if "B_next" in rec:
            Omega_cur = Wt[:, bJ:]
            A_next = rec["A_after"][i0 + bJ:, i0 + bJ:]
            assert np.linalg.norm(rec["B_next"] - Omega_cur @ A_next) <= 1e-12 * scale
        prev = rec["A_after"]


def _separated_matrix(rng, m, n):
    # columns with geometrically spread norms and random directions: QRCP
    # pivot gaps are large at every step
    return rng.standard_normal((m, n)) * (0.7 ** rng.permutation(n))


@pytest.mark.parametrize("seed", range(8))
def test_orthogonal_omega_reduces_to_qrcp(seed):
    """With l = m and Omega orthogonal, sample norms are exact trailing norms,
    so RQRCP makes the pivot decisions of deterministic QRCP (Section 3.1)."""
    rng = np.random.default_rng(seed)
    m, n, b = 24, 20, 4
    A = _separated_matrix(rng, m, n)
    Om = np.linalg.qr(rng.standard_normal((m, m)))[0]
    out = oracle.rqrcp(A, b, m - b, Omega=Om)
    _, _, P = sl.qr(A, pivoting=True, mode="economic")
    if min(out["gaps"][: n - 1]) > 1e-6:
        assert list(out["jpvt"]) == list(P)
    # and brute force on the first steps
    order, gaps = greedy_qrcp_bruteforce(A, 6)
    if min(gaps) > 1e-6:
        assert list(out["jpvt"][:6]) == order


@pytest.mark.parametrize("r,b", [(20, 8), (17, 5), (32, 16)])
def test_exact_rank_is_revealed(r, b):
    A = inputs.rank_r(21, 90, 70, r)
    out = oracle.rqrcp(A, b, 6, seed=3)
    R = np.triu(out["F"][:70])
    nrmA = np.linalg.norm(A)
    assert np.linalg.norm(R[r:, r:]) <= 1e-13 * nrmA
    d = np.abs(np.diag(R))
    assert d[r - 1] > 1e-6 * d[0]
    assert int(np.sum(d > 1e-10 * d[0])) == r


def test_zero_and_nonfinite_inputs():
    out = oracle.rqrcp(np.zeros((20, 15)), 4, 3, seed=1)
    assert np.all(out["F"] == 0) and np.all(out["tau"] == 0)
    assert list(out["jpvt"]) == list(range(15))
    A = inputs.gaussian(1, 20, 15)
    A[3, 7] = np.nan
    out = oracle.rqrcp(A, 4, 3, seed=1)
    assert out["info"] > 0


@settings(max_examples=40, deadline=None)
@given(m=st.integers(1, 14), n=st.integers(1, 14), b=st.integers(1, 6), p=st.integers(0, 5),
       seed=st.integers(0, 2**32 - 1), kind=st.sampled_from(["gauss", "rankdef", "dup"]))
def test_rqrcp_properties(m, n, b, p, seed, kind):
    rng = np.random.default_rng(seed)
    if kind == "gauss":
        A = rng.standard_normal((m, n))
    elif kind == "rankdef":
        r = int(rng.integers(1, min(m, n) + 1))
        A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    else:
        A = rng.standard_normal((m, n))
        A[:, n // 2:] = A[:, : n - n // 2]  # duplicated columns
    out = oracle.rqrcp(A, b, p, seed=seed)
    assert sorted(out["jpvt"]) == list(range(n))
    res, orth = residuals(np.asfortranarray(A), out)
    assert res <= 1e-13 or np.linalg.norm(A) == 0
    assert orth <= 1e-13
