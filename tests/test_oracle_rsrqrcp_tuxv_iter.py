"""Pins for RSRQRCP (Alg. 5: a new compression matrix and sample for every
block) and TUXV with j_max > 1 (Alg. 7: alternating LQ and QR steps)."""

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.linalg.lapack as lapack

import oracle
from oracle import philox
from paper_1509_06820_amd import inputs


def _separated_matrix(rng, m, n):
    # geometrically spread column norms, random directions: the QRCP pivot
    # gaps are large at every step
    return rng.standard_normal((m, n)) * (0.7 ** rng.permutation(n))


def _q_of(F, tau):
    k = len(tau)
    Q, _, _ = lapack.dorgqr(np.asfortranarray(F[:, :k]).copy(), tau)
    return Q


# ---------------------------------------------------------------- RSRQRCP

@pytest.mark.parametrize("seed", range(6))
def test_identity_omega_reduces_rsrqrcp_to_qrcp(seed):
    """With Omega^[J] = I (l = m - i0) every sample is the trailing matrix
    itself, so each block's b steps are the steps of deterministic QRCP:
    the pivots and R of LAPACK dgeqp3."""
    rng = np.random.default_rng(seed)
    m, n, b = 40, 30, 6
    A = _separated_matrix(rng, m, n)
    out = oracle.rsrqrcp(A, b, 0, omegas=lambda J, mJ: np.eye(mJ))
    _, R_ref, P = sl.qr(A, pivoting=True, mode="economic")
    assert min(out["gaps"][: n - 1]) > 1e-6
    assert list(out["jpvt"]) == list(P)
    R = np.triu(out["F"][: min(m, n), :])
    assert np.abs(np.abs(R) - np.abs(R_ref)).max() <= 1e-12 * np.linalg.norm(A)


@pytest.mark.parametrize("seed", range(4))
def test_orthogonal_omega_per_block_reduces_rsrqrcp_to_qrcp(seed):
    """An orthogonal mJ x mJ Omega^[J] keeps every trailing column norm, so
    the pivots are those of QRCP again, whatever the matrices are."""
    rng = np.random.default_rng(100 + seed)
    m, n, b = 28, 22, 5
    A = _separated_matrix(rng, m, n)
    mats = {}

    def om(J, mJ):
        mats[J] = np.linalg.qr(rng.standard_normal((mJ, mJ)))[0]
        return mats[J]

    out = oracle.rsrqrcp(A, b, 0, omegas=om)
    _, _, P = sl.qr(A, pivoting=True, mode="economic")
    assert list(out["jpvt"]) == list(P)
    assert sorted(mats) == list(range(len(mats)))
    assert [mats[J].shape[0] for J in sorted(mats)] == [m - b * J for J in sorted(mats)]


@pytest.mark.parametrize("m,n,b,p", [(150, 97, 16, 5), (97, 150, 16, 8), (64, 64, 64, 8), (120, 80, 13, 3)])
def test_rsrqrcp_ap_equals_qr(m, n, b, p):
    A = inputs.gaussian(m + n, m, n)
    out = oracle.rsrqrcp(A, b, p, seed=m)
    F, tau, jpvt = out["F"], out["tau"], out["jpvt"]
    k = min(m, n)
    assert sorted(jpvt) == list(range(n))
    Q = _q_of(F, tau)
    R = np.triu(F[:k, :])
    nrm = np.linalg.norm(A)
    assert np.linalg.norm(A[:, jpvt] - Q @ R) <= 1e-13 * nrm
    assert np.linalg.norm(Q.T @ Q - np.eye(k)) <= 1e-13


def test_rsrqrcp_first_block_is_rqrcp():
    """Block 0 of Alg. 5 samples A with the Omega of Alg. 4 (key (seed, 0)),
    so its pivots and reflectors are those of RQRCP's first block."""
    A = inputs.with_spectrum(9, 130, 110, inputs.sigma_decade(110, 8))
    b = 16
    rs = oracle.rsrqrcp(A, b, 8, seed=9)
    rq = oracle.rqrcp(A, b, 8, seed=9)
    assert np.array_equal(rs["jpvt"][:b], rq["jpvt"][:b])
    assert np.allclose(rs["F"][:, :b], rq["F"][:, :b], atol=1e-13 * np.linalg.norm(A))


def test_rsrqrcp_blocks_use_independent_streams():
    """Omega^[J] is the Philox stream of key (seed, J): raw words against
    numpy's Philox with the same 128-bit key, and different blocks differ."""
    seed, J = 77, 3
    l, m = 9, 30
    nb = (l * m + 3) // 4
    ref = np.random.Philox(key=(J << 64) | seed).random_raw(4 * nb).reshape(nb, 4)
    assert np.array_equal(philox.raw_words(seed, nb, key1=J), ref)
    z = philox.box_muller(ref).reshape(-1)[: l * m].reshape(l, m)
    assert np.array_equal(philox.omega(seed, l, m, key1=J), z)
    assert not np.allclose(philox.omega(seed, l, m, key1=0), philox.omega(seed, l, m, key1=1))
    assert np.array_equal(philox.omega(seed, l, m, key1=0), philox.omega(seed, l, m))


@pytest.mark.parametrize("r,b", [(20, 8), (17, 5)])
def test_rsrqrcp_reveals_exact_rank(r, b):
    A = inputs.rank_r(31, 90, 70, r)
    out = oracle.rsrqrcp(A, b, 6, seed=31)
    R = np.triu(out["F"][:70, :])
    nrm = np.linalg.norm(A)
    assert np.linalg.norm(R[r:, r:]) <= 1e-12 * nrm
    assert np.abs(np.diag(R)[:r]).min() > 1e-8 * nrm


# ---------------------------------------------------------------- TUXV, j_max > 1

def _tuxv_error(A, out):
    return np.linalg.norm(A - (out["U"] * out["s"]) @ out["VT"]) / np.linalg.norm(A)


@pytest.mark.parametrize("m,n,k", [(90, 70, 10), (70, 110, 16)])
def test_tuxv_error_never_increases_with_jmax(m, n, k):
    """Each step replaces the approximation by the best one with the same
    column (QR step) or row (LQ step) space, so the error never grows and
    never beats Eckart-Young."""
    sig = inputs.sigma_power(min(m, n), 0.93)
    A = inputs.with_spectrum(m * n, m, n, sig)
    errs = [_tuxv_error(A, oracle.tuxv(A, k, 8, 4, seed=2, jmax=j)) for j in range(1, 7)]
    e_opt = inputs.optimal_truncation_error(sig, k)
    for a, c in zip(errs, errs[1:]):
        assert c <= a * (1 + 1e-12)
    assert errs[-1] >= e_opt * (1 - 1e-9)
    assert errs[-1] < errs[0]


def test_tuxv_iterations_converge_to_optimum_with_gap():
    """A spectrum with sigma_{k+1} / sigma_k = 0.1: the alternating steps are
    a subspace iteration and reach the Eckart-Young error."""
    m, n, k = 80, 60, 8
    sig = np.concatenate([np.linspace(2.0, 1.0, k), 0.1 * np.linspace(1.0, 0.5, n - k)])
    A = inputs.with_spectrum(5, m, n, sig)
    e_opt = inputs.optimal_truncation_error(sig, k)
    e = _tuxv_error(A, oracle.tuxv(A, k, 8, 2, seed=5, jmax=8))
    assert abs(e - e_opt) <= 1e-10 * e_opt
    s = oracle.tuxv(A, k, 8, 2, seed=5, jmax=8)["s"]
    assert np.abs(s - sig[:k]).max() <= 1e-10


@pytest.mark.parametrize("jmax", [1, 2, 3, 4])
def test_tuxv_connection_matrix_alternates_and_bases_orthonormal(jmax):
    A = inputs.gaussian(jmax, 60, 50)
    out = oracle.tuxv(A, 12, 4, 4, seed=jmax, jmax=jmax)
    X = out["X"]
    if jmax % 2:
        assert np.array_equal(X, np.triu(X))
    else:
        assert np.array_equal(X, np.tril(X))
    assert np.linalg.norm(out["U"].T @ out["U"] - np.eye(12)) <= 1e-13
    assert np.linalg.norm(out["VT"] @ out["VT"].T - np.eye(12)) <= 1e-13
    assert np.all(np.diff(out["s"]) <= 0)


def test_tuxv_jmax_closed_forms():
    """j_max = 2 gives U1 U1^T A (the best approximation with the columns of
    U1, the basis of the j_max = 1 step); j_max = 3 gives A V2 V2^T with
    span V2 = span(A^T U1)."""
    A = inputs.with_spectrum(3, 70, 55, inputs.sigma_decade(55, 5))
    k = 9
    one = oracle.tuxv(A, k, 8, 4, seed=3, jmax=1)
    U1 = one["U1"]
    two = oracle.tuxv(A, k, 8, 4, seed=3, jmax=2)
    nrm = np.linalg.norm(A)
    assert np.linalg.norm((two["U"] * two["s"]) @ two["VT"] - U1 @ (U1.T @ A)) <= 1e-12 * nrm
    V2 = np.linalg.qr(A.T @ U1)[0]
    three = oracle.tuxv(A, k, 8, 4, seed=3, jmax=3)
    assert np.linalg.norm((three["U"] * three["s"]) @ three["VT"] - (A @ V2) @ V2.T) <= 1e-12 * nrm
