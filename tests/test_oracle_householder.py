"""Pins for reflectors, the compact-WY connection matrix and the unpivoted
blocked QR (Section 2, Section 5.1), against LAPACK (through scipy) and
against explicit products of reflectors."""

import numpy as np
import pytest
import scipy.linalg.lapack as lapack

from oracle import householder as hh
from oracle import qrcp as rq


@pytest.mark.parametrize("seed", range(6))
def test_reflector_matches_lapack_dlarfg(seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(9) * 10.0 ** rng.integers(-3, 4)
    if seed == 1:
        x[0] = 0.0          # sign(0) = +1
    if seed == 2:
        x[0] = -abs(x[0])
    y, tau, beta = hh.reflector(x)
    beta_l, xt, tau_l = lapack.dlarfg(len(x), x[0], x[1:].copy())
    assert np.isclose(beta, beta_l, rtol=1e-14)
    assert np.isclose(tau, tau_l, rtol=1e-14)
    assert np.allclose(y[1:], xt, rtol=1e-13, atol=1e-15)
    H = np.eye(len(x)) - tau * np.outer(y, y)
    e1 = np.zeros(len(x)); e1[0] = beta
    assert np.allclose(H @ x, e1, atol=1e-13 * np.linalg.norm(x))
    assert np.allclose(H @ H.T, np.eye(len(x)), atol=1e-14)


def test_reflector_zero_tail_is_identity():
    y, tau, beta = hh.reflector(np.array([-3.0, 0.0, 0.0]))
    assert tau == 0.0 and beta == -3.0 and np.array_equal(y, [1.0, 0, 0])
    y, tau, beta = hh.reflector(np.zeros(4))
    assert tau == 0.0 and beta == 0.0


@pytest.mark.parametrize("m,n", [(30, 8), (17, 17), (64, 40), (9, 1)])
def test_householder_qr_matches_dgeqrf(m, n):
    A = np.random.default_rng(m * 100 + n).standard_normal((m, n))
    F, tau = hh.householder_qr(A)
    Fl, taul, _, info = lapack.dgeqrf(A.copy())
    assert info == 0
    assert np.allclose(F, Fl, atol=1e-12)
    assert np.allclose(tau, taul, atol=1e-13)


@pytest.mark.parametrize("m,b", [(40, 8), (23, 5), (64, 64)])
def test_larft_is_product_of_reflectors(m, b):
    A = np.random.default_rng(b).standard_normal((m, b))
    F, tau = hh.householder_qr(A)
    Y = hh.unit_lower(F, b)
    T = hh.larft(Y, tau)
    H = np.eye(m)
    for j in range(b):
        H = H @ (np.eye(m) - tau[j] * np.outer(Y[:, j], Y[:, j]))
    assert np.allclose(np.eye(m) - Y @ T @ Y.T, H, atol=1e-13)
    assert np.allclose(np.tril(T, -1), 0)
    # LAPACK dgeqrt returns the same T when its block size covers all columns
    _, Tl, info = lapack.dgeqrt(b, A.copy())
    assert info == 0
    assert np.allclose(T, Tl, atol=1e-13)


def test_form_q_matches_dorgqr():
    A = np.random.default_rng(3).standard_normal((50, 12))
    F, tau = hh.householder_qr(A)
    Q = hh.form_q(F, tau, 12)
    Ql, _, info = lapack.dorgqr(F.copy(), tau)
    assert info == 0
    assert np.allclose(Q, Ql, atol=1e-14)
    assert np.allclose(Q @ np.triu(F[:12]), A, atol=1e-13)


@pytest.mark.parametrize("m,n,b", [(80, 80, 16), (100, 37, 8), (37, 100, 8), (64, 64, 64)])
def test_unpivoted_blocked_qr_matches_dgeqrf(m, n, b):
    # the paper's "qr" comparator: RQRCP with sampling and pivoting removed
    A = np.random.default_rng(7).standard_normal((m, n))
    F, tau = rq.unpivoted_qr(A, b)
    Fl, taul, _, info = lapack.dgeqrf(A.copy())
    assert np.allclose(F, Fl, atol=1e-11)
    assert np.allclose(tau, taul, atol=1e-12)
