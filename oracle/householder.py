"""Householder reflectors and compact-WY blocks (Section 2: H = I - tau y y^T;
Alg. 2 and Section 5.1: Q = I - Y T Y^T with upper-triangular connection
matrix T).

Reading adopted for the reflector scaling (the paper fixes only
tau = 2 / y^T y): the LAPACK dlarfg normalisation, y[0] = 1, which satisfies
that identity.  For x = (alpha, x_tail):
  beta = -sign(alpha) * ||x||,  tau = (beta - alpha) / beta,
  y_tail = x_tail / (alpha - beta),
and tau = 0 (H = I, beta = alpha) when x_tail == 0.  sign(0) = +1.
Norms are plain square roots of sums of squares (no rescaling loop; the
inputs used here are far from overflow or underflow).
"""

import numpy as np


def reflector(x):
    """Return (y, tau, beta) with (I - tau y y^T) x = beta e_1 and y[0] = 1."""
    x = np.asarray(x, dtype=np.float64)
    alpha = x[0]
    tail = x[1:]
    xnorm2 = float(np.dot(tail, tail))
    y = np.zeros_like(x)
    y[0] = 1.0
    if xnorm2 == 0.0:
        return y, 0.0, float(alpha)
    norm = np.sqrt(alpha * alpha + xnorm2)
    beta = -norm if alpha >= 0.0 else norm
    tau = (beta - alpha) / beta
    y[1:] = tail / (alpha - beta)
    return y, float(tau), float(beta)


def apply_reflector(y, tau, C):
    """C <- (I - tau y y^T) C, in place (C has len(y) rows)."""
    if tau == 0.0:
        return C
    w = tau * (y @ C)
    C -= np.outer(y, w)
    return C


def householder_qr(A):
    """Unblocked Householder QR of a tall panel, column by column.

    Returns (F, tau): F holds R on and above the diagonal and the reflector
    tails strictly below it (unit diagonal implicit), as in the in-place
    layout the paper uses for QRCP (Section 2.3).  This is the "qr" step of
    Alg. 4 / Alg. 6 applied to the selected columns.
    """
    F = np.array(A, dtype=np.float64, copy=True)
    m, n = F.shape
    k = min(m, n)
    tau = np.zeros(k)
    for j in range(k):
        y, t, beta = reflector(F[j:, j])
        F[j, j] = beta
        F[j + 1:, j] = y[1:]
        tau[j] = t
        if j + 1 < n:
            apply_reflector(y, t, F[j:, j + 1:])
    return F, tau


def unit_lower(F, k):
    """Explicit m x k reflector block Y from the in-place layout."""
    m = F.shape[0]
    Y = np.tril(F[:, :k], -1)
    Y[np.arange(k), np.arange(k)] = 1.0
    return Y[:m, :k]


def larft(Y, tau):
    """Connection matrix T with H_1 H_2 ... H_b = I - Y T Y^T.

    Forward, columnwise: T[i, i] = tau_i and
    T[:i, i] = -tau_i * T[:i, :i] @ (Y[:, :i]^T y_i)
    (the composition rule of Section 5.1 applied one reflector at a time).
    """
    b = len(tau)
    T = np.zeros((b, b))
    for i in range(b):
        T[i, i] = tau[i]
        if i > 0:
            T[:i, i] = -tau[i] * (T[:i, :i] @ (Y[:, :i].T @ Y[:, i]))
    return T


def form_q(F, tau, ncols=None):
    """First `ncols` columns of Q = H_1 ... H_k, reflectors applied to the
    identity from the last one to the first (explicit Q for TUXV, Alg. 7)."""
    m = F.shape[0]
    k = len(tau)
    if ncols is None:
        ncols = k
    Q = np.zeros((m, ncols))
    Q[np.arange(min(m, ncols)), np.arange(min(m, ncols))] = 1.0
    for j in range(k - 1, -1, -1):
        y = np.concatenate(([1.0], F[j + 1:, j]))
        apply_reflector(y, tau[j], Q[j:, :])
    return Q
