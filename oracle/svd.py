"""TUXV: approximate truncated SVD built on TRQRCP (Section 6, Alg. 7, eq.
tuxv) followed by the SVD of the small connection matrix X that the paper
mentions as an optional refinement.

Readings of points the paper leaves open:
* Alg. 7 produces U from the QR of Z^(1) = A V (its index shift between U^(j+1)
  and eq. tuxv's U^(1) is read this way); its argument tau is unused.
* j_max counts the multiply-and-factorize steps after the first LQ: j_max = 1
  stops after the QR of A V, j_max = 2 adds the LQ of U^T A, and so on; the
  pair (U, V) of the last step and its X are the approximation A ~ U X V^T.
* TRQRCP runs on a copy of A, because A itself is needed again for A V.
* Only k columns of U and V are formed.
* The SVD of X is a one-sided Jacobi SVD (Hestenes); singular values are
  returned in descending order.  A column of U whose singular value is
  exactly zero is left zero.
"""

import numpy as np

from .householder import form_q, householder_qr
from .qrcp import trqrcp


def jacobi_svd(X, tol=1e-15, max_sweeps=80):
    """One-sided Jacobi SVD of a square X: X = Ux diag(s) Vx^T.

    Cyclic-by-rows sweeps over column pairs (i < j).  For each pair the plane
    rotation [[c, s], [-s, c]] (c = 1/sqrt(1+t^2), s = c t,
    t = sign(z)/(|z| + sqrt(1+z^2)), z = (b - a)/(2g) with a = |x_i|^2,
    b = |x_j|^2, g = x_i . x_j) makes the two columns orthogonal; it is skipped
    when |g| <= tol sqrt(a b).  Sweeps stop when none is applied.
    """
    G = np.array(X, dtype=np.float64, copy=True)
    k = G.shape[1]
    V = np.eye(k)
    for _ in range(max_sweeps):
        rotated = False
        for i in range(k - 1):
            for j in range(i + 1, k):
                a = float(G[:, i] @ G[:, i])
                b = float(G[:, j] @ G[:, j])
                g = float(G[:, i] @ G[:, j])
                if abs(g) <= tol * np.sqrt(a * b) or g == 0.0:
                    continue
                rotated = True
                z = (b - a) / (2.0 * g)
                t = (1.0 if z >= 0 else -1.0) / (abs(z) + np.sqrt(1.0 + z * z))
                c = 1.0 / np.sqrt(1.0 + t * t)
                s = c * t
                gi, gj = G[:, i].copy(), G[:, j].copy()
                G[:, i] = c * gi - s * gj
                G[:, j] = s * gi + c * gj
                vi, vj = V[:, i].copy(), V[:, j].copy()
                V[:, i] = c * vi - s * vj
                V[:, j] = s * vi + c * vj
        if not rotated:
            break
    sig = np.sqrt(np.sum(G * G, axis=0))
    order = np.argsort(-sig, kind="stable")
    sig = sig[order]
    G = G[:, order]
    V = V[:, order]
    U = np.zeros_like(G)
    nz = sig > 0
    U[:, nz] = G[:, nz] / sig[nz]
    return U, sig, V.T


def tuxv(A, k, b, p, seed=None, Omega=None, jmax=1):
    """Alg. 7 plus the SVD of X.  Returns dict(U, s, VT, ...).

    TRQRCP -> Z0 = R P^T -> LQ of Z0 (as QR of Z0^T) gives V (n x k) ->
    Z1 = A V -> QR of Z1 gives U1 (m x k) and X (k x k upper).  With
    jmax > 1 the iterations alternate: an even j forms Z = U^T A and its LQ
    (the QR of Z^T = A^T U) gives a new V and a lower triangular X with
    A ~ U X V^T; an odd j forms Z = A V and its QR gives a new U and an upper
    triangular X.  Finally X = Ux diag(s) Vx^T -> U = U Ux, V^T = Vx^T V^T.
    """
    assert jmax >= 1
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    tr = trqrcp(A, k, b, p, seed=seed, Omega=Omega)
    R = np.triu(tr["F"][:k, :])
    Z0 = np.zeros((k, n))
    Z0[:, tr["jpvt"]] = R  # restore the original column order
    Fz, tz = householder_qr(Z0.T)
    V = form_q(Fz, tz, k)
    j = 1
    while True:
        # Multiply Z = A V, QR-factorize it: U, X upper triangular.
        Z1 = A @ V
        Fu, tu = householder_qr(Z1)
        U1 = form_q(Fu, tu, k)
        X = np.triu(Fu[:k, :k])
        if j == jmax:
            break
        # Multiply Z = U^T A, LQ-factorize it (QR of Z^T): V, X lower triangular.
        Fv, tv = householder_qr(A.T @ U1)
        V = form_q(Fv, tv, k)
        X = np.triu(Fv[:k, :k]).T
        if j + 1 == jmax:
            break
        j += 2
    Ux, s, VxT = jacobi_svd(X)
    return dict(U=U1 @ Ux, s=s, VT=VxT @ V.T, X=X, V=V, U1=U1, Z0=Z0, jpvt=tr["jpvt"], trqrcp=tr)
