"""RQRCP (Alg. 4), TRQRCP (Alg. 6) and the unpivoted blocked QR the paper
compares against (Section 7: RQRCP with the sketch and the pivoting taken out).

Conventions (readings of points the paper leaves open):

* Blocks: block J starts at column i0 and has width bJ = min(b, k - i0), so b
  need not divide k (Alg. 4 assumes it does).  Full factorization: k = min(m, n).
* Sample QRCP (Alg. 1 run on the sample for bJ steps): trailing squared norms are
  recomputed from the current sample at every step (not downdated); the
  pivot is the largest one, ties go to the lowest current position, and a
  NaN norm never wins (it ranks as -1).  Swaps are sequential: step t
  exchanges positions t and p_t.
* Permutation: the sequential swaps are applied, in order, to all m rows of A
  (completed R rows included) and to jpvt (0-based original column indices).
* Sample update (eq. update1): W11 = S11 R11^-1 is formed first by forward
  substitution over columns; a column whose R11 diagonal is exactly zero gets
  W11 column 0.  Then B1 = S12 - W11 R12 and B2 = S22.  It is skipped after
  the last block.
* Alg. 6 garbles: its function name (rqrcp) is read as trqrcp, "A{[0]}" as
  A^[0], and qrcp(B^[J], b) as qrcp(B^[J-1], b), as in Alg. 4.
* Alg. 5 (RSRQRCP) sizes its new compression matrix l x (m - Jb) for block
  J = 1, 2, ...; the matrix it multiplies, A^[J-1], has the rows i0..m-1
  (i0 = (J-1) b) of the trailing columns, so the size is read as l x (m - i0)
  and the sample as Omega^[J-1] A(i0:m, i0:n).  Block J (0-based) draws its
  matrix from Philox key (seed, J).
"""

import numpy as np

from .householder import householder_qr, larft, reflector, unit_lower
from .philox import omega as make_omega


def _ranked_norms(nu):
    """Replace NaN by -1 so that it never wins an argmax."""
    nu = np.array(nu, dtype=np.float64, copy=True)
    bad = np.isnan(nu)
    nu[bad] = -1.0
    return nu, bool(bad.any())


def sample_qrcp(B, bJ):
    """Partial QRCP with bJ steps on the l x nJ sample B (Alg. 1 on B).

    Returns dict(S, piv, gaps, refl, info):
      S     transformed sample: S[:, :bJ] upper part = S11, S[:bJ, bJ:] = S12,
            S[bJ:, bJ:] = S22 (the sample reflectors are not kept in S);
      piv   swap partners p_t (local positions), t = 0..bJ-1;
      gaps  relative gap (nu_1 - nu_2) / nu_1 between the two best norms;
      refl  list of (t, y, tau) sample reflectors acting on rows t..l-1;
      info  1-based first step with a non-finite norm, else 0.
    """
    S = np.array(B, dtype=np.float64, copy=True)
    l, n = S.shape
    piv, gaps, refl = [], [], []
    info = 0
    for t in range(bJ):
        nu = np.sum(S[t:, t:] ** 2, axis=0)
        nu, had_nan = _ranked_norms(nu)
        if (had_nan or np.isinf(nu).any()) and info == 0:
            info = t + 1
        j = int(np.argmax(nu))  # first maximum = lowest position on ties
        if len(nu) > 1:
            second = np.max(np.delete(nu, j))
            gaps.append(1.0 if nu[j] <= 0 else float((nu[j] - second) / nu[j]))
        else:
            gaps.append(1.0)
        pt = t + j
        piv.append(pt)
        if pt != t:
            S[:, [t, pt]] = S[:, [pt, t]]
        # Householder on the pivot column, rows t..l-1 (dlarfg convention).
        y, tau, beta = reflector(S[t:, t])
        S[t, t] = beta
        S[t + 1:, t] = 0.0
        if tau != 0.0 and t + 1 < n:
            w = tau * (y @ S[t:, t + 1:])
            S[t:, t + 1:] -= np.outer(y, w)
        refl.append((t, y, tau))
    return dict(S=S, piv=piv, gaps=gaps, refl=refl, info=info)


def apply_swaps(M, piv, offset):
    """Sequential column swaps (offset + t) <-> (offset + p_t) on M, in place."""
    for t, pt in enumerate(piv):
        a, c = offset + t, offset + pt
        if a != c:
            M[..., [a, c]] = M[..., [c, a]]


def sample_update(S, bJ, R11, R12):
    """Eq. update1: B1 = S12 - S11 R11^-1 R12, B2 = S22 (W11 = S11 R11^-1 first)."""
    S11 = np.triu(S[:bJ, :bJ])
    W11 = np.zeros((bJ, bJ))
    for j in range(bJ):  # solve W11 R11 = S11 column by column
        d = R11[j, j]
        if d == 0.0:
            continue
        W11[:, j] = (S11[:, j] - W11[:, :j] @ R11[:j, j]) / d
    B1 = S[:bJ, bJ:] - W11 @ R12
    B2 = S[bJ:, bJ:]
    return np.vstack([B1, B2]), W11


def _setup(A, b, p, seed, Omega):
    A = np.array(A, dtype=np.float64, copy=True, order="F")
    m, n = A.shape
    l = b + p
    if Omega is None:
        Omega = make_omega(seed, l, m)
    Omega = np.asarray(Omega, dtype=np.float64)
    assert Omega.shape == (l, m)
    return A, m, n, l, Omega


def rqrcp(A, b, p, seed=None, Omega=None, k=None, trace=False):
    """Alg. 4 (RQRCP).  Returns dict(F, tau, jpvt, gaps, info[, trace]).

    F is A overwritten in the in-place layout: R on and above the diagonal,
    reflector tails below it.  With k < min(m, n) (truncated RQRCP with
    trailing update), rows k.. of the trailing columns hold the updated
    trailing matrix A^[J].
    """
    A, m, n, l, Omega = _setup(A, b, p, seed, Omega)
    kk = min(m, n) if k is None else k
    jpvt = np.arange(n, dtype=np.int64)
    tau = np.zeros(kk)
    gaps, info, blocks = [], 0, []
    B = Omega @ A  # the sketch B = Omega A of Alg. 4
    i0 = 0
    while i0 < kk:
        bJ = min(b, kk - i0)
        # bJ pivots chosen on the sample (Alg. 1)
        sq = sample_qrcp(B, bJ)
        gaps += sq["gaps"]
        if sq["info"] and not info:
            info = i0 + sq["info"]
        # the same column exchanges on A (every row) and on jpvt
        apply_swaps(A, sq["piv"], i0)
        apply_swaps(jpvt, sq["piv"], i0)
        # Householder QR of the bJ chosen columns
        Fp, tp = householder_qr(A[i0:, i0:i0 + bJ])
        A[i0:, i0:i0 + bJ] = Fp
        tau[i0:i0 + bJ] = tp
        Y = unit_lower(Fp, bJ)
        T = larft(Y, tp)
        # the block's rows of R and the trailing columns: C <- Q^T C
        if i0 + bJ < n:
            C = A[i0:, i0 + bJ:]
            Wt = T.T @ (Y.T @ C)
            C -= Y @ Wt
        rec = None
        if trace:
            rec = dict(i0=i0, bJ=bJ, B=B.copy(), S=sq["S"], refl=sq["refl"], piv=list(sq["piv"]),
                       panel=Fp.copy(), tau=tp.copy(), T=T, A_after=A.copy())
        # next sample by eq. (update1), except after the last block
        if i0 + bJ < kk:
            R11 = np.triu(A[i0:i0 + bJ, i0:i0 + bJ])
            R12 = A[i0:i0 + bJ, i0 + bJ:]
            B, W11 = sample_update(sq["S"], bJ, R11, R12)
            if trace:
                rec["W11"] = W11
                rec["B_next"] = B.copy()
        if trace:
            blocks.append(rec)
        i0 += bJ
    out = dict(F=A, tau=tau, jpvt=jpvt, gaps=np.array(gaps), info=info, Omega=Omega)
    if trace:
        out["trace"] = blocks
    return out


def trqrcp(A, k, b, p, seed=None, Omega=None):
    """Alg. 6 (TRQRCP): truncated RQRCP that never updates the trailing matrix.

    Keeps the explicit reflector block Y (m x k) and the inner products
    W^T = T^T Y^T A (k x n, composed block by block with the Section 5.1
    formula W2^T = T2^T (Y2^T A - (Y2^T Y1) W1^T)).  Selected columns are
    formed as A - Y W^T just before they become reflectors, and new rows of R
    just before the sample update.

    Returns dict(F, tau, jpvt, gaps, info, Y, Wt): F rows 0..k-1 hold R
    (k x n upper trapezoidal), columns 0..k-1 below the diagonal hold the
    reflector tails, and F[k:, k:] holds the permuted original entries.
    """
    A, m, n, l, Omega = _setup(A, b, p, seed, Omega)
    assert 1 <= k <= min(m, n)
    jpvt = np.arange(n, dtype=np.int64)
    tau = np.zeros(k)
    Y = np.zeros((m, k))
    Wt = np.zeros((k, n))
    gaps, info = [], 0
    B = Omega @ A
    i0 = 0
    while i0 < k:
        bJ = min(b, k - i0)
        sq = sample_qrcp(B, bJ)
        gaps += sq["gaps"]
        if sq["info"] and not info:
            info = i0 + sq["info"]
        # the column exchanges on A, on the stored inner products and on jpvt
        apply_swaps(A, sq["piv"], i0)
        apply_swaps(Wt, sq["piv"], i0)
        apply_swaps(jpvt, sq["piv"], i0)
        sel = slice(i0, i0 + bJ)
        trail = slice(i0 + bJ, n)
        # the chosen columns brought up to date: A - Y W^T on them only
        Ahat = A[i0:, sel] - Y[i0:, :i0] @ Wt[:i0, sel]
        Fp, tp = householder_qr(Ahat)
        A[i0:, sel] = Fp
        tau[sel] = tp
        Y2 = unit_lower(Fp, bJ)
        T2 = larft(Y2, tp)
        # the new reflectors' products with the trailing columns (Alg. 6 keeps
        # them instead of updating A)
        Wt[i0:i0 + bJ, trail] = T2.T @ (Y2.T @ A[i0:, trail] - (Y2.T @ Y[i0:, :i0]) @ Wt[:i0, trail])
        Y[i0:, sel] = Y2
        # the block's rows of R: the same correction on those rows only
        A[i0:i0 + bJ, trail] = A[i0:i0 + bJ, trail] - Y[i0:i0 + bJ, :i0 + bJ] @ Wt[:i0 + bJ, trail]
        if i0 + bJ < k:
            R11 = np.triu(A[i0:i0 + bJ, sel])
            R12 = A[i0:i0 + bJ, trail]
            B, _ = sample_update(sq["S"], bJ, R11, R12)
        i0 += bJ
    return dict(F=A, tau=tau, jpvt=jpvt, gaps=np.array(gaps), info=info, Y=Y, Wt=Wt, Omega=Omega)


def rsrqrcp(A, b, p, seed=None, omegas=None, k=None):
    """Alg. 5 (RSRQRCP): RQRCP that draws a new compression matrix for every
    block and samples the updated trailing matrix with it, instead of
    updating the sample by eq. update1.  Returns dict(F, tau, jpvt, gaps, info)
    in the layout of rqrcp.

    omegas, if given, is a function (J, mJ) -> Omega^[J] (any number of rows
    l_J, mJ columns); otherwise block J uses the l x mJ matrix of Philox key
    (seed, J), l = b + p.
    """
    A = np.array(A, dtype=np.float64, copy=True, order="F")
    m, n = A.shape
    l = b + p
    kk = min(m, n) if k is None else k
    jpvt = np.arange(n, dtype=np.int64)
    tau = np.zeros(kk)
    gaps, info = [], 0
    i0, J = 0, 0
    while i0 < kk:
        bJ = min(b, kk - i0)
        mJ = m - i0
        # a new compression matrix for this block and the sample of the
        # trailing matrix it gives
        Om = omegas(J, mJ) if omegas is not None else make_omega(seed, l, mJ, key1=J)
        B = np.asarray(Om, dtype=np.float64) @ A[i0:, i0:]
        # bJ pivots chosen on the sample (Alg. 1)
        sq = sample_qrcp(B, bJ)
        gaps += sq["gaps"]
        if sq["info"] and not info:
            info = i0 + sq["info"]
        # the same column exchanges on A (every row) and on jpvt
        apply_swaps(A, sq["piv"], i0)
        apply_swaps(jpvt, sq["piv"], i0)
        # Householder QR of the chosen columns, then their rows of R and the
        # trailing update
        Fp, tp = householder_qr(A[i0:, i0:i0 + bJ])
        A[i0:, i0:i0 + bJ] = Fp
        tau[i0:i0 + bJ] = tp
        Y = unit_lower(Fp, bJ)
        T = larft(Y, tp)
        if i0 + bJ < n:
            C = A[i0:, i0 + bJ:]
            C -= Y @ (T.T @ (Y.T @ C))
        i0 += bJ
        J += 1
    return dict(F=A, tau=tau, jpvt=jpvt, gaps=np.array(gaps), info=info)


def unpivoted_qr(A, b):
    """Blocked Householder QR without pivoting: RQRCP with the sampling and
    pivoting removed (the paper's "qr" comparator).  Returns (F, tau)."""
    A = np.array(A, dtype=np.float64, copy=True, order="F")
    m, n = A.shape
    k = min(m, n)
    tau = np.zeros(k)
    i0 = 0
    while i0 < k:
        bJ = min(b, k - i0)
        Fp, tp = householder_qr(A[i0:, i0:i0 + bJ])
        A[i0:, i0:i0 + bJ] = Fp
        tau[i0:i0 + bJ] = tp
        if i0 + bJ < n:
            Y = unit_lower(Fp, bJ)
            T = larft(Y, tp)
            C = A[i0:, i0 + bJ:]
            C -= Y @ (T.T @ (Y.T @ C))
        i0 += bJ
    return A, tau
