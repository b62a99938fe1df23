"""Gaussian compression matrix Omega for the sketch (Section 3; drawn in the
first step of Alg. 4, l x m with i.i.d. standard normal entries).

The paper asks only for an l x m matrix with i.i.d. unit-variance Gaussian
entries and names no generator.  Reading adopted here (shared with the GPU
path, each side implementing it independently from the published
definitions):

* Raw words: Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw,
  "Parallel random numbers: as easy as 1, 2, 3", SC'11).  Key = (seed, 0);
  the repeated sketches of Alg. 5 use key (seed, J) for block J.
  Block q (q = 0, 1, ...) is the bijection applied to the 256-bit counter
  (q + 1, 0, 0, 0); it yields four 64-bit words.
* Uniforms: u = ((x >> 12) + 1/2) * 2^-52, exactly representable and
  strictly inside (0, 1) (u ranges over [2^-53, 1 - 2^-53]).
* Normals (Box-Muller, 1958): words (x0, x1) -> r cos(2 pi u1), r sin(2 pi u1)
  with r = sqrt(-2 ln u0); words (x2, x3) likewise.
* Layout: Omega[r, c] (r < l, c < m) is normal number t = r*m + c of the
  stream, i.e. lane t % 4 of block t // 4.  Rows therefore do not depend on
  l, and a larger oversampling p only appends rows.

Pinned in tests against numpy.random.Philox (raw words), against the polar
invariants of Box-Muller, and statistically against the sample-norm law
E||Omega a||^2 = l ||a||^2, Var = 2 l ||a||^4 (Section 3).
"""

import numpy as np

_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

# Multipliers and Weyl key increments of Philox4x64 (SC'11, Table 2 / Sec. 5).
PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
PHILOX_M1 = np.uint64(0xCA5A826395121157)
PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)


def _mulhilo64(a, b):
    """Full 128-bit product of uint64 arrays, returned as (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _MASK32, a >> _S32
    b_lo, b_hi = b & _MASK32, b >> _S32
    p00 = a_lo * b_lo
    p01 = a_lo * b_hi
    p10 = a_hi * b_lo
    p11 = a_hi * b_hi
    mid = (p00 >> _S32) + (p01 & _MASK32) + (p10 & _MASK32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b  # wraps modulo 2^64
    return hi, lo


def philox4x64_10(counter, key):
    """Philox4x64-10 bijection.

    counter: uint64 array of shape (N, 4); key: two uint64 values.
    Returns an (N, 4) uint64 array.  Each round maps (c0, c1, c2, c3) to
    (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)); the key
    is bumped by the Weyl constants between rounds.
    """
    with np.errstate(over="ignore"):
        c = np.array(counter, dtype=np.uint64).reshape(-1, 4).copy()
        k0 = np.uint64(key[0])
        k1 = np.uint64(key[1])
        for rnd in range(10):
            if rnd > 0:
                k0 = k0 + PHILOX_W0
                k1 = k1 + PHILOX_W1
            hi0, lo0 = _mulhilo64(PHILOX_M0, c[:, 0])
            hi1, lo1 = _mulhilo64(PHILOX_M1, c[:, 2])
            c = np.stack([hi1 ^ c[:, 1] ^ k0, lo1, hi0 ^ c[:, 3] ^ k1, lo0], axis=1)
    return c


def raw_words(seed, nblocks, key1=0):
    """The first nblocks Philox blocks of the stream with key (seed, key1)
    ((nblocks, 4))."""
    q = np.arange(nblocks, dtype=np.uint64)
    ctr = np.zeros((nblocks, 4), dtype=np.uint64)
    ctr[:, 0] = q + np.uint64(1)
    seed = int(seed)
    return philox4x64_10(ctr, (seed & 0xFFFFFFFFFFFFFFFF, int(key1) & 0xFFFFFFFFFFFFFFFF))


def uniform52(x):
    """u = ((x >> 12) + 0.5) * 2^-52 in (0, 1); every step is exact."""
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(12)).astype(np.float64) + 0.5) * (2.0 ** -52)


def box_muller(words):
    """Four normals per Philox block (see module docstring)."""
    u = uniform52(words)
    r01 = np.sqrt(-2.0 * np.log(u[:, 0]))
    r23 = np.sqrt(-2.0 * np.log(u[:, 2]))
    a01 = 2.0 * np.pi * u[:, 1]
    a23 = 2.0 * np.pi * u[:, 3]
    return np.stack([r01 * np.cos(a01), r01 * np.sin(a01),
                     r23 * np.cos(a23), r23 * np.sin(a23)], axis=1)


def omega(seed, l, m, key1=0):
    """The l x m compression matrix Omega (Alg. 4 / Alg. 6, first steps).

    key1 selects an independent stream with the same layout: Alg. 5 draws a
    new matrix for every block, block J (0-based) from key (seed, J), so its
    first block uses the Omega of Alg. 4."""
    total = l * m
    nblocks = (total + 3) // 4
    z = box_muller(raw_words(seed, nblocks, key1)).reshape(-1)[:total]
    return z.reshape(l, m)
