// Batched TRQRCP + TUXV (Alg. 6 and Alg. 7 with j_max = 1, Sections 5.1 and
// 6) for many independent small matrices of uneven sizes.
//
// Every stage of the method is ONE persistent launch over the whole batch:
// the products of all matrices go through the grouped GEMM (one list of
// output tiles across every matrix, walked by a grid of at most a few
// workgroups per CU), the latency-bound per-matrix steps (the sample QRCP,
// Cholesky factors of b x b and k x k Gram matrices, the triangular solve of
// the sample update, the SVD of X) run one workgroup per matrix on a grid
// that walks the matrices.  The host builds the whole launch sequence once
// (a plan: every descriptor and tile list uploaded into the caller's
// workspace), after which running the batch enqueues kernels only -- no
// copies, no allocation, no host synchronisation -- so a plan can be
// captured into a HIP graph and replayed.
//
// Orthogonal factors are formed explicitly instead of as Householder
// reflectors: for small matrices every step is then a product over the
// batch plus a tiny per-matrix factorization.  Block J of TRQRCP takes the b
// pivots that the sample QRCP (Alg. 1 on the l x nJ sample, l = b + p)
// chooses, gathers those columns P of A, removes their components along the
// columns Q already found (twice: classical Gram-Schmidt with
// re-orthogonalisation, the explicit form of Alg. 6's A - Y W^T), and
// orthonormalises P by CholeskyQR with a diagonal shift (three passes:
// Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa, "Shifted CholeskyQR
// for computing the QR factorization of ill-conditioned matrices", SISC
// 2020).  The new rows of R are Rr(i0:i0+b, :) = Q_J^T A in the original
// column order, which is exactly Z0 = R P^T of eq. (tuxv).  The sample
// update, eq. (update1), uses R11 and R12 gathered from those rows in the
// sample's column order (R11^-1 R12 does not depend on the signs of the
// rows of R, so the positive-diagonal convention of CholeskyQR gives the
// refreshed sample of the Householder convention).  TUXV: V from the
// CholeskyQR of Z0^T = Rr^T, Z1 = A V, U1 and X from the CholeskyQR of Z1
// (X is the product of the three passes' triangular factors), the SVD of X
// by one-sided Jacobi in LDS, U = U1 Ux and VT = Vx^T V^T.
//
// Limits: l = b + p <= 64 (one sample row per lane), k <= 64 and b | k,
// k <= min(m_i, n_i), n_i <= 8192.
#include <algorithm>
#include <cstring>
#include <vector>

#include "rqrcp.h"
#include "kernels.hpp"

namespace rq {

namespace {

constexpr int BT_T = 512;       // threads of the per-matrix kernels
constexpr int BT_W = BT_T / WAVE;
constexpr int BT_NMAX = 8192;   // sample columns (norms in LDS)
constexpr int BT_KMAX = 64;
constexpr int BT_GP = 16 * 32 * 32;  // doubles of a matrix's Gram partials
constexpr int BT_LD = BT_KMAX + 1;  // LDS pitch of the small matrices
// rows of the batched sample: l rounded up to a multiple of 8 (the rows past l are zero)
__host__ __device__ inline int sample_rows(int l) { return (l + 7) & ~7; }
// dynamic LDS of the sample QRCP: nmax norms (double) and nmax reference norms (float)
inline size_t sample_lds_bytes(int64_t nmax) { return (size_t)((std::max<int64_t>(nmax, 1) * 12 + 15) / 16 * 16); }

// Per-matrix state of a batched run (device resident, built by the plan).
struct BMat {
  int64_t m, n, lda;
  const double* A;
  double* U;
  int64_t ldu;
  double* sigma;
  double* VT;
  int64_t ldvt;
  int64_t* jpvt_out;  // optional: the k pivots
  uint64_t seed;
  double* om;     // Omega^T: m x l, ld m (Omega(r, c) at om[c + r m])
  double* smp;    // sample, row-major: S(r, c) at smp[c + r n], rows padded to a multiple of 8 (zero past l)
  int* jp;        // n: original column at each position
  int* piv;       // b: swap partners of the current block (local positions)
  double* Q;      // m x k, ld m
  double* Rr;     // k x n, ld k
  double* P;      // m x k, ld m
  double* P2;     // m x k, ld m
  double* Rg;     // b x n, ld b
  double* V;      // n x k, ld n
  double* V2;     // n x k, ld n
  double* G;      // k x k (ld k): Q^T P of the panel's re-orthogonalisation
  double* Gp;     // split-K partials of a Gram matrix (BT_GP doubles)
  double* Ri;     // k x k: inverse of the Cholesky factor
  double* X;      // k x k: accumulated triangular factor
  double* W11;    // b x b
  double* Ux;     // k x k
  double* Vx;     // k x k
  double* sg;     // k
  int* info;      // 1 word
};

__device__ __forceinline__ double wsum(double v) { return wave_sum_x(v); }

// ---------------------------------------------------------------- sample QRCP
// Alg. 1 for b steps on the l x nJ sample S of one matrix (row-major: row r
// of the columns i0.. at smp + i0 + r n), one workgroup per matrix and one
// thread per column: a thread holds its column's l rows in registers
// (LMAX >= l), so the inner product with the reflector and the update need
// no cross-lane reduction and the rows of consecutive columns are read and
// written coalesced.  Rows above t are read and written back unchanged (the
// reflector is zero there), which keeps every register index a constant.  Trailing norms
// start exact and are downdated after each step with the column's new
// row-t entry (the reflector keeps the norm of rows >= t), recomputed
// exactly once a norm has fallen below a tenth of its last exact value
// (as the single-matrix kernel does: relative error about 64 eps * 10);
// ties go to the lowest position, a NaN norm never wins; swaps are
// sequential (step t exchanges positions t and p) and are applied to the
// matrix's column order jp at positions i0 + t.
// Dynamic LDS: nmax doubles (norms) then nmax floats (the last exact norm of
// each column, used only by the recomputation test); nmax = the batch's
// largest n, so small matrices leave room for more workgroups per CU.
// LMAX = sample_rows(l): the padding rows are zero, so no row needs a test.
template <int LMAX>
__global__ void __launch_bounds__(BT_T) bt_sample_qrcp_kernel(BMat* __restrict__ mats, int count, int l, int b,
                                                              int64_t i0, int64_t nmax) {
  extern __shared__ double bt_norms[];
  double* nu = bt_norms;
  float* nuref = reinterpret_cast<float*>(bt_norms + nmax);
  __shared__ double v[LMAX];
  __shared__ double rv[BT_W];
  __shared__ int rp[BT_W];
  __shared__ double s_tau;
  __shared__ int s_p;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
  for (int mi = blockIdx.x; mi < count; mi += gridDim.x) {
    BMat& M = mats[mi];
    const int64_t n = M.n, nJ = n - i0;
    const int n32 = (int)n;  // l n < 2^31
    double* S = M.smp + i0;  // S(r, c) at S[c + r n]
    // initial trailing norms (all rows)
    for (int c = tid; c < (int)nJ; c += BT_T) {
      double s2 = 0.0;
#pragma unroll
      for (int r = 0; r < LMAX; ++r) {
        const double x = S[c + r * n32];
        s2 = fma(x, x, s2);
      }
      nu[c] = s2;
      nuref[c] = (float)s2;
    }
    __syncthreads();
    for (int t = 0; t < b; ++t) {
      // argmax over positions >= t (ties: lowest position; NaN ranks -1)
      double bv = -INFINITY;
      int bp = INT_MAX;
      for (int64_t c = t + tid; c < nJ; c += BT_T) {
        double x = nu[c];
        if (x != x) {
          x = -1.0;
          atomicCAS(M.info, 0, (int)(i0 + t + 1));
        }
        if (x > bv) { bv = x; bp = (int)c; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, WAVE);
        const int op = __shfl_xor(bp, off, WAVE);
        if (ov > bv || (ov == bv && op < bp)) { bv = ov; bp = op; }
      }
      if (lane == 0) { rv[w] = bv; rp[w] = bp; }
      __syncthreads();
      if (w == 0) {
        double fv = (lane < BT_W) ? rv[lane] : -INFINITY;
        int fp = (lane < BT_W) ? rp[lane] : INT_MAX;
        for (int off = 32; off > 0; off >>= 1) {
          const double ov = __shfl_xor(fv, off, WAVE);
          const int op = __shfl_xor(fp, off, WAVE);
          if (ov > fv || (ov == fv && op < fp)) { fv = ov; fp = op; }
        }
        const int p = (fp == INT_MAX) ? t : fp;
        // swap columns t and p of the sample (lane = row) and their norms
        const bool inrow = lane < l;
        double xt = inrow ? S[t + lane * n] : 0.0;
        double xp = inrow ? S[p + lane * n] : 0.0;
        if (p != t) {
          if (inrow) {
            S[t + lane * n] = xp;
            S[p + lane * n] = xt;
          }
          if (lane == 0) {
            const double tmp = nu[t];
            nu[t] = nu[p];
            nu[p] = tmp;
            const float tr = nuref[t];
            nuref[t] = nuref[p];
            nuref[p] = tr;
          }
          xt = xp;
        }
        // Householder reflector of column t on rows t..l-1 (dlarfg normalisation)
        const double alpha = __shfl(xt, t, WAVE);
        const double sig = wsum((lane > t && inrow) ? xt * xt : 0.0);
        double tau = 0.0, beta = alpha, scal = 0.0;
        if (sig != 0.0) {
          const double nrm = sqrt(alpha * alpha + sig);
          beta = (alpha >= 0.0) ? -nrm : nrm;
          tau = (beta - alpha) / beta;
          scal = 1.0 / (alpha - beta);
        }
        if (lane < LMAX) v[lane] = (lane < t || !inrow) ? 0.0 : ((lane == t) ? 1.0 : xt * scal);
        if (inrow) S[t + lane * n] = (lane < t) ? xt : ((lane == t) ? beta : 0.0);
        if (lane == 0) {
          s_tau = tau;
          s_p = p;
          M.piv[t] = p;
        }
      }
      __syncthreads();
      const double tau = s_tau;
      // apply to the columns right of t (rows t..l-1) and downdate their
      // trailing norms (rows > t) with the new row-t entry x_t - d (v_t = 1)
      for (int c = t + 1 + tid; c < (int)nJ; c += BT_T) {
        // one running 32-bit offset per pass (recomputed for the store pass,
        // so that no per-row address stays live beside the column)
        double x[LMAX];
        {
          int off = c;
#pragma unroll
          for (int r = 0; r < LMAX; ++r, off += n32) x[r] = S[off];
        }
        const double xt0 = S[c + t * n32];
        // v is read from LDS (one address for the whole workgroup) rather
        // than held in registers next to the column
        double dsum = 0.0;
#pragma unroll
        for (int r = 0; r < LMAX; ++r) dsum = fma(v[r], x[r], dsum);
        const double d = tau * dsum;
        if (tau != 0.0) {
          int off = c;
          asm volatile("" : "+v"(off));
#pragma unroll
          for (int r = 0; r < LMAX; ++r, off += n32) {
            x[r] = fma(-d, v[r], x[r]);
            S[off] = x[r];
          }
        }
        const double xt = xt0 - d;
        double nn = nu[c] - xt * xt;
        if (!(nn >= 0.1 * (double)nuref[c])) {
          double s2 = 0.0;
#pragma unroll
          for (int r = 0; r < LMAX; ++r) s2 = (r > t) ? fma(x[r], x[r], s2) : s2;
          nn = s2;
          nuref[c] = (float)nn;
        }
        nu[c] = nn;
      }
      if (tid == 0) {
        // sequential swap in the column order
        const int p = s_p;
        if (p != t) {
          const int a = M.jp[i0 + t];
          M.jp[i0 + t] = M.jp[i0 + p];
          M.jp[i0 + p] = a;
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- gathers
// GATHER_PANEL: P(:, c) = A(:, jp[i0 + c]), c < b (m rows).
// GATHER_ROWS:  Rg(:, c) = Rr(i0:i0+b, jp[i0 + c]), c < n - i0.
// COPY_PIVOTS:  jpvt_out[c] = jp[c], c < k.
enum { GATHER_PANEL = 0, GATHER_ROWS = 1, COPY_PIVOTS = 2 };

__global__ void __launch_bounds__(256) bt_gather_kernel(BMat* __restrict__ mats, int count, int mode, int64_t i0,
                                                        int b, int k) {
  for (int mi = blockIdx.y; mi < count; mi += gridDim.y) {
    const BMat& M = mats[mi];
    if (mode == GATHER_PANEL) {
      const int64_t tot = M.m * b;
      for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int64_t c = e / M.m, r = e - c * M.m;
        M.P[r + c * M.m] = M.A[r + (int64_t)M.jp[i0 + c] * M.lda];
      }
    } else if (mode == GATHER_ROWS) {
      const int64_t nc = M.n - i0, tot = nc * b;
      for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int64_t c = e / b, r = e - c * b;
        M.Rg[r + c * b] = M.Rr[(i0 + r) + (int64_t)M.jp[i0 + c] * k];
      }
    } else if (M.jpvt_out) {
      for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < k; c += (int64_t)gridDim.x * 256)
        M.jpvt_out[c] = M.jp[c];
    }
  }
}

// jp = identity, info = 0, the sample's padding rows l..L-1 zero
__global__ void __launch_bounds__(256) bt_init_kernel(BMat* __restrict__ mats, int count, int l) {
  const int L = sample_rows(l);
  for (int mi = blockIdx.y; mi < count; mi += gridDim.y) {
    const BMat& M = mats[mi];
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < M.n; c += (int64_t)gridDim.x * 256) {
      M.jp[c] = (int)c;
      for (int r = l; r < L; ++r) M.smp[c + r * M.n] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *M.info = 0;
  }
}

// ---------------------------------------------------------------- Cholesky
// Which Gram matrix a Cholesky launch factors, and of how many rows (for the
// shift): the b x b Gram of the panel (m rows), or the k x k Gram of V
// (n rows) or of Z1 (m rows).
enum { CH_PANEL = 0, CH_V = 1, CH_Z = 2 };

// Split-K of the Gram products that bt_chol_kernel factors: about 256 rows a
// chunk, at most 16 chunks and at most what the partial buffer holds for
// nc x nc; chunk lengths are multiples of 16 (the product's k step).  The
// producer and bt_chol_kernel derive the chunking from the same two numbers.
__host__ __device__ inline int64_t gram_kchunk(int64_t rows, int nc) {
  const int64_t cap = BT_GP / ((int64_t)nc * nc);
  int64_t s = (rows + 255) / 256;
  if (s > 16) s = 16;
  if (s > cap) s = cap;
  if (s < 1) s = 1;
  const int64_t kc = ((rows + s - 1) / s + 15) / 16 * 16;
  return kc < 16 ? 16 : kc;
}
__host__ __device__ inline int gram_chunks(int64_t rows, int nc) {
  return rows > 0 ? (int)((rows + gram_kchunk(rows, nc) - 1) / gram_kchunk(rows, nc)) : 1;
}

// R = chol(G + s I) (upper, R^T R = G + s I) and Ri = R^-1, for the nc x nc
// Gram matrix G held as its split-K partials in M.Gp (ld nc).  shift:
// s = 11 (rows nc + nc (nc + 1)) u tr(G), the first pass of shifted
// CholeskyQR (tr(G) bounds ||X||_2^2 from above); 0 for the later passes.
// A pivot that is not positive (breakdown) is replaced by the smallest
// positive normal so that the pass stays finite, and the matrix's info word
// is set to -4.  With accumulate, X = R X (X = R on the first pass).
__global__ void __launch_bounds__(256) bt_chol_kernel(BMat* __restrict__ mats, int count, int nc, int which,
                                                      int shifted, int accumulate, int first) {
  __shared__ double R[BT_KMAX * BT_LD];
  __shared__ double Ri[BT_KMAX * BT_LD];
  __shared__ double red[256 / WAVE];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
  for (int mi = blockIdx.x; mi < count; mi += gridDim.x) {
    BMat& M = mats[mi];
    // G = the sum of the Gram product's split-K partials (in chunk order)
    const int nz = gram_chunks((which == CH_V) ? M.n : M.m, nc);
    for (int e = tid; e < nc * nc; e += 256) {
      const int j = e / nc, i = e - j * nc;
      double sum = 0.0;
      for (int z = 0; z < nz; ++z) sum += M.Gp[(int64_t)z * nc * nc + i + j * nc];
      R[i + j * BT_LD] = sum;
    }
    __syncthreads();
    if (shifted) {
      double tr = 0.0;
      for (int i = tid; i < nc; i += 256) tr += R[i + i * BT_LD];
      tr = wsum(tr);
      if (lane == 0) red[w] = tr;
      __syncthreads();
      if (tid == 0) {
        double s = 0.0;
        for (int q = 0; q < 256 / WAVE; ++q) s += red[q];
        const double rows = (which == CH_V) ? (double)M.n : (double)M.m;
        const double sh = 11.0 * (rows * nc + (double)nc * (nc + 1)) * 1.1102230246251565e-16 * s;
        red[0] = sh;
      }
      __syncthreads();
      const double sh = red[0];
      for (int i = tid; i < nc; i += 256) R[i + i * BT_LD] += sh;
      __syncthreads();
    }
    // right-looking Cholesky on the upper triangle: row j of R
    for (int j = 0; j < nc; ++j) {
      if (tid == 0) {
        double d = R[j + j * BT_LD];
        if (!(d > 0.0)) {
          d = 2.2250738585072014e-308;
          atomicCAS(M.info, 0, -4);
        }
        R[j + j * BT_LD] = sqrt(d);
      }
      __syncthreads();
      const double rjj = R[j + j * BT_LD];
      for (int c = j + 1 + tid; c < nc; c += 256) R[j + c * BT_LD] /= rjj;
      __syncthreads();
      for (int e = tid; e < (nc - j - 1) * (nc - j - 1); e += 256) {
        const int cc = e / (nc - j - 1), rr = e - cc * (nc - j - 1);
        const int r = j + 1 + rr, c = j + 1 + cc;
        if (r <= c) R[r + c * BT_LD] -= R[j + r * BT_LD] * R[j + c * BT_LD];
      }
      __syncthreads();
    }
    // Ri = R^-1 (upper): column c by back substitution, one thread per column
    for (int c = tid; c < nc; c += 256) {
      for (int i = nc - 1; i >= 0; --i) {
        double s = (i == c) ? 1.0 : 0.0;
        if (i <= c) {
          for (int q = i + 1; q <= c; ++q) s -= R[i + q * BT_LD] * Ri[q + c * BT_LD];
          Ri[i + c * BT_LD] = s / R[i + i * BT_LD];
        } else {
          Ri[i + c * BT_LD] = 0.0;
        }
      }
    }
    __syncthreads();
    for (int e = tid; e < nc * nc; e += 256) {
      const int j = e / nc, i = e - j * nc;
      M.Ri[i + j * nc] = Ri[i + j * BT_LD];
    }
    if (accumulate) {
      // X = R X (both upper triangular); X = R on the first pass
      for (int e = tid; e < nc * nc; e += 256) {
        const int j = e / nc, i = e - j * nc;
        double s = 0.0;
        if (i <= j) {
          if (first) {
            s = R[i + j * BT_LD];
          } else {
            for (int q = i; q <= j; ++q) s += R[i + q * BT_LD] * M.X[q + j * nc];
          }
        }
        Ri[i + j * BT_LD] = s;  // staged: X is read by other threads above
      }
      __syncthreads();
      for (int e = tid; e < nc * nc; e += 256) {
        const int j = e / nc, i = e - j * nc;
        M.X[i + j * nc] = Ri[i + j * BT_LD];
      }
    }
    __syncthreads();
  }
}

// W11 = S11 R11^-1 (b x b): S11 = the sample's leading b x b block (upper
// part), R11 = Rg(:, 0:b) (upper part); column by column as the sample
// update of eq. (update1) reads it; a zero pivot gives a zero column.
__global__ void __launch_bounds__(256) bt_w11_kernel(BMat* __restrict__ mats, int count, int l, int b, int64_t i0) {
  __shared__ double W[BT_KMAX * BT_LD];
  const int tid = threadIdx.x;
  for (int mi = blockIdx.x; mi < count; mi += gridDim.x) {
    const BMat& M = mats[mi];
    const double* S = M.smp + i0;  // S(i, j) at S[j + i n]
    // thread i < b computes row i of W11, left to right
    if (tid < b) {
      const int i = tid;
      for (int j = 0; j < b; ++j) {
        const double d = M.Rg[j + (int64_t)j * b];
        double s = (i <= j) ? S[j + (int64_t)i * M.n] : 0.0;
        for (int q = 0; q < j; ++q) s -= W[i + q * BT_LD] * M.Rg[q + (int64_t)j * b];
        W[i + j * BT_LD] = (d == 0.0) ? 0.0 : s / d;
      }
      for (int j = 0; j < b; ++j) M.W11[i + j * b] = W[i + j * BT_LD];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- SVD of X
// One-sided Jacobi on the k x k X in LDS (the rotation of the single-matrix
// SVD over the round-robin pairs of each sweep), V accumulated; singular
// values in descending order (ties by index), Ux = X V / sigma, Vx = V.
// A pair is rotated by a half wave (32 lanes, one row each) when k <= 32,
// by a whole wave otherwise, so a round's pairs run 16 or 8 at a time
// across the eight waves.
template <bool HALF>
__device__ __forceinline__ double pair_sum(double v) {
  const int lane = (int)(threadIdx.x & (WAVE - 1));
  v += xchg_d<1>(v, lane);
  v += xchg_d<2>(v, lane);
  v += xchg_d<4>(v, lane);
  v += xchg_d<8>(v, lane);
  v += xchg_d<16>(v, lane);
  if (!HALF) v += xchg_d<32>(v, lane);
  return v;
}

template <bool HALF>
__device__ void svd_sweeps(double* X, double* V, int k, int* s_rot, bool& converged) {
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
  const int row = HALF ? (lane & 31) : lane;
  const int slot = HALF ? 2 * w + (lane >> 5) : w;
  constexpr int NSLOT = HALF ? 2 * BT_W : BT_W;
  const int kk = k + (k & 1);
  converged = kk <= 1;
  for (int sweep = 0; sweep < 60 && kk > 1; ++sweep) {
    if (tid == 0) *s_rot = 0;
    __syncthreads();
    for (int r = 0; r < kk - 1; ++r) {
      for (int base = 0; base < kk / 2; base += NSLOT) {
        // every lane takes part in the reductions (zeros for a missing pair)
        const int idx = base + slot;
        int p = 0, q = 0;
        if (idx == 0) { p = kk - 1; q = r; }
        else { p = (r + idx) % (kk - 1); q = (r - idx + kk - 1) % (kk - 1); }
        const bool valid = idx < kk / 2 && p < k && q < k;
        const int i = min(p, q), j = max(p, q);
        const bool in = valid && row < k;
        const double xi = in ? X[row + i * BT_LD] : 0.0;
        const double xj = in ? X[row + j * BT_LD] : 0.0;
        const double sa = pair_sum<HALF>(xi * xi), sb = pair_sum<HALF>(xj * xj), sgm = pair_sum<HALF>(xi * xj);
        if (valid && sgm != 0.0 && fabs(sgm) > 1e-15 * sqrt(sa * sb)) {
          double cs, sn_;
          jacobi_rotation(sa, sb, sgm, cs, sn_);
          if (in) {
            const double vi = V[row + i * BT_LD], vj = V[row + j * BT_LD];
            X[row + i * BT_LD] = cs * xi - sn_ * xj;
            X[row + j * BT_LD] = sn_ * xi + cs * xj;
            V[row + i * BT_LD] = cs * vi - sn_ * vj;
            V[row + j * BT_LD] = sn_ * vi + cs * vj;
          }
          if (row == 0) *s_rot = 1;
        }
      }
      __syncthreads();
    }
    const int rot = *s_rot;
    __syncthreads();
    if (!rot) { converged = true; break; }
  }
}

__global__ void __launch_bounds__(BT_T) bt_svd_kernel(BMat* __restrict__ mats, int count, int k) {
  __shared__ double X[BT_KMAX * BT_LD];
  __shared__ double V[BT_KMAX * BT_LD];
  __shared__ double sn[BT_KMAX];
  __shared__ int s_rot;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
  for (int mi = blockIdx.x; mi < count; mi += gridDim.x) {
    BMat& M = mats[mi];
    for (int e = tid; e < k * k; e += BT_T) {
      const int j = e / k, i = e - j * k;
      X[i + j * BT_LD] = M.X[i + j * k];
      V[i + j * BT_LD] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    bool converged;
    if (k <= 32) svd_sweeps<true>(X, V, k, &s_rot, converged);
    else svd_sweeps<false>(X, V, k, &s_rot, converged);
    if (!converged && tid == 0) atomicCAS(M.info, 0, -2);
    for (int j = w; j < k; j += BT_W) {
      const double x = (lane < k) ? X[lane + j * BT_LD] : 0.0;
      const double s = wsum(x * x);
      if (lane == 0) sn[j] = sqrt(s);
    }
    __syncthreads();
    for (int j = tid; j < k; j += BT_T) {
      const double v = sn[j];
      int rank = 0;
      for (int i = 0; i < k; ++i) rank += (sn[i] > v || (sn[i] == v && i < j)) ? 1 : 0;
      M.sigma[rank] = v;
      const double inv = (v > 0.0) ? 1.0 / v : 0.0;
      for (int rw = 0; rw < k; ++rw) {
        M.Ux[rw + rank * k] = X[rw + j * BT_LD] * inv;
        M.Vx[rw + rank * k] = V[rw + j * BT_LD];
      }
    }
    __syncthreads();
  }
}

}  // namespace

// ======================================================================= plan
// Host side: the plan holds the launch sequence with every device pointer
// resolved; its descriptors and tile lists live in the caller's workspace.
struct BatchOp {
  enum Kind { INIT, OMEGA, GEMM, SQRCP, GATHER, CHOL, W11, SVD } kind = INIT;
  int cfg = GT_64x64;  // GEMM
  bool ta = false, tb = false, f32 = false;
  const GroupedGemm* probs = nullptr;
  const int* tiles = nullptr;
  int64_t ntiles = 0;
  const OmegaJob* jobs = nullptr;  // OMEGA
  int64_t i0 = 0;                  // per-matrix kernels
  int mode = 0, nc = 0, which = 0, shifted = 0, acc = 0, first = 0;
};

}  // namespace rq

struct rq_batch_plan {
  int count = 0;
  int64_t k = 0;
  int b = 0, p = 0, l = 0, precision = RQ_FP64, cfg = rq::GT_64x64;
  int64_t max_n = 0, max_mb = 0, max_m = 0;  // gather grid sizes
  rq::BMat* mats = nullptr;                  // device
  std::vector<rq::BatchOp> ops;
  int wgs = 512;   // persistent grid of the grouped products
  int mwgs = 512;  // grid of the one-workgroup-per-matrix kernels
};

namespace {

using namespace rq;

constexpr int BT_NCALLS_PER_BLOCK = 12;
constexpr int BT_NCALLS_FIXED = 16;

int check_items(const rq_batch_matrix* items, int32_t count, int64_t k, int32_t b, int32_t p, int32_t precision) {
  if (count < 0) return -2;
  if (!items && count > 0) return -1;
  if (k < 1 || k > BT_KMAX) return -3;
  if (b < 1 || k % b != 0) return -4;
  if (p < 0 || b + p > 64) return -5;
  if (precision != RQ_FP64 && precision != RQ_MIXED) return -6;
  for (int i = 0; i < count; ++i) {
    const rq_batch_matrix& it = items[i];
    if (it.m < k || it.m > RQ_MAX_ROWS || it.n < k || it.n > BT_NMAX) return -1;
    if (it.lda < it.m || it.ldu < it.m || it.ldvt < k) return -1;
    if (!it.A || !it.U || !it.sigma || !it.VT) return -1;
  }
  return 0;
}

// Per-matrix buffers, carved in this order from the matrix's region.
void carve_matrix(Carve& cv, int64_t m, int64_t n, int64_t k, int b, int l, BMat& M) {
  M.om = cv.take<double>((size_t)l * m);
  M.smp = cv.take<double>((size_t)sample_rows(l) * n);
  M.jp = cv.take<int>((size_t)n);
  M.piv = cv.take<int>((size_t)b);
  M.Q = cv.take<double>((size_t)m * k);
  M.Rr = cv.take<double>((size_t)k * n);
  M.P = cv.take<double>((size_t)m * k);
  M.P2 = cv.take<double>((size_t)m * k);
  M.Rg = cv.take<double>((size_t)b * n);
  M.V = cv.take<double>((size_t)n * k);
  M.V2 = cv.take<double>((size_t)n * k);
  M.G = cv.take<double>((size_t)k * k);
  M.Gp = cv.take<double>((size_t)BT_GP);
  M.Ri = cv.take<double>((size_t)k * k);
  M.X = cv.take<double>((size_t)k * k);
  M.Ux = cv.take<double>((size_t)k * k);
  M.Vx = cv.take<double>((size_t)k * k);
  M.W11 = cv.take<double>((size_t)b * b);
  M.sg = cv.take<double>((size_t)k);
  M.info = cv.take<int>(1);
}

size_t tiles_bound(const rq_batch_matrix* items, int32_t count, int64_t k, int b, int l) {
  const int nb = (int)(k / b);
  const size_t calls = (size_t)nb * BT_NCALLS_PER_BLOCK + BT_NCALLS_FIXED;
  size_t t = 0;
  for (int i = 0; i < count; ++i) {
    const int64_t m = items[i].m, n = items[i].n;
    // the largest product of a matrix, in the smallest tiles (32 x 32)
    const int64_t tm = (m + 31) / 32, tn = (n + 31) / 32, tk = (k + 31) / 32, tl = (l + 31) / 32;
    t += (size_t)std::max({tl * tn, tk * tn, tm * tk, tn * tk, tk * tk * 16}) * calls;
    // tile indices are 32-bit in the launches (each term is far below 2^62)
    if (t > (size_t)INT32_MAX) return ~(size_t)0;
  }
  return t;
}

// The whole workspace: descriptor region (BMat array, omega jobs, GEMM
// descriptors and tile lists) then the matrices' buffers.
size_t desc_bytes(int32_t count, int64_t k, int b, size_t tiles) {
  const int nb = (int)(k / b);
  const size_t calls = (size_t)nb * BT_NCALLS_PER_BLOCK + BT_NCALLS_FIXED;
  return align_up(sizeof(BMat) * (size_t)count, 256) + align_up(sizeof(OmegaJob) * (size_t)count, 256) +
         calls * (align_up(sizeof(GroupedGemm) * (size_t)count, 256) + 256) + align_up(4 * tiles, 256) + 256;
}

size_t batch_bytes(const rq_batch_matrix* items, int32_t count, int64_t k, int b, int l) {
  Carve cv(nullptr, 0);
  for (int i = 0; i < count; ++i) {
    BMat M;
    carve_matrix(cv, items[i].m, items[i].n, k, b, l, M);
  }
  const size_t tiles = tiles_bound(items, count, k, b, l);
  if (cv.overflowed() || tiles == ~(size_t)0) return ~(size_t)0;  // no workspace can be that large
  return align_up(desc_bytes(count, k, b, tiles), 256) + cv.off + 256;
}

struct Builder {
  rq_batch_plan& plan;
  std::vector<char> img;  // host image of the descriptor region
  size_t off = 0, cap = 0;
  char* dev = nullptr;    // device address of the descriptor region
  std::vector<BMat> mats;
  explicit Builder(rq_batch_plan& pl) : plan(pl) {}

  size_t put_raw(const void* src, size_t bytes) {
    const size_t o = align_up(off, 256);
    if (o + bytes > img.size()) img.resize(o + bytes);
    std::memcpy(img.data() + o, src, bytes);
    off = o + bytes;
    return o;
  }
  // one grouped launch: one product per matrix (spec(i) fills it; a product
  // with an empty output contributes no tile)
  template <class F>
  void gemm(bool ta, bool tb, bool f32, F spec) {
    std::vector<GroupedGemm> probs(plan.count);
    std::vector<int> tiles;
    // the tile of the plan, unless the products are at most 64 columns wide
    // and wider than its tile (the sketch's l = b + p columns with 32 x 32
    // tiles): then 64 x 64, so the long operand is read once
    int cfg = plan.cfg, bm, bn;
    grouped_tile_shape(cfg, &bm, &bn);
    int64_t maxn = 0;
    for (int i = 0; i < plan.count; ++i) {
      GroupedGemm g{};
      spec(i, mats[i], g);
      maxn = std::max<int64_t>(maxn, g.N);
    }
    if (maxn > bn && maxn <= 64) {
      cfg = GT_64x64;
      grouped_tile_shape(cfg, &bm, &bn);
    }
    for (int i = 0; i < plan.count; ++i) {
      GroupedGemm g{};
      spec(i, mats[i], g);
      const int64_t tx = (g.M > 0 && g.N > 0) ? (g.N + bn - 1) / bn : 0;
      const int64_t ty = (g.M > 0 && g.N > 0) ? (g.M + bm - 1) / bm : 0;
      g.tiles_x = std::max<int64_t>(tx, 1);
      g.ntile = std::max<int64_t>(tx * ty, 1);
      if (g.kchunk <= 0) {
        g.kchunk = std::max<int64_t>(g.K, 1);
        g.split_stride = 0;
      }
      const int64_t nz = (g.K > 0) ? (g.K + g.kchunk - 1) / g.kchunk : 1;
      g.tile0 = (int64_t)tiles.size();
      probs[i] = g;
      for (int64_t t = 0; t < tx * ty * nz; ++t) tiles.push_back(i);
    }
    BatchOp op;
    op.kind = BatchOp::GEMM;
    op.cfg = cfg;
    op.ta = ta;
    op.tb = tb;
    op.f32 = f32;
    op.probs = (const GroupedGemm*)(dev + put_raw(probs.data(), sizeof(GroupedGemm) * probs.size()));
    op.ntiles = (int64_t)tiles.size();
    op.tiles = op.ntiles ? (const int*)(dev + put_raw(tiles.data(), 4 * tiles.size())) : nullptr;
    plan.ops.push_back(op);
  }
  void simple(BatchOp::Kind kind, int64_t i0 = 0, int mode = 0, int nc = 0, int which = 0, int shifted = 0,
              int acc = 0, int first = 0) {
    BatchOp op;
    op.kind = kind;
    op.i0 = i0;
    op.mode = mode;
    op.nc = nc;
    op.which = which;
    op.shifted = shifted;
    op.acc = acc;
    op.first = first;
    plan.ops.push_back(op);
  }
  // C = alpha op(A) op(B) + beta C
  static void set(GroupedGemm& g, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                  const double* B, int64_t ldb, double beta, double* C, int64_t ldc) {
    g.M = M; g.N = N; g.K = K; g.alpha = alpha; g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.beta = beta;
    g.C = C; g.ldc = ldc;
  }
  // a Gram product of `rows` rows into the split-K partials (C = M.Gp, ld nc)
  static void split(GroupedGemm& g, int64_t rows, int nc) {
    g.kchunk = gram_kchunk(rows, nc);
    g.split_stride = (int64_t)nc * nc;
  }
  // Three passes of CholeskyQR (the first shifted) of the m x nc matrix X0
  // (ld m), through the buffers X0 -> X1 -> X0 -> out; `which` selects the
  // Gram matrix's row count for the shift; acc accumulates the triangular
  // factors into M.X.
  template <class SelIn, class SelTmp, class SelOut, class SelRows>
  void cholqr3(int nc, int which, int acc, SelIn in, SelTmp tmp, SelOut out, SelRows rows) {
    for (int pass = 0; pass < 3; ++pass) {
      gemm(true, false, false, [&](int, BMat& M, GroupedGemm& g) {
        const double* X = (pass == 1) ? tmp(M) : in(M);
        set(g, nc, nc, rows(M), 1.0, X, rows(M), X, rows(M), 0.0, M.Gp, nc);
        split(g, rows(M), nc);
      });
      simple(BatchOp::CHOL, 0, 0, nc, which, pass == 0, acc, pass == 0);
      gemm(false, false, false, [&](int, BMat& M, GroupedGemm& g) {
        const double* X = (pass == 1) ? tmp(M) : in(M);
        double* Y = (pass == 0) ? tmp(M) : (pass == 1) ? in(M) : out(M);
        set(g, rows(M), nc, nc, 1.0, X, rows(M), M.Ri, nc, 0.0, Y, rows(M));
      });
    }
  }
};

}  // namespace

extern "C" {

int rq_batch_workspace_bytes(const rq_batch_matrix* items, int32_t count, int64_t k, int32_t b, int32_t p,
                             int32_t precision, size_t* bytes) {
  if (!bytes) return -7;
  int rc = check_items(items, count, k, b, p, precision);
  if (rc) return rc;
  const size_t need = batch_bytes(items, count, k, b, b + p);
  if (need == ~(size_t)0) return -1;
  *bytes = need;
  return 0;
}

int rq_batch_plan_create(const rq_batch_matrix* items, int32_t count, int64_t k, int32_t b, int32_t p,
                         int32_t precision, int32_t tile, void* work, size_t work_bytes, rq_batch_plan** out) {
  if (!out) return -10;
  *out = nullptr;
  int rc = check_items(items, count, k, b, p, precision);
  if (rc) return rc;
  if (tile < 0 || tile >= GT_NCFG) return -7;
  const int l = b + p;
  const size_t need = batch_bytes(items, count, k, b, l);
  if (need == ~(size_t)0) return -1;
  if (!work || work_bytes < need) return -9;
  rq_batch_plan* plan = new rq_batch_plan();
  plan->count = count;
  plan->k = k;
  plan->b = b;
  plan->p = p;
  plan->l = l;
  plan->precision = precision;
  plan->cfg = tile;
  {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
      plan->wgs = 2 * cus;
      plan->mwgs = 2 * cus;
    }
  }
  const size_t dbytes = align_up(desc_bytes(count, k, b, tiles_bound(items, count, k, b, l)), 256);
  Builder B(*plan);
  B.dev = (char*)work;
  // the BMat array and the omega jobs come first in the descriptor region
  B.mats.resize(count);
  Carve cv((char*)work + dbytes, work_bytes - dbytes);
  std::vector<OmegaJob> jobs(count);
  int64_t max_n = 0, max_m = 0;
  // matrices in descending size (n, then m): the one-workgroup-per-matrix
  // kernels then start the largest first, so the small ones fill in behind
  // them instead of a large one starting last; every matrix keeps its own
  // buffers, so the order changes no result
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return items[x].n != items[y].n ? items[x].n > items[y].n : items[x].m > items[y].m;
  });
  for (int i = 0; i < count; ++i) {
    const rq_batch_matrix& it = items[order[i]];
    BMat& M = B.mats[i];
    carve_matrix(cv, it.m, it.n, k, b, l, M);
    M.m = it.m; M.n = it.n; M.lda = it.lda; M.A = it.A; M.U = it.U; M.ldu = it.ldu; M.sigma = it.sigma;
    M.VT = it.VT; M.ldvt = it.ldvt; M.jpvt_out = it.jpvt; M.seed = it.seed;
    if (it.info) M.info = it.info;
    jobs[i] = OmegaJob{it.seed, (int64_t)l, it.m, M.om, it.m, 1};  // Omega(r, c) at om[c + r m]
    max_n = std::max(max_n, it.n);
    max_m = std::max(max_m, it.m);
  }
  if (!cv.ok) { delete plan; return -9; }
  plan->max_n = max_n;
  plan->max_m = max_m;
  if (sample_lds_bytes(max_n) > 65536) {
    const void* fns[8] = {(const void*)bt_sample_qrcp_kernel<8>,  (const void*)bt_sample_qrcp_kernel<16>,
                          (const void*)bt_sample_qrcp_kernel<24>, (const void*)bt_sample_qrcp_kernel<32>,
                          (const void*)bt_sample_qrcp_kernel<40>, (const void*)bt_sample_qrcp_kernel<48>,
                          (const void*)bt_sample_qrcp_kernel<56>, (const void*)bt_sample_qrcp_kernel<64>};
    for (const void* fn : fns) {
      if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sample_lds_bytes(max_n)) !=
          hipSuccess) {
        delete plan;
        return -9;
      }
    }
  }
  plan->max_mb = max_m * b;
  plan->mats = (BMat*)(B.dev + B.put_raw(B.mats.data(), sizeof(BMat) * count));
  const OmegaJob* djobs = (const OmegaJob*)(B.dev + B.put_raw(jobs.data(), sizeof(OmegaJob) * count));
  const bool mixed = precision == RQ_MIXED;
  const int nb = (int)(k / b);

  // ---- TRQRCP (Alg. 6) ----
  B.simple(BatchOp::INIT);
  {
    BatchOp op;
    op.kind = BatchOp::OMEGA;
    op.jobs = djobs;
    plan->ops.push_back(op);
  }
  // the sketch B = Omega A (Section 3)
  B.gemm(true, false, mixed, [&](int, BMat& M, GroupedGemm& g) {
    Builder::set(g, M.n, l, M.m, 1.0, M.A, M.lda, M.om, M.m, 0.0, M.smp, M.n);
  });
  for (int J = 0; J < nb; ++J) {
    const int64_t i0 = (int64_t)J * b;
    B.simple(BatchOp::SQRCP, i0);                       // b pivots from the sample
    B.simple(BatchOp::GATHER, i0, GATHER_PANEL);        // P = A(:, pivots)
    if (J > 0) {
      for (int rep = 0; rep < 2; ++rep) {               // P -= Q (Q^T P), twice
        B.gemm(true, false, false, [&](int, BMat& M, GroupedGemm& g) {
          Builder::set(g, i0, b, M.m, 1.0, M.Q, M.m, M.P, M.m, 0.0, M.G, k);
        });
        B.gemm(false, false, false, [&](int, BMat& M, GroupedGemm& g) {
          Builder::set(g, M.m, b, i0, -1.0, M.Q, M.m, M.G, k, 1.0, M.P, M.m);
        });
      }
    }
    B.cholqr3(b, CH_PANEL, 0, [](BMat& M) { return M.P; }, [](BMat& M) { return M.P2; },
              [i0](BMat& M) { return M.Q + i0 * M.m; }, [](BMat& M) { return M.m; });
    // the new rows of R in the original column order: Q_J^T A
    B.gemm(true, false, mixed, [&](int, BMat& M, GroupedGemm& g) {
      Builder::set(g, b, M.n, M.m, 1.0, M.Q + i0 * M.m, M.m, M.A, M.lda, 0.0, M.Rr + i0, k);
    });
    if (J + 1 < nb) {  // the sample update, eq. (update1)
      B.simple(BatchOp::GATHER, i0, GATHER_ROWS);
      B.simple(BatchOp::W11, i0);
      B.gemm(true, true, false, [&](int, BMat& M, GroupedGemm& g) {
        Builder::set(g, M.n - i0 - b, b, b, -1.0, M.Rg + (int64_t)b * b, b, M.W11, b, 1.0, M.smp + (i0 + b), M.n);
      });
    }
  }
  B.simple(BatchOp::GATHER, 0, COPY_PIVOTS);
  // ---- TUXV (Alg. 7, j_max = 1) ----
  // V: CholeskyQR of Z0^T = Rr^T (n x k); the first pass forms Rr Rr^T and Rr^T Ri
  B.gemm(false, true, false, [&](int, BMat& M, GroupedGemm& g) {
    Builder::set(g, k, k, M.n, 1.0, M.Rr, k, M.Rr, k, 0.0, M.Gp, k);
    Builder::split(g, M.n, (int)k);
  });
  B.simple(BatchOp::CHOL, 0, 0, (int)k, CH_V, 1, 0, 1);
  B.gemm(true, false, false, [&](int, BMat& M, GroupedGemm& g) {
    Builder::set(g, M.n, k, k, 1.0, M.Rr, k, M.Ri, k, 0.0, M.V, M.n);
  });
  for (int pass = 1; pass < 3; ++pass) {
    B.gemm(true, false, false, [&](int, BMat& M, GroupedGemm& g) {
      const double* X = (pass == 1) ? M.V : M.V2;
      Builder::set(g, k, k, M.n, 1.0, X, M.n, X, M.n, 0.0, M.Gp, k);
      Builder::split(g, M.n, (int)k);
    });
    B.simple(BatchOp::CHOL, 0, 0, (int)k, CH_V, 0, 0, 0);
    B.gemm(false, false, false, [&](int, BMat& M, GroupedGemm& g) {
      const double* X = (pass == 1) ? M.V : M.V2;
      double* Y = (pass == 1) ? M.V2 : M.V;
      Builder::set(g, M.n, k, k, 1.0, X, M.n, M.Ri, k, 0.0, Y, M.n);
    });
  }
  // Z1 = A V (into P), then U1 (into P2... see cholqr3) and X
  B.gemm(false, false, mixed, [&](int, BMat& M, GroupedGemm& g) {
    Builder::set(g, M.m, k, M.n, 1.0, M.A, M.lda, M.V, M.n, 0.0, M.P, M.m);
  });
  B.cholqr3((int)k, CH_Z, 1, [](BMat& M) { return M.P; }, [](BMat& M) { return M.P2; },
            [](BMat& M) { return M.Q; }, [](BMat& M) { return M.m; });
  B.simple(BatchOp::SVD);
  // U = U1 Ux, VT = Vx^T V^T
  B.gemm(false, false, false, [&](int, BMat& M, GroupedGemm& g) {
    Builder::set(g, M.m, k, k, 1.0, M.Q, M.m, M.Ux, k, 0.0, M.U, M.ldu);
  });
  B.gemm(true, true, false, [&](int, BMat& M, GroupedGemm& g) {
    Builder::set(g, k, M.n, k, 1.0, M.Vx, k, M.V, M.n, 0.0, M.VT, M.ldvt);
  });
  if (B.off > dbytes) {  // cannot happen: the size query bounds the descriptors
    delete plan;
    return -9;
  }
  // the descriptor region (a blocking copy: the plan is ready on return)
  if (hipMemcpy(work, B.img.data(), B.off, hipMemcpyHostToDevice) != hipSuccess) {
    delete plan;
    return RQ_ERR_HIP_BASE + (int)hipErrorInvalidValue;
  }
  *out = plan;
  return 0;
}

int rq_batch_plan_destroy(rq_batch_plan* plan) {
  delete plan;
  return 0;
}

int rq_tuxv_batched(void* stream, const rq_batch_plan* plan) {
  if (!plan) return -2;
  hipStream_t s = (hipStream_t)stream;
  const int count = plan->count;
  if (count == 0) return 0;
  const int l = plan->l, b = plan->b;
  const int k = (int)plan->k;
  const unsigned gy = (unsigned)std::min(count, 65535);
  const unsigned mg = (unsigned)std::min(count, plan->mwgs);
  for (const BatchOp& op : plan->ops) {
    switch (op.kind) {
      case BatchOp::INIT:
        hipLaunchKernelGGL(bt_init_kernel, dim3((unsigned)std::max<int64_t>(1, (plan->max_n + 255) / 256), gy),
                           dim3(256), 0, s, plan->mats, count, l);
        break;
      case BatchOp::OMEGA:
        RQ_TRY_RAW(launch_omega_batched(s, op.jobs, count, (int64_t)l * plan->max_m));
        break;
      case BatchOp::GEMM:
        RQ_TRY_RAW(launch_gemm_grouped(s, op.cfg, op.ta, op.tb, op.f32, op.probs, op.tiles, op.ntiles, plan->wgs));
        break;
      case BatchOp::SQRCP:
        switch (sample_rows(l)) {
#define RQ_BT_SQ(L)                                                                                             \
  case L:                                                                                                     \
    hipLaunchKernelGGL(bt_sample_qrcp_kernel<L>, dim3(mg), dim3(BT_T), sample_lds_bytes(plan->max_n), s,      \
                       plan->mats, count, l, b, op.i0, plan->max_n);                                          \
    break;
          RQ_BT_SQ(8) RQ_BT_SQ(16) RQ_BT_SQ(24) RQ_BT_SQ(32) RQ_BT_SQ(40) RQ_BT_SQ(48) RQ_BT_SQ(56) RQ_BT_SQ(64)
#undef RQ_BT_SQ
          default:
            return -5;
        }
        break;
      case BatchOp::GATHER: {
        const int64_t e = (op.mode == GATHER_PANEL) ? plan->max_mb : (op.mode == GATHER_ROWS) ? plan->max_n * b : k;
        const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((e + 255) / 256, 64));
        hipLaunchKernelGGL(bt_gather_kernel, dim3(gx, gy), dim3(256), 0, s, plan->mats, count, op.mode, op.i0, b, k);
        break;
      }
      case BatchOp::CHOL:
        hipLaunchKernelGGL(bt_chol_kernel, dim3(mg), dim3(256), 0, s, plan->mats, count, op.nc, op.which,
                           op.shifted, op.acc, op.first);
        break;
      case BatchOp::W11:
        hipLaunchKernelGGL(bt_w11_kernel, dim3(mg), dim3(256), 0, s, plan->mats, count, l, b, op.i0);
        break;
      case BatchOp::SVD:
        hipLaunchKernelGGL(bt_svd_kernel, dim3(mg), dim3(BT_T), 0, s, plan->mats, count, k);
        break;
    }
    RQ_HIP(hipGetLastError());
  }
  return 0;
}

}  // extern "C"
