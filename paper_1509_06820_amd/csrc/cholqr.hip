// Householder panel by CholeskyQR2 and Householder reconstruction.
//
// The panel step of Alg. 4 and Alg. 6 is an unpivoted QR of the b chosen
// columns, and the later steps need its Householder form (reflectors Y, tau, connection
// matrix T).  Instead of b sequential column steps, the mJ x b panel P is
// orthogonalised with two Cholesky QR passes and the Householder vectors
// are then recovered from the orthonormal factor (Ballard, Demmel, Grigori,
// Jacobsen, Knight, Nguyen, "Reconstructing Householder vectors from Tall-
// Skinny QR", IPDPS 2014): with E = [I; 0], the LU factorisation without
// pivoting E - Q S = Y U (S diagonal, S_ii = -sign of the current pivot of
// the elimination) gives the unit lower trapezoidal Y, T = U Y1^-T and
// tau = diag(U); R = S R_chol.  In exact arithmetic these are the reflectors
// and R of Householder QR with the LAPACK sign convention.
//
// In RQRCP the sample supplies a preconditioner: the sample QRCP's leading
// block S11 satisfies S11 = W11 R11 (sample update, Sec. 4), so
// X = P S11^-1 = Q W11^-1 is well conditioned and the first Cholesky pass
// runs on X.  Q and R are formed from the first pass's output Q1 (never from
// P times an inverse of S11), so a badly conditioned S11 can make the passes
// fail but cannot make their result inaccurate.
//
// Stages (all on the caller's stream; a device status word `st` records a
// failure, after which the reconstruction is skipped and the column-by-column
// Householder panel runs instead):
//   inv   : M0 = S11^-1                         (1 workgroup)
//   gemm  : X = P M0 (into Y), G1 = X^T X       (matrix cores, split-K)
//   chol1 : M1 = chol(G1)^-1                    (1 workgroup)
//   gemm  : Q1 = X M1, G2 = Q1^T Q1, H = Q1^T P
//   recon : R2 = chol(G2), Q_top = Q1(0:b, :) R2^-1, LU with sign choice,
//           then in four workgroups (each forming the factors): R = S R2^-T H
//           and Y1; tau and T; M3 = -R2^-1 S U^-1; W11
//   gemm  : Y(b:, :) = Q1(b:, :) M3
//   copy  : Y(b:, :) back into the panel storage (skipped on failure)
#include "kernels.hpp"

namespace rq {

namespace {

constexpr int SM_T = 256;    // threads of the small-matrix kernels (thread = row r, column group cg)
constexpr int SM_N = 64;     // matrices are padded to 64 x 64
constexpr int SM_LD = 65;    // LDS leading dimension (odd: no bank conflicts along columns)

// status bits
constexpr int ST_CHOL1 = 1, ST_CHOL2 = 2, ST_ORTH = 4, ST_PIVOT = 8, ST_S11 = 16;

// ---------------------------------------------------------------- LDS helpers
// Matrices live in LDS as M[i + j * SM_LD] (column-major), 64 x 64, padded
// with the identity beyond the active size b.

// Element loops map thread t to row t & 63 and columns (t >> 6) + 4q: no
// integer division in the step loops.
__device__ __forceinline__ int sm_r() { return threadIdx.x & 63; }
__device__ __forceinline__ int sm_cg() { return threadIdx.x >> 6; }

// Global -> LDS and back: each thread's sixteen loads are issued before the
// first of its stores, so a transfer costs one memory latency, not sixteen.
constexpr int SM_PER = SM_N / (SM_T / SM_N);  // elements per thread

__device__ __forceinline__ void sm_load(double* M, const double* G, int64_t rs, int64_t cs, int b, bool upper_only) {
  const int i = sm_r(), cg = sm_cg();
  double v[SM_PER];
#pragma unroll
  for (int q = 0; q < SM_PER; ++q) {
    const int j = cg + q * (SM_T / SM_N);
    // inside b x b: the entry (zero below the diagonal with upper_only);
    // outside: the identity
    const bool in = i < b && j < b && !(upper_only && i > j);
    v[q] = in ? G[(int64_t)i * rs + (int64_t)j * cs] : ((i == j) ? 1.0 : 0.0);
  }
#pragma unroll
  for (int q = 0; q < SM_PER; ++q) M[i + (cg + q * (SM_T / SM_N)) * SM_LD] = v[q];
}

__device__ __forceinline__ void sm_store(const double* M, double* G, int64_t ld, int b) {
  const int i = sm_r(), cg = sm_cg();
  if (i >= b) return;
  double v[SM_PER];
#pragma unroll
  for (int q = 0; q < SM_PER; ++q) v[q] = M[i + (cg + q * (SM_T / SM_N)) * SM_LD];
#pragma unroll
  for (int q = 0; q < SM_PER; ++q) {
    const int j = cg + q * (SM_T / SM_N);
    if (j < b) G[i + (int64_t)j * ld] = v[q];
  }
}

// Products of LDS matrices on the matrix cores: for each of nb batches
// (pointers advanced by boff), the M x N result of op(A) B (K inner, M and N
// multiples of 16, K of 4) is handed element by element to epi(i, j, value).
// TA: op(A)(i, k) = A[k + i * SM_LD], else A[i + k * SM_LD].  16 x 16 tiles
// are dealt to the waves in turn; the operand layout follows the gemm
// kernel's (v_mfma_f64_16x16x4 with swapped operands, lane l / register r
// holding element (l % 16, 4r + l / 16) of the tile).  No barrier inside:
// the caller synchronises before reading what epi wrote.
template <bool TA, class Epi>
__device__ __forceinline__ void sm_mm(const double* A, const double* B, int M, int N, int K, int nb, int boff,
                                      Epi epi) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (M == SM_N && N == SM_N && nb == 1) {
    // full 64 x 64: wave w takes the 32 x 32 quadrant (w & 1, w >> 1) as
    // 2 x 2 tiles, so each operand fragment read from LDS feeds two MFMAs
    const int i0 = 32 * (w & 1), j0 = 32 * (w >> 1);
    double4_t acc[2][2];
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
      for (int b2 = 0; b2 < 2; ++b2) acc[a2][b2] = (double4_t){0.0, 0.0, 0.0, 0.0};
    const int ia = i0 + (lane & 15), jb = j0 + (lane & 15);
#pragma unroll 4
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int ka = k0 + (lane >> 4);
      double af[2], bf[2];
#pragma unroll
      for (int a2 = 0; a2 < 2; ++a2) af[a2] = TA ? A[ka + (ia + 16 * a2) * SM_LD] : A[(ia + 16 * a2) + ka * SM_LD];
#pragma unroll
      for (int b2 = 0; b2 < 2; ++b2) bf[b2] = B[ka + (jb + 16 * b2) * SM_LD];
#pragma unroll
      for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
        for (int b2 = 0; b2 < 2; ++b2)
          acc[a2][b2] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[b2], af[a2], acc[a2][b2], 0, 0, 0);
    }
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
      for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          epi(0, ia + 16 * a2, j0 + 16 * b2 + 4 * r + (lane >> 4), acc[a2][b2][r]);
    return;
  }
  const int tm = M >> 4, tn = N >> 4, per = tm * tn;
  for (int t = w; t < nb * per; t += SM_T / 64) {
    const int bi = t / per, tt = t - bi * per;
    const int i0 = (tt % tm) * 16, j0 = (tt / tm) * 16;
    const double* Ab = A + bi * boff;
    const double* Bb = B + bi * boff;
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    const int ia = i0 + (lane & 15), jb = j0 + (lane & 15);
#pragma unroll 4
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int ka = k0 + (lane >> 4);
      const double af = TA ? Ab[ka + ia * SM_LD] : Ab[ia + ka * SM_LD];
      const double bf = Bb[ka + jb * SM_LD];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bf, af, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) epi(bi, ia, j0 + 4 * r + (lane >> 4), acc[r]);
  }
}

// ---------------------------------------------------------------- blocked factorisations
// The Cholesky and the sign-choosing LU run in blocks of 16.  Within a
// block, wave 0 alone takes the 16 dependent steps without workgroup
// barriers: its lanes hold a 16-wide band of the matrix in registers (the
// step loop is unrolled, so every register index is a constant) and a value
// another lane holds is read with v_readlane into scalar registers.  The
// rank-16 update of the rest of the matrix runs on the matrix cores in all
// four waves.
constexpr int SM_NB = 16;

// 1 / a (a >= 1 here): hardware estimate and two Newton steps.
__device__ __forceinline__ double rcp_nr(double a) {
  double r = __builtin_amdgcn_rcp(a);
  r = fma(r, fma(-a, r, 1.0), r);
  r = fma(r, fma(-a, r, 1.0), r);
  return r;
}

// 1 / sqrt(a), a > 0: hardware estimate and two Newton steps
// y <- y (3 - a y^2) / 2.
__device__ __forceinline__ double rsqrt_nr(double a) {
  double y = __builtin_amdgcn_rsq(a);
  const double h = 0.5 * a;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

__device__ __forceinline__ double lane_val(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// In-place Cholesky G = R^T R of the upper triangle of G (64 x 64, LDS;
// R upper, lower part zeroed).  Returns false (uniformly) if a pivot is not
// positive.  Block k0: lane c holds G(k0:k0+16, c), the row band of R.
__device__ __forceinline__ bool sm_chol(double* G, int* flag) {
  __shared__ double rowbuf[SM_N];  // row p of R, for the broadcast reads
  if (threadIdx.x == 0) *flag = 0;
  __syncthreads();
#pragma unroll
  for (int k0 = 0; k0 < SM_N; k0 += SM_NB) {  // unrolled: every lane index below is a constant
    if (threadIdx.x < SM_N) {
      const int c = threadIdx.x;
      double a[SM_NB];
#pragma unroll
      for (int i = 0; i < SM_NB; ++i) a[i] = G[(k0 + i) + c * SM_LD];
      // Step i's pivot chain (pivot, reciprocal square root, row scaling,
      // the next pivot row's update, read with v_readlane) is formed first,
      // and the next pivot's reciprocal square root inside step i, so that
      // it overlaps step i's updates of the rows further down.  Those take
      // row p of R through LDS: each lane stores its R(p, c), and every lane
      // reads the entries it needs at one address (a broadcast), in order
      // within the wave.
      bool ok = true;
      double d = lane_val(a[0], k0);
      double dd = (d > 0.0) ? d : 1.0;
      double isd = rsqrt_nr(dd);
#pragma unroll
      for (int i = 0; i < SM_NB; ++i) {
        const int p = k0 + i;
        ok = ok && (d > 0.0);
        const double sd = dd * isd;
        const double r = (c > p) ? a[i] * isd : ((c == p) ? sd : 0.0);  // R(p, c)
        a[i] = r;
        rowbuf[c] = r;
        __builtin_amdgcn_wave_barrier();
        if (i + 1 < SM_NB) {
          a[i + 1] = fma(-lane_val(r, p + 1), r, a[i + 1]);
          d = lane_val(a[i + 1], p + 1);
          dd = (d > 0.0) ? d : 1.0;
          isd = rsqrt_nr(dd);
        }
#pragma unroll
        for (int q = i + 2; q < SM_NB; ++q) a[q] = fma(-rowbuf[k0 + q], r, a[q]);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int i = 0; i < SM_NB; ++i) G[(k0 + i) + c * SM_LD] = (c >= k0 + i) ? a[i] : 0.0;
      if (c == 0 && !ok) *flag = 1;
    }
    __syncthreads();
    const int n2 = SM_N - k0 - SM_NB;
    if (n2 > 0) {
      // G22 -= R12^T R12
      const double* R12 = G + k0 + (k0 + SM_NB) * SM_LD;
      double* G22 = G + (k0 + SM_NB) * (1 + SM_LD);
      sm_mm<true>(R12, R12, n2, n2, SM_NB, 1, 0, [&](int, int i, int j, double v) { G22[i + j * SM_LD] -= v; });
      __syncthreads();
    }
  }
  return *flag == 0;
}

// Lane src's value in every lane of the wave, through the LDS crossbar
// (ds_bpermute: no memory access and no scalar registers, so a step's
// broadcasts can all be in flight at once).
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const int addr = src << 2;
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// The 16 elimination steps of block k0 in wave 0 (lane r holds
// A(r, k0:k0+16) in a).  FULL: every step of the block is an ordinary one
// (p < b and p != mJ - 1), so the steps need no branches.
template <bool FULL>
__device__ __forceinline__ void lu_block_steps(double (&a)[SM_NB], int k0, int r, int b, int64_t mJ, double* sgn) {
#pragma unroll
  for (int i = 0; i < SM_NB; ++i) {
    const int p = k0 + i;
    if (FULL || p < b) {
      // the pivot row's entries right of the pivot, from lane p
      double u[SM_NB];
#pragma unroll
      for (int j = i + 1; j < SM_NB; ++j) u[j] = lane_bcast(a[j], p);
      const double c0 = lane_val(a[i], p);
      if (!FULL && p == mJ - 1) {
        if (r == 0) sgn[p] = (c0 >= 0.0) ? 1.0 : -1.0;
        if (r == p) a[i] = 0.0;
      } else {
        const double sg = (c0 >= 0.0) ? -1.0 : 1.0;
        const double piv = 1.0 + fabs(c0);
        const double f = -sg * rcp_nr(piv);
        const double l = (r > p) ? a[i] * f : 0.0;  // L(r, p)
        a[i] = (r > p) ? l : ((r == p) ? piv : a[i]);
#pragma unroll
        for (int j = i + 1; j < SM_NB; ++j) a[j] = fma(-l, u[j], a[j]);
        if (r == 0) sgn[p] = sg;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// LU without pivoting of E - Q S on the top b x b block (in A, 64 x 64 LDS,
// identity padded), with the sign choice of Householder reconstruction: at
// step i with c0 = Q'(i, i), S_ii = -sign(c0) (sign(0) = +1), U(i, i) =
// 1 + |c0|, L(r, i) = -S_ii Q'(r, i) / U(i, i), Q'(r, c) -= L(r, i) Q'(i, c).
// The last column of a square panel (i = mJ - 1) has no row below: there
// S_ii = sign(c0) and U(i, i) = 0.  On return A holds L (unit, below the
// diagonal), U(i, i) on the diagonal and Q' above it; sgn[i] = S_ii.
// Block k0: wave 0 eliminates the 16 columns k0..k0+15 with lane r holding
// A(r, k0:k0+16) (steps without barriers, the pivot row's entries taken by
// ds_bpermute broadcasts); then the row band U12 = L11^-1 A12 (rows k0..k0+15, the
// columns right of the block) by forward substitution, one thread per
// column; then A22 -= L21 U12 on the matrix cores.
__device__ __forceinline__ void sm_lu_sign(double* A, double* sgn, int b, int64_t mJ) {
#pragma unroll
  for (int k0 = 0; k0 < SM_N; k0 += SM_NB) {  // unrolled: every lane index below is a constant
    if (k0 >= b) break;
    if (threadIdx.x < SM_N) {
      const int r = threadIdx.x;
      double a[SM_NB];
#pragma unroll
      for (int j = 0; j < SM_NB; ++j) a[j] = A[r + (k0 + j) * SM_LD];
      const bool full = k0 + SM_NB <= b && !(mJ - 1 >= k0 && mJ - 1 < k0 + SM_NB);
      if (full)
        lu_block_steps<true>(a, k0, r, b, mJ, sgn);
      else
        lu_block_steps<false>(a, k0, r, b, mJ, sgn);
#pragma unroll
      for (int j = 0; j < SM_NB; ++j)
        if (r >= k0) A[r + (k0 + j) * SM_LD] = a[j];
    }
    __syncthreads();
    const int n2 = SM_N - k0 - SM_NB;
    if (n2 > 0 && k0 + SM_NB < b) {
      // U12 = L11^-1 A12: column c = k0 + 16 + t, rows k0..k0+15, in order
      const int t = threadIdx.x;
      if (t < n2) {
        const int c = k0 + SM_NB + t;
        double x[SM_NB];
#pragma unroll
        for (int q = 0; q < SM_NB; ++q) x[q] = A[(k0 + q) + c * SM_LD];
#pragma unroll
        for (int q = 1; q < SM_NB; ++q)
#pragma unroll
          for (int pp = 0; pp < q; ++pp) x[q] = fma(-A[(k0 + q) + (k0 + pp) * SM_LD], x[pp], x[q]);
#pragma unroll
        for (int q = 0; q < SM_NB; ++q) A[(k0 + q) + c * SM_LD] = x[q];
      }
      __syncthreads();
      // A22 -= L21 U12
      const double* L21 = A + (k0 + SM_NB) + k0 * SM_LD;
      const double* U12 = A + k0 + (k0 + SM_NB) * SM_LD;
      double* A22 = A + (k0 + SM_NB) * (1 + SM_LD);
      sm_mm<false>(L21, U12, n2, n2, SM_NB, 1, 0, [&](int, int i, int j, double v) { A22[i + j * SM_LD] -= v; });
      __syncthreads();
    }
  }
  __syncthreads();
}

// Inverse of an upper-triangular matrix by recursive doubling:
// inv([A B; 0 C]) = [inv(A), -inv(A) B inv(C); 0, inv(C)], block size 16, 32.
// The four diagonal 16 x 16 blocks by back substitution (one wave each), the
// doubling levels on the matrix cores.  R and Ri
// must differ; W is scratch (SM_N * SM_LD).  Returns false (uniformly) if a
// diagonal entry is zero; *flag is set to match.
__device__ __forceinline__ bool sm_tri_inv(const double* R, double* Ri, double* W, int* flag) {
  __shared__ int zero_diag[SM_T / 64];  // per wave: its diagonal block has a zero
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // blocks below the diagonal blocks are zero (no barrier before the
  // diagonal blocks: those write other entries of Ri and read only R)
  for (int e = threadIdx.x; e < SM_N * SM_N; e += SM_T) {
    const int i = e & (SM_N - 1), j = e >> 6;
    if ((i >> 4) > (j >> 4)) Ri[i + j * SM_LD] = 0.0;
  }
  {
    // diagonal block w, one wave: lane j < 16 forms column j of the block's
    // inverse by back substitution; column k of the block, R(o:o+k, o+k), is
    // read from LDS at the same address by every lane (a broadcast, off the
    // substitution's dependency chain, so the reads of later steps can be
    // issued early: these kernels run one workgroup per CU, registers are
    // plentiful), the reciprocal of R(o+k, o+k) from lane k with v_readlane
    const int o = SM_NB * w, j = lane & 15;
    double x[SM_NB];
#pragma unroll
    for (int i = 0; i < SM_NB; ++i) x[i] = (i == j) ? 1.0 : 0.0;
    const double dj = R[(o + j) + (o + j) * SM_LD];
    const bool zero = __any(lane < SM_NB && dj == 0.0);
    if (lane == 0) zero_diag[w] = zero ? 1 : 0;
    const double rdj = (dj != 0.0) ? 1.0 / dj : 0.0;
#pragma unroll
    for (int k = SM_NB - 1; k >= 0; --k) {
      const double xk = x[k] * lane_val(rdj, k);
      x[k] = xk;
      const double* colk = R + o + (o + k) * SM_LD;
#pragma unroll
      for (int i = 0; i < k; ++i) x[i] = fma(-colk[i], xk, x[i]);
    }
    if (lane < SM_NB) {
#pragma unroll
      for (int i = 0; i < SM_NB; ++i) Ri[(o + i) + (o + j) * SM_LD] = x[i];
    }
  }
  __syncthreads();
  for (int sz = 16; sz <= 32; sz <<= 1) {
    const int nb = SM_N / (2 * sz), boff = 2 * sz * (1 + SM_LD);
    // W = B inv(C) for each pair of diagonal blocks
    sm_mm<false>(R + sz * SM_LD, Ri + sz * (1 + SM_LD), sz, sz, sz, nb, boff,
                 [&](int bi, int i, int j, double v) { W[bi * boff + i + (sz + j) * SM_LD] = v; });
    __syncthreads();
    // off-diagonal block = -inv(A) W
    sm_mm<false>(Ri, W + sz * SM_LD, sz, sz, sz, nb, boff,
                 [&](int bi, int i, int j, double v) { Ri[bi * boff + i + (sz + j) * SM_LD] = -v; });
    __syncthreads();
  }
  // (the barriers of the doubling levels order the flags' stores before
  // these reads)
  const bool ok = !(zero_diag[0] | zero_diag[1] | zero_diag[2] | zero_diag[3]);
  if (threadIdx.x == 0) *flag = ok ? 0 : 1;
  return ok;
}

// C = A B (all 64 x 64 in LDS, C distinct from A and B).
__device__ void sm_mul(const double* A, const double* B, double* C) {
  sm_mm<false>(A, B, SM_N, SM_N, SM_N, 1, 0, [&](int, int i, int j, double v) { C[i + j * SM_LD] = v; });
  __syncthreads();
}

// ---------------------------------------------------------------- kernels
// M0 = S11^-1 (S11 = S[i*srs + j*scs], upper b x b).  A zero diagonal marks
// the status word and leaves the preconditioner unused.
__global__ void __launch_bounds__(SM_T) inv_kernel(int b, const double* S, int64_t srs, int64_t scs, double* M0,
                                                   int* st) {
  extern __shared__ __align__(16) double sm[];
  __shared__ int flag;
  double* A = sm;
  double* Ai = sm + SM_N * SM_LD;
  double* W = sm + 2 * SM_N * SM_LD;
  sm_load(A, S, srs, scs, b, true);
  __syncthreads();
  const bool ok = sm_tri_inv(A, Ai, W, &flag);
  if (!ok) {
    if (threadIdx.x == 0) atomicOr(st, ST_S11);
    return;
  }
  sm_store(Ai, M0, b, b);
}

// M1 = chol(G1)^-1.
__global__ void __launch_bounds__(SM_T) chol1_kernel(int b, const double* G1, double* M1, int* st) {
  extern __shared__ __align__(16) double sm[];
  __shared__ int flag;
  __shared__ int s_skip;
  if (threadIdx.x == 0) s_skip = *st;
  __syncthreads();
  if (s_skip) return;
  double* G = sm;
  double* Ri = sm + SM_N * SM_LD;
  double* W = sm + 2 * SM_N * SM_LD;
  sm_load(G, G1, 1, b, b, true);
  __syncthreads();
  if (!sm_chol(G, &flag) || !sm_tri_inv(G, Ri, W, &flag)) {
    if (threadIdx.x == 0) atomicOr(st, ST_CHOL1);
    return;
  }
  sm_store(Ri, M1, b, b);
}

// Second Cholesky pass, sign-choosing LU of E - Q S on the top block, and
// the Householder quantities.  Q1 (ld ldq) is the first pass's output,
// G2 = Q1^T Q1 and H = Q1^T P; with R2 = chol(G2) the orthonormal factor is
// Q = Q1 R2^-1 and R = S Q^T P = S R2^-T H.  Forming Q and R from Q1 rather
// than from P keeps the preconditioner's conditioning out of both.
__global__ void __launch_bounds__(SM_T) recon_kernel(int b, int64_t mJ, const double* G2, const double* H,
                                                     const double* Q1, int64_t ldq, double* P, int64_t ldp, double* Y,
                                                     int64_t ldy, double* tau, double* T, double* M3, int* st,
                                                     const double* M1, double* W11) {
  extern __shared__ __align__(16) double sm[];
  __shared__ int flag;
  __shared__ int s_skip;
  __shared__ double sgn[SM_N];
  __shared__ double wmax[SM_T / 64];
  // All three inputs are read up front (thread (r, cg) holds entries
  // (r, cg + 4 q)), so their latencies overlap.
  const int r = sm_r(), cg = sm_cg();
  double g2r[SM_N / 4], q1r[SM_N / 4], hr[SM_N / 4];
#pragma unroll
  for (int q = 0; q < SM_N / 4; ++q) {
    const int c = cg + 4 * q;
    const bool in = r < b && c < b;
    const double id = (r == c) ? 1.0 : 0.0;
    g2r[q] = in ? G2[r + (int64_t)c * b] : id;
    q1r[q] = in ? Q1[r + (int64_t)c * ldq] : id;
    hr[q] = in ? H[r + (int64_t)c * b] : 0.0;
  }
  if (threadIdx.x == 0) s_skip = *st;
  __syncthreads();
  if (s_skip) return;
  double* A = sm;
  double* B = sm + SM_N * SM_LD;
  double* C = sm + 2 * SM_N * SM_LD;
  double* D = sm + 3 * SM_N * SM_LD;
  // E = G2 - I; its largest entry decides how R2 = chol(G2) is formed (G2
  // must be close to the identity after the first pass)
  {
    double em = 0.0;
#pragma unroll
    for (int q = 0; q < SM_N / 4; ++q) em = fmax(em, fabs(g2r[q] - ((r == cg + 4 * q) ? 1.0 : 0.0)));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) em = fmax(em, __shfl_xor(em, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = em;
    if (threadIdx.x == 0) flag = 0;
  }
  __syncthreads();
  const double emax = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
  if (!(emax <= 0.25)) {
    if (threadIdx.x == 0) atomicOr(st, ST_ORTH);
    return;
  }
  if (emax <= 1e-10) {
    // R2 = I + F with F = U(E) - U(F^T F) (U: strict upper part plus half
    // the diagonal) and R2^-1 = I - F + F^2 - ...; at |E| <= 1e-10 every
    // term past U(E) is below 64 |E|^2 < 1e-18, so R2^-1 = I - U(E).
#pragma unroll
    for (int q = 0; q < SM_N / 4; ++q) {
      const int c = cg + 4 * q;
      const double e = g2r[q] - ((r == c) ? 1.0 : 0.0);
      B[r + c * SM_LD] = (r < c) ? -e : ((r == c) ? 1.0 - 0.5 * e : 0.0);
    }
    __syncthreads();
  } else if (emax <= 1e-6) {
    // G2 = I + E with E tiny: R2 = I + F, F = U(E) - U(F^T F) gives
    // F = U0 - U(U0^T U0) with error O(|E|^3), and R2^-1 = I - F + F^2 with
    // error O(|F|^3) -- both far below rounding at |E| <= 1e-6.  B = U0,
    // then A = F, then B = R2^-1.
#pragma unroll
    for (int q = 0; q < SM_N / 4; ++q) {
      const int c = cg + 4 * q;
      const double e = g2r[q] - ((r == c) ? 1.0 : 0.0);
      B[r + c * SM_LD] = (r < c) ? e : ((r == c) ? 0.5 * e : 0.0);
    }
    __syncthreads();
    sm_mm<true>(B, B, SM_N, SM_N, SM_N, 1, 0, [&](int, int i, int j, double v) { D[i + j * SM_LD] = v; });
    __syncthreads();
    for (int c = cg; c < SM_N; c += SM_T / SM_N) {
      const double u = (r < c) ? D[r + c * SM_LD] : ((r == c) ? 0.5 * D[r + c * SM_LD] : 0.0);
      A[r + c * SM_LD] = B[r + c * SM_LD] - u;
    }
    __syncthreads();
    sm_mm<false>(A, A, SM_N, SM_N, SM_N, 1, 0, [&](int, int i, int j, double v) { D[i + j * SM_LD] = v; });
    __syncthreads();
    for (int c = cg; c < SM_N; c += SM_T / SM_N)
      B[r + c * SM_LD] = (r == c ? 1.0 : 0.0) - A[r + c * SM_LD] + D[r + c * SM_LD];
    __syncthreads();
  } else {
#pragma unroll
    for (int q = 0; q < SM_N / 4; ++q) {  // the upper triangle
      const int c = cg + 4 * q;
      A[r + c * SM_LD] = (r <= c) ? g2r[q] : 0.0;
    }
    __syncthreads();
    if (!sm_chol(A, &flag)) {
      if (threadIdx.x == 0) atomicOr(st, ST_CHOL2);
      return;
    }
    // B = R2^-1 (C scratch)
    if (!sm_tri_inv(A, B, C, &flag)) {
      if (threadIdx.x == 0) atomicOr(st, ST_CHOL2);
      return;
    }
  }
  // A = Q_top = Q1(0:b, 0:b) R2^-1 (full b x b); Q1's top block is staged
  // in C first so the products read LDS only; D = H
#pragma unroll
  for (int q = 0; q < SM_N / 4; ++q) {
    const int c = cg + 4 * q;
    C[r + c * SM_LD] = q1r[q];
    D[r + c * SM_LD] = hr[q];
  }
  __syncthreads();
  sm_mm<false>(C, B, SM_N, SM_N, SM_N, 1, 0,
               [&](int, int i, int j, double v) { A[i + j * SM_LD] = (i < b && j < b) ? v : 0.0; });
  __syncthreads();
  // LU of E - Q S by right-looking elimination on Q alone: at step i the
  // pivot column c = Q'(i:, i); S_ii = -sign(c_0) (sign(0) = +1); pivot
  // p_i = 1 + |c_0|; L(r, i) = -S_ii Q'(r, i) / p_i; Q'(r, j) -= L(r, i) Q'(i, j).
  // A column with no row below its diagonal (the last one of a square panel)
  // is left alone by Householder QR (tau = 0): there S_ii = sign(c_0) and the
  // pivot is 0.
  sm_lu_sign(A, sgn, b, mJ);
  // C = U (U(i, j) = -S_jj Q'(i, j) above the diagonal, pivots on it);
  // A keeps L1 below the diagonal.  Padding stays identity.  (Thread (r, cg)
  // reads its sixteen entries before it writes any: A and C are distinct,
  // which the compiler cannot see.)
  {
    double av[SM_N / 4], sv[SM_N / 4];
#pragma unroll
    for (int q = 0; q < SM_N / 4; ++q) {
      const int c = cg + 4 * q;
      av[q] = A[r + c * SM_LD];
      sv[q] = sgn[c];
    }
#pragma unroll
    for (int q = 0; q < SM_N / 4; ++q) {
      const int c = cg + 4 * q;
      double u;
      if (r < b && c < b) u = (r < c) ? -sv[q] * av[q] : (r == c ? av[q] : 0.0);
      else u = (r == c) ? 1.0 : 0.0;
      C[r + c * SM_LD] = u;
    }
  }
  __syncthreads();
  // The four products that follow use only the factors above, so each
  // workgroup of the launch (which all computed them) takes one.
  const int task = blockIdx.x;
  if (task == 0) {
    // outputs of the top block: R(i, j) = S_ii sum_k R2^-1(k, i) H(k, j) on and
    // above the diagonal, Y1 below it
    sm_mm<true>(B, D, SM_N, SM_N, SM_N, 1, 0, [&](int, int i, int j, double v) {
      if (i < b && j < b) {
        if (i <= j) {
          P[i + (int64_t)j * ldp] = sgn[i] * v;
          Y[i + (int64_t)j * ldy] = (i == j) ? 1.0 : 0.0;
        } else {
          const double y = A[i + j * SM_LD];
          P[i + (int64_t)j * ldp] = y;
          Y[i + (int64_t)j * ldy] = y;
        }
      }
    });
    return;
  }
  if (task == 1) {
    // tau and T = U inv(Y1^T)
    for (int i = threadIdx.x; i < b; i += SM_T) tau[i] = C[i + i * SM_LD];
    // D = Y1^T (unit upper) padded (reads before writes, as for C above)
    {
      double yv[SM_N / 4];
#pragma unroll
      for (int q = 0; q < SM_N / 4; ++q) yv[q] = A[(cg + 4 * q) + r * SM_LD];
#pragma unroll
      for (int q = 0; q < SM_N / 4; ++q) {
        const int c = cg + 4 * q;
        double v;
        if (r < b && c < b) v = (r < c) ? yv[q] : (r == c ? 1.0 : 0.0);
        else v = (r == c) ? 1.0 : 0.0;
        D[r + c * SM_LD] = v;
      }
    }
    __syncthreads();
    sm_tri_inv(D, A, B, &flag);   // A = inv(Y1^T) (unit diagonal: never singular)
    sm_mm<false>(C, A, SM_N, SM_N, SM_N, 1, 0, [&](int, int i, int j, double v) {
      if (i < b && j < b) T[i + (int64_t)j * b] = v;
    });
    return;
  }
  // B = -R2^-1 S (columns scaled; padding zero), for M3 and W11: each
  // thread rewrites only its own entries
#pragma unroll
  for (int q = 0; q < SM_N / 4; ++q) {
    const int c = cg + 4 * q;
    B[r + c * SM_LD] = (r <= c && r < b && c < b) ? -sgn[c] * B[r + c * SM_LD] : 0.0;
  }
  if (task == 2) {
    if (mJ <= b) return;  // no rows below the top block
    __syncthreads();
    // M3 = -R2^-1 S inv(U): A = inv(U) (D scratch)
    if (!sm_tri_inv(C, A, D, &flag)) {  // pivots are >= 1 here: cannot happen
      if (threadIdx.x == 0) atomicOr(st, ST_PIVOT);
      return;
    }
    sm_mm<false>(B, A, SM_N, SM_N, SM_N, 1, 0, [&](int, int i, int j, double v) {
      if (i < b && j < b) M3[i + (int64_t)j * b] = v;
    });
    return;
  }
  if (W11) {
    // W11 = S11 R11^-1 of the sample update (eq. update1): with the panel
    // preconditioned by X = P S11^-1, X = Q R2 R1 (the two Cholesky factors,
    // R1^-1 = M1) and R11 = S R2 R1 S11, so W11 = M1 R2^-1 S -- upper
    // triangular, formed from factors at hand.
#pragma unroll
    for (int q = 0; q < SM_N / 4; ++q) {
      const int c = cg + 4 * q;
      D[r + c * SM_LD] = (r <= c && r < b && c < b) ? M1[r + (int64_t)c * b] : 0.0;
    }
    __syncthreads();
    sm_mm<false>(D, B, SM_N, SM_N, SM_N, 1, 0, [&](int, int i, int j, double v) {
      if (i < b && j < b) W11[i + (int64_t)j * b] = (i <= j) ? -v : 0.0;
    });
  }
}

// The fallback panel's tail (runs only when the CholeskyQR panel failed,
// after the column panel):
//  * T of its reflectors: G = Y^T Y, then the forward recurrence
//    T(i, i) = tau_i, T(0:i, i) = -tau_i T(0:i, 0:i) G(0:i, i);
//  * with W, W11 = S11 R11^-1 of the sample update (eq. update1), b x b upper
//    triangular.  A zero pivot R11(j, j) gives a zero column j of W11 and
//    takes row j of R11 out of the later columns; that is W11 = S~ R~^-1
//    with column j of S~ zeroed and row and column j of R~ replaced by the
//    unit vector.
// (When the CholeskyQR panel succeeds, the reconstruction has written T and
// W11 from its own factors.)
__global__ void __launch_bounds__(SM_T) fallback_tail_kernel(int64_t mJ, int b, const double* __restrict__ Y,
                                                             int64_t ldy, const double* __restrict__ tau,
                                                             double* __restrict__ T, const int* st, const double* S,
                                                             int64_t srs, int64_t scs, const double* R, int64_t ldr,
                                                             double* W) {
  extern __shared__ __align__(16) double sm[];
  __shared__ int flag;
  __shared__ int s_failed;
  if (threadIdx.x == 0) s_failed = (*st != 0);
  __syncthreads();
  if (!s_failed) return;
  {
    double* Gs = sm;
    double* Ts = sm + SM_N * SM_N;
    for (int e = threadIdx.x; e < b * b; e += SM_T) {
      const int i = e % b, j = e / b;
      double acc = 0.0;
      if (i <= j)
        for (int64_t r = 0; r < mJ; ++r) acc += Y[r + i * ldy] * Y[r + j * ldy];
      Gs[e] = acc;
      Ts[e] = 0.0;
    }
    __syncthreads();
    for (int i = 0; i < b; ++i) {
      const int r = threadIdx.x;
      if (r < i) {
        double h = 0.0;
        for (int q = r; q < i; ++q) h += Ts[r + q * b] * Gs[q + i * b];
        Ts[r + i * b] = -tau[i] * h;
      } else if (r == i) {
        Ts[i + i * b] = tau[i];
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < b * b; e += SM_T) T[e] = Ts[e];
    __syncthreads();
  }
  if (!W) return;
  double* Rt = sm;
  double* Ri = sm + SM_N * SM_LD;
  double* Wk = sm + 2 * SM_N * SM_LD;
  double* St = sm + 3 * SM_N * SM_LD;
  __shared__ int zero_piv[SM_N];
  sm_load(Rt, R, 1, ldr, b, true);
  sm_load(St, S, srs, scs, b, true);
  __syncthreads();
  if (threadIdx.x < SM_N) zero_piv[threadIdx.x] = Rt[threadIdx.x + threadIdx.x * SM_LD] == 0.0;
  __syncthreads();
  {
    const int r = sm_r();
    for (int c = sm_cg(); c < SM_N; c += SM_T / SM_N) {
      if (zero_piv[c]) St[r + c * SM_LD] = 0.0;
      if (zero_piv[c] || zero_piv[r]) Rt[r + c * SM_LD] = (r == c) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  sm_tri_inv(Rt, Ri, Wk, &flag);
  sm_mm<false>(St, Ri, SM_N, SM_N, SM_N, 1, 0, [&](int, int i, int j, double v) {
    if (i < b && j < b) W[i + (int64_t)j * b] = (i <= j) ? v : 0.0;
  });
}

constexpr size_t SM_LDS = 4 * SM_N * SM_LD * sizeof(double);

int set_lds(const void* fn) {
  RQ_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)SM_LDS));
  return 0;
}

}  // namespace

int launch_fallback_tail(hipStream_t s, int64_t mJ, int bJ, const double* Y, int64_t ldy, const double* tau,
                         double* T, const int* st, const double* S, int64_t srs, int64_t scs, const double* R,
                         int64_t ldr, double* W) {
  static bool init = false;
  if (!init) {
    RQ_TRY_RAW(set_lds((const void*)fallback_tail_kernel));
    init = true;
  }
  hipLaunchKernelGGL(fallback_tail_kernel, dim3(1), dim3(SM_T), SM_LDS, s, mJ, bJ, Y, ldy, tau, T, st, S, srs, scs, R,
                     ldr, W);
  RQ_HIP(hipGetLastError());
  return 0;
}

size_t cholqr_scratch_elems(int64_t mmax, int bmax) {
  // Q1 (mmax x b), G1, G2, H, M0, M1, M3 (b x b each)
  return (size_t)mmax * bmax + 6 * (size_t)bmax * bmax;
}

// Panel (mJ x bJ, ld ldp) -> in-place Householder layout, tau, explicit Y
// (ld ldy) and T (bJ x bJ).  S11 (optional): the sample's leading block,
// element (i, j) at S11[i*srs + j*scs].  `st` is a device status word the
// caller zeroes; nonzero on return means the fallback must run.  Y doubles
// as the first pass's X = P S11^-1.
int launch_panel_cholqr(hipStream_t s, double* P, int64_t ldp, int64_t mJ, int bJ, const double* S11, int64_t srs,
                        int64_t scs, double* tau, double* Y, int64_t ldy, double* T, double* scratch,
                        double* splitk, size_t splitk_elems, int* st, double* W11) {
  static bool init = false;
  if (!init) {
    RQ_TRY_RAW(set_lds((const void*)inv_kernel));
    RQ_TRY_RAW(set_lds((const void*)chol1_kernel));
    RQ_TRY_RAW(set_lds((const void*)recon_kernel));
    init = true;
  }
  const int b = bJ;
  double* Q1 = scratch;
  double* G1 = Q1 + mJ * (int64_t)b;
  double* G2 = G1 + b * b;
  double* H = G2 + b * b;
  double* M0 = H + b * b;
  double* M1 = M0 + b * b;
  double* M3 = M1 + b * b;
  const double* X = P;
  int64_t ldx = ldp;
  if (S11) {
    hipLaunchKernelGGL(inv_kernel, dim3(1), dim3(SM_T), SM_LDS, s, b, S11, srs, scs, M0, st);
    RQ_HIP(hipGetLastError());
    RQ_TRY_RAW(launch_gemm(s, false, false, mJ, b, b, 1.0, P, ldp, M0, b, 0.0, Y, ldy, nullptr, 0));
    X = Y;
    ldx = ldy;
  }
  RQ_TRY_RAW(launch_gemm(s, true, false, b, b, mJ, 1.0, X, ldx, X, ldx, 0.0, G1, b, splitk, splitk_elems));
  hipLaunchKernelGGL(chol1_kernel, dim3(1), dim3(SM_T), SM_LDS, s, b, G1, M1, st);
  RQ_HIP(hipGetLastError());
  RQ_TRY_RAW(launch_gemm(s, false, false, mJ, b, b, 1.0, X, ldx, M1, b, 0.0, Q1, mJ, nullptr, 0));
  // [G2 H] = Q1^T [Q1 P] in one launch (H follows G2 in the scratch, ld b)
  RQ_TRY_RAW(launch_gemm_pair(s, b, b, mJ, 1.0, Q1, mJ, Q1, mJ, P, ldp, 0.0, G2, b, splitk, splitk_elems));
  // four workgroups: each forms the factors, then one of the four products
  hipLaunchKernelGGL(recon_kernel, dim3(4), dim3(SM_T), SM_LDS, s, b, mJ, G2, H, Q1, mJ, P, ldp, Y, ldy, tau, T, M3,
                     st, (const double*)M1, S11 ? W11 : nullptr);
  RQ_HIP(hipGetLastError());
  // (the panel launch that follows copies Y(b:mJ, :) into P when st is 0)
  if (mJ > b)
    RQ_TRY_RAW(launch_gemm(s, false, false, mJ - b, b, b, 1.0, Q1 + b, mJ, M3, b, 0.0, Y + b, ldy, nullptr, 0));
  return 0;
}

}  // namespace rq
