// Sample QRCP (Alg. 4 step "get b column pivots from the sample", i.e. Alg. 1
// run for bJ steps on the l x nJ sample), column swaps of A, the connection
// matrix T of a reflector block, the W11 = S11 R11^-1 factor of the sample
// update (eq. update1) and small data-movement kernels.
//
// The sample is stored transposed: Bt is nJ x l column-major, so B(r, c) =
// Bt[c + r*ldbt] and a thread that owns a sample column reads it with
// coalesced row-by-row loads across the wave.
#include <float.h>
#include "kernels.hpp"

namespace rq {

namespace {

constexpr int SQ_THREADS = 256;
constexpr int SQ_MAXP = 64;     // workgroups of the sample QRCP launch
constexpr int SQ_MAXK = 16;     // candidates per workgroup (P > 1)
constexpr int SQ_MAXCPT = 4;    // sample columns per thread in the scan
constexpr int SQ_FLAG_GO = 64;  // flags[64]: round released by workgroup 0
constexpr int SQ_FLAG_T0 = 65;  // flags[65]: pivots certified so far

struct SqParams {
  double* Bt;
  int64_t ldbt;
  int l;
  int64_t nJ;
  int bJ;
  int* piv;
  int* info;
  int info_base;
  double* refl;
  double* rtau;
  long long* cand_pos;
  double* theta;
  unsigned* flags;
  int* err;
  int P;
  int K;
};

__device__ __forceinline__ double ranked(double nu) { return (nu != nu) ? -1.0 : nu; }

// Squared trailing norm over rows from..LMAX-1 (rows >= l are zero), summed
// in increasing row order.  The scan and the candidate steps use this same
// function, so both see bitwise identical norms for identical columns.
template <int LMAX>
__device__ __forceinline__ double trailing_norm2(const double (&col)[LMAX], int from) {
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < LMAX; ++r) s += (r >= from) ? col[r] * col[r] : 0.0;
  return s;
}

// col <- (I - tau v v^T) col.  v is zero above its first row and below row l,
// so the full-length loops leave those rows of col exactly unchanged.
template <int LMAX>
__device__ __forceinline__ void apply_reflector(double (&col)[LMAX], const double* v, double tau) {
  double dot = 0.0;
#pragma unroll
  for (int r = 0; r < LMAX; ++r) dot += v[r] * col[r];
  dot *= tau;
  // re-read v from LDS below instead of keeping LMAX values live in registers
  asm volatile("" ::: "memory");
#pragma unroll
  for (int r = 0; r < LMAX; ++r) col[r] -= dot * v[r];
}

// Block-wide argmax over (value, position) with the pivot ranking
// (larger value, then lower position).  256 threads.
__device__ __forceinline__ void block_argmax(double& v, long long& p, double* sv, long long* sp) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    double ov = __shfl_xor(v, off, WAVE);
    long long op = __shfl_xor(p, off, WAVE);
    if (ov > v || (ov == v && op < p)) { v = ov; p = op; }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { sv[w] = v; sp[w] = p; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bv = sv[0];
    long long bp = sp[0];
    for (int q = 1; q < SQ_THREADS / WAVE; ++q)
      if (sv[q] > bv || (sv[q] == bv && sp[q] < bp)) { bv = sv[q]; bp = sp[q]; }
    sv[4] = bv;
    sp[4] = bp;
  }
  __syncthreads();
  v = sv[4];
  p = sp[4];
  __syncthreads();
}

template <int LMAX>
__device__ __forceinline__ void load_col(const SqParams& a, int64_t c, double (&col)[LMAX]) {
#pragma unroll
  for (int r = 0; r < LMAX; ++r) col[r] = (r < a.l) ? a.Bt[c + (int64_t)r * a.ldbt] : 0.0;
}

// Scan: apply reflectors [a0, t0) to every unselected column (positions
// >= t0) of this workgroup's slab, write it back, and (if select) compute the
// trailing norms over rows >= t0, pick this workgroup's K best columns as
// candidates and record theta = the best norm among the rest.
template <int LMAX>
__device__ void sq_scan(const SqParams& a, int me, int a0, int t0, bool select, double* vs, double* vtau,
                        double* snu, long long* spos, double* sv, long long* sp) {
  const int tid = threadIdx.x;
  const int nr = t0 - a0;
  for (int e = tid; e < nr * LMAX; e += SQ_THREADS) {
    const int s = e / LMAX, r = e - s * LMAX;
    vs[e] = (r < a.l) ? a.refl[r + (int64_t)(a0 + s) * a.l] : 0.0;
  }
  for (int s = tid; s < nr; s += SQ_THREADS) vtau[s] = a.rtau[a0 + s];
  __syncthreads();

  const int64_t rem = a.nJ - t0;
  const int64_t w = (rem + a.P - 1) / a.P;
  const int64_t lo = t0 + (int64_t)me * w;
  const int64_t hi = min(a.nJ, lo + w);
  const int cnt = (int)max<int64_t>(0, hi - lo);
  bool bad = false;
#pragma unroll 1
  for (int e = tid; e < cnt; e += SQ_THREADS) {
    const int64_t c = lo + e;
    double col[LMAX];
    load_col<LMAX>(a, c, col);
#pragma unroll 1
    for (int s = 0; s < nr; ++s) apply_reflector<LMAX>(col, vs + s * LMAX, vtau[s]);
    if (nr > 0) {
#pragma unroll
      for (int r = 0; r < LMAX; ++r)
        if (r < a.l) a.Bt[c + (int64_t)r * a.ldbt] = col[r];
    }
    if (select) {
      const double x = trailing_norm2<LMAX>(col, t0);
      if (!(x <= DBL_MAX)) bad = true;
      snu[e] = ranked(x);
      spos[e] = c;
    }
  }
  if (!select) return;
  if (bad && a.info) atomicCAS(a.info, 0, a.info_base + t0 + 1);
  __syncthreads();

  long long* cand = a.cand_pos + (int64_t)me * a.K;
  if (a.K >= cnt) {
    // every column of the slab is a candidate; nothing is left out
    for (int e = tid; e < a.K; e += SQ_THREADS) cand[e] = (e < cnt) ? spos[e] : -1;
    if (tid == 0) a.theta[me] = -INFINITY;
    __syncthreads();
    return;
  }
  for (int k = 0; k <= a.K; ++k) {
    double bv = -INFINITY;
    long long bp = LLONG_MAX;
    for (int e = tid; e < cnt; e += SQ_THREADS) {
      const long long pp = spos[e];
      const double vv = snu[e];
      if (pp != LLONG_MAX && (vv > bv || (vv == bv && pp < bp))) { bv = vv; bp = pp; }
    }
    block_argmax(bv, bp, sv, sp);
    if (k == a.K) {
      if (tid == 0) a.theta[me] = (bp == LLONG_MAX) ? -INFINITY : bv;
      break;
    }
    if (tid == 0) cand[k] = (bp == LLONG_MAX) ? -1 : bp;
    if (bp != LLONG_MAX) {
      const int e = (int)(bp - lo);
      if (e >= 0 && e < cnt && (e % SQ_THREADS) == tid) spos[e] = LLONG_MAX;  // taken
    }
    __syncthreads();
  }
  __syncthreads();
}

// Candidate steps (workgroup 0): greedy QRCP on the gathered candidates as
// long as the winner provably beats every column left out of the candidate
// set (its norm exceeds the largest left-out norm at the start of the round,
// which bounds all later ones).  Returns the number of pivots fixed so far.
template <int LMAX>
__device__ int sq_steps(const SqParams& a, int t0, double* vsh, double* sv, long long* sp, double* sscal) {
  const int tid = threadIdx.x;
  const int C = a.P * a.K;
  double col[LMAX];
  long long pos = -1;
  bool active = false;
  if (tid < C) pos = a.cand_pos[tid];
  if (pos >= 0) {
    active = true;
    load_col<LMAX>(a, pos, col);
  } else {
#pragma unroll
    for (int r = 0; r < LMAX; ++r) col[r] = 0.0;
  }
  double theta = -INFINITY;
  for (int q = 0; q < a.P; ++q) theta = fmax(theta, a.theta[q]);
  const double bound = (theta > 0.0) ? theta * (1.0 + 1e-12) : theta;

  int t = t0;
  while (t < a.bJ) {
    double nu = active ? ranked(trailing_norm2<LMAX>(col, t)) : -INFINITY;
    long long p = active ? pos : LLONG_MAX;
    block_argmax(nu, p, sv, sp);
    if (t > t0 && !(nu > bound)) break;
    if (p == LLONG_MAX) break;  // no candidate left (cannot happen for bJ <= C)
    const bool winner = active && pos == p;
    if (tid == 0) a.piv[t] = (int)p;
    // Sequential swap t <-> p: the column now at position t moves to p.
    if (p != t && tid < a.l) {
      const double v = a.Bt[t + (int64_t)tid * a.ldbt];
      a.Bt[p + (int64_t)tid * a.ldbt] = v;
    }
    if (active && !winner && pos == t) pos = p;
    __syncthreads();
    if (winner) {
      // Householder reflector of col[t..l) (LAPACK dlarfg normalisation).
      double alpha = 0.0, xn2 = 0.0;
#pragma unroll
      for (int r = 0; r < LMAX; ++r) {
        alpha = (r == t) ? col[r] : alpha;
        xn2 += (r > t) ? col[r] * col[r] : 0.0;
      }
      double tau = 0.0, beta = alpha, scal = 0.0;
      if (xn2 != 0.0) {
        const double nrm = sqrt(alpha * alpha + xn2);
        beta = (alpha >= 0.0) ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
#pragma unroll
      for (int r = 0; r < LMAX; ++r) {
        const double v = (r == t) ? 1.0 : ((r > t) ? col[r] * scal : 0.0);
        vsh[r] = v;
        if (r < a.l) {
          a.refl[r + (int64_t)t * a.l] = v;
          a.Bt[t + (int64_t)r * a.ldbt] = (r < t) ? col[r] : (r == t ? beta : 0.0);
        }
      }
      sscal[0] = tau;
      a.rtau[t] = tau;
      active = false;
    }
    __syncthreads();
    if (active) apply_reflector<LMAX>(col, vsh, sscal[0]);
    ++t;
    __syncthreads();
  }
  return t;
}

template <int LMAX>
__global__ void __launch_bounds__(SQ_THREADS) sample_qrcp_kernel(SqParams a) {
  __shared__ double vs[64 * LMAX];  // up to 64 reflectors
  __shared__ double vtau[64];
  __shared__ double vsh[LMAX];
  __shared__ double snu[SQ_THREADS * SQ_MAXCPT];
  __shared__ long long spos[SQ_THREADS * SQ_MAXCPT];
  __shared__ double sv[8];
  __shared__ long long sp[8];
  __shared__ double sscal[2];
  const int me = blockIdx.x;
  if (earlier_failure(a.err)) return;
  int a0 = 0, t0 = 0;
  for (unsigned round = 1;; ++round) {
    const bool select = t0 < a.bJ;
    sq_scan<LMAX>(a, me, a0, t0, select, vs, vtau, snu, spos, sv, sp);
    if (!select) break;
    publish_flag(a.flags, me, round);
    if (me == 0) {
      if (!wait_flags(a.flags, a.P, round, a.err)) return;
      const int tn = sq_steps<LMAX>(a, t0, vsh, sv, sp, sscal);
      if (threadIdx.x == 0) a.flags[SQ_FLAG_T0] = (unsigned)tn;
      publish_flag(a.flags + SQ_FLAG_GO, 0, round);
    }
    if (!wait_one(a.flags + SQ_FLAG_GO, round, a.err, nullptr)) return;
    const int tn = (int)__hip_atomic_load(&a.flags[SQ_FLAG_T0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a0 = t0;
    t0 = tn;
    __syncthreads();
  }
}

template <int LMAX>
int launch_sq(hipStream_t s, SqParams& a) {
  void* args[] = {&a};
  RQ_HIP(hipLaunchCooperativeKernel((const void*)sample_qrcp_kernel<LMAX>, dim3(a.P), dim3(SQ_THREADS), args, 0, s));
  return 0;
}

// ------------------------------------------------------------------ swaps
constexpr int SW_ROWS = 64;

__global__ void __launch_bounds__(256) apply_swaps_kernel(const int* __restrict__ piv, int bJ, int64_t offset,
                                                          double* M, int64_t ldm, int64_t rows, int64_t* jpvt) {
  __shared__ int dst[128], src[128];
  __shared__ int npair;
  __shared__ double tile[128 * SW_ROWS];
  __shared__ int64_t itile[128];
  const int tid = threadIdx.x;
  if (tid == 0) npair = 0;
  __syncthreads();
  // Destinations: positions 0..bJ-1 and every partner p_t >= bJ (first occurrence).
  if (tid < 2 * bJ) {
    int q = -1;
    if (tid < bJ) {
      q = tid;
    } else {
      const int t = tid - bJ;
      const int pt = piv[t];
      bool first = pt >= bJ;
      for (int s2 = 0; s2 < t && first; ++s2)
        if (piv[s2] == pt) first = false;
      if (first) q = pt;
    }
    if (q >= 0) {
      // content of position q after the swaps: undo them from the last one
      int sidx = q;
      for (int s2 = bJ - 1; s2 >= 0; --s2) {
        const int ps = piv[s2];
        if (sidx == s2) sidx = ps;
        else if (sidx == ps) sidx = s2;
      }
      if (sidx != q) {
        const int k = atomicAdd(&npair, 1);
        dst[k] = q;
        src[k] = sidx;
      }
    }
  }
  __syncthreads();
  const int np = npair;
  if (np == 0) return;
  const int64_t r0 = (int64_t)blockIdx.x * SW_ROWS;
  for (int e = tid; e < np * SW_ROWS; e += 256) {
    const int k = e / SW_ROWS, rr = e - k * SW_ROWS;
    const int64_t r = r0 + rr;
    if (r < rows) tile[e] = M[r + (offset + src[k]) * ldm];
  }
  if (jpvt && blockIdx.x == 0 && tid < np) itile[tid] = jpvt[offset + src[tid]];
  __syncthreads();
  for (int e = tid; e < np * SW_ROWS; e += 256) {
    const int k = e / SW_ROWS, rr = e - k * SW_ROWS;
    const int64_t r = r0 + rr;
    if (r < rows) M[r + (offset + dst[k]) * ldm] = tile[e];
  }
  if (jpvt && blockIdx.x == 0 && tid < np) jpvt[offset + dst[tid]] = itile[tid];
}

// ------------------------------------------------------------------ T factor
// T[i,i] = tau_i;  T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i]   (G = Y^T Y)
__global__ void __launch_bounds__(64) larft_kernel(int bJ, const double* __restrict__ G, const double* __restrict__ tau,
                                                   double* __restrict__ T) {
  __shared__ double Gs[64 * 64];
  __shared__ double Ts[64 * 64];
  const int r = threadIdx.x;
  for (int e = r; e < bJ * bJ; e += 64) { Gs[e] = G[e]; Ts[e] = 0.0; }
  __syncthreads();
  for (int i = 0; i < bJ; ++i) {
    const double ti = tau[i];
    if (r < i) {
      double h = 0.0;
      for (int q = r; q < i; ++q) h += Ts[r + q * bJ] * Gs[q + i * bJ];
      Ts[r + i * bJ] = -ti * h;
    } else if (r == i) {
      Ts[i + i * bJ] = ti;
    }
    __syncthreads();
  }
  for (int e = r; e < bJ * bJ; e += 64) T[e] = Ts[e];
}

// ------------------------------------------------------------------ W11
// Row i of W solves W R = S: W(i, j) = (S(i, j) - sum_{i<=q<j} W(i,q) R(q,j)) / R(j,j),
// with column j of W set to zero when R(j, j) == 0.
__global__ void __launch_bounds__(64) w11_kernel(int bJ, const double* __restrict__ S, int64_t srs, int64_t scs,
                                                 const double* __restrict__ R, int64_t ldr, double* __restrict__ W) {
  __shared__ double Rs[64 * 64];
  __shared__ double Ws[64 * 65];
  const int i = threadIdx.x;
  for (int e = i; e < bJ * bJ; e += 64) {
    const int rr = e % bJ, cc = e / bJ;
    Rs[e] = (rr <= cc) ? R[rr + cc * ldr] : 0.0;
  }
  __syncthreads();
  if (i < bJ) {
    for (int j = 0; j < bJ; ++j) {
      double v = 0.0;
      const double d = Rs[j + j * bJ];
      if (j >= i && d != 0.0) {
        double acc = S[(int64_t)i * srs + (int64_t)j * scs];
        for (int q = i; q < j; ++q) acc -= Ws[i + q * 65] * Rs[q + j * bJ];
        v = acc / d;
      }
      Ws[i + j * 65] = v;
    }
    for (int j = 0; j < bJ; ++j) W[i + j * bJ] = Ws[i + j * 65];
  }
}

// ------------------------------------------------------------------ utilities
__global__ void fill_kernel(unsigned* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void copy2d_kernel(int64_t rows, int64_t cols, const double* __restrict__ src, int64_t lds,
                              double* __restrict__ dst, int64_t ldd) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t j = idx / rows, i = idx - j * rows;
  dst[i + j * ldd] = src[i + j * lds];
}

__global__ void set_identity_kernel(int64_t rows, int64_t cols, double* M, int64_t ldm) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t j = idx / rows, i = idx - j * rows;
  M[i + j * ldm] = (i == j) ? 1.0 : 0.0;
}

__global__ void scatter_rt_kernel(int64_t k, int64_t n, const double* __restrict__ R, int64_t ldr,
                                  const int64_t* __restrict__ jpvt, double* __restrict__ Z, int64_t ldz) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= k * n) return;
  const int64_t j = idx / k, i = idx - j * k;
  Z[jpvt[j] + i * ldz] = (i <= j) ? R[i + j * ldr] : 0.0;
}

__global__ void triu_copy_kernel(int64_t k, const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                                 int64_t ldd) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= k * k) return;
  const int64_t j = idx / k, i = idx - j * k;
  dst[i + j * ldd] = (i <= j) ? src[i + j * lds] : 0.0;
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

size_t sample_qrcp_flag_words() { return 128; }

int launch_sample_qrcp(hipStream_t s, double* Bt, int64_t ldbt, int l, int64_t nJ, int bJ, int* piv, int* info,
                       int info_base, const SampleQrcpWork& w) {
  if (bJ <= 0 || nJ <= 0) return 0;
  SqParams a;
  a.Bt = Bt; a.ldbt = ldbt; a.l = l; a.nJ = nJ; a.bJ = bJ; a.piv = piv; a.info = info; a.info_base = info_base;
  a.refl = w.refl; a.rtau = w.rtau; a.cand_pos = w.cand_pos; a.theta = w.theta; a.flags = w.flags; a.err = w.err;
  int64_t P = (nJ + SQ_THREADS - 1) / SQ_THREADS;
  if (P > SQ_MAXP) P = SQ_MAXP;
  if ((nJ + P - 1) / P > (int64_t)SQ_THREADS * SQ_MAXCPT) return -4;  // n too large for this kernel
  a.P = (int)P;
  a.K = (P == 1) ? SQ_THREADS : std::min(SQ_MAXK, SQ_THREADS / (int)P);
  if (l <= 32) return launch_sq<32>(s, a);
  if (l <= 64) return launch_sq<64>(s, a);
  if (l <= 80) return launch_sq<80>(s, a);
  if (l <= 128) return launch_sq<128>(s, a);
  return -7;
}

int launch_apply_swaps(hipStream_t s, const int* piv, int bJ, int64_t offset, double* M, int64_t ldm, int64_t rows,
                       int64_t* jpvt) {
  if (bJ <= 0) return 0;
  const unsigned grid = std::max<unsigned>(1u, blocks_for(rows, SW_ROWS));
  hipLaunchKernelGGL(apply_swaps_kernel, dim3(grid), dim3(256), 0, s, piv, bJ, offset, M, ldm, rows, jpvt);
  RQ_HIP(hipGetLastError());
  return 0;
}

int launch_larft(hipStream_t s, int bJ, const double* G, const double* tau, double* T) {
  hipLaunchKernelGGL(larft_kernel, dim3(1), dim3(64), 0, s, bJ, G, tau, T);
  RQ_HIP(hipGetLastError());
  return 0;
}

int launch_w11(hipStream_t s, int bJ, const double* S, int64_t srs, int64_t scs, const double* R, int64_t ldr,
               double* W) {
  hipLaunchKernelGGL(w11_kernel, dim3(1), dim3(64), 0, s, bJ, S, srs, scs, R, ldr, W);
  RQ_HIP(hipGetLastError());
  return 0;
}

int launch_fill(hipStream_t s, void* p, size_t words) {
  if (!words) return 0;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, (unsigned*)p, words);
  RQ_HIP(hipGetLastError());
  return 0;
}

int launch_copy2d(hipStream_t s, int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst,
                  int64_t ldd) {
  if (rows <= 0 || cols <= 0) return 0;
  hipLaunchKernelGGL(copy2d_kernel, dim3(blocks_for(rows * cols, 256)), dim3(256), 0, s, rows, cols, src, lds, dst,
                     ldd);
  RQ_HIP(hipGetLastError());
  return 0;
}

int launch_set_identity(hipStream_t s, int64_t rows, int64_t cols, double* M, int64_t ldm) {
  if (rows <= 0 || cols <= 0) return 0;
  hipLaunchKernelGGL(set_identity_kernel, dim3(blocks_for(rows * cols, 256)), dim3(256), 0, s, rows, cols, M, ldm);
  RQ_HIP(hipGetLastError());
  return 0;
}

int launch_scatter_rt(hipStream_t s, int64_t k, int64_t n, const double* R, int64_t ldr, const int64_t* jpvt,
                      double* Z0T, int64_t ldz) {
  if (k <= 0 || n <= 0) return 0;
  hipLaunchKernelGGL(scatter_rt_kernel, dim3(blocks_for(k * n, 256)), dim3(256), 0, s, k, n, R, ldr, jpvt, Z0T, ldz);
  RQ_HIP(hipGetLastError());
  return 0;
}

int launch_triu_copy(hipStream_t s, int64_t k, const double* src, int64_t lds, double* dst, int64_t ldd) {
  if (k <= 0) return 0;
  hipLaunchKernelGGL(triu_copy_kernel, dim3(blocks_for(k * k, 256)), dim3(256), 0, s, k, src, lds, dst, ldd);
  RQ_HIP(hipGetLastError());
  return 0;
}

}  // namespace rq
