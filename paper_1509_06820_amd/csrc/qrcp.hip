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

constexpr int SQ_THREADS = 1024;
constexpr int SQ_MAXP = 64;      // workgroups of the sample QRCP launch
constexpr int SQ_MAXCPT = 4;     // passes over the slab in the scan
constexpr int SQ_FLAG_GO = 64;   // flags[64]: round released by workgroup 0
constexpr int SQ_FLAG_T0 = 65;   // flags[65]: pivots certified so far
constexpr int SQ_BMAX = 64;

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

// A sample column is held by LANES adjacent lanes; lane `sub` owns rows
// sub*RPL .. sub*RPL+RPL-1 (rows >= l are zero).
template <int LANES>
__device__ __forceinline__ double grp_sum(double v) {
#pragma unroll
  for (int off = 1; off < LANES; off <<= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

template <int LMAX, int LANES>
__device__ __forceinline__ void sq_load(const SqParams& a, int64_t c, int sub, double (&col)[LMAX / LANES]) {
  constexpr int RPL = LMAX / LANES;
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int r = sub * RPL + i;
    col[i] = (r < a.l) ? a.Bt[c + (int64_t)r * a.ldbt] : 0.0;
  }
}

// Squared norm over rows >= from.  Lane partial sums run in increasing row
// order and are combined pairwise, so every lane of the group -- and the scan
// and the candidate steps -- get bitwise identical values.
template <int LMAX, int LANES>
__device__ __forceinline__ double sq_norm2(const double (&col)[LMAX / LANES], int sub, int from) {
  constexpr int RPL = LMAX / LANES;
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < RPL; ++i) s += (sub * RPL + i >= from) ? col[i] * col[i] : 0.0;
  return grp_sum<LANES>(s);
}

// col <- (I - tau v v^T) col, v in LDS (zero above its first row and below row l).
template <int LMAX, int LANES>
__device__ __forceinline__ void sq_apply(double (&col)[LMAX / LANES], int sub, const double* v, double tau) {
  constexpr int RPL = LMAX / LANES;
  double d = 0.0;
#pragma unroll
  for (int i = 0; i < RPL; ++i) d += v[sub * RPL + i] * col[i];
  d = grp_sum<LANES>(d) * tau;
  asm volatile("" ::: "memory");
#pragma unroll
  for (int i = 0; i < RPL; ++i) col[i] -= d * v[sub * RPL + i];
}

__device__ __forceinline__ bool key_before(double v1, long long p1, double v2, long long p2) {
  return (v1 > v2) || (v1 == v2 && p1 < p2);
}

// Block-wide argmax over (value, position), SQ_THREADS threads.
__device__ __forceinline__ void block_argmax(double& v, long long& p, double* sv, long long* sp) {
#pragma unroll
  for (int off = 1; off < WAVE; off <<= 1) {
    const double ov = __shfl_xor(v, off, WAVE);
    const long long op = __shfl_xor(p, off, WAVE);
    if (key_before(ov, op, v, p)) { v = ov; p = op; }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { sv[w] = v; sp[w] = p; }
  __syncthreads();
  if (threadIdx.x < WAVE) {
    constexpr int NW = SQ_THREADS / WAVE;
    double bv = (threadIdx.x < NW) ? sv[threadIdx.x] : -INFINITY;
    long long bp = (threadIdx.x < NW) ? sp[threadIdx.x] : LLONG_MAX;
#pragma unroll
    for (int off = 1; off < NW; off <<= 1) {
      const double ov = __shfl_xor(bv, off, WAVE);
      const long long op = __shfl_xor(bp, off, WAVE);
      if (key_before(ov, op, bv, bp)) { bv = ov; bp = op; }
    }
    if (threadIdx.x == 0) { sv[NW] = bv; sp[NW] = bp; }
  }
  __syncthreads();
  v = sv[SQ_THREADS / WAVE];
  p = sp[SQ_THREADS / WAVE];
}

// Sort n (power of two) keys in LDS: descending value, ascending position.
__device__ void bitonic_sort_keys(double* kv, long long* kp, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < n / 2; t += SQ_THREADS) {
        const int lo = 2 * stride * (t / stride) + (t % stride);
        const int hi = lo + stride;
        const bool up = ((lo & size) == 0);  // this run sorted "best first"
        const double v1 = kv[lo], v2 = kv[hi];
        const long long p1 = kp[lo], p2 = kp[hi];
        const bool swap = up ? key_before(v2, p2, v1, p1) : key_before(v1, p1, v2, p2);
        if (swap) { kv[lo] = v2; kv[hi] = v1; kp[lo] = p2; kp[hi] = p1; }
      }
      __syncthreads();
    }
  }
}

struct SqShared {
  double* vs;       // reflectors of the scan, SQ_BMAX x LMAX (aliases vlog)
  double* vlog;     // reflectors found in this round (SQ_BMAX x LMAX)
  double* slog;     // S columns of this round's pivots (SQ_BMAX x LMAX)
  double* vsh;      // 2 x LMAX current reflector (double buffered)
  double* kv;       // sort keys (values)
  long long* kp;    // sort keys (positions)
  double* sv;
  long long* sp;
  double* scal;     // tau log (SQ_BMAX) + current tau (2)
  int* plog;        // pivot log (SQ_BMAX)
  int* misc;
};

// Scan: apply reflectors [a0, t0) to every unselected column (positions >=
// t0) of this workgroup's slab and write it back; if `select`, rank the slab
// by trailing norm over rows >= t0, publish the K best positions as
// candidates and theta = the best norm left out.
template <int LMAX, int LANES>
__device__ void sq_scan(const SqParams& a, int me, int a0, int t0, bool select, const SqShared& sh) {
  constexpr int RPL = LMAX / LANES;
  constexpr int COLS = SQ_THREADS / LANES;
  const int tid = threadIdx.x, sub = tid % LANES, grp = tid / LANES;
  const int nr = t0 - a0;
  for (int e = tid; e < nr * LMAX; e += SQ_THREADS) {
    const int s = e / LMAX, r = e - s * LMAX;
    sh.vs[e] = (r < a.l) ? a.refl[r + (int64_t)(a0 + s) * a.l] : 0.0;
  }
  for (int s = tid; s < nr; s += SQ_THREADS) sh.scal[s] = a.rtau[a0 + s];
  __syncthreads();

  const int64_t rem = a.nJ - t0;
  const int64_t w = (rem + a.P - 1) / a.P;
  const int64_t lo = t0 + (int64_t)me * w;
  const int64_t hi = min(a.nJ, lo + w);
  const int cnt = (int)max<int64_t>(0, hi - lo);
  bool bad = false;
  for (int e0 = 0; e0 < cnt; e0 += COLS) {
    const int e = e0 + grp;
    const bool have = e < cnt;
    const int64_t c = lo + (have ? e : 0);
    double col[RPL];
    sq_load<LMAX, LANES>(a, c, sub, col);
    for (int s = 0; s < nr; ++s) sq_apply<LMAX, LANES>(col, sub, sh.vs + s * LMAX, sh.scal[s]);
    if (have && nr > 0) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int r = sub * RPL + i;
        if (r >= a0 && r < a.l) a.Bt[c + (int64_t)r * a.ldbt] = col[i];
      }
    }
    if (select) {
      const double x = sq_norm2<LMAX, LANES>(col, sub, t0);
      if (have && !(x <= DBL_MAX)) bad = true;
      if (have && sub == 0) { sh.kv[e] = ranked(x); sh.kp[e] = c; }
    }
  }
  if (!select) return;
  if (bad && a.info) atomicCAS(a.info, 0, a.info_base + t0 + 1);
  long long* cand = a.cand_pos + (int64_t)me * a.K;
  if (a.K >= cnt) {
    __syncthreads();
    for (int e = tid; e < a.K; e += SQ_THREADS) cand[e] = (e < cnt) ? sh.kp[e] : -1;
    if (tid == 0) a.theta[me] = -INFINITY;
    return;
  }
  int n2 = 1;
  while (n2 < cnt) n2 <<= 1;
  for (int e = cnt + tid; e < n2; e += SQ_THREADS) { sh.kv[e] = -INFINITY; sh.kp[e] = LLONG_MAX; }
  __syncthreads();
  bitonic_sort_keys(sh.kv, sh.kp, n2);
  for (int e = tid; e < a.K; e += SQ_THREADS) cand[e] = sh.kp[e];
  if (tid == 0) a.theta[me] = sh.kv[a.K];
}

// Candidate steps (workgroup 0): greedy QRCP on the gathered candidates as
// long as the winner provably beats every column left out of the candidate
// set (its norm exceeds the largest left-out norm at the start of the round,
// which bounds all later ones).  Nothing is written to global memory inside
// the loop; the round's pivots, reflectors, S columns and column moves are
// written at the end.  Returns the number of pivots fixed so far.
template <int LMAX, int LANES>
__device__ int sq_steps(const SqParams& a, int t0, const SqShared& sh) {
  constexpr int RPL = LMAX / LANES;
  const int tid = threadIdx.x, sub = tid % LANES, grp = tid / LANES;
  const int C = a.P * a.K;
  double col[RPL];
  long long pos = (grp < C) ? a.cand_pos[grp] : -1;
  bool active = pos >= 0;
  sq_load<LMAX, LANES>(a, active ? pos : 0, sub, col);
  double theta = -INFINITY;
  for (int q = 0; q < a.P; ++q) theta = fmax(theta, a.theta[q]);
  const double bound = (theta > 0.0) ? theta * (1.0 + 1e-12) : theta;

  int t = t0;
  while (t < a.bJ) {
    double nu = active ? ranked(sq_norm2<LMAX, LANES>(col, sub, t)) : -INFINITY;
    long long p = active ? pos : LLONG_MAX;
    block_argmax(nu, p, sh.sv, sh.sp);
    if ((t > t0 && !(nu > bound)) || p == LLONG_MAX) break;
    const bool winner = active && pos == p;
    double* vsh = sh.vsh + (t & 1) * LMAX;
    if (winner) {
      // Householder reflector of rows t..l-1 (LAPACK dlarfg normalisation)
      double alpha_part = 0.0, xn2 = 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int r = sub * RPL + i;
        alpha_part += (r == t) ? col[i] : 0.0;
        xn2 += (r > t) ? col[i] * col[i] : 0.0;
      }
      const double alpha = grp_sum<LANES>(alpha_part);
      xn2 = grp_sum<LANES>(xn2);
      double tau = 0.0, beta = alpha, scal = 0.0;
      if (xn2 != 0.0) {
        const double nrm = sqrt(alpha * alpha + xn2);
        beta = (alpha >= 0.0) ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      const int slot = t - t0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int r = sub * RPL + i;
        const double v = (r == t) ? 1.0 : ((r > t) ? col[i] * scal : 0.0);
        vsh[r] = v;
        sh.vlog[slot * LMAX + r] = v;
        sh.slog[slot * LMAX + r] = (r < t) ? col[i] : ((r == t) ? beta : 0.0);
      }
      if (sub == 0) {
        sh.scal[SQ_BMAX + (t & 1)] = tau;
        sh.scal[slot] = tau;
        sh.plog[slot] = (int)p;
      }
      active = false;
    }
    // sequential swap t <-> p: a candidate sitting at position t moves to p
    if (active && pos == t) pos = p;
    __syncthreads();
    if (active) sq_apply<LMAX, LANES>(col, sub, vsh, sh.scal[SQ_BMAX + (t & 1)]);
    ++t;
  }
  __syncthreads();
  const int tn = t;
  const int nt = tn - t0;
  // pivots, reflectors
  for (int e = tid; e < nt * a.l; e += SQ_THREADS) {
    const int s = e / a.l, r = e - s * a.l;
    a.refl[r + (int64_t)(t0 + s) * a.l] = sh.vlog[s * LMAX + r];
  }
  for (int s = tid; s < nt; s += SQ_THREADS) {
    a.rtau[t0 + s] = sh.scal[s];
    a.piv[t0 + s] = sh.plog[s];
  }
  // Column moves of this round: position q >= tn named as a partner receives
  // the round-start column found by undoing the swaps from the last one.
  int* dst = sh.misc;           // SQ_BMAX destinations
  int* src = sh.misc + SQ_BMAX; // their sources
  int* nmv = sh.misc + 2 * SQ_BMAX;
  if (tid == 0) *nmv = 0;
  __syncthreads();
  if (tid < nt) {
    const int q = sh.plog[tid];
    bool first = q >= tn;
    for (int s2 = 0; s2 < tid && first; ++s2)
      if (sh.plog[s2] == q) first = false;
    if (first) {
      int x = q;
      for (int s2 = nt - 1; s2 >= 0; --s2) {
        const int ps = sh.plog[s2], ts = t0 + s2;
        if (x == ts) x = ps;
        else if (x == ps) x = ts;
      }
      const int k = atomicAdd(nmv, 1);
      dst[k] = q;
      src[k] = x;
    }
  }
  __syncthreads();
  const int nm = *nmv;
  double* stage = sh.vlog;  // reused: reflectors are already written out
  for (int e = tid; e < nm * a.l; e += SQ_THREADS) {
    const int k = e / a.l, r = e - k * a.l;
    stage[k * LMAX + r] = a.Bt[src[k] + (int64_t)r * a.ldbt];
  }
  __syncthreads();
  for (int e = tid; e < nm * a.l; e += SQ_THREADS) {
    const int k = e / a.l, r = e - k * a.l;
    a.Bt[dst[k] + (int64_t)r * a.ldbt] = stage[k * LMAX + r];
  }
  for (int e = tid; e < nt * a.l; e += SQ_THREADS) {
    const int s = e / a.l, r = e - s * a.l;
    a.Bt[(t0 + s) + (int64_t)r * a.ldbt] = sh.slog[s * LMAX + r];
  }
  return tn;
}

// LDS: [vlog = vs] [slog | sort keys] [vsh] [argmax] [tau log] [pivot log] [moves]
// (the sort keys live only in the scan, the S-column log only in the steps)
template <int LMAX, int LANES>
constexpr size_t sq_region_b() {
  constexpr size_t slog = (size_t)SQ_BMAX * LMAX * 8;
  constexpr size_t keys = (size_t)(SQ_THREADS / LANES) * SQ_MAXCPT * 16;
  return slog > keys ? slog : keys;
}

template <int LMAX, int LANES>
constexpr size_t sq_lds_bytes() {
  return (size_t)SQ_BMAX * LMAX * 8 + sq_region_b<LMAX, LANES>() + 2 * LMAX * 8 + 64 * 8 + (SQ_BMAX + 4) * 8 +
         SQ_BMAX * 4 + 3 * SQ_BMAX * 4 + 64;
}

template <int LMAX, int LANES>
__global__ void __launch_bounds__(SQ_THREADS) sample_qrcp_kernel(SqParams a) {
  extern __shared__ double smem[];
  SqShared sh;
  char* base = (char*)smem;
  sh.vlog = (double*)base; base += (size_t)SQ_BMAX * LMAX * 8;
  sh.vs = sh.vlog;
  sh.slog = (double*)base;
  sh.kv = (double*)base;
  sh.kp = (long long*)(base + (size_t)(SQ_THREADS / LANES) * SQ_MAXCPT * 8);
  base += sq_region_b<LMAX, LANES>();
  sh.vsh = (double*)base; base += 2 * LMAX * 8;
  sh.sv = (double*)base; base += 32 * 8;
  sh.sp = (long long*)base; base += 32 * 8;
  sh.scal = (double*)base; base += (SQ_BMAX + 4) * 8;
  sh.plog = (int*)base; base += SQ_BMAX * 4;
  sh.misc = (int*)base;
  const int me = blockIdx.x;
  if (earlier_failure(a.err)) return;
  int a0 = 0, t0 = 0;
  for (unsigned round = 1;; ++round) {
    const bool select = t0 < a.bJ;
    sq_scan<LMAX, LANES>(a, me, a0, t0, select, sh);
    if (!select) break;
    publish_flag(a.flags, me, round);
    if (me == 0) {
      if (!wait_flags(a.flags, a.P, round, a.err)) return;
      const int tn = sq_steps<LMAX, LANES>(a, t0, sh);
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

template <int LMAX, int LANES>
int launch_sq(hipStream_t s, SqParams& a) {
  constexpr int COLS = SQ_THREADS / LANES;
  int64_t P = (a.nJ + COLS - 1) / COLS;
  if (P > SQ_MAXP) P = SQ_MAXP;
  if ((a.nJ + P - 1) / P > (int64_t)COLS * SQ_MAXCPT) return -4;  // n too large for this kernel
  a.P = (int)P;
  a.K = (P == 1) ? COLS : std::max(1, COLS / (int)P);
  const size_t lds = sq_lds_bytes<LMAX, LANES>();
  static_assert(sq_lds_bytes<LMAX, LANES>() <= 160 * 1024, "LDS budget");
  static bool attr_set = false;
  if (!attr_set) {
    RQ_HIP(hipFuncSetAttribute((const void*)sample_qrcp_kernel<LMAX, LANES>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr_set = true;
  }
  void* args[] = {&a};
  RQ_HIP(hipLaunchCooperativeKernel((const void*)sample_qrcp_kernel<LMAX, LANES>, dim3(a.P), dim3(SQ_THREADS), args,
                                    lds, s));
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

// Fallback T: G = Y^T Y accumulated by one workgroup, then the recurrence.
__global__ void __launch_bounds__(256) larft_gated_kernel(int64_t mJ, int bJ, const double* __restrict__ Y,
                                                          int64_t ldy, const double* __restrict__ tau,
                                                          double* __restrict__ T, const int* gate) {
  __shared__ double Gs[64 * 64];
  __shared__ double Ts[64 * 64];
  __shared__ int s_gate;
  if (threadIdx.x == 0) s_gate = *gate;
  __syncthreads();
  if (s_gate == 0) return;
  for (int e = threadIdx.x; e < bJ * bJ; e += 256) {
    const int i = e % bJ, j = e / bJ;
    double acc = 0.0;
    if (i <= j)
      for (int64_t r = 0; r < mJ; ++r) acc += Y[r + i * ldy] * Y[r + j * ldy];
    Gs[e] = acc;
    Ts[e] = 0.0;
  }
  __syncthreads();
  for (int i = 0; i < bJ; ++i) {
    const int r = threadIdx.x;
    if (r < i) {
      double h = 0.0;
      for (int q = r; q < i; ++q) h += Ts[r + q * bJ] * Gs[q + i * bJ];
      Ts[r + i * bJ] = -tau[i] * h;
    } else if (r == i) {
      Ts[i + i * bJ] = tau[i];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < bJ * bJ; e += 256) T[e] = Ts[e];
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
  if (bJ > SQ_BMAX) return -5;
  SqParams a;
  a.Bt = Bt; a.ldbt = ldbt; a.l = l; a.nJ = nJ; a.bJ = bJ; a.piv = piv; a.info = info; a.info_base = info_base;
  a.refl = w.refl; a.rtau = w.rtau; a.cand_pos = w.cand_pos; a.theta = w.theta; a.flags = w.flags; a.err = w.err;
  if (l <= 32) return launch_sq<32, 4>(s, a);
  if (l <= 64) return launch_sq<64, 4>(s, a);
  if (l <= 80) return launch_sq<80, 4>(s, a);
  if (l <= 128) return launch_sq<128, 8>(s, a);
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

int launch_larft_gated(hipStream_t s, int64_t mJ, int bJ, const double* Y, int64_t ldy, const double* tau, double* T,
                       const int* gate) {
  hipLaunchKernelGGL(larft_gated_kernel, dim3(1), dim3(256), 0, s, mJ, bJ, Y, ldy, tau, T, gate);
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
