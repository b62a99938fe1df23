// Sample QRCP (the pivot-selection step of Alg. 4: Alg. 1 run for bJ steps on
// the l x nJ sample), column swaps of A, the connection
// matrix T of a reflector block, the W11 = S11 R11^-1 factor of the sample
// update (eq. update1) and small data-movement kernels.
//
// The sample is stored column-major with its rows padded to a register tile
// (sample_rows_padded(l) = LMAX rows, the rows past l zero): column c is the
// LMAX contiguous doubles at S + c * LMAX, so a thread that owns a column
// reads and writes it with 16-byte accesses at immediate offsets.
#include <float.h>
#include <type_traits>
#include "kernels.hpp"
#include "gemm_tile.hpp"

namespace rq {

namespace {

constexpr int SQ_T = 256;      // threads per workgroup = slab width = candidate capacity
constexpr int SQ_BMAX = 64;    // pivots per call at most
constexpr int SQ_MAXP = 256;   // workgroups (slabs) at most, so nJ <= 65536
constexpr int SQ_LCAP = 128;   // rows of a candidate buffer
// Words of one workgroup's theta entry: a whole 128-byte line, so that no two
// workgroups (which may sit on different XCDs, each with its own L2) ever
// write the same line.
constexpr int SQ_TH = 16;

struct SqParams {
  double* S;        // sample, column c at S + c * LMAX
  int l;
  int64_t nJ;
  int bJ;
  int* piv;
  int* info;
  int info_base;
  double* cand;     // 2 buffers of SQ_T columns of SQ_LCAP rows; column of slot i at [buf][i * LMAX]
  int* cand_idx;    // 2 buffers of 2 x SQ_T: logical position (-1: empty slot), physical column
  double* theta;    // 2 buffers of SQ_MAXP entries, SQ_TH words apart
  unsigned* flags;  // [0]: arrival counter (zeroed by the caller)
  int* err;
  int P;
  int K;
};

template <int LMAX>
struct SqLds {
  // the scan's row pairs (rows 8 i + 2 q, 8 i + 2 q + 1) and the steps'
  // 16-byte reads of a quad lane's LMAX / 4 rows need LMAX to be a multiple of 8
  static_assert(LMAX % 8 == 0 && LMAX <= SQ_LCAP, "sample register tile");
  double vlog[SQ_BMAX * LMAX];        // reflector of step t (zero above row t, one at row t)
  // Quad layout (row 4 i + q at [q * LMAX / 4 + i]): during a round, the
  // reflectors of its steps; at its end they are copied to vlog and their
  // rows take the final sample columns of the round's pivots.
  double vq[SQ_BMAX * LMAX];
  double taus[SQ_BMAX];
  double kv[SQ_T];                    // ranking keys sorted per wave: trailing norm, position
  int kp[SQ_T];
  int rk[SQ_T];                       // rank of each lane's column
  int plog[SQ_BMAX];                  // position of the pivot chosen at step t
  int wonstep[SQ_T];                  // step at which candidate slot i became a pivot (-1: none)
  double betas[SQ_BMAX];              // beta of the pivot of step t
  int pphys[SQ_BMAX];                 // its physical column
  double rv[2][SQ_T / WAVE];          // per-wave argmax
  int rp[2][SQ_T / WAVE];
  double theta;
  int bad;
  int nvalid;
};

__device__ __forceinline__ double ranked(double nu) { return (nu != nu) ? -1.0 : nu; }

// 1 / a for a > 0: hardware reciprocal estimate and two Newton steps
// (within an ulp or so of the rounded quotient).
__device__ __forceinline__ double rcp_nr(double a) {
  double r = __builtin_amdgcn_rcp(a);
  r = fma(r, fma(-a, r, 1.0), r);
  r = fma(r, fma(-a, r, 1.0), r);
  return r;
}

__device__ __forceinline__ bool better(double v1, int p1, double v2, int p2) {
  return (v1 > v2) || (v1 == v2 && p1 < p2);
}

// The same test without short-circuit evaluation (both operands loaded and
// compared unconditionally, no branch): 0 or 1.
__device__ __forceinline__ int beats(double v1, int p1, double v2, int p2) {
  return (int)(v1 > v2) | ((int)(v1 == v2) & (int)(p1 < p2));
}

// Values every thread reads from the same LDS word are uniform, but the
// compiler cannot know it; taking them from the first lane lets it keep the
// step index and everything derived from it in scalar registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Householder reflector of a column whose pivot-row entry is alpha and whose
// rows below have squared norm sig (dlarfg normalisation: beta = -sign(alpha)
// ||x||, tau = (beta - alpha) / beta, v = x / (alpha - beta) below the pivot
// row; an exactly zero tail gives tau = 0 and beta = alpha).  With
// q = |alpha| + ||x|| (no cancellation), tau = q / ||x|| and
// 1 / (alpha - beta) = sign(alpha) / q: two independent reciprocals.
__device__ __forceinline__ void sq_reflector(double alpha, double sig, double& tau, double& beta, double& scal) {
  const double nrm = sqrt(fma(alpha, alpha, sig));
  const double sg = (alpha >= 0.0) ? 1.0 : -1.0;
  const double q = fabs(alpha) + nrm;
  const bool zero = !(sig != 0.0);
  tau = zero ? 0.0 : q * rcp_nr(nrm);
  beta = zero ? alpha : -sg * nrm;
  scal = zero ? 0.0 : sg * rcp_nr(q);
}

// Maximum over the wave by DPP moves within rows of 16 lanes, then the four
// row results read as scalars.
__device__ __forceinline__ double dpp_pull(double v, int ctrl_id) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  switch (ctrl_id) {
    case 0:  // quad_perm [1, 0, 3, 2]
      lo = __builtin_amdgcn_update_dpp(lo, lo, 0xB1, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(hi, hi, 0xB1, 0xF, 0xF, false);
      break;
    case 1:  // quad_perm [2, 3, 0, 1]
      lo = __builtin_amdgcn_update_dpp(lo, lo, 0x4E, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(hi, hi, 0x4E, 0xF, 0xF, false);
      break;
    case 2:  // row_half_mirror
      lo = __builtin_amdgcn_update_dpp(lo, lo, 0x141, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(hi, hi, 0x141, 0xF, 0xF, false);
      break;
    default:  // row_mirror
      lo = __builtin_amdgcn_update_dpp(lo, lo, 0x140, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(hi, hi, 0x140, 0xF, 0xF, false);
      break;
  }
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Exchanges across rows of 16 lanes and across the wave halves (gfx950
// v_permlane16_swap / v_permlane32_swap): with both operands the same value,
// the two results hold the value of the lane itself and of its partner
// row (half), in some order.
__device__ __forceinline__ double xrow16_max(double v) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
  return fmax(__hiloint2double(hi[0], lo[0]), __hiloint2double(hi[1], lo[1]));
}
__device__ __forceinline__ double xrow32_max(double v) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
  return fmax(__hiloint2double(hi[0], lo[0]), __hiloint2double(hi[1], lo[1]));
}
__device__ __forceinline__ int dpp_pull_i(int v, int ctrl_id) {
  switch (ctrl_id) {
    case 0: return __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);
    case 1: return __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);
    case 2: return __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false);
    default: return __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false);
  }
}

// Maximum over the wave: DPP within rows of 16 lanes, then row and half
// exchanges.  Every lane gets the result.
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_pull(v, 0));
  v = fmax(v, dpp_pull(v, 1));
  v = fmax(v, dpp_pull(v, 2));
  v = fmax(v, dpp_pull(v, 3));
  v = xrow16_max(v);
  return xrow32_max(v);
}

__device__ __forceinline__ int wave_min_i(int v) {
  v = min(v, dpp_pull_i(v, 0));
  v = min(v, dpp_pull_i(v, 1));
  v = min(v, dpp_pull_i(v, 2));
  v = min(v, dpp_pull_i(v, 3));
  {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = min((int)r[0], (int)r[1]);
  }
  {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    v = min((int)r[0], (int)r[1]);
  }
  return v;
}

// Wave-level (value, position) argmax: the largest value, ties to the lowest
// position.  Values must not be NaN; every lane of the wave active.  Uniform
// result.  The position is read from the first lane at the maximum; only
// when lanes at the maximum disagree on it (equal values at different
// positions) does a second reduction take the lowest.
__device__ __forceinline__ void wave_argmax_vp(double v, int p, double& bv, int& bp) {
  bv = uni(wave_max(v));
  const bool top = v == bv;
  const int first = (int)__builtin_ctzll(__ballot(top));
  const int p0 = __builtin_amdgcn_readlane(p, first);
  if (__ballot(top && p != p0) == 0ull) bp = p0;
  else bp = uni(wave_min_i(top ? p : INT_MAX));
}

// Quad lanes (tid & ~3 .. tid | 3) exchange values with DPP quad permutes.
template <int CTRL>
__device__ __forceinline__ double qperm(double v) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// Sum over the quad; every lane gets the same bits (the two additions are
// the same pairs in either order).
__device__ __forceinline__ double quad_sum(double v) {
  v += qperm<0xB1>(v);
  return v + qperm<0x4E>(v);
}
// The value of quad lane qs (uniform) in every lane of the quad.
__device__ __forceinline__ double quad_bcast(double v, int qs) {
  switch (qs) {
    case 0: return qperm<0x00>(v);
    case 1: return qperm<0x55>(v);
    case 2: return qperm<0xAA>(v);
    default: return qperm<0xFF>(v);
  }
}

// Row-quad helpers: x[c][i] is row 4 i + q (q = quad lane) of column c.

// e[c] = x[c][ri] for a uniform ri (binary branch tree on ri).
template <int RQ, int LO, int HI>
__device__ __forceinline__ void sq_pick_rows(const double (&x)[4][RQ], int ri, double (&e)[4]) {
  if constexpr (HI - LO == 1) {
    double e0 = x[0][LO], e1 = x[1][LO], e2 = x[2][LO], e3 = x[3][LO];
    // the leaf's values pass through an empty asm statement, so the leaves
    // cannot be merged into one access with a computed register index
    asm volatile("; row pick" : "+v"(e0), "+v"(e1), "+v"(e2), "+v"(e3));
    e[0] = e0;
    e[1] = e1;
    e[2] = e2;
    e[3] = e3;
  } else {
    constexpr int MID = (LO + HI) / 2;
    if (ri < MID) sq_pick_rows<RQ, LO, MID>(x, ri, e);
    else sq_pick_rows<RQ, MID, HI>(x, ri, e);
  }
}

template <int RQ>
__device__ __forceinline__ void sq_copy_col(const double (&xc)[RQ], double (&y)[RQ]) {
#pragma unroll
  for (int i = 0; i < RQ; ++i) y[i] = xc[i];
}

// Sum over the quad of y[i]^2 for rows 4 i + q >= f (uniform f): every row
// index i > f / 4 counts, i == f / 4 counts in lanes q >= f % 4.
template <int RQ>
__device__ __forceinline__ double sq_tail2_one(const double (&y)[RQ], int q, int f) {
  const int fi = f >> 2, fq = f & 3;
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int i = 0; i < RQ; ++i) {
    const double m = (i > fi) ? 1.0 : ((i == fi && q >= fq) ? 1.0 : 0.0);
    acc[i & 1] = fma(y[i] * m, y[i], acc[i & 1]);
  }
  return quad_sum(acc[0] + acc[1]);
}

// The same for the four columns.
template <int RQ>
__device__ __forceinline__ void sq_tail2(const double (&x)[4][RQ], int q, int f, double (&out)[4]) {
  const int fi = f >> 2, fq = f & 3;
  double acc[4][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
  for (int i = 0; i < RQ; ++i) {
    const double m = (i > fi) ? 1.0 : ((i == fi && q >= fq) ? 1.0 : 0.0);
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c][i & 1] = fma(x[c][i] * m, x[c][i], acc[c][i & 1]);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) out[c] = quad_sum(acc[c][0] + acc[c][1]);
}

// Integer value of quad lane qs (a constant) in every lane of the quad.
template <int QS>
__device__ __forceinline__ int quad_bcast_i(int v) {
  return __builtin_amdgcn_update_dpp(v, v, QS * 0x55, 0xF, 0xF, false);
}

// One pass over this workgroup's slab of SQ_T columns: apply the reflectors
// of steps [a0, t0), write the columns back (on the last pass, a column
// whose position changed goes to its final position), and, if `select`,
// publish the K best columns by trailing norm over rows >= t0 as candidates
// together with theta = the best norm left out.  The sample has LMAX rows
// (rows past l are zero and stay zero).
//
// Four lanes (a quad) share four slab columns, in row pairs: quad lane q
// holds rows 8 i + 2 q and 8 i + 2 q + 1 of all four (x[c][2 i + h]), so the
// quad reads each column with whole 64-byte segments and each reflector
// value a lane reads from LDS serves four columns; the partial sums are
// combined by DPP quad permutes.  Column c of quad g is slab column 4 g + c,
// the column whose bookkeeping (logical position, selected flag) lane
// 4 g + c holds.
template <int LMAX>
__device__ void sq_scan(const SqParams& a, SqLds<LMAX>& L, int me, int a0, int t0, bool select, int buf,
                        int pos_s, bool sel_s) {
  constexpr int RQ = LMAX / 4, NI = LMAX / 8;
  const int tid = threadIdx.x, q = tid & 3;
  int posc[4];
  int64_t colc[4];
  bool minec[4];
  {
    const int sel = sel_s ? 1 : 0;
    const int p4[4] = {quad_bcast_i<0>(pos_s), quad_bcast_i<1>(pos_s), quad_bcast_i<2>(pos_s),
                       quad_bcast_i<3>(pos_s)};
    const int s4[4] = {quad_bcast_i<0>(sel), quad_bcast_i<1>(sel), quad_bcast_i<2>(sel), quad_bcast_i<3>(sel)};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      posc[c] = p4[c];
      colc[c] = (int64_t)me * SQ_T + (tid & ~3) + c;
      minec[c] = colc[c] < a.nJ && s4[c] == 0;
    }
  }
  double x[4][RQ];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double2* col = reinterpret_cast<const double2*>(a.S + colc[c] * LMAX + 2 * q);
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const double2 w = minec[c] ? col[4 * i] : make_double2(0.0, 0.0);
      x[c][2 * i] = w.x;
      x[c][2 * i + 1] = w.y;
    }
  }
  for (int s = a0; s < t0; ++s) {
    const double tau = uni(L.taus[s]);
    const double2* vp = reinterpret_cast<const double2*>(L.vlog + s * LMAX + 2 * q);
    double2 v[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) v[i] = vp[4 * i];
    double acc[4][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        acc[c][0] = fma(x[c][2 * i], v[i].x, acc[c][0]);
        acc[c][1] = fma(x[c][2 * i + 1], v[i].y, acc[c][1]);
      }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double d = tau * quad_sum(acc[c][0] + acc[c][1]);
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        x[c][2 * i] = fma(-d, v[i].x, x[c][2 * i]);
        x[c][2 * i + 1] = fma(-d, v[i].y, x[c][2 * i + 1]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const bool move = !select && posc[c] != colc[c];
    if (minec[c] && (move || t0 > a0)) {
      double2* col = reinterpret_cast<double2*>(a.S + (move ? (int64_t)posc[c] : colc[c]) * LMAX + 2 * q);
#pragma unroll
      for (int i = 0; i < NI; ++i) col[4 * i] = make_double2(x[c][2 * i], x[c][2 * i + 1]);
    }
  }
  if (!select) return;
  // trailing squared norms (rows >= t0) of the quad's columns; lane q ranks column q
  double nu = 0.0;
  {
    double acc[4][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const double m0 = (8 * i + 2 * q >= t0) ? 1.0 : 0.0;
      const double m1 = (8 * i + 2 * q + 1 >= t0) ? 1.0 : 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        acc[c][0] = fma(x[c][2 * i] * m0, x[c][2 * i], acc[c][0]);
        acc[c][1] = fma(x[c][2 * i + 1] * m1, x[c][2 * i + 1], acc[c][1]);
      }
    }
    double n4[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) n4[c] = quad_sum(acc[c][0] + acc[c][1]);
    nu = (q == 0) ? n4[0] : (q == 1) ? n4[1] : (q == 2) ? n4[2] : n4[3];
  }
  const bool mine = (q == 0) ? minec[0] : (q == 1) ? minec[1] : (q == 2) ? minec[2] : minec[3];
  const double kv = mine ? ranked(nu) : -INFINITY;
  const int kp = mine ? pos_s : INT_MAX;
  if (tid == 0) { L.bad = 0; L.nvalid = SQ_T; }
  int rank = SQ_T;
  {
  // rank of this column among the slab: the number of columns that beat it
  // (larger trailing norm, ties to the lower position); the K best become
  // candidates and the one of rank K gives theta.  Each wave sorts its 64
  // keys (bitonic network over lanes), then an entry's rank is its index in
  // its wave plus, for each other wave, the length of that wave's sorted
  // prefix that beats it (binary search in LDS).
  {
    const int lane = tid & (WAVE - 1), w = tid / WAVE;
    double sv = kv;
    int sp = kp, sl = tid;
    // in a best-first run the lower lane of a pair keeps the better key, in
    // a best-last run the worse one
    auto stage = [&](auto size_c, auto stride_c) __attribute__((always_inline)) {
      constexpr int SIZE = decltype(size_c)::value, STRIDE = decltype(stride_c)::value;
      const double ov = xchg_d<STRIDE>(sv, lane);
      const int op = xchg_i<STRIDE>(sp, lane);
      const int ol = xchg_i<STRIDE>(sl, lane);
      const bool lower = (lane & STRIDE) == 0;
      const bool best_first = (lane & SIZE) == 0;
      const bool ob = beats(ov, op, sv, sp) != 0;
      const bool take = (lower == best_first) ? ob : (!ob && (ov != sv || op != sp));
      sv = take ? ov : sv;
      sp = take ? op : sp;
      sl = take ? ol : sl;
    };
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I4 = std::integral_constant<int, 4>;
    using I8 = std::integral_constant<int, 8>;
    using I16 = std::integral_constant<int, 16>;
    using I32 = std::integral_constant<int, 32>;
    using I64 = std::integral_constant<int, 64>;
    stage(I2{}, I1{});
    stage(I4{}, I2{}); stage(I4{}, I1{});
    stage(I8{}, I4{}); stage(I8{}, I2{}); stage(I8{}, I1{});
    stage(I16{}, I8{}); stage(I16{}, I4{}); stage(I16{}, I2{}); stage(I16{}, I1{});
    stage(I32{}, I16{}); stage(I32{}, I8{}); stage(I32{}, I4{}); stage(I32{}, I2{}); stage(I32{}, I1{});
    stage(I64{}, I32{}); stage(I64{}, I16{}); stage(I64{}, I8{}); stage(I64{}, I4{}); stage(I64{}, I2{});
    stage(I64{}, I1{});
    L.kv[tid] = sv;
    L.kp[tid] = sp;
    __syncthreads();
    if (mine && !(nu <= DBL_MAX)) L.bad = 1;
    int rk = lane;
#pragma unroll
    for (int w2 = 0; w2 < SQ_T / WAVE; ++w2) {
      if (w2 == w) continue;
      // number of entries of wave w2 that beat (sv, sp): first index whose key does not
      int lo = 0, hi = WAVE;
#pragma unroll
      for (int it = 0; it < 7; ++it) {
        if (lo < hi) {
          const int mid = (lo + hi) >> 1;
          const int qi = w2 * WAVE + mid;
          if (beats(L.kv[qi], L.kp[qi], sv, sp)) lo = mid + 1;
          else hi = mid;
        }
      }
      rk += lo;
    }
    L.rk[sl] = rk;
    if (sp == INT_MAX) atomicMin(&L.nvalid, rk);  // empty entries rank after all valid ones
  }
  __syncthreads();
  rank = L.rk[tid];
  }
  __syncthreads();
  if (L.bad && tid == 0 && a.info) atomicCAS(a.info, 0, a.info_base + t0 + 1);
  const int nvalid = L.nvalid;  // min over empty entries of their rank, or SQ_T
  double* cb = a.cand + (size_t)buf * SQ_LCAP * SQ_T;
  int* ib = a.cand_idx + (size_t)buf * 2 * SQ_T;
  const int rk4[4] = {quad_bcast_i<0>(rank), quad_bcast_i<1>(rank), quad_bcast_i<2>(rank), quad_bcast_i<3>(rank)};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (minec[c] && rk4[c] < a.K) {
      // candidate columns are stored in the steps' quad layout: row r at
      // (r mod 4) RQ + r / 4; this lane holds rows r = 8 i + 2 q + h
      const int slot = me * a.K + rk4[c];
      double* col = cb + (size_t)slot * LMAX;
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int r = 8 * i + 2 * q + h;
          col[(r & 3) * RQ + (r >> 2)] = x[c][2 * i + h];
        }
      if (q == c) {
        ib[slot] = posc[c];
        ib[SQ_T + slot] = (int)colc[c];
      }
    }
  }
  if (tid < a.K && tid >= nvalid) ib[me * a.K + tid] = -1;
  if (mine && rank == a.K) a.theta[((size_t)buf * SQ_MAXP + me) * SQ_TH] = kv;
  if (tid == 0 && a.K >= nvalid) a.theta[((size_t)buf * SQ_MAXP + me) * SQ_TH] = -INFINITY;
}

// Arrival barrier over the P workgroups: every workgroup adds one to the
// counter after its candidates are visible device-wide and waits until the
// counter reaches round * P.  Bounded: on timeout the error word is set.
__device__ bool sq_barrier(const SqParams& a, unsigned round) {
  __shared__ int s_bad;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x < WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (threadIdx.x == 0) {
      __hip_atomic_fetch_add(&a.flags[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned target = round * (unsigned)a.P;
      long spins = 0;
      int bad = 0;
      while (__hip_atomic_load(&a.flags[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++spins > SPIN_LIMIT) { bad = 1; atomicExch(a.err, 1); break; }
        __builtin_amdgcn_s_sleep(1);
      }
      s_bad = bad;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(s_bad) == 0;
}

// Sample QRCP (Alg. 1 for bJ steps, Alg. 4) by certified candidate rounds.
// Each round every workgroup updates its slab of 256 columns and proposes its
// K best columns; all workgroups then run the same greedy steps on the
// gathered candidates (so they all hold the round's reflectors without a
// second exchange) for as long as the winner provably beats every column
// left out: its trailing norm must exceed theta, the largest left-out norm at
// the start of the round, which bounds the left-out norms later in the round
// (they only shrink) -- with a relative margin of 1e-10 for rounding.  The
// steps are the sequential ones of the algorithm: swap of positions t and p,
// Householder reflector of the pivot column (LAPACK normalisation), update of
// the remaining candidates.  Within a step, each wave's best candidate forms
// its reflector and stores it before the one barrier of the step, so the
// winner's reflector is ready as soon as the winner is known.  Columns are
// never moved during the rounds; each thread tracks the logical position of
// its slab column.
template <int LMAX>
__device__ __forceinline__ void sample_qrcp_body(const SqParams& a, const int me) {
  extern __shared__ __align__(16) double smem[];
  SqLds<LMAX>& L = *reinterpret_cast<SqLds<LMAX>*>(smem);
  const int tid = threadIdx.x, wv_id = tid / WAVE;
  // the sequential pivot steps are the critical path: ahead of the waves of
  // a trailing update that may share the CU
  __builtin_amdgcn_s_setprio(3);
  if (earlier_failure(a.err)) return;
  const int64_t c_s = (int64_t)me * SQ_T + tid;
  int pos_s = (int)c_s;   // logical position of this thread's slab column
  bool sel_s = false;     // selected as a pivot
  int a0 = 0, t0 = 0;
  __syncthreads();
  for (unsigned round = 1;; ++round) {
    const bool select = t0 < a.bJ;
    const int buf = round & 1;
    sq_scan<LMAX>(a, L, me, a0, t0, select, buf, pos_s, sel_s);
    if (!select) break;
    if (!sq_barrier(a, round)) return;

    // gather the candidates (identical in every workgroup).  Four lanes (a
    // quad) share four candidate columns: quad lane q holds rows 4 i + q,
    // i < RQ, of all four, so each reflector value a lane reads from LDS
    // serves four columns, and the quad's partial sums are combined by DPP.
    constexpr int RQ = LMAX / 4;
    const int C = a.P * a.K;
    const double* cb = a.cand + (size_t)buf * SQ_LCAP * SQ_T;
    const int* ib = a.cand_idx + (size_t)buf * 2 * SQ_T;
    const int q = tid & 3;
    int pos[4], phys[4];
    unsigned act = 0;  // bit c: column c of the quad is still a candidate
    double x[4][RQ];
    // The left-out norms, the slot indices and the slot columns are all read
    // before any of them is used (one memory round trip): a slot's column is
    // read whether or not the slot holds a candidate (the buffer has SQ_T
    // slots) and zeroed afterwards when it does not.
    double thv[SQ_MAXP / WAVE];
    if (tid < WAVE) {
#pragma unroll
      for (int k = 0; k < SQ_MAXP / WAVE; ++k) {
        const int qq = tid + k * WAVE;
        thv[k] = (qq < a.P) ? a.theta[((size_t)buf * SQ_MAXP + qq) * SQ_TH] : -INFINITY;
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int sl = (tid & ~3) + c;
      const bool in = sl < C;
      pos[c] = in ? ib[sl] : -1;
      phys[c] = in ? ib[SQ_T + sl] : -1;
      const double2* col = reinterpret_cast<const double2*>(cb + (size_t)sl * LMAX + q * RQ);
#pragma unroll
      for (int i = 0; i < RQ / 2; ++i) {
        const double2 w = in ? col[i] : make_double2(0.0, 0.0);
        x[c][2 * i] = w.x;
        x[c][2 * i + 1] = w.y;
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const bool on = pos[c] >= 0;
      if (on) act |= 1u << c;
      else pos[c] = INT_MAX;
#pragma unroll
      for (int i = 0; i < RQ; ++i) x[c][i] = on ? x[c][i] : 0.0;
    }
    L.wonstep[tid] = -1;
    if (tid < WAVE) {
      double th = thv[0];
#pragma unroll
      for (int k = 1; k < SQ_MAXP / WAVE; ++k) th = fmax(th, thv[k]);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) th = fmax(th, __shfl_xor(th, off, WAVE));
      if (tid == 0) L.theta = th;
    }
    __syncthreads();
    const double theta = uni(L.theta);
    const double bound = (theta > 0.0) ? theta * (1.0 + 1e-10) : theta;

    int t = t0;
    // Per column (the same in the quad's four lanes): alpha = x[t] and the
    // trailing squared norm nu of rows >= t.  nu is downdated after each
    // step (the reflector keeps the norm of rows >= t, so rows > t keep it
    // minus the new row-t entry squared) and recomputed once it falls below
    // a tenth of its last exact value, which bounds its relative error by
    // about 64 eps * 10; the pivot's reflector always uses the exact norm
    // of its column.
    double alpha[4], nu[4], nu_ref[4];
    // eg[c] = x[c][gi]: the rows 4 gi .. 4 gi + 3 of each column across the
    // quad, the group that holds the next pivot row.  It gets the same update
    // as x, so it is picked out of x (a branch tree) only when the pivot row
    // enters a new group, once in four steps.
    double eg[4];
    int gi = t >> 2;
    {
      sq_pick_rows<RQ, 0, RQ>(x, gi, eg);
#pragma unroll
      for (int c = 0; c < 4; ++c) alpha[c] = quad_bcast(eg[c], t & 3);
      sq_tail2<RQ>(x, q, t, nu);
#pragma unroll
      for (int c = 0; c < 4; ++c) nu_ref[c] = nu[c];
    }
    while (t < a.bJ) {
      t = uni(t);
      const int par = t & 1;
      // the quad's best column (the same in its four lanes)
      double bv = -INFINITY;
      int bp = INT_MAX, bc = 0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const bool on = (act >> c) & 1u;
        const double val = on ? ranked(nu[c]) : -INFINITY;
        const int pc = on ? pos[c] : INT_MAX;
        if (beats(val, pc, bv, bp)) { bv = val; bp = pc; bc = c; }
      }
      double vwave;
      int pwave;
      wave_argmax_vp(bv, bp, vwave, pwave);
      if ((tid & (WAVE - 1)) == 0) { L.rv[par][wv_id] = vwave; L.rp[par][wv_id] = pwave; }
      __syncthreads();
      // the best of the four waves' results: a two-level tree (beats is a
      // strict order, so the result is the one a sequential scan gives)
      static_assert(SQ_T / WAVE == 4, "four waves per workgroup");
      double v;
      int p;
      {
        const double v0 = uni(L.rv[par][0]), v1 = uni(L.rv[par][1]);
        const double v2 = uni(L.rv[par][2]), v3 = uni(L.rv[par][3]);
        const int p0 = uni(L.rp[par][0]), p1 = uni(L.rp[par][1]);
        const int p2 = uni(L.rp[par][2]), p3 = uni(L.rp[par][3]);
        const bool b10 = beats(v1, p1, v0, p0), b32 = beats(v3, p3, v2, p2);
        const double va = b10 ? v1 : v0, vb = b32 ? v3 : v2;
        const int pa = b10 ? p1 : p0, pb = b32 ? p3 : p2;
        const bool bba = beats(vb, pb, va, pa);
        v = bba ? vb : va;
        p = bba ? pb : pa;
      }
      if ((t > t0 && !(v > bound)) || p == INT_MAX) break;
      double* vt = L.vq + t * LMAX;
      if (pwave == p) {
        // this wave holds the winner: column cw of one quad becomes pivot t.
        // Its exact tail norm, its reflector (dlarfg normalisation) and the
        // normalised reflector in quad layout (zero above row t, one at row
        // t, the column below times 1 / (alpha - beta)) are formed by the
        // whole wave with the winner's column index made uniform; only the
        // winner's quad stores.
        const bool is_w = bp == p;
        const unsigned long long wm = __ballot(is_w);
        const int cw = __builtin_amdgcn_readlane(bc, (int)__builtin_ctzll(wm));
        const int ti = t >> 2, tq = t & 3;
        auto win = [&](const double (&xc)[RQ], double al) __attribute__((always_inline)) {
          const double sg2 = sq_tail2_one<RQ>(xc, q, t + 1);
          double r_tau, r_beta, r_scal;
          sq_reflector(al, sg2, r_tau, r_beta, r_scal);
          if (is_w) {
            double2* dst = reinterpret_cast<double2*>(vt + q * RQ);
#pragma unroll
            for (int i2 = 0; i2 < RQ / 2; ++i2) {
              double e[2];
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                const int i = 2 * i2 + h;
                const double sv = xc[i] * r_scal;
                const double bnd = (q < tq) ? 0.0 : ((q == tq) ? 1.0 : sv);
                e[h] = (i < ti) ? 0.0 : ((i > ti) ? sv : bnd);
              }
              dst[i2] = make_double2(e[0], e[1]);
            }
            if (q == 0) {
              L.taus[t] = r_tau;
              L.betas[t] = r_beta;
              L.plog[t] = p;
            }
          }
        };
        // one copy of the code per column (the empty asm statements keep
        // the compiler from merging them into an indexed access of x)
        if (cw == 0) {
          asm volatile("; winner column 0");
          win(x[0], alpha[0]);
        } else if (cw == 1) {
          asm volatile("; winner column 1");
          win(x[1], alpha[1]);
        } else if (cw == 2) {
          asm volatile("; winner column 2");
          win(x[2], alpha[2]);
        } else {
          asm volatile("; winner column 3");
          win(x[3], alpha[3]);
        }
        if (is_w) {
          int ph = phys[0];
#pragma unroll
          for (int c = 1; c < 4; ++c)
            if (cw == c) ph = phys[c];
          if (q == 0) {
            L.pphys[t] = ph;
            L.wonstep[(tid & ~3) + cw] = t;
          }
          act &= ~(1u << cw);
        }
      }
      // sequential swap: the column at position t moves to p
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (((act >> c) & 1u) && pos[c] == t) pos[c] = p;
      __syncthreads();
      {
        const double tau = uni(L.taus[t]);
        {
          const int gn = (t + 1) >> 2;
          if (gn != gi) {  // row t + 1 starts a new group (picked before this step's update)
            gi = gn < RQ ? gn : RQ - 1;
            sq_pick_rows<RQ, 0, RQ>(x, gi, eg);
          }
        }
        const double vg = vt[q * RQ + gi];  // this lane's reflector entry in that group
        double vr[RQ];
        const double2* src = reinterpret_cast<const double2*>(vt + q * RQ);
#pragma unroll
        for (int i2 = 0; i2 < RQ / 2; ++i2) {
          const double2 w = src[i2];
          vr[2 * i2] = w.x;
          vr[2 * i2 + 1] = w.y;
        }
        double dp[4][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
        for (int i = 0; i < RQ; ++i)
#pragma unroll
          for (int c = 0; c < 4; ++c) dp[c][i & 1] = fma(vr[i], x[c][i], dp[c][i & 1]);
        double d[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double s4 = quad_sum(dp[c][0] + dp[c][1]);
          d[c] = ((act >> c) & 1u) ? tau * s4 : 0.0;
        }
#pragma unroll
        for (int i = 0; i < RQ; ++i)
#pragma unroll
          for (int c = 0; c < 4; ++c) x[c][i] = fma(-d[c], vr[i], x[c][i]);
#pragma unroll
        for (int c = 0; c < 4; ++c) eg[c] = fma(-d[c], vg, eg[c]);
        // downdate with the new row-t entries alpha - d (v[t] = 1)
        bool redo = false;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double xt = alpha[c] - d[c];
          nu[c] -= xt * xt;
          redo = redo || (((act >> c) & 1u) && !(nu[c] >= 0.1 * nu_ref[c]));
        }
        if (__ballot(redo)) {
          double ex[4];
          sq_tail2<RQ>(x, q, t + 1, ex);
#pragma unroll
          for (int c = 0; c < 4; ++c)
            if (!(nu[c] >= 0.1 * nu_ref[c])) { nu[c] = ex[c]; nu_ref[c] = ex[c]; }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) alpha[c] = quad_bcast(eg[c], (t + 1) & 3);
      }
      ++t;
    }
    const int tn = t;
    __syncthreads();
    for (int s = t0; s < tn; ++s) {
      if (c_s == L.pphys[s]) sel_s = true;
      else if (pos_s == s) pos_s = L.plog[s];
    }
    if (me == 0 && tid >= t0 && tid < tn) a.piv[tid] = L.plog[tid];
    // the round's reflectors in row order, for the later scans
    for (int e = tid; e < (tn - t0) * LMAX; e += SQ_T) {
      const int st = t0 + e / LMAX, r = e % LMAX;
      L.vlog[st * LMAX + r] = L.vq[st * LMAX + (r & 3) * (LMAX / 4) + (r >> 2)];
    }
    __syncthreads();
    // S columns of this round's pivots (quad layout): rows above the pivot
    // row as they were when it was chosen, beta on it, zeros below
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int wt = L.wonstep[(tid & ~3) + c];
      if (wt >= 0) {
        const double bw = L.betas[wt];
        double2* st = reinterpret_cast<double2*>(L.vq + wt * LMAX + q * RQ);
#pragma unroll
        for (int i2 = 0; i2 < RQ / 2; ++i2) {
          double e[2];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int r = 4 * (2 * i2 + h) + q;
            e[h] = (r < wt) ? x[c][2 * i2 + h] : ((r == wt) ? bw : 0.0);
          }
          st[i2] = make_double2(e[0], e[1]);
        }
      }
    }

    if (tn == t0) {  // no candidate left although steps remain: cannot happen for bJ <= nJ
      if (tid == 0) atomicExch(a.err, 1);
      return;
    }
    a0 = uni(t0);
    t0 = uni(tn);
  }
  // the pivot columns of the sample go to positions 0..bJ-1 (workgroup 0
  // owns those physical columns, and its own reads of them are done)
  if (me == 0) {
    __syncthreads();
    for (int e = tid; e < a.bJ * LMAX; e += SQ_T) {
      const int j = e / LMAX, r = e % LMAX;
      a.S[e] = L.vq[j * LMAX + (r & 3) * (LMAX / 4) + (r >> 2)];
    }
  }
}

template <int LMAX>
__global__ void __launch_bounds__(SQ_T) sample_qrcp_kernel(SqParams a) {
  sample_qrcp_body<LMAX>(a, blockIdx.x);
}

// The trailing update C -= A B (M x N, reduction K = the block size) that
// runs in the same launch as the next block's sample QRCP: workgroups P..
// of the grid walk its 128 x 64 tiles, the first P run the sample QRCP.  One
// launch on one stream orders both before the next block's swaps with no
// event between streams, and the tiles compute exactly what the ordinary
// trailing-update launch computes.
struct UpdParams {
  int64_t M, N, K;
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
  int64_t tiles_x, tiles;
};

template <int LMAX, typename Acc>
__global__ void __launch_bounds__(SQ_T) sample_qrcp_update_kernel(SqParams a, UpdParams u) {
  if ((int)blockIdx.x < a.P) {
    sample_qrcp_body<LMAX>(a, blockIdx.x);
    return;
  }
  const int64_t wg = (int64_t)blockIdx.x - a.P, nwg = (int64_t)gridDim.x - a.P;
  for (int64_t t = wg; t < u.tiles; t += nwg) {
    // four waves of 32 x 64 (each its own rows of the tile; measured a
    // little faster here than 2 x 2 waves of 64 x 32, with the same
    // products in the same order)
    gemm_tile<128, 64, 16, 4, 1, false, false, double, double, Acc, false>(
        u.M, u.N, u.K, -1.0, u.A, u.lda, u.B, u.ldb, 1.0, u.C, u.ldc, u.K, 0, nullptr, 0, 0, t % u.tiles_x,
        t / u.tiles_x, 0);
    __syncthreads();  // the next tile's LDS stores after every wave's last reads
  }
}

// launch_sq_update's answer when the sample QRCP's workgroups leave no
// place for the update's (not an error code: every error is negative or
// at least RQ_ERR_HIP_BASE)
constexpr int SQ_NO_ROOM = 1;

template <int LMAX, typename Acc>
int launch_sq_update(hipStream_t s, SqParams& a, const BesideUpdate& b) {
  constexpr size_t lds = std::max(sizeof(SqLds<LMAX>), gemm_lds_bytes<128, 64, 16, Acc>());
  static_assert(lds <= 160 * 1024, "LDS budget");
  auto kern = sample_qrcp_update_kernel<LMAX, Acc>;
  static int resident = 0;
  if (!resident) {
    RQ_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int occ = 0, dev = 0, cus = 0;
    RQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, SQ_T, lds));
    RQ_HIP(hipGetDevice(&dev));
    RQ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    resident = occ * cus;
  }
  UpdParams u;
  u.M = b.M; u.N = b.N; u.K = b.K; u.A = b.A; u.lda = b.lda; u.B = b.B; u.ldb = b.ldb; u.C = b.C; u.ldc = b.ldc;
  u.tiles_x = (b.N + 63) / 64;
  u.tiles = u.tiles_x * ((b.M + 127) / 128);
  // every workgroup of the grid must be resident at once (the sample QRCP's
  // wait on each other; the update's are dispatched after them): the update
  // gets at most the places the sample QRCP leaves, and none left means no
  // room (the caller then runs the two one after the other)
  const int64_t room = (int64_t)resident - a.P;
  if (room < 1) return SQ_NO_ROOM;
  const int64_t wgs = std::max<int64_t>(1, std::min<int64_t>({b.wgs, u.tiles, room}));
  hipLaunchKernelGGL(kern, dim3((unsigned)(a.P + wgs)), dim3(SQ_T), lds, s, a, u);
  RQ_HIP(hipGetLastError());
  return 0;
}

template <int LMAX>
int launch_sq_alone(hipStream_t s, SqParams& a);

template <int LMAX>
int launch_sq(hipStream_t s, SqParams& a, const BesideUpdate* upd) {
  const int64_t P = (a.nJ + SQ_T - 1) / SQ_T;
  if (P > SQ_MAXP) return -4;  // n too large for this kernel
  a.P = (int)P;
  // K even where it can be: with 8 B per row and LMAX = 8 x (odd) (40, 72),
  // an even K makes each workgroup's K candidate columns whole 128-byte
  // lines, so two workgroups never write one line of the candidate buffer
  // (above 128 workgroups K is 1)
  a.K = std::max(1, (SQ_T / a.P) & ~1);
  if (upd && upd->M > 0 && upd->N > 0 && upd->K > 0) {
    const int rc = upd->f32 ? launch_sq_update<LMAX, float>(s, a, *upd) : launch_sq_update<LMAX, double>(s, a, *upd);
    if (rc != SQ_NO_ROOM) return rc;
    // the sample QRCP fills every place on the device: the update follows it
    // as an ordinary launch (the same products, so the same bits)
    const int rs = launch_sq_alone<LMAX>(s, a);
    if (rs) return rs;
    const BesideUpdate& b = *upd;
    return b.f32 ? launch_gemm_f32(s, false, false, b.M, b.N, b.K, -1.0, b.A, b.lda, b.B, b.ldb, 1.0, b.C, b.ldc,
                                   nullptr, 0)
                 : launch_gemm(s, false, false, b.M, b.N, b.K, -1.0, b.A, b.lda, b.B, b.ldb, 1.0, b.C, b.ldc, nullptr,
                               0);
  }
  return launch_sq_alone<LMAX>(s, a);
}

template <int LMAX>
int launch_sq_alone(hipStream_t s, SqParams& a) {
  constexpr size_t lds = sizeof(SqLds<LMAX>);
  static_assert(lds <= 160 * 1024, "LDS budget");
  // The P workgroups wait on each other, so all of them must be resident
  // at once: checked here against the occupancy of one CU times the CU
  // count.  An ordinary launch, not a cooperative one: a cooperative
  // dispatch leaves the queue idle for 12-15 us on each side, and on a
  // stream that runs nothing else beside it every workgroup of a grid this
  // size starts at once.  Should other work on the device hold a workgroup
  // back for too long, the bounded waits end the call with info = -1.
  static int resident = 0;
  if (!resident) {
    RQ_HIP(hipFuncSetAttribute((const void*)sample_qrcp_kernel<LMAX>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    int occ = 0, dev = 0, cus = 0;
    RQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, sample_qrcp_kernel<LMAX>, SQ_T, lds));
    RQ_HIP(hipGetDevice(&dev));
    RQ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    resident = occ * cus;
  }
  if (a.P > resident) return RQ_ERR_HIP_BASE + (int)hipErrorCooperativeLaunchTooLarge;
  hipLaunchKernelGGL(sample_qrcp_kernel<LMAX>, dim3(a.P), dim3(SQ_T), lds, s, a);
  RQ_HIP(hipGetLastError());
  return 0;
}

// ------------------------------------------------------------------ swaps
constexpr int SW_ROWS = 16;  // rows per workgroup (8192 rows: 512 workgroups)

template <typename T>
__global__ void __launch_bounds__(256) apply_swaps_kernel(const int* __restrict__ piv, int bJ, int64_t offset,
                                                          T* M, int64_t ldm, int64_t rows, int64_t* jpvt) {
  __shared__ int dst[128], src[128];
  __shared__ int npair;
  __shared__ int pv[SQ_BMAX];
  __shared__ T tile[128 * SW_ROWS];
  __shared__ int64_t itile[128];
  const int tid = threadIdx.x;
  if (tid == 0) npair = 0;
  if (tid < bJ) pv[tid] = piv[tid];  // the swap list is read from global memory once
  __syncthreads();
  // Destinations: positions 0..bJ-1 and every partner p_t >= bJ (first occurrence).
  if (tid < 2 * bJ) {
    int q = -1;
    if (tid < bJ) {
      q = tid;
    } else {
      const int t = tid - bJ;
      const int pt = pv[t];
      bool first = pt >= bJ;
      for (int s2 = 0; s2 < t && first; ++s2)
        if (pv[s2] == pt) first = false;
      if (first) q = pt;
    }
    if (q >= 0) {
      // content of position q after the swaps: undo them from the last one
      int sidx = q;
      for (int s2 = bJ - 1; s2 >= 0; --s2) {
        const int ps = pv[s2];
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

// ------------------------------------------------------------------ utilities
__global__ void fill_kernel(unsigned* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void zero_rows_kernel(int64_t r0, int64_t r1, int64_t cols, double* M, int64_t ldm) {
  const int64_t rows = r1 - r0;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t j = idx / rows, i = r0 + (idx - j * rows);
  M[i + j * ldm] = 0.0;
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

// Vp(i, c) = V(jpvt[i], c): the rows of V in the column order of A P.
__global__ void gather_rows_kernel(int64_t n, int64_t k, const double* __restrict__ V, int64_t ldv,
                                   const int64_t* __restrict__ jpvt, double* __restrict__ Vp, int64_t ldp) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * k) return;
  const int64_t c = idx / n, i = idx - c * n;
  Vp[i + c * ldp] = V[jpvt[i] + c * ldv];
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
int sample_rows_padded(int l) {
  return l <= 32 ? 32 : l <= 40 ? 40 : l <= 48 ? 48 : l <= 64 ? 64 : l <= 72 ? 72 : l <= 80 ? 80 : l <= 128 ? 128 : -1;
}
size_t sample_qrcp_cand_elems() { return 2 * (size_t)SQ_LCAP * SQ_T; }
size_t sample_qrcp_idx_elems() { return 2 * 2 * (size_t)SQ_T; }
size_t sample_qrcp_theta_elems() { return 2 * (size_t)SQ_MAXP * SQ_TH; }

int sample_qrcp_workgroups(int64_t nJ) { return (int)((nJ + SQ_T - 1) / SQ_T); }

int launch_sample_qrcp(hipStream_t s, double* S, int64_t lds, int l, int64_t nJ, int bJ, int* piv, int* info,
                       int info_base, const SampleQrcpWork& w, const BesideUpdate* upd) {
  if (bJ <= 0 || nJ <= 0) return 0;
  if (bJ > SQ_BMAX || bJ > nJ) return -5;
  if (lds != sample_rows_padded(l)) return -6;
  SqParams a;
  a.S = S; a.l = l; a.nJ = nJ; a.bJ = bJ; a.piv = piv; a.info = info; a.info_base = info_base;
  a.cand = w.cand; a.cand_idx = w.cand_idx; a.theta = w.theta; a.flags = w.flags; a.err = w.err;
  if (l <= 32) return launch_sq<32>(s, a, upd);
  if (l <= 40) return launch_sq<40>(s, a, upd);
  if (l <= 48) return launch_sq<48>(s, a, upd);
  if (l <= 64) return launch_sq<64>(s, a, upd);
  if (l <= 72) return launch_sq<72>(s, a, upd);
  if (l <= 80) return launch_sq<80>(s, a, upd);
  if (l <= 128) return launch_sq<128>(s, a, upd);
  return -7;
}

int launch_apply_swaps(hipStream_t s, const int* piv, int bJ, int64_t offset, double* M, int64_t ldm, int64_t rows,
                       int64_t* jpvt) {
  if (bJ <= 0) return 0;
  if (bJ > SQ_BMAX) return -5;
  const unsigned grid = std::max<unsigned>(1u, blocks_for(rows, SW_ROWS));
  hipLaunchKernelGGL(apply_swaps_kernel<double>, dim3(grid), dim3(256), 0, s, piv, bJ, offset, M, ldm, rows, jpvt);
  RQ_HIP(hipGetLastError());
  return 0;
}

int launch_apply_swaps_f32(hipStream_t s, const int* piv, int bJ, int64_t offset, float* M, int64_t ldm,
                           int64_t rows) {
  if (bJ <= 0) return 0;
  if (bJ > SQ_BMAX) return -5;
  const unsigned grid = std::max<unsigned>(1u, blocks_for(rows, SW_ROWS));
  hipLaunchKernelGGL(apply_swaps_kernel<float>, dim3(grid), dim3(256), 0, s, piv, bJ, offset, M, ldm, rows,
                     (int64_t*)nullptr);
  RQ_HIP(hipGetLastError());
  return 0;
}

int launch_fill(hipStream_t s, void* p, size_t words) {
  if (!words) return 0;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, (unsigned*)p, words);
  RQ_HIP(hipGetLastError());
  return 0;
}

int launch_zero_rows(hipStream_t s, int64_t r0, int64_t r1, int64_t cols, double* M, int64_t ldm) {
  if (r1 <= r0 || cols <= 0) return 0;
  hipLaunchKernelGGL(zero_rows_kernel, dim3(blocks_for((r1 - r0) * cols, 256)), dim3(256), 0, s, r0, r1, cols, M, ldm);
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

int launch_gather_rows(hipStream_t s, int64_t n, int64_t k, const double* V, int64_t ldv, const int64_t* jpvt,
                       double* Vp, int64_t ldp) {
  if (n <= 0 || k <= 0) return 0;
  hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks_for(n * k, 256)), dim3(256), 0, s, n, k, V, ldv, jpvt, Vp, ldp);
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
