// The FP64 (and mixed-precision) GEMM tile of the matrix cores: one
// workgroup of 256 threads computes one BM x BN tile of C = alpha op(A)
// op(B) + beta C over one chunk of the reduction.  Shared by the GEMM
// kernels (gemm.hip) and by the sample QRCP's launch that runs the
// look-ahead trailing update beside it (qrcp.hip); the tiling, the operand
// layout and the pipelines are described in gemm.hip.
#pragma once
#include <type_traits>
#include "kernels.hpp"

namespace rq {

namespace {

typedef float float4_t __attribute__((ext_vector_type(4)));

template <int BM, int BN, int BK, typename Acc>
constexpr size_t gemm_lds_bytes() {
  return (size_t)2 * BK * ((BM + 2) + (BN + 2)) * sizeof(Acc);
}

template <typename Acc>
struct Acc4;
template <>
struct Acc4<double> { typedef double4_t type; };
template <>
struct Acc4<float> { typedef float4_t type; };

// PAIR: the columns j >= nsplit of op(B) come from a second matrix B2 (column
// j - nsplit of op(B2), leading dimension ldb2), so that one launch forms
// op(A) [B B2] from two operands that are not adjacent in memory.
template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, typename TAe, typename TBe, typename Acc,
          bool PAIR>
__device__ __forceinline__ void gemm_tile(int64_t M, int64_t N, int64_t K, double alpha, const TAe* __restrict__ A,
                                          int64_t lda, const TBe* __restrict__ B, int64_t ldb, double beta,
                                          double* __restrict__ C, int64_t ldc, int64_t kchunk, int64_t split_stride,
                                          const TBe* __restrict__ B2, int64_t ldb2, int64_t nsplit, int64_t bx,
                                          int64_t by, int64_t bz) {
  typedef typename Acc4<Acc>::type acc4_t;
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  constexpr int ALD = BM + 2, BLD = BN + 2;  // padded rows: no bank conflicts between k rows
  constexpr int A_PER = BM * BK / 256, B_PER = BK * BN / 256;
  static_assert(A_PER * 256 == BM * BK && B_PER * 256 == BK * BN, "tile/threads mismatch");
  static_assert(WM * WN == 4, "four waves");
  // two LDS stages: the tiles of step k+1 are stored while step k computes
  extern __shared__ __align__(16) double gsm_raw[];
  Acc* gsm = reinterpret_cast<Acc*>(gsm_raw);
  Acc* As = gsm;                   // [2][BK][ALD]
  Acc* Bs = gsm + 2 * BK * ALD;    // [2][BK][BLD]

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int64_t i0 = by * BM;
  const int64_t j0 = bx * BN;
  const int64_t kbeg = bz * kchunk;
  const int64_t kend = min(K, kbeg + kchunk);
  double* Cz = C + bz * split_stride;

  // The accumulators start from beta * C (lane holds C(i, j) for
  // i = row0 + lane%16, j = col0 + 4r + lane/16): all C loads are issued
  // together, ahead of the first operand tiles, and alpha is folded into the
  // A tile, so the epilogue is stores only.
  acc4_t acc[TM][TN];
  constexpr bool F64 = std::is_same<Acc, double>::value;
  const int64_t ri = i0 + wm * WTM + (lane & 15);
  // column of accumulator register r: cj + 16 b + CR * r
  const int64_t cj = j0 + wn * WTN + (F64 ? (lane >> 4) : 4 * (lane >> 4));
  constexpr int CR = F64 ? 4 : 1;
  // (FP32 accumulators start from zero instead: beta C is added in FP64 in
  // the epilogue, so that C keeps its FP64 precision.)
  if (F64 && beta != 0.0) {
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gi = ri + a * 16, gj = cj + b * 16 + CR * r;
          acc[a][b][r] = (Acc)((gi < M && gj < N) ? Cz[gi + gj * ldc] : 0.0);
        }
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[a][b][r] *= (Acc)beta;
  } else {
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[a][b][r] = (Acc)0;
  }

  auto compute = [&](int stage) {
    const Acc* as = As + stage * BK * ALD;
    const Acc* bs = Bs + stage * BK * BLD;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      Acc af[TM], bf[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) af[a] = as[(kk + (lane >> 4)) * ALD + wm * WTM + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < TN; ++b) bf[b] = bs[(kk + (lane >> 4)) * BLD + wn * WTN + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          if constexpr (std::is_same<Acc, double>::value)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[b], af[a], acc[a][b], 0, 0, 0);
          else
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[b], af[a], acc[a][b], 0, 0, 0);
        }
    }
  };

  if constexpr (BM * BN <= 64 * 64) {
    // Tiles up to 64 x 64 (few accumulators): prefetch distance two.
    // Register set s % 2 receives the tiles of step s two steps ahead and LDS
    // stage s % 2 one step ahead.  The loads have no branches: an element
    // outside the matrix or past the chunk's end is read at the clamped
    // position and zeroed when it is stored to LDS, so the loads are issued
    // unconditionally, the number in flight is the same on every path, and
    // the wait before an LDS store covers only the older register set.
    TAe ra[2][A_PER];
    TBe rb[2][B_PER];
    auto load_tiles = [&](int64_t k0, TAe* ra_, TBe* rb_) {
#pragma unroll
      for (int e = 0; e < A_PER; ++e) {
        const int idx = tid + e * 256;
        int ii, kk;
        if (TA) { kk = idx % BK; ii = idx / BK; } else { ii = idx % BM; kk = idx / BM; }
        const int64_t gi = i0 + ii, gk = k0 + kk;
        const int64_t gic = gi < M ? gi : M - 1, gkc = gk < kend ? gk : kend - 1;
        ra_[e] = TA ? A[gkc + gic * lda] : A[gic + gkc * lda];
      }
#pragma unroll
      for (int e = 0; e < B_PER; ++e) {
        const int idx = tid + e * 256;
        int jj, kk;
        if (TB) { jj = idx % BN; kk = idx / BN; } else { kk = idx % BK; jj = idx / BK; }
        const int64_t gj = j0 + jj, gk = k0 + kk;
        const int64_t gjc = gj < N ? gj : N - 1, gkc = gk < kend ? gk : kend - 1;
        const TBe* src;
        if constexpr (PAIR) {
          const bool second = gjc >= nsplit;
          const int64_t g2 = second ? gjc - nsplit : gjc;
          const TBe* base = second ? B2 : B;
          const int64_t ld = second ? ldb2 : ldb;
          src = TB ? base + g2 + gkc * ld : base + gkc + g2 * ld;
        } else {
          src = TB ? B + gjc + gkc * ldb : B + gkc + gjc * ldb;
        }
        rb_[e] = *src;
      }
    };
    auto store_tiles = [&](int stage, int64_t k0, const TAe* ra_, const TBe* rb_) {
      Acc* as = As + stage * BK * ALD;
      Acc* bs = Bs + stage * BK * BLD;
#pragma unroll
      for (int e = 0; e < A_PER; ++e) {
        const int idx = tid + e * 256;
        int ii, kk;
        if (TA) { kk = idx % BK; ii = idx / BK; } else { ii = idx % BM; kk = idx / BM; }
        const bool ok = i0 + ii < M && k0 + kk < kend;
        as[kk * ALD + ii] = ok ? (Acc)(alpha * (double)ra_[e]) : (Acc)0;
      }
#pragma unroll
      for (int e = 0; e < B_PER; ++e) {
        const int idx = tid + e * 256;
        int jj, kk;
        if (TB) { jj = idx % BN; kk = idx / BN; } else { kk = idx % BK; jj = idx / BK; }
        const bool ok = j0 + jj < N && k0 + kk < kend;
        bs[kk * BLD + jj] = ok ? (Acc)rb_[e] : (Acc)0;
      }
    };
    if (kbeg < kend) {
      const int64_t nsteps = (kend - kbeg + BK - 1) / BK;
      load_tiles(kbeg, ra[0], rb[0]);
      load_tiles(kbeg + BK, ra[1], rb[1]);
      store_tiles(0, kbeg, ra[0], rb[0]);
      __syncthreads();
      // steps st and st + 1 per iteration while step st + 2 exists; no
      // branch lies between a load and its LDS store, so the compiler does
      // not sink the loads past one
      int64_t st = 0;
      for (; st + 2 < nsteps; st += 2) {
        load_tiles(kbeg + (st + 2) * BK, ra[0], rb[0]);
        __builtin_amdgcn_sched_barrier(0);  // the loads stay ahead of the products
        compute(0);
        store_tiles(1, kbeg + (st + 1) * BK, ra[1], rb[1]);
        __syncthreads();
        load_tiles(kbeg + (st + 3) * BK, ra[1], rb[1]);
        __builtin_amdgcn_sched_barrier(0);
        compute(1);
        store_tiles(0, kbeg + (st + 2) * BK, ra[0], rb[0]);
        __syncthreads();
      }
      // the last one or two steps: stage 0 holds step st, set 1 step st + 1
      compute(0);
      if (st + 1 < nsteps) {
        store_tiles(1, kbeg + (st + 1) * BK, ra[1], rb[1]);
        __syncthreads();
        compute(1);
      }
    }
  } else {
    // Larger tiles (more accumulators, less room for a second register
    // set): prefetch distance one; the loads of step k + 1 are issued before
    // step k computes.
    TAe ra[A_PER];
    TBe rb[B_PER];
    auto load_tiles = [&](int64_t k0) {
#pragma unroll
      for (int e = 0; e < A_PER; ++e) {
        const int idx = tid + e * 256;
        int ii, kk;
        if (TA) { kk = idx % BK; ii = idx / BK; } else { ii = idx % BM; kk = idx / BM; }
        const int64_t gi = i0 + ii, gk = k0 + kk;
        TAe v = (TAe)0;
        if (gi < M && gk < kend) v = TA ? A[gk + gi * lda] : A[gi + gk * lda];
        ra[e] = v;
      }
#pragma unroll
      for (int e = 0; e < B_PER; ++e) {
        const int idx = tid + e * 256;
        int jj, kk;
        if (TB) { jj = idx % BN; kk = idx / BN; } else { kk = idx % BK; jj = idx / BK; }
        const int64_t gj = j0 + jj, gk = k0 + kk;
        TBe v = (TBe)0;
        if (gj < N && gk < kend) {
          if constexpr (PAIR) {
            if (gj >= nsplit) {
              const int64_t g2 = gj - nsplit;
              v = TB ? B2[g2 + gk * ldb2] : B2[gk + g2 * ldb2];
            } else {
              v = TB ? B[gj + gk * ldb] : B[gk + gj * ldb];
            }
          } else {
            v = TB ? B[gj + gk * ldb] : B[gk + gj * ldb];
          }
        }
        rb[e] = v;
      }
    };
    auto store_tiles = [&](int stage) {
      Acc* as = As + stage * BK * ALD;
      Acc* bs = Bs + stage * BK * BLD;
#pragma unroll
      for (int e = 0; e < A_PER; ++e) {
        const int idx = tid + e * 256;
        int ii, kk;
        if (TA) { kk = idx % BK; ii = idx / BK; } else { ii = idx % BM; kk = idx / BM; }
        as[kk * ALD + ii] = (Acc)(alpha * (double)ra[e]);
      }
#pragma unroll
      for (int e = 0; e < B_PER; ++e) {
        const int idx = tid + e * 256;
        int jj, kk;
        if (TB) { jj = idx % BN; kk = idx / BN; } else { kk = idx % BK; jj = idx / BK; }
        bs[kk * BLD + jj] = (Acc)rb[e];
      }
    };
    if (kbeg < kend) {
      load_tiles(kbeg);
      store_tiles(0);
      __syncthreads();
      int stage = 0;
      for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
        const bool more = k0 + BK < kend;
        if (more) load_tiles(k0 + BK);
        const Acc* as = As + stage * BK * ALD;
        const Acc* bs = Bs + stage * BK * BLD;
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
          Acc af[TM], bf[TN];
#pragma unroll
          for (int a = 0; a < TM; ++a) af[a] = as[(kk + (lane >> 4)) * ALD + wm * WTM + a * 16 + (lane & 15)];
#pragma unroll
          for (int b = 0; b < TN; ++b) bf[b] = bs[(kk + (lane >> 4)) * BLD + wn * WTN + b * 16 + (lane & 15)];
#pragma unroll
          for (int a = 0; a < TM; ++a)
#pragma unroll
            for (int b = 0; b < TN; ++b) {
              if constexpr (std::is_same<Acc, double>::value)
                acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[b], af[a], acc[a][b], 0, 0, 0);
              else
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[b], af[a], acc[a][b], 0, 0, 0);
            }
        }
        if (more) store_tiles(stage ^ 1);
        __syncthreads();
        stage ^= 1;
      }
    }
  }

#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = ri + a * 16, gj = cj + b * 16 + CR * r;
        if (gi < M && gj < N) {
          double v = (double)acc[a][b][r];
          if (!F64 && beta != 0.0) v += beta * Cz[gi + gj * ldc];
          Cz[gi + gj * ldc] = v;
        }
      }
}

}  // namespace

}  // namespace rq
