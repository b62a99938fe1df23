// FP64 GEMM on the gfx950 matrix cores (v_mfma_f64_16x16x4_f64).
//
//   C(i, j) = alpha * sum_k opA(i, k) opB(k, j) + beta * C(i, j)
//   opA(i, k) = TA ? A[k + i*lda] : A[i + k*lda]
//   opB(k, j) = TB ? B[j + k*ldb] : B[k + j*ldb]
//   C column-major with leading dimension ldc.
//
// Used for every block-reflector product of the method: the sketch B = Omega A,
// W^T = T^T (Y^T A), the trailing update A -= Y W^T, the TRQRCP inner-product
// composition, the sample-update product W11 R12 and the TUXV products.
//
// Tiling: a workgroup of 256 threads (4 waves, WM x WN) owns a BM x BN tile of
// C; operand tiles of depth BK are staged through LDS with register
// prefetch of the next tile.  The MFMA is issued with its operands swapped
// (B-fragment first) so that lane l, register r of a 16x16 accumulator holds
// C(i0 + l%16, j0 + 4r + l/16): sixteen consecutive rows of one column of
// the column-major C, which makes the C loads and stores 128-byte coalesced.
//
// Split-K (grid.z > 1) writes partial sums to a scratch buffer; a second
// kernel adds them in a fixed order (deterministic, no atomics).
#include "kernels.hpp"

namespace rq {

namespace {

template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB>
__global__ void __launch_bounds__(256) gemm_kernel(int64_t M, int64_t N, int64_t K, double alpha,
                                                   const double* __restrict__ A, int64_t lda,
                                                   const double* __restrict__ B, int64_t ldb, double beta,
                                                   double* __restrict__ C, int64_t ldc, int64_t kchunk,
                                                   int64_t split_stride) {
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  constexpr int APAD = 2, BPAD = 2;
  constexpr int A_PER = BM * BK / 256, B_PER = BK * BN / 256;
  static_assert(A_PER * 256 == BM * BK && B_PER * 256 == BK * BN, "tile/threads mismatch");
  __shared__ double As[BK][BM + APAD];
  __shared__ double Bs[BK][BN + BPAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int64_t i0 = (int64_t)blockIdx.y * BM;
  const int64_t j0 = (int64_t)blockIdx.x * BN;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = min(K, kbeg + kchunk);
  double* Cz = C + (int64_t)blockIdx.z * split_stride;

  double4_t acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = (double4_t){0.0, 0.0, 0.0, 0.0};

  double ra[A_PER], rb[B_PER];

  auto load_tiles = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < A_PER; ++e) {
      const int idx = tid + e * 256;
      int ii, kk;
      if (TA) { kk = idx % BK; ii = idx / BK; } else { ii = idx % BM; kk = idx / BM; }
      const int64_t gi = i0 + ii, gk = k0 + kk;
      double v = 0.0;
      if (gi < M && gk < kend) v = TA ? A[gk + gi * lda] : A[gi + gk * lda];
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < B_PER; ++e) {
      const int idx = tid + e * 256;
      int jj, kk;
      if (TB) { jj = idx % BN; kk = idx / BN; } else { kk = idx % BK; jj = idx / BK; }
      const int64_t gj = j0 + jj, gk = k0 + kk;
      double v = 0.0;
      if (gj < N && gk < kend) v = TB ? B[gj + gk * ldb] : B[gk + gj * ldb];
      rb[e] = v;
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int e = 0; e < A_PER; ++e) {
      const int idx = tid + e * 256;
      int ii, kk;
      if (TA) { kk = idx % BK; ii = idx / BK; } else { ii = idx % BM; kk = idx / BM; }
      As[kk][ii] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < B_PER; ++e) {
      const int idx = tid + e * 256;
      int jj, kk;
      if (TB) { jj = idx % BN; kk = idx / BN; } else { kk = idx % BK; jj = idx / BK; }
      Bs[kk][jj] = rb[e];
    }
  };

  if (kbeg < kend) {
    load_tiles(kbeg);
    for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
      store_tiles();
      __syncthreads();
      if (k0 + BK < kend) load_tiles(k0 + BK);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        double af[TM], bf[TN];
#pragma unroll
        for (int a = 0; a < TM; ++a) af[a] = As[kk + (lane >> 4)][wm * WTM + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < TN; ++b) bf[b] = Bs[kk + (lane >> 4)][wn * WTN + b * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[b], af[a], acc[a][b], 0, 0, 0);
      }
      __syncthreads();
    }
  }

  // Epilogue: lane holds C(i, j) for i = row0 + lane%16, j = col0 + 4r + lane/16.
#pragma unroll
  for (int a = 0; a < TM; ++a) {
    const int64_t gi = i0 + wm * WTM + a * 16 + (lane & 15);
#pragma unroll
    for (int b = 0; b < TN; ++b) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gj = j0 + wn * WTN + b * 16 + 4 * r + (lane >> 4);
        if (gi < M && gj < N) {
          double* p = Cz + gi + gj * ldc;
          double v = alpha * acc[a][b][r];
          if (beta != 0.0) v += beta * (*p);
          *p = v;
        }
      }
    }
  }
}

// C = alpha * sum_z P[z] + beta * C   (P[z] is M x N with leading dimension M)
__global__ void __launch_bounds__(256) splitk_reduce_kernel(int64_t M, int64_t N, int splits,
                                                            const double* __restrict__ P, double alpha,
                                                            double beta, double* __restrict__ C, int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = M * N;
  if (idx >= total) return;
  const int64_t j = idx / M, i = idx - j * M;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += P[(int64_t)z * total + idx];
  double v = alpha * s;
  double* c = C + i + j * ldc;
  if (beta != 0.0) v += beta * (*c);
  *c = v;
}

// Same sum for many splits: a workgroup reduces 16 consecutive outputs; its
// 16 thread groups each add every 16th partial (128-byte coalesced reads),
// then the 16 group sums are added in LDS in a fixed order.
__global__ void __launch_bounds__(256) splitk_reduce_many_kernel(int64_t M, int64_t N, int splits,
                                                                 const double* __restrict__ P, double alpha,
                                                                 double beta, double* __restrict__ C, int64_t ldc) {
  __shared__ double part[16][17];
  const int64_t total = M * N;
  const int ol = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int64_t o = (int64_t)blockIdx.x * 16 + ol;
  double s = 0.0;
  if (o < total)
    for (int z = g; z < splits; z += 16) s += P[(int64_t)z * total + o];
  part[g][ol] = s;
  __syncthreads();
  if (threadIdx.x < 16 && o < total) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += part[q][ol];
    const int64_t j = o / M, i = o - j * M;
    double v = alpha * acc;
    double* c = C + i + j * ldc;
    if (beta != 0.0) v += beta * (*c);
    *c = v;
  }
}

template <int BM, int BN, int BK, int WM, int WN>
int launch_tiles(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                 int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int splits,
                 int64_t kchunk, int64_t split_stride) {
  dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM), (unsigned)splits);
  dim3 block(256);
  if (!ta && !tb)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, BK, WM, WN, false, false>), grid, block, 0, s, M, N, K, alpha, A, lda,
                       B, ldb, beta, C, ldc, kchunk, split_stride);
  else if (ta && !tb)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, BK, WM, WN, true, false>), grid, block, 0, s, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc, kchunk, split_stride);
  else if (!ta && tb)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, BK, WM, WN, false, true>), grid, block, 0, s, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc, kchunk, split_stride);
  else
    hipLaunchKernelGGL((gemm_kernel<BM, BN, BK, WM, WN, true, true>), grid, block, 0, s, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc, kchunk, split_stride);
  RQ_HIP(hipGetLastError());
  return 0;
}

}  // namespace

// Small outputs with a long reduction (Gram matrices of tall panels, b x n
// products with n short) are split along K: "gram mode" for outputs of at
// most 64 x 128 (up to 256 splits of >= 32 rows), the general split for
// short-and-wide outputs (up to 8 splits).
constexpr int GRAM_MAXS = 256;
constexpr int64_t GRAM_MINK = 32;

bool gram_mode(int64_t M, int64_t N, int64_t K) { return M <= 64 && N <= 128 && K >= 256; }

size_t gemm_scratch_elems(int64_t M, int64_t N, int64_t K) {
  size_t e = 0;
  if (M <= 128 && K >= 1024) e = (size_t)M * (size_t)N * 8;
  if (gram_mode(M, N, K)) {
    const int64_t s = std::min<int64_t>(GRAM_MAXS, (K + GRAM_MINK - 1) / GRAM_MINK);
    e = std::max(e, (size_t)M * (size_t)N * (size_t)s);
  }
  return e;
}

int launch_gemm(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* scratch,
                size_t scratch_elems) {
  if (M <= 0 || N <= 0) return 0;
  if (K <= 0) {
    // C = beta * C
    if (beta == 1.0) return 0;
    return launch_scale(s, M, N, beta, C, ldc);
  }
  constexpr int BM = 64, BN = 64, BK = 16;
  const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  int splits = 1;
  int64_t kchunk = K;
  bool many = false;
  if (scratch && gram_mode(M, N, K)) {
    kchunk = std::max<int64_t>(GRAM_MINK, (K + GRAM_MAXS - 1) / GRAM_MAXS);
    kchunk = (kchunk + BK - 1) / BK * BK;
    splits = (int)((K + kchunk - 1) / kchunk);
    while (splits > 1 && (size_t)splits * (size_t)M * (size_t)N > scratch_elems) {
      kchunk *= 2;
      splits = (int)((K + kchunk - 1) / kchunk);
    }
    many = true;
  } else if (scratch && M <= 128 && K >= 1024) {
    // aim for >= 1024 workgroups, at least 512 reduction steps per split
    int64_t want = (1024 + tiles - 1) / tiles;
    int64_t maxs = K / 512;
    splits = (int)std::max<int64_t>(1, std::min<int64_t>({want, maxs, 8}));
    while (splits > 1 && (size_t)splits * (size_t)M * (size_t)N > scratch_elems) --splits;
    kchunk = (K + splits - 1) / splits;
    kchunk = (kchunk + BK - 1) / BK * BK;
  }
  if (splits == 1)
    return launch_tiles<BM, BN, BK, 2, 2>(s, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, 1, K, 0);
  int rc = launch_tiles<BM, BN, BK, 2, 2>(s, ta, tb, M, N, K, 1.0, A, lda, B, ldb, 0.0, scratch, M, splits, kchunk,
                                          M * N);
  if (rc) return rc;
  const int64_t total = M * N;
  if (many) {
    hipLaunchKernelGGL(splitk_reduce_many_kernel, dim3((unsigned)((total + 15) / 16)), dim3(256), 0, s, M, N, splits,
                       (const double*)scratch, alpha, beta, C, ldc);
  } else {
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, M, N, splits,
                       (const double*)scratch, alpha, beta, C, ldc);
  }
  RQ_HIP(hipGetLastError());
  return 0;
}

namespace {
__global__ void __launch_bounds__(256) scale_kernel(int64_t M, int64_t N, double beta, double* C, int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t j = idx / M, i = idx - j * M;
  C[i + j * ldc] *= beta;
}
}  // namespace

int launch_scale(hipStream_t s, int64_t M, int64_t N, double beta, double* C, int64_t ldc) {
  if (M <= 0 || N <= 0) return 0;
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((M * N + 255) / 256)), dim3(256), 0, s, M, N, beta, C, ldc);
  RQ_HIP(hipGetLastError());
  return 0;
}

}  // namespace rq
