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
// C (128 x 64 for the large updates, 64 x 64 otherwise); operand tiles of
// depth BK are staged through two LDS buffers with register prefetch (two
// steps ahead for tiles up to 64 x 64, one step for the 128 x 64 tiles),
// and C is loaded into the accumulators before the k loop.  The MFMA is
// issued with its operands swapped (B-fragment first) so that lane l,
// register r of a 16x16 accumulator holds C(i0 + l%16, j0 + 4r + l/16):
// sixteen consecutive rows of one column of the column-major C, which makes
// the C loads and stores 128-byte coalesced.
//
// Split-K (grid.z > 1) writes partial sums to a scratch buffer; a second
// kernel adds them in a fixed order (deterministic, no atomics).
//
// The same kernel, instantiated with FP32 accumulation, serves the mixed-
// precision products: operands are read in their stored precision (one of
// them an FP32 copy of A), rounded to FP32 into the LDS tiles and multiplied
// on v_mfma_f32_16x16x4_f32, whose operands are laid out as those of the
// FP64 instruction but whose accumulator registers run along the other
// index: with the operands swapped, register r of lane l holds
// C(i0 + l%16, j0 + 4 (l/16) + r).  C and the split-K partials stay FP64.
#include <type_traits>
#include "kernels.hpp"
#include "gemm_tile.hpp"

namespace rq {

namespace {

// One output tile per workgroup (grid tiles_x x tiles_y x splits).
template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, typename TAe = double, typename TBe = double,
          typename Acc = double, bool PAIR = false>
__global__ void __launch_bounds__(256, 2)
    gemm_kernel(int64_t M, int64_t N, int64_t K, double alpha, const TAe* __restrict__ A, int64_t lda,
                const TBe* __restrict__ B, int64_t ldb, double beta, double* __restrict__ C, int64_t ldc,
                int64_t kchunk, int64_t split_stride, const TBe* __restrict__ B2, int64_t ldb2, int64_t nsplit) {
  gemm_tile<BM, BN, BK, WM, WN, TA, TB, TAe, TBe, Acc, PAIR>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk,
                                                             split_stride, B2, ldb2, nsplit, blockIdx.x, blockIdx.y,
                                                             blockIdx.z);
}

// Grouped products (the batched engine): the tiles of many independent
// products in one persistent launch.  Workgroup g walks the tile list
// t = g, g + gridDim.x, ...; tile t belongs to product tile_prob[t] and is
// its tile t - tile0: chunk z = (t - tile0) / ntile of the reduction (split
// K, partial products to C + z split_stride), then row-major tile order.
template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, typename Acc>
__global__ void __launch_bounds__(256, 2)
    gemm_grouped_kernel(const GroupedGemm* __restrict__ probs,
                                                           const int* __restrict__ tile_prob, int64_t ntiles) {
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int pi = __builtin_amdgcn_readfirstlane(tile_prob[t]);
    const GroupedGemm& g = probs[pi];
    const int64_t lt = t - g.tile0;
    const int64_t z = lt / g.ntile, tl = lt - z * g.ntile;
    gemm_tile<BM, BN, BK, WM, WN, TA, TB, double, double, Acc, false>(
        g.M, g.N, g.K, g.alpha, g.A, g.lda, g.B, g.ldb, g.beta, g.C, g.ldc, g.kchunk, g.split_stride, nullptr, 0, 0,
        tl % g.tiles_x, tl / g.tiles_x, z);
    __syncthreads();  // the next tile's LDS stores after every wave's last reads
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

struct PairB {
  const void* B2 = nullptr;  // null: no second operand
  int64_t ldb2 = 0;
  int64_t nsplit = 0;
};

template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, typename TAe, typename TBe, typename Acc,
          bool PAIR = false>
int launch_one(hipStream_t s, dim3 grid, int64_t M, int64_t N, int64_t K, double alpha, const TAe* A, int64_t lda,
               const TBe* B, int64_t ldb, double beta, double* C, int64_t ldc, int64_t kchunk,
               int64_t split_stride, const PairB& pb = PairB()) {
  constexpr size_t lds = gemm_lds_bytes<BM, BN, BK, Acc>();
  static bool attr = false;
  if (!attr) {
    RQ_HIP(hipFuncSetAttribute((const void*)gemm_kernel<BM, BN, BK, WM, WN, TA, TB, TAe, TBe, Acc, PAIR>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  hipLaunchKernelGGL((gemm_kernel<BM, BN, BK, WM, WN, TA, TB, TAe, TBe, Acc, PAIR>), grid, dim3(256), lds, s, M, N,
                     K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, split_stride, (const TBe*)pb.B2, pb.ldb2,
                     pb.nsplit);
  RQ_HIP(hipGetLastError());
  return 0;
}

template <int BM, int BN, int BK, int WM, int WN, typename TAe, typename TBe, typename Acc>
int launch_tiles(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const TAe* A,
                 int64_t lda, const TBe* B, int64_t ldb, double beta, double* C, int64_t ldc, int splits,
                 int64_t kchunk, int64_t split_stride) {
  dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM), (unsigned)splits);
  if (!ta && !tb)
    return launch_one<BM, BN, BK, WM, WN, false, false, TAe, TBe, Acc>(s, grid, M, N, K, alpha, A, lda, B, ldb, beta,
                                                                       C, ldc, kchunk, split_stride);
  if (ta && !tb)
    return launch_one<BM, BN, BK, WM, WN, true, false, TAe, TBe, Acc>(s, grid, M, N, K, alpha, A, lda, B, ldb, beta,
                                                                      C, ldc, kchunk, split_stride);
  if (!ta && tb)
    return launch_one<BM, BN, BK, WM, WN, false, true, TAe, TBe, Acc>(s, grid, M, N, K, alpha, A, lda, B, ldb, beta,
                                                                      C, ldc, kchunk, split_stride);
  return launch_one<BM, BN, BK, WM, WN, true, true, TAe, TBe, Acc>(s, grid, M, N, K, alpha, A, lda, B, ldb, beta, C,
                                                                   ldc, kchunk, split_stride);
}

}  // namespace

// Small outputs with a long reduction (Gram matrices of tall panels) are
// split along K: "gram mode" for outputs of at most 64 x 128, up to 256
// splits of >= 32 rows.
constexpr int GRAM_MAXS = 256;
constexpr int64_t GRAM_MINK = 32;

bool gram_mode(int64_t M, int64_t N, int64_t K) { return M <= 64 && N <= 128 && K >= 256; }

// Short-wide outputs with a long reduction (b x n products Y^T A, l x n
// sketches Omega A): one row of tiles (64 x 64 up to 64 rows, 128 x 64 up
// to 128, so that B is read once), up to WIDE_MAXS splits of at least
// wide_mink(K) rows, aiming at about 2048 workgroups (eight per CU).  Short
// reductions (the last blocks' Y^T A) take chunks down to 64 rows: there the
// launch is latency-bound and more workgroups shorten it (at 512 rows, 27 ->
// 10 us per product).
constexpr int WIDE_MAXS = 16;

static bool wide_mode(int64_t M, int64_t K) { return M <= 128 && K >= 256; }
static int64_t wide_mink(int64_t K) { return K >= 2048 ? 256 : 64; }

size_t gemm_scratch_elems(int64_t M, int64_t N, int64_t K) {
  size_t e = 0;
  if (wide_mode(M, K)) e = (size_t)M * (size_t)N * WIDE_MAXS;
  if (gram_mode(M, N, K)) {
    const int64_t s = std::min<int64_t>(GRAM_MAXS, (K + GRAM_MINK - 1) / GRAM_MINK);
    e = std::max(e, (size_t)M * (size_t)N * (size_t)s);
  }
  return e;
}

template <typename TAe, typename TBe, typename Acc>
static int gemm_dispatch(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const TAe* A,
                         int64_t lda, const TBe* B, int64_t ldb, double beta, double* C, int64_t ldc, double* scratch,
                         size_t scratch_elems, const PairB& pb = PairB()) {
  if (M <= 0 || N <= 0) return 0;
  if (K <= 0) {
    // C = beta * C
    if (beta == 1.0) return 0;
    return launch_scale(s, M, N, beta, C, ldc);
  }
  constexpr int BK = 16;
  int splits = 1;
  int64_t kchunk = K;
  enum { SMALL, BIG, WIDE } shape = SMALL;  // WIDE: split-K with the SMALL tiles (BIG ones above 64 rows)
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
  } else if (scratch && wide_mode(M, K)) {
    shape = (M <= 64) ? WIDE : BIG;
    const int64_t tiles = (N + 63) / 64;
    const int64_t want = (2048 + tiles - 1) / tiles;
    const int64_t maxs = K / wide_mink(K);
    splits = (int)std::max<int64_t>(1, std::min<int64_t>({want, maxs, (int64_t)WIDE_MAXS}));
    while (splits > 1 && (size_t)splits * (size_t)M * (size_t)N > scratch_elems) --splits;
    kchunk = (K + splits - 1) / splits;
    kchunk = (kchunk + BK - 1) / BK * BK;
    splits = (int)((K + kchunk - 1) / kchunk);
  } else if (M >= 128 && N >= 128) {
    shape = BIG;
  }
  auto tiles = [&](double al, double be, double* out, int64_t ldo, int64_t stride) {
    if constexpr (std::is_same<TAe, double>::value && std::is_same<TBe, double>::value &&
                  std::is_same<Acc, double>::value) {
      if (pb.B2) {  // launch_gemm_pair: A transposed, B not, 64 x 64 tiles
        dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)splits);
        return launch_one<64, 64, BK, 2, 2, true, false, double, double, double, true>(
            s, grid, M, N, K, al, A, lda, B, ldb, be, out, ldo, kchunk, stride, pb);
      }
    }
    switch (shape) {
      case BIG:
        return launch_tiles<128, 64, BK, 2, 2, TAe, TBe, Acc>(s, ta, tb, M, N, K, al, A, lda, B, ldb, be, out, ldo,
                                                              splits, kchunk, stride);
      default:
        return launch_tiles<64, 64, BK, 2, 2, TAe, TBe, Acc>(s, ta, tb, M, N, K, al, A, lda, B, ldb, be, out, ldo,
                                                             splits, kchunk, stride);
    }
  };
  if (splits == 1) return tiles(alpha, beta, C, ldc, 0);
  int rc = tiles(1.0, 0.0, scratch, M, M * N);
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

int launch_gemm(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* scratch,
                size_t scratch_elems) {
  return gemm_dispatch<double, double, double>(s, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, scratch,
                                               scratch_elems);
}

namespace {
template <int BM, int BN, bool TA, bool TB, typename Acc>
int launch_grouped_one(hipStream_t s, const GroupedGemm* probs, const int* tile_prob, int64_t ntiles, int wgs) {
  constexpr size_t lds = gemm_lds_bytes<BM, BN, 16, Acc>();
  auto fn = gemm_grouped_kernel<BM, BN, 16, 2, 2, TA, TB, Acc>;
  static bool attr = false;
  if (!attr) {
    RQ_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ntiles, wgs));
  hipLaunchKernelGGL(fn, dim3(g), dim3(256), lds, s, probs, tile_prob, ntiles);
  RQ_HIP(hipGetLastError());
  return 0;
}

template <int BM, int BN, typename Acc>
int launch_grouped_tr(hipStream_t s, bool ta, bool tb, const GroupedGemm* probs, const int* tile_prob, int64_t ntiles,
                      int wgs) {
  if (!ta && !tb) return launch_grouped_one<BM, BN, false, false, Acc>(s, probs, tile_prob, ntiles, wgs);
  if (ta && !tb) return launch_grouped_one<BM, BN, true, false, Acc>(s, probs, tile_prob, ntiles, wgs);
  if constexpr (std::is_same<Acc, double>::value) {
    if (!ta && tb) return launch_grouped_one<BM, BN, false, true, Acc>(s, probs, tile_prob, ntiles, wgs);
    return launch_grouped_one<BM, BN, true, true, Acc>(s, probs, tile_prob, ntiles, wgs);
  } else {
    return -2;  // FP32 grouped products: no transposed second operand
  }
}
}  // namespace

void grouped_tile_shape(int cfg, int* bm, int* bn) {
  *bm = (cfg == GT_128x64) ? 128 : (cfg == GT_32x32) ? 32 : 64;
  *bn = (cfg == GT_32x32) ? 32 : 64;
}

int launch_gemm_grouped(hipStream_t s, int cfg, bool ta, bool tb, bool f32, const GroupedGemm* probs,
                        const int* tile_prob, int64_t ntiles, int wgs) {
  if (ntiles <= 0) return 0;
  switch (cfg) {
    case GT_32x32:
      return f32 ? launch_grouped_tr<32, 32, float>(s, ta, tb, probs, tile_prob, ntiles, wgs)
                 : launch_grouped_tr<32, 32, double>(s, ta, tb, probs, tile_prob, ntiles, wgs);
    case GT_128x64:
      return f32 ? launch_grouped_tr<128, 64, float>(s, ta, tb, probs, tile_prob, ntiles, wgs)
                 : launch_grouped_tr<128, 64, double>(s, ta, tb, probs, tile_prob, ntiles, wgs);
    default:
      return f32 ? launch_grouped_tr<64, 64, float>(s, ta, tb, probs, tile_prob, ntiles, wgs)
                 : launch_grouped_tr<64, 64, double>(s, ta, tb, probs, tile_prob, ntiles, wgs);
  }
}

int launch_gemm_pair(hipStream_t s, int64_t M, int64_t N1, int64_t K, double alpha, const double* A, int64_t lda,
                     const double* B1, int64_t ldb1, const double* B2, int64_t ldb2, double beta, double* C,
                     int64_t ldc, double* scratch, size_t scratch_elems) {
  if (M > 64 || N1 > 64) {  // outside the one-launch shape: two products
    RQ_TRY_RAW(launch_gemm(s, true, false, M, N1, K, alpha, A, lda, B1, ldb1, beta, C, ldc, scratch, scratch_elems));
    return launch_gemm(s, true, false, M, N1, K, alpha, A, lda, B2, ldb2, beta, C + N1 * ldc, ldc, scratch,
                       scratch_elems);
  }
  PairB pb;
  pb.B2 = B2;
  pb.ldb2 = ldb2;
  pb.nsplit = N1;
  return gemm_dispatch<double, double, double>(s, true, false, M, 2 * N1, K, alpha, A, lda, B1, ldb1, beta, C, ldc,
                                               scratch, scratch_elems, pb);
}

int launch_gemm_f32(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const float* A,
                    int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* scratch,
                    size_t scratch_elems) {
  return gemm_dispatch<float, double, float>(s, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, scratch,
                                             scratch_elems);
}

int launch_gemm_f32(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                    int64_t lda, const float* B, int64_t ldb, double beta, double* C, int64_t ldc, double* scratch,
                    size_t scratch_elems) {
  return gemm_dispatch<double, float, float>(s, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, scratch,
                                             scratch_elems);
}

int launch_gemm_f32(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                    int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* scratch,
                    size_t scratch_elems) {
  return gemm_dispatch<double, double, float>(s, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, scratch,
                                              scratch_elems);
}

namespace {
__global__ void __launch_bounds__(256) scale_kernel(int64_t M, int64_t N, double beta, double* C, int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t j = idx / M, i = idx - j * M;
  C[i + j * ldc] *= beta;
}
}  // namespace

namespace {
// dst = src rounded to FP32 (and dst64 = src when given); one thread per
// element, rows contiguous.
__global__ void __launch_bounds__(256) to_f32_kernel(int64_t rows, int64_t cols, const double* __restrict__ src,
                                                     int64_t lds, float* __restrict__ dst, int64_t ldd,
                                                     double* __restrict__ dst64, int64_t ld64) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t j = idx / rows, i = idx - j * rows;
  const double v = src[i + j * lds];
  dst[i + j * ldd] = (float)v;
  if (dst64) dst64[i + j * ld64] = v;
}
}  // namespace

int launch_to_f32(hipStream_t s, int64_t rows, int64_t cols, const double* src, int64_t lds, float* dst, int64_t ldd,
                  double* dst64, int64_t ld64) {
  if (rows <= 0 || cols <= 0) return 0;
  hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)((rows * cols + 255) / 256)), dim3(256), 0, s, rows, cols, src,
                     lds, dst, ldd, dst64, ld64);
  RQ_HIP(hipGetLastError());
  return 0;
}

int launch_scale(hipStream_t s, int64_t M, int64_t N, double beta, double* C, int64_t ldc) {
  if (M <= 0 || N <= 0) return 0;
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((M * N + 255) / 256)), dim3(256), 0, s, M, N, beta, C, ldc);
  RQ_HIP(hipGetLastError());
  return 0;
}

}  // namespace rq
