// The sketch B = Omega A of Section 3 on the BF16 matrix cores, for the
// mixed-precision paths (RQ_MIXED): the sample only steers the pivot choice
// (the method already works with norms of a random projection, not the true
// column norms), so its operands are rounded to BF16 and the products
// accumulated in FP32 (v_mfma_f32_16x16x32_bf16); the result is stored in
// FP64, the precision of everything the sample QRCP does with it.
//
// Tiling: a workgroup (256 threads, four waves) owns all l <= 128 rows of
// the output and 64 of its columns (so A is read once), over a chunk of the
// reduction index m (split-K, chunks of whole 32-deep steps, a fixed-order
// reduction afterwards).  Per 32-deep step the Omega tile (128 x 32) and the
// A tile (32 x 64) are rounded to BF16 and stored in LDS with the reduction
// index contiguous, so that each MFMA operand (eight consecutive k of one
// row or column) is one 16-byte LDS read; the next step's tiles are loaded
// into registers while the current one multiplies.  A column of A (32
// consecutive values of one column) is read by four lanes with 16-byte loads
// when the pointer and leading dimension allow it.
//
// Operands are issued as (A fragment, Omega fragment), so that lane l,
// register r of an accumulator holds S(i0 + l%16, j0 + 4 (l/16) + r): sixteen
// consecutive rows of one column of the column-major output.
#include <type_traits>
#include "kernels.hpp"

namespace rq {

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int SB_M = 128;   // output rows (l <= 128)
constexpr int SB_N = 64;    // output columns per workgroup
constexpr int SB_K = 32;    // reduction depth per step
constexpr int SB_KP = 40;   // LDS row pitch in BF16 elements (80 bytes: rows land on different banks)
constexpr int SB_T = 256;

struct alignas(16) SketchLds {
  __bf16 om[2][SB_M * SB_KP];
  __bf16 a[2][SB_N * SB_KP];
};

template <typename TA>
struct ARegs;
template <>
struct ARegs<double> { double v[8]; };
template <>
struct ARegs<float> { float v[8]; };

// VEC: A's columns start on 16-byte boundaries (pointer and lda), so a
// lane's eight consecutive values are read with 16-byte loads.
template <typename TA, bool VEC>
__global__ void __launch_bounds__(SB_T) sketch_bf16_kernel(int l, int64_t n, int64_t m, const double* __restrict__ Om,
                                                           int64_t ldo, const TA* __restrict__ A, int64_t lda,
                                                           double* __restrict__ C, int64_t ldc, int64_t kchunk,
                                                           int64_t split_stride) {
  __shared__ SketchLds sm;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t j0 = (int64_t)blockIdx.x * SB_N;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = min(m, kbeg + kchunk);
  double* Cz = C + (int64_t)blockIdx.z * split_stride;
  const int tm = (l + 15) >> 4;  // 16-row tiles of the output that hold rows < l

  // Omega tile: thread -> row i = tid % 128, sixteen k (half = tid / 128)
  const int oi = tid & (SB_M - 1), oh = tid >> 7;
  // A tile: thread -> column j = tid / 4 of the tile, eight k (quarter tid % 4)
  const int aj = tid >> 2, aq = tid & 3;
  const int64_t gj = j0 + aj;

  double ro[16];
  ARegs<TA> ra;

  auto load = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int64_t k = k0 + oh * 16 + e;
      ro[e] = (oi < l && k < kend) ? Om[oi + k * ldo] : 0.0;
    }
    const int64_t kk = k0 + aq * 8;
    if (gj < n) {
      const TA* src = A + kk + gj * lda;
      if (VEC && kk + 8 <= kend) {
        if constexpr (std::is_same<TA, double>::value) {
          const double4_t* p4 = reinterpret_cast<const double4_t*>(src);
          const double4_t x = p4[0], y = p4[1];
#pragma unroll
          for (int e = 0; e < 4; ++e) { ra.v[e] = x[e]; ra.v[4 + e] = y[e]; }
        } else {
          typedef float float8_t __attribute__((ext_vector_type(8)));
          const float8_t x = *reinterpret_cast<const float8_t*>(src);
#pragma unroll
          for (int e = 0; e < 8; ++e) ra.v[e] = x[e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) ra.v[e] = (kk + e < kend) ? src[e] : (TA)0;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) ra.v[e] = (TA)0;
    }
  };
  auto store = [&](int st) {
    bf16x8_t o0, o1, a8;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      o0[e] = (__bf16)(float)ro[e];
      o1[e] = (__bf16)(float)ro[8 + e];
      a8[e] = (__bf16)(float)ra.v[e];
    }
    *reinterpret_cast<bf16x8_t*>(&sm.om[st][oi * SB_KP + oh * 16]) = o0;
    *reinterpret_cast<bf16x8_t*>(&sm.om[st][oi * SB_KP + oh * 16 + 8]) = o1;
    *reinterpret_cast<bf16x8_t*>(&sm.a[st][aj * SB_KP + aq * 8]) = a8;
  };

  f32x4_t acc[SB_M / 16];
#pragma unroll
  for (int a = 0; a < SB_M / 16; ++a) acc[a] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  if (kbeg < kend) {
    load(kbeg);
    store(0);
    __syncthreads();
    int st = 0;
    for (int64_t k0 = kbeg; k0 < kend; k0 += SB_K) {
      const bool more = k0 + SB_K < kend;
      if (more) load(k0 + SB_K);
      // this wave's 16 columns, eight consecutive k per lane
      const bf16x8_t bf = *reinterpret_cast<const bf16x8_t*>(&sm.a[st][(w * 16 + (lane & 15)) * SB_KP + 8 * (lane >> 4)]);
#pragma unroll
      for (int a = 0; a < SB_M / 16; ++a) {
        if (a < tm) {
          const bf16x8_t of =
              *reinterpret_cast<const bf16x8_t*>(&sm.om[st][(a * 16 + (lane & 15)) * SB_KP + 8 * (lane >> 4)]);
          acc[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf, of, acc[a], 0, 0, 0);
        }
      }
      if (more) store(st ^ 1);
      __syncthreads();
      st ^= 1;
    }
  }
  // lane l, register r: S(16 a + l%16, j0 + 16 w + 4 (l/16) + r)
#pragma unroll
  for (int a = 0; a < SB_M / 16; ++a) {
    if (a < tm) {
      const int i = a * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t j = j0 + w * 16 + 4 * (lane >> 4) + r;
        if (i < l && j < n) Cz[i + j * ldc] = (double)acc[a][r];
      }
    }
  }
}

// S(i, j) = sum over splits z of P[z](i, j) in a fixed order (P[z] is l x n, ld l).
__global__ void __launch_bounds__(256) sketch_reduce_kernel(int l, int64_t n, int splits, const double* __restrict__ P,
                                                            double* __restrict__ S, int64_t lds) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)l * n;
  if (idx >= total) return;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += P[(int64_t)z * total + idx];
  const int64_t j = idx / l, i = idx - j * l;
  S[i + j * lds] = s;
}

constexpr int SB_MAXS = 16;
constexpr int64_t SB_MINK = 256;

template <typename TA>
int sketch_impl(hipStream_t s, int64_t l, int64_t n, int64_t m, const double* Om, int64_t ldo, const TA* A,
                int64_t lda, double* S, int64_t lds, double* scratch, size_t scratch_elems) {
  if (l <= 0 || n <= 0) return 0;
  if (l > SB_M) return -3;
  if (m <= 0) return launch_zero_rows(s, 0, l, n, S, lds);
  // split along m toward about 2048 workgroups (eight per CU), chunks of
  // whole 32-deep steps, at least 256 deep
  const int64_t tiles = (n + SB_N - 1) / SB_N;
  int splits = 1;
  if (scratch) {
    const int64_t want = (2048 + tiles - 1) / tiles;
    splits = (int)std::max<int64_t>(1, std::min<int64_t>({want, m / SB_MINK, (int64_t)SB_MAXS}));
    while (splits > 1 && (size_t)splits * (size_t)l * (size_t)n > scratch_elems) --splits;
  }
  int64_t kchunk = (m + splits - 1) / splits;
  kchunk = (kchunk + SB_K - 1) / SB_K * SB_K;
  splits = (int)((m + kchunk - 1) / kchunk);
  constexpr size_t vec_bytes = 16;
  const bool vec = ((uintptr_t)A % vec_bytes == 0) && ((lda * (int64_t)sizeof(TA)) % (int64_t)vec_bytes == 0);
  dim3 grid((unsigned)tiles, 1, (unsigned)splits);
  double* out = splits > 1 ? scratch : S;
  const int64_t ldout = splits > 1 ? l : lds;
  const int64_t stride = splits > 1 ? l * n : 0;
  if (vec)
    hipLaunchKernelGGL((sketch_bf16_kernel<TA, true>), grid, dim3(SB_T), 0, s, (int)l, n, m, Om, ldo, A, lda, out,
                       ldout, kchunk, stride);
  else
    hipLaunchKernelGGL((sketch_bf16_kernel<TA, false>), grid, dim3(SB_T), 0, s, (int)l, n, m, Om, ldo, A, lda, out,
                       ldout, kchunk, stride);
  RQ_HIP(hipGetLastError());
  if (splits > 1) {
    const int64_t total = l * n;
    hipLaunchKernelGGL(sketch_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (int)l, n, splits,
                       (const double*)scratch, S, lds);
    RQ_HIP(hipGetLastError());
  }
  return 0;
}

}  // namespace

int launch_sketch_bf16(hipStream_t s, int64_t l, int64_t n, int64_t m, const double* Omega, int64_t ldo,
                       const double* A, int64_t lda, double* S, int64_t lds, double* scratch, size_t scratch_elems) {
  return sketch_impl<double>(s, l, n, m, Omega, ldo, A, lda, S, lds, scratch, scratch_elems);
}

int launch_sketch_bf16(hipStream_t s, int64_t l, int64_t n, int64_t m, const double* Omega, int64_t ldo,
                       const float* A, int64_t lda, double* S, int64_t lds, double* scratch, size_t scratch_elems) {
  return sketch_impl<float>(s, l, n, m, Omega, ldo, A, lda, S, lds, scratch, scratch_elems);
}

}  // namespace rq
