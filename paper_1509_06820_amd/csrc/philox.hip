// Gaussian compression matrix Omega (Section 3: i.i.d. unit-variance Gaussian
// entries; Alg. 4 and Alg. 6 draw it once per factorization).
//
// Generator: Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11),
// key (seed, key1) -- key1 = 0 for Alg. 4 and Alg. 6, key1 = J for block J of
// Alg. 5, which draws a new matrix per block; block q is the bijection of
// counter (q + 1, 0, 0, 0).
// Uniforms u = ((x >> 12) + 1/2) 2^-52 lie strictly inside (0, 1).
// Box-Muller (1958) turns words (x0, x1) into r cos(2 pi u1), r sin(2 pi u1)
// with r = sqrt(-2 ln u0), and (x2, x3) likewise.  Normal number
// t = r*m + c of the stream is Omega(r, c), so rows do not depend on l.
#include "kernels.hpp"

namespace rq {

namespace {

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox_block(uint64_t q, uint64_t seed, uint64_t key1, uint64_t out[4]) {
  uint64_t c0 = q + 1, c1 = 0, c2 = 0, c3 = 0;
  uint64_t k0 = seed, k1 = key1;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd > 0) { k0 += kW0; k1 += kW1; }
    const uint64_t lo0 = kM0 * c0, hi0 = __umul64hi(kM0, c0);
    const uint64_t lo1 = kM1 * c2, hi1 = __umul64hi(kM1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

__device__ __forceinline__ double u52(uint64_t x) {
  return ((double)(x >> 12) + 0.5) * 0x1.0p-52;
}

// One thread per Philox block (four consecutive stream positions), grid-
// stride so that any l * m fits a bounded grid.  Omega(r, c) is stored at
// out[r * rs + c * cs].
__global__ void __launch_bounds__(256) omega_kernel(uint64_t seed, uint64_t key1, int64_t l, int64_t m,
                                                     double* out, int64_t rs, int64_t cs) {
  const int64_t total = l * m;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q * 4 < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    uint64_t w[4];
    philox_block((uint64_t)q, seed, key1, w);
    const double two_pi = 2.0 * M_PI;
    double z[4];
    const double r01 = sqrt(-2.0 * log(u52(w[0])));
    const double r23 = sqrt(-2.0 * log(u52(w[2])));
    const double a01 = two_pi * u52(w[1]);
    const double a23 = two_pi * u52(w[3]);
    z[0] = r01 * cos(a01);
    z[1] = r01 * sin(a01);
    z[2] = r23 * cos(a23);
    z[3] = r23 * sin(a23);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t t = q * 4 + i;
      if (t < total) {
        const int64_t r = t / m, c = t - r * m;
        out[r * rs + c * cs] = z[i];
      }
    }
  }
}

// The same numbers for the matrices of a batch: grid.y walks the jobs.
__global__ void __launch_bounds__(256) omega_batched_kernel(const OmegaJob* __restrict__ jobs, int count) {
  for (int j = blockIdx.y; j < count; j += gridDim.y) {
    const OmegaJob jb = jobs[j];
    const int64_t total = jb.l * jb.m;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q * 4 < total;
         q += (int64_t)gridDim.x * blockDim.x) {
      uint64_t w[4];
      philox_block((uint64_t)q, jb.seed, 0, w);
      const double two_pi = 2.0 * M_PI;
      const double r01 = sqrt(-2.0 * log(u52(w[0])));
      const double r23 = sqrt(-2.0 * log(u52(w[2])));
      const double a01 = two_pi * u52(w[1]);
      const double a23 = two_pi * u52(w[3]);
      const double z[4] = {r01 * cos(a01), r01 * sin(a01), r23 * cos(a23), r23 * sin(a23)};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t t = q * 4 + i;
        if (t < total) {
          const int64_t r = t / jb.m, c = t - r * jb.m;
          jb.out[r * jb.rs + c * jb.cs] = z[i];
        }
      }
    }
  }
}

}  // namespace

int launch_omega_batched(hipStream_t s, const OmegaJob* jobs, int count, int64_t max_elems) {
  if (count <= 0 || max_elems <= 0) return 0;
  const int64_t blocks = (max_elems + 3) / 4;
  const unsigned gx = (unsigned)std::min<int64_t>((blocks + 255) / 256, 64);
  const unsigned gy = (unsigned)std::min(count, 65535);
  hipLaunchKernelGGL(omega_batched_kernel, dim3(gx, gy), dim3(256), 0, s, jobs, count);
  RQ_HIP(hipGetLastError());
  return 0;
}

int launch_omega(hipStream_t s, uint64_t seed, int64_t l, int64_t m, double* out, int64_t rs, int64_t cs,
                 uint64_t key1) {
  const int64_t blocks = (l * m + 3) / 4;
  if (blocks == 0) return 0;
  const int64_t grid = std::min<int64_t>((blocks + 255) / 256, 65536);
  hipLaunchKernelGGL(omega_kernel, dim3((unsigned)grid), dim3(256), 0, s, seed, key1, l, m, out, rs, cs);
  RQ_HIP(hipGetLastError());
  return 0;
}

}  // namespace rq
