// Shared device/host helpers for the gfx950 RQRCP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace rq {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int WAVE = 64;

// Error codes returned by the C ABI (negative: bad argument index, LAPACK style).
constexpr int RQ_ERR_HIP_BASE = 1000;   // hipError_t + 1000
constexpr int RQ_ERR_COOP = 2001;       // cooperative launch rejected (grid does not fit)

#define RQ_HIP(call)                                                   \
  do {                                                                 \
    hipError_t _e = (call);                                            \
    if (_e != hipSuccess) return ::rq::RQ_ERR_HIP_BASE + (int)_e;      \
  } while (0)

#define RQ_TRY_RAW(x)        \
  do {                       \
    int _rc = (x);           \
    if (_rc) return _rc;     \
  } while (0)

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Value of lane ^ STRIDE (STRIDE a power of two below 64) without LDS: DPP
// within rows of 16 lanes, gfx950 permlane swaps across rows and halves
// (with both operands equal, result 1 holds the partner row's value in the
// even rows and result 0 in the odd rows).
template <int STRIDE>
__device__ __forceinline__ int xchg_i(int v, int lane) {
  if constexpr (STRIDE == 1) {
    return __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  } else if constexpr (STRIDE == 2) {
    return __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  } else if constexpr (STRIDE == 4) {
    const int up = __builtin_amdgcn_update_dpp(v, v, 0x104, 0xF, 0xF, false);   // row_shl:4 (lane + 4)
    const int dn = __builtin_amdgcn_update_dpp(v, v, 0x114, 0xF, 0xF, false);   // row_shr:4 (lane - 4)
    return (lane & 4) ? dn : up;
  } else if constexpr (STRIDE == 8) {
    return __builtin_amdgcn_update_dpp(v, v, 0x128, 0xF, 0xF, false);  // row_ror:8
  } else if constexpr (STRIDE == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (lane & 16) ? (int)r[0] : (int)r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (lane & 32) ? (int)r[0] : (int)r[1];
  }
}
template <int STRIDE>
__device__ __forceinline__ double xchg_d(double v, int lane) {
  return __hiloint2double(xchg_i<STRIDE>(__double2hiint(v), lane), xchg_i<STRIDE>(__double2loint(v), lane));
}

// Sum over the wave by xor butterflies (DPP and permlane exchanges, no LDS):
// every lane ends with the same bits, since each step adds the same pair in
// either order.
__device__ __forceinline__ double wave_sum_x(double v) {
  const int lane = (int)(threadIdx.x & (WAVE - 1));
  v += xchg_d<1>(v, lane);
  v += xchg_d<2>(v, lane);
  v += xchg_d<4>(v, lane);
  v += xchg_d<8>(v, lane);
  v += xchg_d<16>(v, lane);
  v += xchg_d<32>(v, lane);
  return v;
}

// (value, position) ranking used for pivot selection: larger value wins,
// ties go to the lower position.  NaN values must be mapped to -1 before.
__device__ __forceinline__ bool rank_better(double v1, long p1, double v2, long p2) {
  return (v1 > v2) || (v1 == v2 && p1 < p2);
}

__device__ __forceinline__ void wave_argmax(double& v, long& p) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    double ov = __shfl_xor(v, off, WAVE);
    long op = __shfl_xor(p, off, WAVE);
    if (rank_better(ov, op, v, p)) { v = ov; p = op; }
  }
}

// ---------------------------------------------------------------- cross-WG exchange
// Workgroups of one cooperative launch exchange data through global memory.
// A publisher writes its payload; every wave waits until its stores are
// acknowledged, the workgroup synchronises, and wave 0 issues one
// agent-scope release fence (write-back of the L2 for the other XCDs) before
// thread 0 stores the epoch into its flag.  A consumer's wave 0 polls the
// flags (one lane per flag) with agent-scope atomic loads and issues one
// agent-scope acquire fence (invalidation of this CU's L1 and of stale L2
// lines) before the workgroup synchronises, so every wave then reads the
// payload from memory.  Only one wave per workgroup pays for the cache
// maintenance.  Waits are bounded: after SPIN_LIMIT polls the wait fails, the
// error word is set and the caller returns, so a broken exchange ends the
// kernel instead of hanging it.
constexpr long SPIN_LIMIT = 1L << 20;

// Jacobi rotation of a column pair with squared norms a, b and inner
// product g (Rutishauser's form): z = (b - a) / (2 g),
// t = sign(z) / (|z| + sqrt(1 + z^2)), c = 1 / sqrt(1 + t^2), s = c t.
// The quotients and square roots use the hardware reciprocal and
// reciprocal-square-root estimates refined by two Newton steps each (a few
// ulps, which the rotation's own rounding dwarfs), so the dependent chain
// is a couple of dozen FMAs instead of the long expansions of the correctly
// rounded operations.  For |z| > 1e150 (1 + z^2 would overflow)
// t = 1 / (2 z) to working accuracy.
__device__ __forceinline__ double jr_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double jr_rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}
__device__ __forceinline__ void jacobi_rotation(double a, double b, double g, double& c, double& s) {
  const double z = (b - a) * jr_rcp(2.0 * g);
  const double az = fabs(z);
  double t;
  if (az > 1e150) {
    t = 0.5 * jr_rcp(z);
  } else {
    const double q = fma(z, z, 1.0);
    const double sq = q * jr_rsqrt(q);
    t = jr_rcp(az + sq);
    t = (z >= 0.0) ? t : -t;
  }
  c = jr_rsqrt(fma(t, t, 1.0));
  s = c * t;
}

// A cooperative kernel starts by checking the error word: once one stage has
// timed out, the later stages of the same call return at once.
// Thread 0 reads the word and broadcasts it, so the whole workgroup takes
// the same branch.
__device__ __forceinline__ bool earlier_failure(const int* err) {
  __shared__ int s_fail;
  if (threadIdx.x == 0) s_fail = __hip_atomic_load((int*)err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(s_fail) != 0;
}

__device__ __forceinline__ void publish_flag(unsigned* flags, int me, unsigned epoch) {
  // every wave waits for its own stores to be acknowledged ...
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // ... then one wave writes the cache back device-wide and raises the flag
  if (threadIdx.x < WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (threadIdx.x == 0) __hip_atomic_store(&flags[me], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Wait until flags[q] >= epoch for q in [0, P).  Returns false on timeout.
__device__ __forceinline__ bool wait_flags(const unsigned* flags, int P, unsigned epoch, int* err) {
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  if (threadIdx.x < WAVE) {
    long spins = 0;
    for (int base = 0; base < P; base += WAVE) {
      int q = base + (int)threadIdx.x;
      bool done = false;
      while (!done) {
        unsigned f = (q < P) ? __hip_atomic_load((unsigned*)&flags[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : epoch;
        done = __all(f >= epoch);
        if (!done) {
          if (++spins > SPIN_LIMIT) {
            if (threadIdx.x == 0) { s_bad = 1; atomicExch(err, 1); }
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      if (!done) break;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  // the acquire above invalidated this CU's caches; the barrier orders the
  // other waves' reads after it
  __syncthreads();
  return s_bad == 0;
}

// Wait for one flag to reach `epoch`; the flag's value is returned in *seen.
__device__ __forceinline__ bool wait_one(const unsigned* flag, unsigned epoch, int* err, unsigned* seen) {
  __shared__ int s_bad;
  __shared__ unsigned s_seen;
  if (threadIdx.x == 0) {
    s_bad = 0;
    long spins = 0;
    unsigned f;
    while ((f = __hip_atomic_load((unsigned*)flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < epoch) {
      if (++spins > SPIN_LIMIT) { s_bad = 1; atomicExch(err, 1); break; }
      __builtin_amdgcn_s_sleep(1);
    }
    s_seen = f;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (seen) *seen = s_seen;
  return s_bad == 0;
}

// ---------------------------------------------------------------- host helpers
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over the caller's workspace (host side bookkeeping only).
struct Carve {
  char* base;
  size_t off;
  size_t cap;
  bool ok;
  explicit Carve(void* b, size_t c) : base((char*)b), off(0), cap(c), ok(true) {}
  // A request whose size overflows size_t saturates `off` (and fails `ok`),
  // so a size query can never wrap round to a small number.
  template <class T>
  T* take(size_t count) {
    constexpr size_t kMax = ~(size_t)0 - 511;
    size_t bytes = 0;
    if (off > kMax || __builtin_mul_overflow(count, sizeof(T), &bytes) || bytes > kMax - align_up(off, 256)) {
      off = ~(size_t)0;
      ok = false;
      return nullptr;
    }
    size_t o = align_up(off, 256);
    bytes = align_up(bytes, 256);
    off = o + bytes;
    if (off > cap) ok = false;
    return base ? (T*)(base + o) : nullptr;
  }
  bool overflowed() const { return off == ~(size_t)0; }
};
// p + k for a carved pointer: stays null in a size query (no arithmetic on null)
template <class T>
inline T* carved_at(T* p, size_t k) {
  return p ? p + k : nullptr;
}

}  // namespace rq
