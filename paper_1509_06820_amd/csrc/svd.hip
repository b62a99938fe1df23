// SVD of the k x k connection matrix X of TUXV (Section 6: a small SVD of X
// turns U X V^T into a truncated SVD and refines the approximation).
//
// One-sided Jacobi (Hestenes): plane rotations orthogonalise pairs of columns
// of X; the rotations are accumulated in V, so that on convergence
// X V = U Sigma.  Pairs are visited in the parallel round-robin (circle)
// order: in round r player k'-1 meets player r and players (r+i, r-i) mod
// (k'-1) meet for i = 1..k'/2-1 (k' = k rounded up to even; a pair with the
// padding player is skipped), so the k'/2 rotations of a round touch
// disjoint columns and run concurrently.  A rotation of columns (i, j) uses
// z = (b - a) / (2 g), t = sign(z) / (|z| + sqrt(1 + z^2)), c = 1/sqrt(1+t^2),
// s = c t with a = |x_i|^2, b = |x_j|^2, g = x_i . x_j, and is skipped when
// |g| <= tol sqrt(a b).  Sweeps stop after one without rotations.
// Singular values are returned in descending order with U = X V / sigma
// (a column with sigma == 0 is left zero).  The rounds of a sweep run on
// k/8 workgroups (one wave per column pair, four pairs each) that meet at an
// arrival barrier after every round (k < 128 and k > 576; in between, the
// block kernel below).
#include "kernels.hpp"

namespace rq {

namespace {

constexpr int SVD_THREADS = 1024;

__device__ __forceinline__ void rr_pair(int r, int idx, int kk, int& p, int& q) {
  const int n1 = kk - 1;
  if (idx == 0) {
    p = kk - 1;
    q = r;
  } else {
    p = (r + idx) % n1;
    q = (r - idx + n1) % n1;
  }
}

// Rotation sweeps spread over P workgroups (all resident at once): in each
// round wave w of workgroup me takes pairs idx = 4 me + w, 4 me + w + 4 P,
// ... of the round-robin order, and the workgroups meet at an arrival
// barrier before the next round reads the rotated columns.  A wave that
// rotated during the sweep marks the sweep's flag; after the sweep's last
// barrier every workgroup reads it, so all of them stop after the same sweep.
// flags[0]: arrival counter, flags[1 + s]: sweep s rotated (zeroed by the
// caller).  A last sweep that still rotated sets the error word to 2 (no
// convergence within max_sweeps) unless an earlier failure set it.
constexpr int JW_T = 256;             // threads of a sweep workgroup: four waves, one column pair each
constexpr int JW_PAIRS = JW_T / WAVE;  // column pairs a workgroup rotates at once
constexpr int JW_MAXK = 1024;

__device__ bool jw_barrier(unsigned* flags, int P, unsigned round, int* err) {
  __shared__ int s_bad;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x < WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (threadIdx.x == 0) {
      __hip_atomic_fetch_add(&flags[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned target = round * (unsigned)P;
      long spins = 0;
      int bad = 0;
      while (__hip_atomic_load(&flags[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++spins > SPIN_LIMIT) { bad = 1; atomicExch(err, 1); break; }
        __builtin_amdgcn_s_sleep(1);
      }
      s_bad = bad;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(s_bad) == 0;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Each wave rotates one column pair of the round (RPT rows per lane, the
// three inner products reduced within the wave by xor butterflies, no LDS), so a workgroup
// handles four pairs and the round's k/2 pairs need k/8 workgroups; a wave
// that rotated anything during a sweep sets that sweep's flag once, just
// before the sweep's last barrier.
template <int RPT>
__global__ void __launch_bounds__(JW_T) jacobi_sweeps_kernel(int k, double* X, int64_t ldx, double* V, int64_t ldv,
                                                              double tol, int max_sweeps, unsigned* flags, int* err) {
  if (earlier_failure(err)) return;
  const int P = gridDim.x, lane = threadIdx.x & (WAVE - 1);
  const int slot = blockIdx.x * JW_PAIRS + (int)(threadIdx.x / WAVE), nslots = P * JW_PAIRS;
  const int kk = k + (k & 1), npairs = kk / 2;
  unsigned round = 0;
  for (int sweep = 0; sweep < max_sweeps && kk > 1; ++sweep) {
    bool rotated = false;
    for (int r = 0; r < kk - 1; ++r) {
      for (int idx = slot; idx < npairs; idx += nslots) {
        int p, q;
        rr_pair(r, idx, kk, p, q);
        if (p >= k || q >= k) continue;
        const int i = min(p, q), j = max(p, q);
        double* xi = X + (int64_t)i * ldx;
        double* xj = X + (int64_t)j * ldx;
        double* vi = V + (int64_t)i * ldv;
        double* vj = V + (int64_t)j * ldv;
        // the pair's columns of X and V are all read up front (one memory
        // round trip per round)
        double u[RPT], v[RPT], a2[RPT], b2[RPT];
#pragma unroll
        for (int e = 0; e < RPT; ++e) {
          const int row = lane + e * WAVE;
          const bool in = row < k;
          u[e] = in ? xi[row] : 0.0;
          v[e] = in ? xj[row] : 0.0;
          a2[e] = in ? vi[row] : 0.0;
          b2[e] = in ? vj[row] : 0.0;
        }
        double sa = 0.0, sb = 0.0, sg = 0.0;
#pragma unroll
        for (int e = 0; e < RPT; ++e) {
          sa = fma(u[e], u[e], sa);
          sb = fma(v[e], v[e], sb);
          sg = fma(u[e], v[e], sg);
        }
        sa = wave_sum_x(sa);
        sb = wave_sum_x(sb);
        sg = wave_sum_x(sg);
        if (sg != 0.0 && fabs(sg) > tol * sqrt(sa * sb)) {
          double cs, sn_;
          jacobi_rotation(sa, sb, sg, cs, sn_);
#pragma unroll
          for (int e = 0; e < RPT; ++e) {
            const int row = lane + e * WAVE;
            if (row < k) {
              xi[row] = cs * u[e] - sn_ * v[e];
              xj[row] = sn_ * u[e] + cs * v[e];
              vi[row] = cs * a2[e] - sn_ * b2[e];
              vj[row] = sn_ * a2[e] + cs * b2[e];
            }
          }
          rotated = true;
        }
      }
      if (r == kk - 2 && rotated && lane == 0) atomicOr(&flags[1 + sweep], 1u);
      if (!jw_barrier(flags, P, ++round, err)) return;
    }
    const unsigned rot = __hip_atomic_load(&flags[1 + sweep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__builtin_amdgcn_readfirstlane(rot) == 0u) break;
    if (sweep == max_sweeps - 1 && blockIdx.x == 0 && threadIdx.x == 0) atomicCAS(err, 0, 2);
  }
}

// ---------------------------------------------------------------- block Jacobi
// For larger k the rounds above cost a device-wide barrier each (k - 1 per
// sweep), which dominates.  The block variant splits the columns into nb
// blocks of BW and pairs the blocks in the same round-robin order: in each
// outer round workgroup g takes block pair (I, J), copies those 2 BW columns
// of X and of V into LDS, rotates column pairs there (a group of
// G = 512 / BW lanes per pair, BW pairs at a time, a workgroup barrier
// between inner rounds) and writes both back; the workgroups meet at a
// device-wide barrier after each outer round only (nb - 1 per sweep).  Each
// column pair is rotated once per sweep, as in the round kernel: the pairs
// inside a block in the sweep's first outer round (where every block meets
// one other: the full round-robin over the 2 BW columns), the pairs across
// I and J in the round where I and J meet (BW inner rounds, column l of I
// with column (l + s) mod BW of J).  Running full round-robin sweeps over
// the 2 BW columns in every outer round instead rotated each column 2 BW - 1
// times per round and cost V twice the loss of orthogonality.  Every
// rotation is the scalar one (same formulas, same threshold); a sweep in
// which no workgroup rotated ends the iteration.
constexpr int BJ_T = 512;
constexpr size_t BJ_LDS_MAX = 150 * 1024;
constexpr int BJ_MINK = 128;  // smaller k: the round kernel (few rounds, cheap barriers)

template <int G>
__device__ __forceinline__ double group_sum(double v) {
  const int lane = (int)(threadIdx.x & (WAVE - 1));
  if constexpr (G >= 2) v += xchg_d<1>(v, lane);
  if constexpr (G >= 4) v += xchg_d<2>(v, lane);
  if constexpr (G >= 8) v += xchg_d<4>(v, lane);
  if constexpr (G >= 16) v += xchg_d<8>(v, lane);
  if constexpr (G >= 32) v += xchg_d<16>(v, lane);
  if constexpr (G >= 64) v += xchg_d<32>(v, lane);
  return v;
}

// LDS of a block pair: 2 BW columns of X and of V, kpad = RPL * (512 / BW)
// rows each (rows past k zero), pitch kpad + 1.
template <int BW, int RPL>
constexpr size_t bj_lds_bytes() {
  return (size_t)2 * (2 * BW) * (RPL * (BJ_T / BW) + 1) * sizeof(double);
}

// BW columns per block, RPL rows per lane in an inner round (k <= RPL * G).
template <int BW, int RPL>
__global__ void __launch_bounds__(BJ_T) jacobi_block_kernel(int k, double* X, int64_t ldx, double* V, int64_t ldv,
                                                             double tol, int max_sweeps, unsigned* flags, int* err) {
  constexpr int C2 = 2 * BW;            // columns held by a workgroup
  constexpr int G = BJ_T / BW;          // lanes per column pair in an inner round
  constexpr int KPAD = RPL * G;         // rows held per column (zero past k)
  constexpr int KP = KPAD + 1;          // LDS pitch
  static_assert(G <= WAVE && (G & (G - 1)) == 0, "group within a wave");
  static_assert(bj_lds_bytes<BW, RPL>() <= BJ_LDS_MAX, "LDS budget");
  extern __shared__ __align__(16) double bj_smem[];
  double* Xs = bj_smem;                 // C2 columns of X
  double* Vs = bj_smem + (size_t)C2 * KP;  // the same columns of V
  __shared__ int s_rot;
  if (earlier_failure(err)) return;
  const int tid = threadIdx.x, P = gridDim.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int nb = 2 * P;                 // blocks (the last ones may be partly or wholly padding)
  const int pi = tid / G, gl = tid % G; // inner pair slot and lane within its group
  unsigned round = 0;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    bool any = false;
    for (int r = 0; r < nb - 1; ++r) {
      int bi, bj;
      rr_pair(r, blockIdx.x, nb, bi, bj);
      auto gcol = [&](int l) { return (l < BW) ? bi * BW + l : bj * BW + (l - BW); };
      // the two blocks' columns of X and V into LDS: wave w takes columns
      // w, w + 8, ..., a lane per row (coalesced), zeros past k; all of a
      // lane's loads are issued before the first LDS store
      {
        constexpr int NCW = C2 / (BJ_T / WAVE);     // columns per wave
        constexpr int NRC = (KPAD + WAVE - 1) / WAVE;  // row chunks per column
        double lx[NCW][NRC], lv[NCW][NRC];
#pragma unroll
        for (int cc = 0; cc < NCW; ++cc) {
          const int c = gcol(wv + cc * (BJ_T / WAVE));
          const bool cin = c < k;
          const double* xc = X + (int64_t)(cin ? c : 0) * ldx;
          const double* vc = V + (int64_t)(cin ? c : 0) * ldv;
#pragma unroll
          for (int h = 0; h < NRC; ++h) {
            const int row = lane + h * WAVE;
            const bool in = cin && row < k;
            lx[cc][h] = in ? xc[row] : 0.0;
            lv[cc][h] = in ? vc[row] : 0.0;
          }
        }
#pragma unroll
        for (int cc = 0; cc < NCW; ++cc) {
          const int l = wv + cc * (BJ_T / WAVE);
#pragma unroll
          for (int h = 0; h < NRC; ++h) {
            const int row = lane + h * WAVE;
            if (row < KPAD) {
              Xs[l * KP + row] = lx[cc][h];
              Vs[l * KP + row] = lv[cc][h];
            }
          }
        }
      }
      if (tid == 0) s_rot = 0;
      __syncthreads();
      auto rotate_if = [&](double (&u)[RPL], double (&v)[RPL], double (&a2)[RPL], double (&b2)[RPL])
          __attribute__((always_inline)) {
        double sa = 0.0, sb = 0.0, sg = 0.0;
#pragma unroll
        for (int e = 0; e < RPL; ++e) {
          sa = fma(u[e], u[e], sa);
          sb = fma(v[e], v[e], sb);
          sg = fma(u[e], v[e], sg);
        }
        sa = group_sum<G>(sa);
        sb = group_sum<G>(sb);
        sg = group_sum<G>(sg);
        if (sg != 0.0 && fabs(sg) > tol * sqrt(sa * sb)) {
          double cs, sn_;
          jacobi_rotation(sa, sb, sg, cs, sn_);
#pragma unroll
          for (int e = 0; e < RPL; ++e) {
            const double x1 = u[e], x2 = v[e], y1 = a2[e], y2 = b2[e];
            u[e] = cs * x1 - sn_ * x2;
            v[e] = sn_ * x1 + cs * x2;
            a2[e] = cs * y1 - sn_ * y2;
            b2[e] = sn_ * y1 + cs * y2;
          }
          if (gl == 0) s_rot = 1;
          return true;
        }
        return false;
      };
      if (r == 0) {
        // every pair of the 2 BW columns once (round-robin), from LDS
        for (int ir = 0; ir < C2 - 1; ++ir) {
          int p, q;
          rr_pair(ir, pi, C2, p, q);
          const int i = min(p, q), j = max(p, q);
          double* xi = Xs + i * KP + gl;
          double* xj = Xs + j * KP + gl;
          double* vi = Vs + i * KP + gl;
          double* vj = Vs + j * KP + gl;
          double u[RPL], v[RPL], a2[RPL], b2[RPL];
#pragma unroll
          for (int e = 0; e < RPL; ++e) {
            u[e] = xi[G * e];
            v[e] = xj[G * e];
            a2[e] = vi[G * e];
            b2[e] = vj[G * e];
          }
          if (rotate_if(u, v, a2, b2)) {
#pragma unroll
            for (int e = 0; e < RPL; ++e) {
              xi[G * e] = u[e];
              xj[G * e] = v[e];
              vi[G * e] = a2[e];
              vj[G * e] = b2[e];
            }
          }
          __syncthreads();
        }
      } else {
        // column pi of I against column (pi + s) mod BW of J, s = 0..BW-1:
        // the group keeps its column of I in registers and reads and writes
        // only the J columns in LDS
        double u[RPL], a2[RPL];
        {
          const double* xi = Xs + pi * KP + gl;
          const double* vi = Vs + pi * KP + gl;
#pragma unroll
          for (int e = 0; e < RPL; ++e) {
            u[e] = xi[G * e];
            a2[e] = vi[G * e];
          }
        }
        for (int ir = 0; ir < BW; ++ir) {
          const int j = BW + ((pi + ir) & (BW - 1));
          double* xj = Xs + j * KP + gl;
          double* vj = Vs + j * KP + gl;
          double v[RPL], b2[RPL];
#pragma unroll
          for (int e = 0; e < RPL; ++e) {
            v[e] = xj[G * e];
            b2[e] = vj[G * e];
          }
          if (rotate_if(u, v, a2, b2)) {
#pragma unroll
            for (int e = 0; e < RPL; ++e) {
              xj[G * e] = v[e];
              vj[G * e] = b2[e];
            }
          }
          __syncthreads();
        }
        double* xi = Xs + pi * KP + gl;
        double* vi = Vs + pi * KP + gl;
#pragma unroll
        for (int e = 0; e < RPL; ++e) {
          xi[G * e] = u[e];
          vi[G * e] = a2[e];
        }
        __syncthreads();
      }
      if (s_rot) any = true;
      // the columns back to X and V
      for (int l = wv; l < C2; l += BJ_T / WAVE) {
        const int c = gcol(l);
        if (c < k) {
          double* xc = X + (int64_t)c * ldx;
          double* vc = V + (int64_t)c * ldv;
#pragma unroll
          for (int row = lane; row < KPAD; row += WAVE) {
            if (row < k) {
              xc[row] = Xs[l * KP + row];
              vc[row] = Vs[l * KP + row];
            }
          }
        }
      }
      if (r == nb - 2 && any && tid == 0) atomicOr(&flags[1 + sweep], 1u);
      if (!jw_barrier(flags, P, ++round, err)) return;
    }
    const unsigned rot = __hip_atomic_load(&flags[1 + sweep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__builtin_amdgcn_readfirstlane(rot) == 0u) break;
    if (sweep == max_sweeps - 1 && blockIdx.x == 0 && threadIdx.x == 0) atomicCAS(err, 0, 2);
  }
}

// Launch of the block kernel for BW, RPL (RPL * 512 / BW >= k).
template <int BW, int RPL>
int launch_bj(hipStream_t s, int k, double* X, int64_t ldx, double* V, int64_t ldv, int max_sweeps, unsigned* flags,
              int* err) {
  constexpr size_t lds = bj_lds_bytes<BW, RPL>();
  int nb = (k + BW - 1) / BW;
  nb += nb & 1;
  const int P = nb / 2;
  static int res = 0;
  auto kern = jacobi_block_kernel<BW, RPL>;
  const void* fn = (const void*)kern;
  if (!res) {
    RQ_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int occ = 0, dev = 0, cus = 0;
    RQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, BJ_T, lds));
    RQ_HIP(hipGetDevice(&dev));
    RQ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    res = std::max(1, occ * cus);
  }
  if (P > res) return RQ_ERR_HIP_BASE + (int)hipErrorCooperativeLaunchTooLarge;
  hipLaunchKernelGGL(kern, dim3(P), dim3(BJ_T), lds, s, k, X, ldx, V, ldv, 1e-15, max_sweeps, flags, err);
  RQ_HIP(hipGetLastError());
  return 0;
}

// The block kernel for this k (RPL = rows per lane), or 1 when k is outside
// its range (the round kernel then runs).
int dispatch_bj(hipStream_t s, int k, double* X, int64_t ldx, double* V, int64_t ldv, int max_sweeps,
                unsigned* flags, int* err) {
  if (k < BJ_MINK) return 1;
  if (k <= 9 * 32) {  // blocks of 16 columns, 32 lanes per pair
    switch ((k + 31) / 32) {
      case 4: return launch_bj<16, 4>(s, k, X, ldx, V, ldv, max_sweeps, flags, err);
      case 5: return launch_bj<16, 5>(s, k, X, ldx, V, ldv, max_sweeps, flags, err);
      case 6: return launch_bj<16, 6>(s, k, X, ldx, V, ldv, max_sweeps, flags, err);
      case 7: return launch_bj<16, 7>(s, k, X, ldx, V, ldv, max_sweeps, flags, err);
      case 8: return launch_bj<16, 8>(s, k, X, ldx, V, ldv, max_sweeps, flags, err);
      default: return launch_bj<16, 9>(s, k, X, ldx, V, ldv, max_sweeps, flags, err);
    }
  }
  if (k <= 9 * 64) {  // blocks of 8 columns, 64 lanes per pair
    switch ((k + 63) / 64) {
      case 5: return launch_bj<8, 5>(s, k, X, ldx, V, ldv, max_sweeps, flags, err);
      case 6: return launch_bj<8, 6>(s, k, X, ldx, V, ldv, max_sweeps, flags, err);
      case 7: return launch_bj<8, 7>(s, k, X, ldx, V, ldv, max_sweeps, flags, err);
      case 8: return launch_bj<8, 8>(s, k, X, ldx, V, ldv, max_sweeps, flags, err);
      default: return launch_bj<8, 9>(s, k, X, ldx, V, ldv, max_sweeps, flags, err);
    }
  }
  return 1;
}

// Column norms of the rotated X, singular values in descending order (ties
// by index), U = X V / sigma (a column with sigma == 0 is left zero).
__global__ void __launch_bounds__(SVD_THREADS) jacobi_finish_kernel(int k, const double* X, int64_t ldx,
                                                                     const double* V, int64_t ldv, double* U,
                                                                     int64_t ldu, double* sigma, double* Vout,
                                                                     int64_t ldvo, const int* err) {
  __shared__ double sn[1024];
  const int tid = threadIdx.x;
  for (int j = tid / WAVE; j < k; j += SVD_THREADS / WAVE) {
    const double* xj = X + (int64_t)j * ldx;
    double s = 0.0;
    for (int row = tid & (WAVE - 1); row < k; row += WAVE) s += xj[row] * xj[row];
    s = wave_sum(s);
    if ((tid & (WAVE - 1)) == 0) sn[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < k; j += SVD_THREADS) {
    const double v = sn[j];
    int rank = 0;
    for (int i = 0; i < k; ++i) rank += (sn[i] > v || (sn[i] == v && i < j)) ? 1 : 0;
    sigma[rank] = v;
    const double inv = (v > 0.0) ? 1.0 / v : 0.0;
    for (int row = 0; row < k; ++row) {
      U[row + (int64_t)rank * ldu] = X[row + (int64_t)j * ldx] * inv;
      Vout[row + (int64_t)rank * ldvo] = V[row + (int64_t)j * ldv];
    }
  }
}

__global__ void identity_kernel(int k, double* V, int64_t ldv, unsigned* flags, int nflags) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (int64_t)k * k) {
    const int64_t j = e / k, i = e - j * k;
    V[i + j * ldv] = (i == j) ? 1.0 : 0.0;
  }
  if (e < nflags) flags[e] = 0u;
}

}  // namespace

int launch_jacobi_svd(hipStream_t s, int k, double* X, int64_t ldx, double* U, int64_t ldu, double* sigma, double* V,
                      int64_t ldv, const SvdWork& w) {
  if (k <= 0) return 0;
  if (k > JW_MAXK) return -3;
  if (!w.flags || !w.err) return -3;
  constexpr int MAX_SWEEPS = 60;
  // w.tmp holds the accumulated rotations (k x k)
  const int64_t ke = (int64_t)k * k;
  const int nflags = 1 + MAX_SWEEPS;
  hipLaunchKernelGGL(identity_kernel, dim3((unsigned)((std::max<int64_t>(ke, nflags) + 255) / 256)), dim3(256), 0, s,
                     k, w.tmp, (int64_t)k, w.flags, nflags);
  RQ_HIP(hipGetLastError());
  {
    const int rc = dispatch_bj(s, k, X, ldx, w.tmp, (int64_t)k, MAX_SWEEPS, w.flags, w.err);
    if (rc <= 0) {
      if (rc < 0) return rc;
      hipLaunchKernelGGL(jacobi_finish_kernel, dim3(1), dim3(SVD_THREADS), 0, s, k, (const double*)X, ldx,
                         (const double*)w.tmp, (int64_t)k, U, ldu, sigma, V, ldv, (const int*)w.err);
      RQ_HIP(hipGetLastError());
      return 0;
    }
  }
  const int kk = k + (k & 1);
  // one wave per column pair of a round, four per workgroup
  int P = std::max(1, (kk / 2 + JW_PAIRS - 1) / JW_PAIRS);
  double tol = 1e-15;
  int ksw = k;
  int64_t ldt = k;
  int maxs = MAX_SWEEPS;
  static_assert(16 * WAVE >= JW_MAXK, "rows per lane");
  // An ordinary launch after a residency check (occupancy of one CU times
  // the CU count; at most k/8 = 128 workgroups of 256 threads): the
  // workgroups wait on each other at the round barriers, whose waits are
  // bounded, so a workgroup held back by other work makes the call report
  // info = -1 instead of hanging.
  static int resident[3] = {0, 0, 0};
  const int which = (k <= 4 * WAVE) ? 0 : (k <= 8 * WAVE) ? 1 : 2;
  const void* fns[3] = {(const void*)jacobi_sweeps_kernel<4>, (const void*)jacobi_sweeps_kernel<8>,
                        (const void*)jacobi_sweeps_kernel<16>};
  if (!resident[which]) {
    int occ = 0, dev = 0, cus = 0;
    RQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fns[which], JW_T, 0));
    RQ_HIP(hipGetDevice(&dev));
    RQ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    resident[which] = std::max(1, occ * cus);
  }
  if (P > resident[which]) return RQ_ERR_HIP_BASE + (int)hipErrorCooperativeLaunchTooLarge;
  if (which == 0)
    hipLaunchKernelGGL(jacobi_sweeps_kernel<4>, dim3(P), dim3(JW_T), 0, s, ksw, X, ldx, w.tmp, ldt, tol, maxs,
                       w.flags, w.err);
  else if (which == 1)
    hipLaunchKernelGGL(jacobi_sweeps_kernel<8>, dim3(P), dim3(JW_T), 0, s, ksw, X, ldx, w.tmp, ldt, tol, maxs,
                       w.flags, w.err);
  else
    hipLaunchKernelGGL(jacobi_sweeps_kernel<16>, dim3(P), dim3(JW_T), 0, s, ksw, X, ldx, w.tmp, ldt, tol, maxs,
                       w.flags, w.err);
  RQ_HIP(hipGetLastError());
  hipLaunchKernelGGL(jacobi_finish_kernel, dim3(1), dim3(SVD_THREADS), 0, s, k, (const double*)X, ldx,
                     (const double*)w.tmp, (int64_t)k, U, ldu, sigma, V, ldv, (const int*)w.err);
  RQ_HIP(hipGetLastError());
  return 0;
}

}  // namespace rq
