// Householder QR of an mJ x bJ panel (the "qr" step of Alg. 4 / Alg. 6 on the
// b selected columns), in place in the LAPACK layout: R on and above the
// diagonal, reflector tails below it, tau per column; the explicit unit-lower
// reflector block Y is written as well for the block-reflector products.
//
// One launch (see launch_panel).  Workgroup q owns rows [256 q, 256 q + 256) of the
// panel in registers (thread = one column x 32 rows).  For column j every
// workgroup forms its partial inner products of column j with columns j..bJ-1
// over its rows below j, publishes them (plus row j if it owns it), and after
// one exchange every workgroup adds the partials in the same order, builds
// the same reflector (LAPACK dlarfg normalisation) and updates its rows.
#include "kernels.hpp"

namespace rq {

namespace {

constexpr int PN_THREADS = 512;
constexpr int PN_RPT = 32;
constexpr int PN_GROUPS = PN_THREADS / 64;
constexpr int PN_RB = PN_GROUPS * PN_RPT;  // 256 rows per workgroup

struct PanelParams {
  double* P;
  int64_t ldp;
  int64_t mJ;
  int bJ;
  double* tau;
  double* Y;
  int64_t ldy;
  double* slots;    // bJ * NP * 64 partial sums
  double* rowslot;  // bJ * 64 values of row j
  unsigned* flags;
  int* err;
  const int* gate;
  int copy_y;  // with gate: a launch whose gate is 0 copies Y(bJ:mJ, :) into P
  int NP;
};

// Rows per workgroup of the copy of Y(b:mJ, :) into P(b:mJ, :).
constexpr int CP_ROWS = 64;

// Y -> P for rows [r0, r1) (r0 >= b, r1 - r0 <= CP_ROWS), by the NT threads
// of one workgroup, consecutive threads on consecutive rows; every load of
// the thread is issued before its first store.
template <int NT>
__device__ __forceinline__ void copy_y_rows(const PanelParams& a, int64_t r0, int64_t r1) {
  constexpr int PER = CP_ROWS * 64 / NT;
  const int rows = (int)(r1 - r0);  // at most CP_ROWS
  if (rows <= 0) return;
  const int tot = rows * a.bJ;
  double v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = (int)threadIdx.x + q * NT;
    const int j = e / rows, i = e - j * rows;
    v[q] = (e < tot) ? a.Y[r0 + i + j * a.ldy] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = (int)threadIdx.x + q * NT;
    const int j = e / rows, i = e - j * rows;
    if (e < tot) a.P[r0 + i + j * a.ldp] = v[q];
  }
}

// The copy alone, for panels too tall for the column panel's grid: runs only
// if *gate is 0.
__global__ void __launch_bounds__(256) ycopy_gated_kernel(PanelParams a) {
  __shared__ int s_gate;
  if (threadIdx.x == 0) s_gate = *a.gate;
  __syncthreads();
  if (s_gate != 0) return;
  const int64_t q = blockIdx.x;
  copy_y_rows<256>(a, std::max<int64_t>(q * CP_ROWS, a.bJ), std::min<int64_t>(a.mJ, q * CP_ROWS + CP_ROWS));
}

__global__ void __launch_bounds__(PN_THREADS) panel_kernel(PanelParams a) {
  __shared__ double xs[PN_RB];
  __shared__ double part[PN_GROUPS][64];
  __shared__ double rowj[64];
  __shared__ double dsum[64], rowv[64], wv[64];
  __shared__ double hh[4];
  const int tid = threadIdx.x, c = tid & 63, g = tid >> 6;
  const int me = blockIdx.x;
  // row indices fit in 32 bits (mJ < 2^31 is checked by the launcher)
  const int mJ = (int)a.mJ;
  const int r0 = me * PN_RB + g * PN_RPT;
  const int wlo = me * PN_RB;
  const int whi = min(mJ, wlo + PN_RB);
  const int bJ = a.bJ;
  if (a.gate) {
    __shared__ int s_gate;
    if (threadIdx.x == 0) s_gate = *a.gate;
    __syncthreads();
    if (s_gate == 0) {  // the CholeskyQR panel succeeded: workgroup q copies its CP_ROWS rows
      const int64_t q = me;
      if (a.copy_y)
        copy_y_rows<PN_THREADS>(a, std::max<int64_t>(q * CP_ROWS, bJ), std::min<int64_t>(a.mJ, q * CP_ROWS + CP_ROWS));
      return;
    }
  }
  if (me >= a.NP) return;  // workgroups beyond the column panel's (they serve the copy)
  if (earlier_failure(a.err)) return;

  double v[PN_RPT];
#pragma unroll
  for (int rr = 0; rr < PN_RPT; ++rr) {
    const int row = r0 + rr;
    v[rr] = (row < mJ && c < bJ) ? a.P[row + c * a.ldp] : 0.0;
  }

  for (int j = 0; j < bJ; ++j) {
    if (c == j) {
#pragma unroll
      for (int rr = 0; rr < PN_RPT; ++rr) xs[g * PN_RPT + rr] = v[rr];
    }
#pragma unroll
    for (int rr = 0; rr < PN_RPT; ++rr)
      if (r0 + rr == j) rowj[c] = v[rr];
    __syncthreads();
    double s = 0.0;
    if (c >= j && c < bJ) {
#pragma unroll
      for (int rr = 0; rr < PN_RPT; ++rr) {
        const int row = r0 + rr;
        if (row > j && row < mJ) s += xs[g * PN_RPT + rr] * v[rr];
      }
    }
    part[g][c] = s;
    __syncthreads();
    if (tid < 64) {
      double d = 0.0;
#pragma unroll
      for (int q = 0; q < PN_GROUPS; ++q) d += part[q][tid];
      a.slots[((int64_t)j * a.NP + me) * 64 + tid] = d;
      if (j >= wlo && j < whi) a.rowslot[(int64_t)j * 64 + tid] = rowj[tid];
    }
    publish_flag(a.flags, me, (unsigned)(j + 1));
    if (!wait_flags(a.flags, a.NP, (unsigned)(j + 1), a.err)) return;
    // all partials are loaded at once (row group g reads workgroups g, g+16, ...)
    {
      double d = 0.0;
      for (int q = g; q < a.NP; q += PN_GROUPS) d += a.slots[((int64_t)j * a.NP + q) * 64 + c];
      part[g][c] = d;
      if (tid < 64) rowv[tid] = a.rowslot[(int64_t)j * 64 + tid];
    }
    __syncthreads();
    if (tid < 64) {
      double d = 0.0;
#pragma unroll
      for (int q = 0; q < PN_GROUPS; ++q) d += part[q][tid];
      dsum[tid] = d;
    }
    __syncthreads();
    if (tid == 0) {
      const double alpha = rowv[j];
      const double xn2 = dsum[j];
      double tau = 0.0, beta = alpha, scal = 0.0;
      if (xn2 != 0.0) {
        const double nrm = sqrt(alpha * alpha + xn2);
        beta = (alpha >= 0.0) ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      hh[0] = tau; hh[1] = beta; hh[2] = scal;
      if (me == 0) a.tau[j] = tau;
    }
    __syncthreads();
    if (tid < 64) wv[tid] = (tid > j && tid < bJ) ? hh[0] * (rowv[tid] + hh[2] * dsum[tid]) : 0.0;
    __syncthreads();
    const double beta = hh[1], scal = hh[2], w = wv[c];
#pragma unroll
    for (int rr = 0; rr < PN_RPT; ++rr) {
      const int row = r0 + rr;
      if (row > j && row < mJ) {
        const double y = xs[g * PN_RPT + rr] * scal;
        if (c > j) v[rr] -= y * w;
        else if (c == j) v[rr] = y;
      } else if (row == j) {
        if (c > j) v[rr] -= w;
        else if (c == j) v[rr] = beta;
      }
    }
    __syncthreads();
  }

  if (c < bJ) {
#pragma unroll
    for (int rr = 0; rr < PN_RPT; ++rr) {
      const int row = r0 + rr;
      if (row < mJ) {
        a.P[row + c * a.ldp] = v[rr];
        a.Y[row + c * a.ldy] = (row < c) ? 0.0 : (row == c ? 1.0 : v[rr]);
      }
    }
  }
}

}  // namespace

size_t panel_slot_elems(int64_t mmax, int bmax) {
  const int64_t np = (mmax + PN_RB - 1) / PN_RB;
  return (size_t)bmax * (size_t)np * 64 + (size_t)bmax * 64;
}

int launch_panel(hipStream_t s, double* P, int64_t ldp, int64_t mJ, int bJ, double* tau, double* Y, int64_t ldy,
                 const PanelWork& w, bool copy_y) {
  if (bJ <= 0 || mJ <= 0) return 0;
  if (bJ > 64) return -6;
  if (mJ >= (int64_t)1 << 31) return -3;
  PanelParams a;
  a.P = P; a.ldp = ldp; a.mJ = mJ; a.bJ = bJ; a.tau = tau; a.Y = Y; a.ldy = ldy;
  a.NP = (int)((mJ + PN_RB - 1) / PN_RB);
  a.slots = w.slots;
  a.rowslot = w.slots + (size_t)bJ * a.NP * 64;
  a.flags = w.flags;
  a.err = w.err;
  a.gate = w.gate;
  a.copy_y = (copy_y && w.gate) ? 1 : 0;
  // An ordinary launch, not a cooperative one: the kernel is the fallback of
  // the CholeskyQR panel and almost always leaves at its gate, before any
  // exchange, and a cooperative dispatch costs the queue tens of
  // microseconds per block.  Its NP workgroups (one per 256 rows, 512
  // threads each) wait on each other, so they must fit the device at once:
  // checked here against one CU's occupancy times the CU count (the caller
  // turns a panel too tall for that into an error).  The exchange waits are
  // bounded, so a workgroup held back by other work on the device makes the
  // call report failure (info = -1) instead of hanging.
  static int resident = 0;
  if (!resident) {
    int occ = 0, dev = 0, cus = 0;
    RQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, panel_kernel, PN_THREADS, 0));
    RQ_HIP(hipGetDevice(&dev));
    RQ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    resident = std::max(1, occ * cus);
  }
  // the copy takes one workgroup per CP_ROWS rows; the column panel's
  // workgroups are the first NP (the others leave at once when it runs)
  const int64_t ncopy = a.copy_y ? (mJ + CP_ROWS - 1) / CP_ROWS : 0;
  if (a.NP > resident) {
    if (a.copy_y) {  // the copy still runs when the CholeskyQR panel succeeded
      hipLaunchKernelGGL(ycopy_gated_kernel, dim3((unsigned)ncopy), dim3(256), 0, s, a);
      RQ_HIP(hipGetLastError());
    }
    return RQ_PANEL_TOO_TALL;
  }
  hipLaunchKernelGGL(panel_kernel, dim3((unsigned)std::max<int64_t>(a.NP, ncopy)), dim3(PN_THREADS), 0, s, a);
  RQ_HIP(hipGetLastError());
  return 0;
}

}  // namespace rq
