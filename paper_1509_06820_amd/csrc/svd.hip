// SVD of the k x k connection matrix X of TUXV (Section 6: "feasible to obtain
// slightly better approximations by taking the SVD of X").
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
// (a column with sigma == 0 is left zero).
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

__device__ __forceinline__ double group_sum(double v, int tpp) {
  for (int off = tpp >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

__global__ void __launch_bounds__(SVD_THREADS) jacobi_kernel(int k, double* X, int64_t ldx, double* V, int64_t ldv,
                                                             double* U, int64_t ldu, double* sigma, double* Vout,
                                                             int64_t ldvo, double tol, int max_sweeps) {
  __shared__ int rotated;
  __shared__ double sn[1024];
  const int tid = threadIdx.x;
  const int kk = k + (k & 1);
  const int npairs = kk / 2;
  int tpp = SVD_THREADS / max(npairs, 1);
  int pw = 1;
  while (pw * 2 <= tpp && pw < 64) pw *= 2;
  tpp = pw;
  const int groups = SVD_THREADS / tpp;
  const int grp = tid / tpp, sub = tid % tpp;

  for (int64_t e = tid; e < (int64_t)k * k; e += SVD_THREADS) {
    const int64_t j = e / k, i = e - j * k;
    V[i + j * ldv] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();

  for (int sweep = 0; sweep < max_sweeps && kk > 1; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < kk - 1; ++r) {
      for (int idx = grp; idx < npairs; idx += groups) {
        int p, q;
        rr_pair(r, idx, kk, p, q);
        if (p >= k || q >= k) continue;
        const int i = min(p, q), j = max(p, q);
        double* xi = X + (int64_t)i * ldx;
        double* xj = X + (int64_t)j * ldx;
        double sa = 0.0, sb = 0.0, sg = 0.0;
        for (int row = sub; row < k; row += tpp) {
          const double u = xi[row], w = xj[row];
          sa += u * u;
          sb += w * w;
          sg += u * w;
        }
        sa = group_sum(sa, tpp);
        sb = group_sum(sb, tpp);
        sg = group_sum(sg, tpp);
        if (sg != 0.0 && fabs(sg) > tol * sqrt(sa * sb)) {
          const double z = (sb - sa) / (2.0 * sg);
          const double t = ((z >= 0.0) ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
          const double cs = 1.0 / sqrt(1.0 + t * t);
          const double sn_ = cs * t;
          for (int row = sub; row < k; row += tpp) {
            const double u = xi[row], w = xj[row];
            xi[row] = cs * u - sn_ * w;
            xj[row] = sn_ * u + cs * w;
          }
          double* vi = V + (int64_t)i * ldv;
          double* vj = V + (int64_t)j * ldv;
          for (int row = sub; row < k; row += tpp) {
            const double u = vi[row], w = vj[row];
            vi[row] = cs * u - sn_ * w;
            vj[row] = sn_ * u + cs * w;
          }
          if (sub == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }

  // column norms
  for (int j = grp; j < k; j += groups) {
    const double* xj = X + (int64_t)j * ldx;
    double s = 0.0;
    for (int row = sub; row < k; row += tpp) s += xj[row] * xj[row];
    s = group_sum(s, tpp);
    if (sub == 0) sn[j] = sqrt(s);
  }
  __syncthreads();
  // descending order, ties by index
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

}  // namespace

int launch_jacobi_svd(hipStream_t s, int k, double* X, int64_t ldx, double* U, int64_t ldu, double* sigma, double* V,
                      int64_t ldv, const SvdWork& w) {
  if (k <= 0) return 0;
  if (k > 1024) return -3;
  // w.tmp holds the accumulated rotations (k x k)
  hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(SVD_THREADS), 0, s, k, X, ldx, w.tmp, (int64_t)k, U, ldu, sigma, V,
                     ldv, 1e-15, 60);
  RQ_HIP(hipGetLastError());
  return 0;
}

}  // namespace rq
