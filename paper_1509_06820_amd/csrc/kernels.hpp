// Host-side launchers of the gfx950 kernels (internal to the library).
#pragma once

#include <algorithm>
#include "common.hpp"

namespace rq {

// Omega(r, c) -> out[r*rs + c*cs], r < l, c < m (Philox4x64-10 + Box-Muller).
int launch_omega(hipStream_t s, uint64_t seed, int64_t l, int64_t m, double* out, int64_t rs, int64_t cs,
                 uint64_t key1 = 0);
// Omega of each matrix of a batch: job j writes the l x m matrix of its seed
// (column-major, ld) -- the same numbers as launch_omega.  jobs: device array;
// max_elems bounds l * m over the jobs.
struct OmegaJob {
  uint64_t seed;
  int64_t l, m;
  double* out;   // Omega(r, c) at out[r * rs + c * cs]
  int64_t rs, cs;
};
int launch_omega_batched(hipStream_t s, const OmegaJob* jobs, int count, int64_t max_elems);

// C = alpha * opA * opB + beta * C  (see gemm.hip).  `scratch` (may be null)
// enables split-K for short-wide outputs; gemm_scratch_elems gives its size.
int launch_gemm(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* scratch,
                size_t scratch_elems);
// C (M x 2 N1, ldc) = alpha A^T [B1 B2] + beta C, with A K x M and B1, B2 K x N1
// (separate arrays): one launch for M, N1 <= 64.
int launch_gemm_pair(hipStream_t s, int64_t M, int64_t N1, int64_t K, double alpha, const double* A, int64_t lda,
                     const double* B1, int64_t ldb1, const double* B2, int64_t ldb2, double beta, double* C,
                     int64_t ldc, double* scratch, size_t scratch_elems);
size_t gemm_scratch_elems(int64_t M, int64_t N, int64_t K);
// One product of a grouped launch: C = alpha op(A) op(B) + beta C (M x N,
// reduction K), tiles_x = tiles per row of output tiles, tile0 = index of
// its first tile in the launch's tile list.
struct GroupedGemm {
  int64_t M, N, K;
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
  double alpha, beta;
  int64_t tiles_x, tile0;
  // split-K: the reduction runs in chunks of kchunk (K: no split); chunk z
  // writes its partial product to C + z * split_stride (beta 0); ntile =
  // output tiles of one chunk
  int64_t kchunk, split_stride, ntile;
};
// Tile shapes of the grouped launches (output rows x columns per workgroup).
enum { GT_64x64 = 0, GT_32x32 = 1, GT_128x64 = 2, GT_NCFG = 3 };
void grouped_tile_shape(int cfg, int* bm, int* bn);
// All tiles of the products probs[0..] (device arrays; tile_prob[t] = the
// product of tile t) in one persistent launch of at most wgs workgroups.
// f32: operands rounded to FP32 on the FP32 matrix cores (no transposed
// second operand), FP64 C.  Every product of a launch has the same
// transposes.
int launch_gemm_grouped(hipStream_t s, int cfg, bool ta, bool tb, bool f32, const GroupedGemm* probs,
                        const int* tile_prob, int64_t ntiles, int wgs);
// The same products on the FP32 matrix cores (operands rounded to FP32,
// FP32 accumulation, FP64 C), with one operand stored in FP32.
int launch_gemm_f32(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const float* A,
                    int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* scratch,
                    size_t scratch_elems);
int launch_gemm_f32(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                    int64_t lda, const float* B, int64_t ldb, double beta, double* C, int64_t ldc, double* scratch,
                    size_t scratch_elems);
int launch_gemm_f32(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                    int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* scratch,
                    size_t scratch_elems);
// Sketch S (l x n, ld lds) = Omega (l x m, ld ldo) A (m x n, ld lda) on the
// BF16 matrix cores: both operands rounded to BF16, FP32 accumulation, FP64
// output; split along m when scratch (gemm_scratch_elems(l, n, m)) is given.
int launch_sketch_bf16(hipStream_t s, int64_t l, int64_t n, int64_t m, const double* Omega, int64_t ldo,
                       const double* A, int64_t lda, double* S, int64_t lds, double* scratch, size_t scratch_elems);
int launch_sketch_bf16(hipStream_t s, int64_t l, int64_t n, int64_t m, const double* Omega, int64_t ldo,
                       const float* A, int64_t lda, double* S, int64_t lds, double* scratch, size_t scratch_elems);
// dst (FP32, rows x cols, ld ldd) = src (FP64, ld lds) rounded to nearest;
// with dst64, also an FP64 copy in the same pass.
int launch_to_f32(hipStream_t s, int64_t rows, int64_t cols, const double* src, int64_t lds, float* dst, int64_t ldd,
                  double* dst64 = nullptr, int64_t ld64 = 0);
int launch_scale(hipStream_t s, int64_t M, int64_t N, double beta, double* C, int64_t ldc);

// Sample QRCP (Alg. 1 on the sample, bJ steps) in place on the l x nJ sample.
struct SampleQrcpWork {
  double* cand;        // sample_qrcp_cand_elems(): candidate columns (double buffered)
  int* cand_idx;       // sample_qrcp_idx_elems(): their positions and physical columns
  double* theta;       // sample_qrcp_theta_elems(): best left-out norm per workgroup
  unsigned* flags;     // arrival counter (zeroed by the caller)
  int* err;
};
size_t sample_qrcp_flag_words();
// Rows of the sample as the sample QRCP stores it (l rounded up to its
// register tile: 32, 40, 48, 64, 72, 80 or 128; -1 if l > 128).
int sample_rows_padded(int l);
size_t sample_qrcp_cand_elems();
size_t sample_qrcp_idx_elems();
size_t sample_qrcp_theta_elems();
// S is the sample, column-major with ld lds == sample_rows_padded(l) (rows
// past l zero).
// Workgroups of the sample QRCP on a sample of nJ columns (all resident at once).
int sample_qrcp_workgroups(int64_t nJ);
// With upd: the same launch also runs the trailing update C -= A B (M x N,
// reduction K; A ld lda, B ld ldb, C ld ldc; the products on the FP32 matrix
// cores with f32) on `wgs` more workgroups -- the previous block's rows below
// its R12, which the sample QRCP does not touch.
struct BesideUpdate {
  int64_t M = 0, N = 0, K = 0;
  const double* A = nullptr;
  int64_t lda = 0;
  const double* B = nullptr;
  int64_t ldb = 0;
  double* C = nullptr;
  int64_t ldc = 0;
  bool f32 = false;
  int64_t wgs = 0;
};
int launch_sample_qrcp(hipStream_t s, double* S, int64_t lds, int l, int64_t nJ, int bJ, int* piv, int* info,
                       int info_base, const SampleQrcpWork& w, const BesideUpdate* upd = nullptr);

// Apply the sequential swaps (offset+t) <-> (offset+piv[t]), t < bJ, to the
// columns of an R x ncols matrix (double) and optionally to an int64 vector.
int launch_apply_swaps(hipStream_t s, const int* piv, int bJ, int64_t offset, double* M, int64_t ldm, int64_t rows,
                       int64_t* jpvt);
// The same composed permutation applied to an FP32 copy (no jpvt).
int launch_apply_swaps_f32(hipStream_t s, const int* piv, int bJ, int64_t offset, float* M, int64_t ldm,
                           int64_t rows);

// Householder panel QR (in-place layout), tau, explicit unit-lower Y, one
// column at a time.  With `gate` set, the kernel runs only if *gate != 0;
// with copy_y as well, a launch whose gate is 0 (the CholeskyQR panel
// succeeded) copies Y(bJ:mJ, :) into P(bJ:mJ, :) instead.
struct PanelWork {
  double* slots;       // bmax * 256 * 64 + bmax * 64 doubles
  unsigned* flags;     // 256 words (zeroed by the caller)
  int* err;
  const int* gate;
};
size_t panel_slot_elems(int64_t mmax, int bmax);
// launch_panel's return value when its workgroups cannot all be resident.
constexpr int RQ_PANEL_TOO_TALL = RQ_ERR_HIP_BASE + (int)hipErrorCooperativeLaunchTooLarge;
int launch_panel(hipStream_t s, double* P, int64_t ldp, int64_t mJ, int bJ, double* tau, double* Y, int64_t ldy,
                 const PanelWork& w, bool copy_y);

// Panel by CholeskyQR2 + Householder reconstruction (see cholqr.hip).
size_t cholqr_scratch_elems(int64_t mmax, int bmax);
int launch_panel_cholqr(hipStream_t s, double* P, int64_t ldp, int64_t mJ, int bJ, const double* S11, int64_t srs,
                        int64_t scs, double* tau, double* Y, int64_t ldy, double* T, double* scratch,
                        double* splitk, size_t splitk_elems, int* st, double* W11 = nullptr);

// After the column panel (runs only if *st != 0, i.e. the CholeskyQR panel
// failed): T (bJ x bJ, ld bJ) of the panel's reflectors from Y (mJ x bJ, ld
// ldy) and tau, and, with W non-null, W11 = S11 R11^{-1} (upper triangular,
// ld bJ; zero-diagonal columns of R11 give 0), S11(i, j) = S[i*srs + j*scs],
// R11 the panel's R (ld ldr).
int launch_fallback_tail(hipStream_t s, int64_t mJ, int bJ, const double* Y, int64_t ldy, const double* tau,
                         double* T, const int* st, const double* S, int64_t srs, int64_t scs, const double* R,
                         int64_t ldr, double* W);

// Small utilities.
int launch_fill(hipStream_t s, void* p, size_t words32);  // zero-fill 32-bit words
// M(r0:r1, 0:cols) = 0
int launch_zero_rows(hipStream_t s, int64_t r0, int64_t r1, int64_t cols, double* M, int64_t ldm);
int launch_copy2d(hipStream_t s, int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst,
                  int64_t ldd);
int launch_set_identity(hipStream_t s, int64_t rows, int64_t cols, double* M, int64_t ldm);
// Z0T(jpvt[j], i) = R(i, j) for i <= j (upper trapezoidal R, k x n) else 0.
// Vp(i, :) = V(jpvt[i], :) for i < n (k columns).
int launch_gather_rows(hipStream_t s, int64_t n, int64_t k, const double* V, int64_t ldv, const int64_t* jpvt,
                       double* Vp, int64_t ldp);
int launch_scatter_rt(hipStream_t s, int64_t k, int64_t n, const double* R, int64_t ldr, const int64_t* jpvt,
                      double* Z0T, int64_t ldz);
// Upper-triangular part of a k x k block (zeros below the diagonal).
int launch_triu_copy(hipStream_t s, int64_t k, const double* src, int64_t lds, double* dst, int64_t ldd);

// One-sided Jacobi SVD of a k x k matrix X (in place: X -> U Sigma), V
// accumulated, singular values sorted descending.
struct SvdWork {
  double* colnorm;     // k
  int* order;          // k
  unsigned* flags;
  int* err;
  double* tmp;         // k * k
};
int launch_jacobi_svd(hipStream_t s, int k, double* X, int64_t ldx, double* U, int64_t ldu, double* sigma,
                      double* V, int64_t ldv, const SvdWork& w);

}  // namespace rq
