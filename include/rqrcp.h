/*
 * rqrcp.h -- C ABI of the gfx950 (MI355X) library for randomized QR with
 * column pivoting (Duersch & Gu, "Randomized QR with Column Pivoting",
 * arXiv 1509.06820).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * - Matrices are column-major, double precision, with a leading dimension
 *   ld >= max(1, rows).  Every pointer to matrix/vector data is a DEVICE
 *   pointer owned by the caller; the library never allocates or frees
 *   device memory.  Scratch memory is the caller's `work` buffer of at least
 *   rq_workspace_bytes(...) bytes (device memory, 256-byte aligned).
 * - `stream` is a hipStream_t (passed as void*; NULL = default stream).  The
 *   calls only ENQUEUE work: they return as soon as the kernels are queued
 *   and the results are valid once the stream reaches that point.  Calls
 *   that share a `work` buffer must be ordered on one stream.
 * - Return value (enqueue status): 0 on success; -i when argument i (1-based)
 *   is invalid, LAPACK xerbla style; -100 when the workspace is too small;
 *   1000 + hipError_t on a HIP runtime error (including a kernel whose
 *   workgroups must all be resident at once and do not fit the device).
 * - `info` (device int32, may be NULL) is written by the kernels: 0 = no
 *   issue; j > 0 = a non-finite sample norm was first met around pivot step j
 *   (the factorization still completes; a NaN norm never wins a pivot
 *   choice); -1 = an internal cross-workgroup wait timed out (results are
 *   invalid; possible when other work on the device keeps a workgroup of the
 *   sample QRCP from starting for a long time).
 * - Empty matrices: for m = 0 or n = 0 the factorizations write only jpvt
 *   (the identity) and info (0); rq_sketch with m = 0 writes B = 0.
 * - Limits of this version: 1 <= b <= 64, 0 <= p, b + p <= 128, n <= 65536,
 *   k <= 1024 for rq_tuxv and rq_tuxv_iter.
 * - Pivot indices are 0-based int64.  jpvt[j] is the original index of column
 *   j of A P.
 */
#ifndef RQRCP_H
#define RQRCP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Operation codes for rq_workspace_bytes. */
enum {
  RQ_OP_RQRCP = 0,        /* rq_rqrcp / rq_rqrcp_omega          */
  RQ_OP_TRQRCP = 1,       /* rq_trqrcp / rq_trqrcp_omega        */
  RQ_OP_TUXV = 2,         /* rq_tuxv / rq_tuxv_omega            */
  RQ_OP_QR = 3,           /* rq_unpivoted_qr                    */
  RQ_OP_SAMPLE_QRCP = 4,  /* rq_sample_qrcp                     */
  RQ_OP_SVD = 5,          /* rq_small_svd                       */
  RQ_OP_RSRQRCP = 6,      /* rq_rsrqrcp                         */
  RQ_OP_TUXV_MIXED = 7,   /* rq_tuxv_mixed                      */
  RQ_OP_TRQRCP_MIXED = 8  /* rq_trqrcp_mixed                    */
};

/* Largest j_max accepted by rq_tuxv_iter. */
#define RQ_TUXV_MAX_ITER 64

/* Library version string (static storage). */
const char* rq_version(void);

/*
 * Look-ahead switch for rq_rqrcp / rq_rqrcp_omega (host-side, process-wide).
 * With it on (the default, unless the environment sets RQRCP_LOOKAHEAD=0)
 * each block's trailing update below the new rows of R runs on a second,
 * library-owned stream of the current device, beside the sample update and
 * the next block's sample QRCP (which touch other data); the caller's stream
 * waits for it before the next block's column swaps, so the call still
 * completes in the caller's stream order.  Off: every kernel on the caller's
 * stream.  Results are bitwise the same either way.  Returns the previous
 * setting (0 or 1).
 */
int rq_set_lookahead(int32_t on);

/*
 * Workspace size in bytes for operation `op` at the given sizes (host-only
 * query, no GPU work).  k is ignored for RQ_OP_RQRCP and RQ_OP_QR.
 * Returns 0 on success or -i for an invalid argument i.
 */
int rq_workspace_bytes(int32_t op, int64_t m, int64_t n, int64_t k, int32_t b, int32_t p, size_t* bytes);

/*
 * RQRCP -- Alg. 4 (Section 5), full factorization with k = min(m, n):
 * A P = Q R with Q = H_0 ... H_{k-1}.
 *   Omega (l x m, l = b + p) is drawn from `seed` (Philox4x64-10 + Box-Muller,
 *   see rq_omega); the sample B = Omega A picks each block of b pivots by a
 *   partial QRCP of the l x n sample; the selected columns get a Householder
 *   panel and a compact-WY update of the trailing matrix; the sample is then
 *   refreshed by eq. (update1) instead of being re-drawn.
 *   On exit A holds R on and above the diagonal and the Householder vectors
 *   below it (unit diagonal implicit; the LAPACK dgeqp3 layout), tau[k]
 *   holds the reflector coefficients (H_i = I - tau_i y_i y_i^T) and jpvt[n]
 *   the column permutation.
 *   Arguments: 1 stream, 2 m, 3 n, 4 A (in/out, m x n, device), 5 lda,
 *   6 b (block size), 7 p (oversampling), 8 seed, 9 jpvt (out, n int64),
 *   10 tau (out, min(m,n)), 11 work, 12 work_bytes, 13 info (out, device).
 */
int rq_rqrcp(void* stream, int64_t m, int64_t n, double* A, int64_t lda, int32_t b, int32_t p, uint64_t seed,
             int64_t* jpvt, double* tau, void* work, size_t work_bytes, int32_t* info);

/* As rq_rqrcp with a caller-supplied compression matrix Omega (l x m,
 * column-major, leading dimension ldo >= l, device; argument 8 = Omega,
 * 9 = ldo; the later arguments shift by one). */
int rq_rqrcp_omega(void* stream, int64_t m, int64_t n, double* A, int64_t lda, int32_t b, int32_t p,
                   const double* Omega, int64_t ldo, int64_t* jpvt, double* tau, void* work, size_t work_bytes,
                   int32_t* info);

/*
 * RSRQRCP -- Alg. 5 (Section 5), repeated-sampling RQRCP: the factorization
 * of rq_rqrcp, except that every block J = 0, 1, ... (starting at column
 * i0 = J b) draws a new compression matrix Omega^[J] (l x (m - i0), Philox
 * key (seed, J), same normal map and layout as rq_omega) and samples the
 * updated trailing matrix, B = Omega^[J] A(i0:m, i0:n), instead of updating
 * the previous sample by eq. (update1).  Block 0 therefore makes the pivot
 * choices of rq_rqrcp's first block.  The paper gives it as the comparison
 * that shows what the sample update saves.
 *   Outputs and layout as rq_rqrcp; workspace: rq_workspace_bytes with
 *   RQ_OP_RSRQRCP.
 *   Arguments: 1 stream, 2 m, 3 n, 4 A (in/out, m x n, device), 5 lda,
 *   6 b, 7 p, 8 seed, 9 jpvt (out, n int64), 10 tau (out, min(m,n)),
 *   11 work, 12 work_bytes, 13 info (out, device).
 */
int rq_rsrqrcp(void* stream, int64_t m, int64_t n, double* A, int64_t lda, int32_t b, int32_t p, uint64_t seed,
               int64_t* jpvt, double* tau, void* work, size_t work_bytes, int32_t* info);

/*
 * TRQRCP -- Alg. 6 (Section 5.1): truncated RQRCP to rank k that never
 * updates the trailing matrix; it keeps the reflector block Y and the inner
 * products W^T = T^T Y^T A and forms selected columns A - Y W^T and new rows
 * of R on demand.  On exit rows 0..k-1 of A hold R (k x n upper trapezoidal),
 * columns 0..k-1 below the diagonal hold the Householder vectors, and the
 * block A(k:m, k:n) holds the PERMUTED ORIGINAL entries (unlike dgeqp3).
 * jpvt[0..k-1] are the pivots; jpvt[k..n-1] is the swap-induced order of the
 * other columns.  tau has k entries.  1 <= k <= min(m, n).
 * Arguments: 1 stream, 2 m, 3 n, 4 k, 5 A, 6 lda, 7 b, 8 p, 9 seed, 10 jpvt,
 * 11 tau, 12 work, 13 work_bytes, 14 info.
 */
int rq_trqrcp(void* stream, int64_t m, int64_t n, int64_t k, double* A, int64_t lda, int32_t b, int32_t p,
              uint64_t seed, int64_t* jpvt, double* tau, void* work, size_t work_bytes, int32_t* info);

/*
 * TRQRCP in mixed precision (not in the paper): as rq_trqrcp, but the two
 * products that stream the whole matrix -- the sketch Omega A and each
 * block's Y2^T A -- run on the FP32 matrix cores (operands rounded to FP32,
 * FP32 accumulation, FP64 results) from an FP32 copy of A that the call
 * makes in its workspace and permutes along with A.  The sample QRCP, the
 * panels, reflectors, T and the column swaps stay FP64, so Q is orthonormal
 * to FP64 accuracy and A(k:m, k:n) still holds the permuted original
 * entries exactly; R and the selected columns carry FP32 rounding of the
 * products (about sqrt(m) 6e-8 relative), and pivots may differ from the
 * FP64 path where two sample norms lie within that rounding.
 * Arguments as rq_trqrcp; workspace: rq_workspace_bytes with
 * RQ_OP_TRQRCP_MIXED (RQ_OP_TRQRCP plus 4 m n bytes).
 */
int rq_trqrcp_mixed(void* stream, int64_t m, int64_t n, int64_t k, double* A, int64_t lda, int32_t b, int32_t p,
                    uint64_t seed, int64_t* jpvt, double* tau, void* work, size_t work_bytes, int32_t* info);

int rq_trqrcp_omega(void* stream, int64_t m, int64_t n, int64_t k, double* A, int64_t lda, int32_t b, int32_t p,
                    const double* Omega, int64_t ldo, int64_t* jpvt, double* tau, void* work, size_t work_bytes,
                    int32_t* info);

/*
 * TUXV -- Alg. 7 with j_max = 1 (Section 6, eq. tuxv) followed by the SVD of
 * the k x k connection matrix X: A ~= U diag(sigma) VT.
 *   TRQRCP on a copy of A -> Z0 = R P^T -> V from the QR of Z0^T -> Z1 = A V
 *   -> U1, X from the QR of Z1 -> X = Ux diag(sigma) Vx^T (one-sided Jacobi)
 *   -> U = U1 Ux, VT = Vx^T V^T.
 *   A is read-only.  Outputs: U (m x k, orthonormal columns, ldu >= m),
 *   sigma (k, descending, >= 0), VT (k x n, orthonormal rows, ldvt >= k).
 *   Singular vectors are defined up to sign.
 * Arguments: 1 stream, 2 m, 3 n, 4 k, 5 A, 6 lda, 7 b, 8 p, 9 seed, 10 U,
 * 11 ldu, 12 sigma, 13 VT, 14 ldvt, 15 work, 16 work_bytes, 17 info.
 */
int rq_tuxv(void* stream, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, int32_t b, int32_t p,
            uint64_t seed, double* U, int64_t ldu, double* sigma, double* VT, int64_t ldvt, void* work,
            size_t work_bytes, int32_t* info);

int rq_tuxv_omega(void* stream, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, int32_t b, int32_t p,
                  const double* Omega, int64_t ldo, double* U, int64_t ldu, double* sigma, double* VT, int64_t ldvt,
                  void* work, size_t work_bytes, int32_t* info);

/*
 * TUXV in mixed precision (j_max = 1): the three products that stream the
 * whole matrix -- the sketch Omega A, the per-block Y2^T A of TRQRCP and
 * Z = A V -- run on the FP32 matrix cores (operands rounded to FP32, FP32
 * accumulation) from an FP32 copy of A made inside the call and permuted
 * along with A; the panels, reflectors, T, the rows of R, the sample QRCP,
 * the orthogonal factors and the SVD of X stay FP64.  The FP32 rounding of
 * those products (relative ~ sqrt(n) 6e-8) is far below the truncation
 * errors this path is meant for; an approximation whose error approaches
 * it needs rq_tuxv.  Pivots may differ from rq_tuxv's where two sample
 * norms lie within the FP32 rounding of each other.  Arguments as rq_tuxv;
 * workspace: RQ_OP_TUXV_MIXED (RQ_OP_TUXV plus 4 m n + 8 n k bytes).
 */
int rq_tuxv_mixed(void* stream, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, int32_t b, int32_t p,
                  uint64_t seed, double* U, int64_t ldu, double* sigma, double* VT, int64_t ldvt, void* work,
                  size_t work_bytes, int32_t* info);

/*
 * TUXV with j_max >= 1 iterations -- Alg. 7 (Section 6): after the first LQ,
 * steps alternate between the QR of Z = A V (new U, upper triangular X) and
 * the LQ of Z = U^T A, computed as the QR of A^T U (new V, lower triangular
 * X); j_max counts these steps, so j_max = 1 is rq_tuxv.  Each step can only
 * lower the error ||A - U X V^T||_F (the best approximation with the new
 * column or row space).  The SVD of the last X gives the outputs, as in
 * rq_tuxv.  Workspace: RQ_OP_TUXV.
 * Arguments: 1 stream, 2 m, 3 n, 4 k, 5 A, 6 lda, 7 b, 8 p, 9 seed,
 * 10 jmax (1 <= jmax <= RQ_TUXV_MAX_ITER), 11 U, 12 ldu, 13 sigma, 14 VT,
 * 15 ldvt, 16 work, 17 work_bytes, 18 info.
 */
int rq_tuxv_iter(void* stream, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, int32_t b, int32_t p,
                 uint64_t seed, int32_t jmax, double* U, int64_t ldu, double* sigma, double* VT, int64_t ldvt,
                 void* work, size_t work_bytes, int32_t* info);

/*
 * Unpivoted blocked Householder QR (the paper's "qr" comparator, Section 7:
 * RQRCP with sampling and pivoting removed), same output layout as rq_rqrcp
 * without jpvt.  Arguments: 1 stream, 2 m, 3 n, 4 A, 5 lda, 6 b, 7 tau,
 * 8 work, 9 work_bytes, 10 info.
 */
int rq_unpivoted_qr(void* stream, int64_t m, int64_t n, double* A, int64_t lda, int32_t b, double* tau, void* work,
                    size_t work_bytes, int32_t* info);

/*
 * Compression matrix alone (Section 3: i.i.d. N(0,1) entries): Omega(r, c),
 * r < l, c < m, is normal number r*m + c of the stream for `seed`:
 * Philox4x64-10 (Salmon et al., SC'11) with key (seed, 0), block q = counter
 * (q+1, 0, 0, 0); u = ((x >> 12) + 1/2) 2^-52; Box-Muller on word pairs
 * (0,1) and (2,3).  Output column-major l x m with ldo >= l.
 * Arguments: 1 stream, 2 seed, 3 l, 4 m, 5 Omega (out), 6 ldo.
 */
int rq_omega(void* stream, uint64_t seed, int64_t l, int64_t m, double* Omega, int64_t ldo);

/*
 * Sketch alone (Alg. 4, "form the initial sample"): B = Omega A with Omega
 * drawn from `seed` as in rq_omega; B is l x n column-major (ldb >= l).
 * Arguments: 1 stream, 2 m, 3 n, 4 A, 5 lda, 6 l, 7 seed, 8 B, 9 ldb,
 * 10 work, 11 work_bytes (RQ_OP_RQRCP workspace with b = l, p = 0 suffices).
 */
int rq_sketch(void* stream, int64_t m, int64_t n, const double* A, int64_t lda, int32_t l, uint64_t seed, double* B,
              int64_t ldb, void* work, size_t work_bytes);

/*
 * Partial QRCP of a sample alone (Alg. 1 run for bsteps steps on an l x n
 * matrix, the "qrcp(B, b)" step of Alg. 4): trailing squared norms are
 * recomputed at every step, the largest wins with ties to the lowest
 * position, swaps are sequential (step t exchanges positions t and piv[t]).
 * On exit B (l x n, ldb >= l, in/out) holds S: the first bsteps columns are
 * upper triangular (S11 above S21 = 0), the rest hold S12 / S22.
 * Arguments: 1 stream, 2 l, 3 n, 4 bsteps (<= min(64, l, n)), 5 B, 6 ldb,
 * 7 piv (out, bsteps int32, device), 8 work, 9 work_bytes, 10 info.
 */
int rq_sample_qrcp(void* stream, int32_t l, int64_t n, int32_t bsteps, double* B, int64_t ldb, int32_t* piv,
                   void* work, size_t work_bytes, int32_t* info);

/*
 * SVD of a small square matrix alone (the SVD of X in TUXV): X = U diag(s) V^T
 * by one-sided Jacobi.  X (k x k, ldx) is overwritten.  U (ldu), V (ldv) are
 * k x k outputs, sigma descending.
 * Arguments: 1 stream, 2 k, 3 X, 4 ldx, 5 U, 6 ldu, 7 sigma, 8 V, 9 ldv,
 * 10 work, 11 work_bytes.
 */
int rq_small_svd(void* stream, int32_t k, double* X, int64_t ldx, double* U, int64_t ldu, double* sigma, double* V,
                 int64_t ldv, void* work, size_t work_bytes);

/*
 * Stage timing (host side, for measurement).  Between rq_profile_start() and
 * rq_profile_stop() every entry point records a pair of HIP events on its
 * stream around each stage of the method (classes 0..rq_profile_classes()-1,
 * named by rq_profile_name), together with the stage's algorithmic bytes
 * and flops.  rq_profile_stop() waits for the recorded events and
 * accumulates per class; rq_profile_get() then returns the launch count,
 * total milliseconds, algorithmic bytes and flops of a class.  Not
 * reentrant across host threads that profile concurrently.
 * rq_profile_select(mask) limits the recording to the classes whose bit is
 * set in mask (all classes by default), so that a timed run can carry the
 * events of one stage only.
 */
int rq_profile_start(void);
int rq_profile_select(uint32_t class_mask);
int rq_profile_stop(void);
int rq_profile_get(int32_t cls, int64_t* count, double* total_ms, double* bytes, double* flops);
const char* rq_profile_name(int32_t cls);
int32_t rq_profile_classes(void);

#ifdef __cplusplus
}
#endif

#endif /* RQRCP_H */
