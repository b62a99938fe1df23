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
 *   is invalid, LAPACK xerbla style (a workspace smaller than the size query
 *   makes its size argument invalid); 1000 + hipError_t on a HIP runtime
 *   error (including a kernel whose workgroups must all be resident at once
 *   and do not fit the device).
 * - `info` (device int32, may be NULL) is written by the kernels: 0 = no
 *   issue; j > 0 = a non-finite sample norm was first met around pivot step j
 *   (the factorization still completes; a NaN norm never wins a pivot
 *   choice); -1 = an internal cross-workgroup wait timed out (results are
 *   invalid; possible when other work on the device keeps a workgroup of the
 *   sample QRCP from starting for a long time); -2 = the SVD of X (TUXV) did
 *   not converge within its sweep limit (the outputs are then the last
 *   sweep's, still orthonormal but not fully diagonalising X).
 * - Empty matrices: for m = 0 or n = 0 the factorizations write only jpvt
 *   (the identity) and info (0); rq_sketch with m = 0 writes B = 0.
 * - Limits of this version: 1 <= b <= 64, 0 <= p, b + p <= 128, n <= 65536,
 *   m <= RQ_MAX_ROWS (and m, n <= RQ_MAX_ROWS for rq_sketch and rq_omega, so
 *   that no size computed by the library can overflow), k <= 1024 for
 *   rq_tuxv and rq_tuxv_iter, and m small enough for the fallback panel's
 *   workgroups (one per 256 rows) to be resident together (checked at
 *   launch; about 10^5 rows on MI355X).  The size queries reject what the
 *   entry points would reject.
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
  RQ_OP_RSRQRCP = 6       /* rq_rsrqrcp                         */
};

/*
 * Arithmetic of the products that stream the whole matrix (argument
 * `precision` of rq_rqrcp, rq_trqrcp, rq_tuxv, rq_sketch and
 * rq_workspace_bytes; the method itself does not fix a precision -- this is
 * an extension).  The panels, Householder vectors, T, the sample QRCP and
 * its norms, the sample update, the column swaps and the SVD of X are FP64
 * at every level.
 *   RQ_FP64       : everything in FP64 (the FP64 matrix cores).
 *   RQ_MIXED      : the sketch Omega A and the products with A itself --
 *                   RQRCP's Y^T A and trailing update, TRQRCP's Y2^T A,
 *                   TUXV's A V -- on the FP32 matrix cores (operands rounded
 *                   to FP32, FP32 accumulation, results added to FP64
 *                   storage).  Rounding floor about sqrt(m) 6e-8 relative to
 *                   ||A||: sample norms, pivots and truncation errors below
 *                   it are not resolved.
 *   RQ_MIXED_BF16 : as RQ_MIXED, but the sketch on the BF16 matrix cores
 *                   (Omega and A rounded to BF16, FP32 accumulation): the
 *                   sample only steers the pivots (Section 3), but its
 *                   rounding (at most 2^-8 ||Omega||_F ||A||_F, typically
 *                   1e-4 of it) limits which trailing norms the pivot choice
 *                   can tell apart, so this level suits truncations whose
 *                   relative error is well above 1e-3.
 */
enum { RQ_FP64 = 0, RQ_MIXED = 1, RQ_MIXED_BF16 = 2 };

/* Largest row count (m) accepted by any entry point or size query. */
#define RQ_MAX_ROWS ((int64_t)1 << 40)

/* Largest j_max accepted by rq_tuxv_iter. */
#define RQ_TUXV_MAX_ITER 64

/* Library version string (static storage). */
const char* rq_version(void);

/*
 * Look-ahead switch for rq_rqrcp / rq_rqrcp_omega (host-side, process-wide;
 * on by default).  With it on, each block's trailing update below the new
 * rows of R runs in the next block's sample-QRCP launch, on workgroups of
 * its own beside the sample QRCP's (which touches only the sample), instead
 * of right after those rows; everything stays on the caller's stream, in
 * its order.  Results are bitwise the same either way.  Returns the
 * previous setting (0 or 1).
 */
int rq_set_lookahead(int32_t on);

/*
 * Workspace size in bytes for operation `op` at the given sizes and
 * precision (host-only query, no GPU work).  k is ignored for RQ_OP_RQRCP,
 * RQ_OP_RSRQRCP and RQ_OP_QR; precision other than RQ_FP64 is accepted for
 * RQ_OP_RQRCP, RQ_OP_TRQRCP and RQ_OP_TUXV.  For RQ_OP_SAMPLE_QRCP, m is
 * the sample's row count l (1..128), n its column count and b the pivot
 * steps (b <= l, b <= n); RQ_OP_SVD reads only k (1..1024; m, n, p are
 * not used, b must still lie in 1..64).  Sizes beyond the limits of the
 * entry points (m > RQ_MAX_ROWS, n > 65536) are rejected, never wrapped.
 * Arguments: 1 op, 2 m, 3 n, 4 k, 5 b, 6 p, 7 precision, 8 bytes (out, host).
 * Returns 0 on success or -i for an invalid argument i.
 */
int rq_workspace_bytes(int32_t op, int64_t m, int64_t n, int64_t k, int32_t b, int32_t p, int32_t precision,
                       size_t* bytes);

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
 *   With precision = RQ_MIXED (or RQ_MIXED_BF16) the sketch, each block's
 *   Y^T A and the trailing update run on the lower-precision matrix cores:
 *   A stays FP64 in memory and receives FP32-rounded updates, so the
 *   factorization carries about sqrt(n) 6e-8 relative rounding, and pivots
 *   may differ from the FP64 path where two sample norms lie within the
 *   sketch's rounding of each other.
 *   Arguments: 1 stream, 2 m, 3 n, 4 A (in/out, m x n, device), 5 lda,
 *   6 b (block size), 7 p (oversampling), 8 seed, 9 precision (RQ_FP64,
 *   RQ_MIXED or RQ_MIXED_BF16), 10 jpvt (out, n int64), 11 tau (out, min(m,n)), 12 work,
 *   13 work_bytes, 14 info (out, device).
 */
int rq_rqrcp(void* stream, int64_t m, int64_t n, double* A, int64_t lda, int32_t b, int32_t p, uint64_t seed,
             int32_t precision, int64_t* jpvt, double* tau, void* work, size_t work_bytes, int32_t* info);

/*
 * RQRCP without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  The factorization is rq_rqrcp's (same kernels,
 * bitwise the same results), with every kernel on the caller's stream (no
 * look-ahead stream), and its scratch is a static device array of
 * RQ_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on
 * until the process ends.  The call allocates nothing.  Calls on one device
 * share that array: calls that overlap on one device (different streams, or
 * host threads without ordering) race and give wrong results; calls ordered
 * on one stream are fine (each clears what must start at zero).
 * Sizes whose rq_workspace_bytes(RQ_OP_RQRCP, ...) exceeds the array are
 * rejected with RQ_ERR_SCRATCH_TOO_SMALL before anything is enqueued
 * (8192 x 8192 with b = 64, p = 8 needs 91 MiB and fits).
 * Arguments: as rq_rqrcp without work and work_bytes: 1 stream, 2 m, 3 n,
 * 4 A, 5 lda, 6 b, 7 p, 8 seed, 9 precision, 10 jpvt, 11 tau, 12 info.
 */
#define RQ_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
#define RQ_ERR_SCRATCH_TOO_SMALL 2002
int rq_rqrcp_noalloc(void* stream, int64_t m, int64_t n, double* A, int64_t lda, int32_t b, int32_t p,
                     uint64_t seed, int32_t precision, int64_t* jpvt, double* tau, int32_t* info);

/* As rq_rqrcp in FP64 with a caller-supplied compression matrix Omega
 * (l x m, column-major, leading dimension ldo >= l, device; a test hook):
 * arguments 1-7 as rq_rqrcp, 8 Omega, 9 ldo, 10 jpvt, 11 tau, 12 work,
 * 13 work_bytes, 14 info. */
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
 * With precision = RQ_MIXED the sketch and each block's Y2^T A run on the
 * FP32 matrix cores (RQ_MIXED_BF16: the sketch on the BF16 ones), both from
 * an FP32 copy of A that
 * the call makes in its workspace and permutes along with A (see RQ_MIXED);
 * Q stays orthonormal to FP64 accuracy and A(k:m, k:n) still holds the
 * permuted original entries exactly, while R and the selected columns carry
 * FP32 rounding of the products (about sqrt(m) 6e-8 relative).
 * Arguments: 1 stream, 2 m, 3 n, 4 k, 5 A, 6 lda, 7 b, 8 p, 9 seed,
 * 10 precision, 11 jpvt, 12 tau, 13 work, 14 work_bytes, 15 info.
 */
int rq_trqrcp(void* stream, int64_t m, int64_t n, int64_t k, double* A, int64_t lda, int32_t b, int32_t p,
              uint64_t seed, int32_t precision, int64_t* jpvt, double* tau, void* work, size_t work_bytes,
              int32_t* info);

/* As rq_trqrcp in FP64 with a caller-supplied Omega (a test hook):
 * arguments 1-8 as rq_trqrcp, 9 Omega, 10 ldo, 11 jpvt, 12 tau, 13 work,
 * 14 work_bytes, 15 info. */
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
 * With precision = RQ_MIXED the sketch, TRQRCP's Y2^T A and Z1 = A V run on
 * the FP32 matrix cores (RQ_MIXED_BF16: the sketch on the BF16 ones; A V in
 * FP64 below RQ_MIXED_FP64_BELOW, see RQ_MIXED), from an FP32 copy of A made
 * inside the call and permuted along with A; the panels, reflectors, T, the
 * rows of R, the sample QRCP, the orthogonal factors and the SVD of X stay
 * FP64, so U and V are orthonormal to FP64 accuracy and only the
 * approximation carries the FP32 rounding of the products (relative about
 * sqrt(n) 6e-8), far below the truncation errors this path is meant for.
 * Arguments: 1 stream, 2 m, 3 n, 4 k, 5 A, 6 lda, 7 b, 8 p, 9 seed,
 * 10 precision, 11 U, 12 ldu, 13 sigma, 14 VT, 15 ldvt, 16 work,
 * 17 work_bytes, 18 info.
 */
int rq_tuxv(void* stream, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, int32_t b, int32_t p,
            uint64_t seed, int32_t precision, double* U, int64_t ldu, double* sigma, double* VT, int64_t ldvt,
            void* work, size_t work_bytes, int32_t* info);

/* As rq_tuxv in FP64 with a caller-supplied Omega (a test hook):
 * arguments 1-8 as rq_tuxv, 9 Omega, 10 ldo, 11 U, 12 ldu, 13 sigma, 14 VT,
 * 15 ldvt, 16 work, 17 work_bytes, 18 info. */
int rq_tuxv_omega(void* stream, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, int32_t b, int32_t p,
                  const double* Omega, int64_t ldo, double* U, int64_t ldu, double* sigma, double* VT, int64_t ldvt,
                  void* work, size_t work_bytes, int32_t* info);

/*
 * TUXV with j_max >= 1 iterations -- Alg. 7 (Section 6): after the first LQ,
 * steps alternate between the QR of Z = A V (new U, upper triangular X) and
 * the LQ of Z = U^T A, computed as the QR of A^T U (new V, lower triangular
 * X); j_max counts these steps, so j_max = 1 is rq_tuxv.  Each step can only
 * lower the error ||A - U X V^T||_F (the best approximation with the new
 * column or row space).  The SVD of the last X gives the outputs, as in
 * rq_tuxv.  FP64 only; workspace: RQ_OP_TUXV with RQ_FP64.
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
 * Sketch alone (the first step of Alg. 4, Section 3): B = Omega A with Omega
 * drawn from `seed` as in rq_omega, in the given precision (RQ_FP64, RQ_MIXED:
 * FP32 matrix cores, RQ_MIXED_BF16: BF16 matrix cores); B is l x n
 * column-major (ldb >= l).
 * Arguments: 1 stream, 2 m, 3 n, 4 A, 5 lda, 6 l, 7 seed, 8 precision, 9 B,
 * 10 ldb, 11 work, 12 work_bytes (RQ_OP_RQRCP workspace with b = l, p = 0
 * suffices).
 */
int rq_sketch(void* stream, int64_t m, int64_t n, const double* A, int64_t lda, int32_t l, uint64_t seed,
              int32_t precision, double* B, int64_t ldb, void* work, size_t work_bytes);

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
 * Batched TRQRCP + TUXV (Alg. 6, Alg. 7 with j_max = 1 and the SVD of X,
 * Sections 5.1 and 6) for many independent matrices of uneven sizes with a
 * common rank k, block b and oversampling p.  Each matrix gets the result of
 * rq_tuxv (A ~= U diag(sigma) VT, its own seed for Omega) -- the same pivots
 * and, up to rounding, the same sigma and U diag(sigma) VT; the orthogonal
 * factors are formed explicitly (Gram-Schmidt against the earlier blocks and
 * shifted CholeskyQR, three passes) instead of as reflectors.  Every stage
 * of the method is one launch over the whole batch (grouped products over
 * the output tiles of all matrices, one workgroup per matrix for the sample
 * QRCP, the small factorizations and the SVD).
 *   Usage: rq_batch_workspace_bytes -> allocate `work` -> rq_batch_plan_create
 *   (builds the launch sequence and uploads its descriptors into `work` with
 *   a blocking copy; the plan refers to the matrices' device buffers named
 *   in items) -> rq_tuxv_batched (enqueues kernels only: no copy, no
 *   allocation, no synchronisation, so it can be captured in a HIP graph and
 *   replayed; calls that share a plan must be ordered on one stream) ->
 *   rq_batch_plan_destroy.
 *   precision: RQ_FP64 or RQ_MIXED (the sketch, Q_J^T A and A V on the FP32
 *   matrix cores).  tile: the output tile of the grouped products
 *   (RQ_TILE_64x64, RQ_TILE_32x32, RQ_TILE_128x64).
 *   Limits: 1 <= k <= 64, b divides k, b + p <= 64, k <= m_i, k <= n_i <= 8192.
 *   info (per matrix, optional): 0, j > 0 (non-finite sample norm at pivot
 *   step j), -2 (the SVD of X did not converge), -4 (a CholeskyQR pass met a
 *   non-positive pivot: numerically rank-deficient columns; the result is
 *   then not reliable).
 */
typedef struct {
  int64_t m, n;          /* A is m x n */
  const double* A;       /* device, column-major, lda >= m (read only) */
  int64_t lda;
  double* U;             /* out: m x k, ldu >= m */
  int64_t ldu;
  double* sigma;         /* out: k, descending */
  double* VT;            /* out: k x n, ldvt >= k */
  int64_t ldvt;
  int64_t* jpvt;         /* out (may be NULL): the k pivots */
  int32_t* info;         /* out (may be NULL): device status word */
  uint64_t seed;         /* Omega of this matrix, as rq_omega */
} rq_batch_matrix;

typedef struct rq_batch_plan rq_batch_plan;
enum { RQ_TILE_64x64 = 0, RQ_TILE_32x32 = 1, RQ_TILE_128x64 = 2 };

/* Workspace bytes of a batch.  Arguments: 1 items (host array), 2 count,
 * 3 k, 4 b, 5 p, 6 precision, 7 bytes (out, host).  -1: an item is invalid. */
int rq_batch_workspace_bytes(const rq_batch_matrix* items, int32_t count, int64_t k, int32_t b, int32_t p,
                             int32_t precision, size_t* bytes);
/* Arguments: 1 items, 2 count, 3 k, 4 b, 5 p, 6 precision, 7 tile, 8 work
 * (device), 9 work_bytes, 10 plan (out, host). */
int rq_batch_plan_create(const rq_batch_matrix* items, int32_t count, int64_t k, int32_t b, int32_t p,
                         int32_t precision, int32_t tile, void* work, size_t work_bytes, rq_batch_plan** plan);
/* Arguments: 1 stream, 2 plan. */
int rq_tuxv_batched(void* stream, const rq_batch_plan* plan);
int rq_batch_plan_destroy(rq_batch_plan* plan);

/*
 * Test hook: per-block dump of the sample (host-side, process-wide; not for
 * concurrent use).  With `buf` non-null, rq_rqrcp, rq_rqrcp_omega, rq_trqrcp
 * and rq_trqrcp_omega copy, right before each block's sample QRCP, the
 * sample that block works on -- B^[0] = Omega A for the first block, the
 * sample refreshed by eq. (update1) of Section 4 for every later one -- into
 * buf: block J (starting at column i0 = J b) stores its l x (n - i0) sample
 * column-major with leading dimension l at element offset
 * l * sum_{J' < J} (n - J' b).  A block whose sample does not fit in
 * `capacity` elements (and every block after it) is not stored.  The rest
 * of a block's state needs no dump: its pivots, tau and rows of R are final
 * once the block is done and appear unchanged in the call's outputs.
 * buf = NULL turns the dump off.  Arguments: 1 buf (device, FP64),
 * 2 capacity (elements).  Returns 0, or -2 for a negative capacity.
 */
int rq_set_block_dump(double* buf, int64_t capacity);

/*
 * Test hook: the panel factorization path (host-side, process-wide).
 * mode 0 (default): CholeskyQR2 with Householder reconstruction, and the
 * column-by-column Householder panel only where CholeskyQR reports failure;
 * mode 1: the column-by-column Householder panel (the "qr" step of Alg. 4 /
 * Alg. 6 computed as in Alg. 1 without pivoting) and the forward T
 * recurrence for every block, with the sample update forming
 * W11 = S11 R11^-1 by its own triangular solve.  Returns the previous mode,
 * or -1 for an invalid mode.
 */
int rq_set_panel_path(int32_t mode);

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
