// C ABI and host-side drivers: RQRCP (Alg. 4), TRQRCP (Alg. 6), TUXV (Alg. 7
// with j_max = 1 plus the SVD of X) and the unpivoted blocked QR comparator.
// The drivers only enqueue kernels (on the caller's stream, and for RQRCP's
// look-ahead on a second library-owned stream joined back by events); pivot
// indices and all intermediate state stay on the device (no host
// synchronisation).
#include <atomic>
#include <mutex>
#include <type_traits>

#include "rqrcp.h"
#include "kernels.hpp"
#include "prof.hpp"

namespace rq {

namespace {

constexpr int FLAG_STRIDE = 512;  // 32-bit flag words per block (sample QRCP + panel)

__global__ void iota64_kernel(int64_t n, int64_t* v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = i;
}

// info: the sample QRCP's non-finite-norm step, or -(error word) when a
// stage failed (1: a cross-workgroup wait timed out, 2: the SVD of X hit its
// sweep limit, 3: the fallback panel was needed and does not fit the device)
__global__ void finish_kernel(const int* err, const int* info_ws, int32_t* info) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int v = *info_ws;
    if (*err) v = -*err;
    *info = v;
  }
}

// *w = v when the gate word is nonzero (or always, without a gate)
__global__ void set_word_kernel(int* w, int v, const int* gate) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && (!gate || *gate != 0)) *w = v;
}

int launch_set_word(hipStream_t s, int* w, int v, const int* gate = nullptr) {
  hipLaunchKernelGGL(set_word_kernel, dim3(1), dim3(64), 0, s, w, v, gate);
  RQ_HIP(hipGetLastError());
  return 0;
}

__global__ void transpose_kernel(int64_t rows, int64_t cols, const double* __restrict__ src, int64_t lds,
                                 double* __restrict__ dst, int64_t ldd) {
  // dst(j, i) = src(i, j), src rows x cols
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t j = idx / rows, i = idx - j * rows;
  dst[j + i * ldd] = src[i + j * lds];
}

int launch_iota(hipStream_t s, int64_t n, int64_t* v) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(iota64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, v);
  RQ_HIP(hipGetLastError());
  return 0;
}

int launch_transpose(hipStream_t s, int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst,
                     int64_t ldd) {
  if (rows <= 0 || cols <= 0) return 0;
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((rows * cols + 255) / 256)), dim3(256), 0, s, rows, cols, src,
                     lds, dst, ldd);
  RQ_HIP(hipGetLastError());
  return 0;
}

#define RQ_TRY(x)            \
  do {                       \
    int _rc = (x);           \
    if (_rc) return _rc;     \
  } while (0)

// ------------------------------------------------------------------ workspace
// Every operation carves its buffers from the caller's workspace with the
// same code path used by rq_workspace_bytes (base pointer null = size query).
struct Common {
  unsigned* flags;   // nblk * FLAG_STRIDE words
  int* err;          // 1 word
  int* info;         // 1 word
  size_t flag_words;
};

void carve_common(Carve& cv, int64_t nblk, Common& c) {
  c.flag_words = (size_t)nblk * FLAG_STRIDE + 64;
  c.flags = cv.take<unsigned>(c.flag_words);
  c.err = (int*)carved_at(c.flags, (size_t)nblk * FLAG_STRIDE);
  c.info = carved_at(c.err, 1);
}

struct SampleBufs {
  double* omega;      // l x m (ld l)
  double* smp;        // sample, ls x n (ld ls = sample_rows_padded(l)); rows past l are zero
  int ls;
  SampleQrcpWork sq;
  int* piv;           // b
  double* w11;        // b x b
};

void carve_sample(Carve& cv, int64_t m, int64_t n, int b, int l, SampleBufs& sb) {
  sb.omega = cv.take<double>((size_t)l * m);
  sb.ls = std::max(sample_rows_padded(l), l);
  sb.smp = cv.take<double>((size_t)n * sb.ls);
  sb.sq.cand = cv.take<double>(sample_qrcp_cand_elems());
  sb.sq.cand_idx = cv.take<int>(sample_qrcp_idx_elems());
  sb.sq.theta = cv.take<double>(sample_qrcp_theta_elems());
  sb.piv = cv.take<int>(b);
  sb.w11 = cv.take<double>((size_t)b * b);
}

struct BlockBufs {
  double* panel_slots;
  double* G;          // b x b
  double* T;          // b x b
  double* zbuf;       // b x n
  double* wt;         // b x n
  double* splitk;
  size_t splitk_elems;
  double* cq;         // CholeskyQR scratch
};

void carve_block(Carve& cv, int64_t m, int64_t n, int b, BlockBufs& bb) {
  bb.panel_slots = cv.take<double>(panel_slot_elems(m, b));
  bb.cq = cv.take<double>(cholqr_scratch_elems(m, b));
  bb.G = cv.take<double>((size_t)b * b);
  bb.T = cv.take<double>((size_t)b * b);
  bb.zbuf = cv.take<double>((size_t)b * std::max<int64_t>(n, 1));
  bb.wt = cv.take<double>((size_t)b * std::max<int64_t>(n, 1));
  bb.splitk_elems =
      std::max<size_t>({gemm_scratch_elems(b, n, m), gemm_scratch_elems(b, 2 * b, m), (size_t)1});
  bb.splitk = cv.take<double>(bb.splitk_elems);
}

// Words of a block's flag region: [0, 128) sample QRCP, [128, 384) panel
// fallback, 448 panel status (nonzero: CholeskyQR failed, fallback runs).
constexpr int FLAG_PANEL_STATUS = 448;

PanelWork panel_work(const BlockBufs& bb, const Common& c, int64_t J) {
  PanelWork w;
  w.slots = bb.panel_slots;
  w.flags = c.flags + (size_t)J * FLAG_STRIDE + 128;
  w.err = c.err;
  w.gate = (const int*)(c.flags + (size_t)J * FLAG_STRIDE + FLAG_PANEL_STATUS);
  return w;
}

SampleQrcpWork sq_work(const SampleBufs& sb, const Common& c, int64_t J) {
  SampleQrcpWork w = sb.sq;
  w.flags = c.flags + (size_t)J * FLAG_STRIDE;
  w.err = c.err;
  return w;
}

int64_t nblocks(int64_t k, int b) { return (k + b - 1) / b; }

// Algorithmic flops of a block's sample QRCP: Householder steps t < bJ on
// the l x nJ sample, each a norm and a reflector on rows t..l-1 applied to the
// nJ - t - 1 columns to its right (norm maintenance, which an implementation
// may do by recomputation or downdating, is not counted).
double sample_qrcp_flops(int l, int64_t nJ, int bJ) {
  double f = 0.0;
  for (int t = 0; t < bJ; ++t) f += 4.0 * (double)(l - t) * (double)(nJ - t - 1) + 3.0 * (double)(l - t);
  return f;
}

// Test hooks (process-wide): the panel path and the per-block sample dump.
std::atomic<int> g_panel_mode{0};
std::atomic<double*> g_dump{nullptr};
std::atomic<int64_t> g_dump_cap{0};

// Copies block J's sample (l x nJ, ld ls) into the dump buffer, if one is set
// and the block fits; `off` accumulates the element offset across blocks.
int dump_sample(hipStream_t s, const double* smp, int ls, int l, int64_t nJ, int64_t& off) {
  double* buf = g_dump.load(std::memory_order_relaxed);
  if (!buf) return 0;
  const int64_t need = (int64_t)l * nJ;
  if (off >= 0 && off + need <= g_dump_cap.load(std::memory_order_relaxed)) {
    RQ_TRY(launch_copy2d(s, l, nJ, smp, ls, buf + off, l));
    off += need;
  } else {
    off = -1;  // this block and the later ones are not stored
  }
  return 0;
}

// ------------------------------------------------------------------ pieces
// Panel QR of A(i0:m, i0:i0+bJ) + connection matrix T of its reflectors:
// CholeskyQR2 + Householder reconstruction (preconditioned by the sample's
// S11 when given), with the column-by-column Householder panel as fallback.
// W11 (with S11): where the panel writes S11 R11^-1 for the sample update
// (the reconstruction from its own factors, or the fallback's tail from R11).
int panel_and_t(hipStream_t s, double* A, int64_t lda, int64_t m, int64_t i0, int bJ, double* tau, double* Y,
                int64_t ldy, const BlockBufs& bb, const Common& c, int64_t J, const double* S11 = nullptr,
                int64_t srs = 0, int64_t scs = 0, double* W11 = nullptr) {
  const int64_t mJ = m - i0;
  const double dm = (double)mJ, db = (double)bJ;
  PanelWork pw = panel_work(bb, c, J);
  int* st = (int*)pw.gate;
  ProfScope ps(PC_PANEL, s, 32.0 * dm * db, 6.0 * dm * db * db);
  const bool forced = g_panel_mode.load(std::memory_order_relaxed) == 1;
  if (forced) {
    RQ_TRY(launch_set_word(s, st, 1));  // the status word that selects the column panel
  } else {
    RQ_TRY(launch_panel_cholqr(s, A + i0 + i0 * lda, lda, mJ, bJ, S11, srs, scs, tau, Y, ldy, bb.T, bb.cq, bb.splitk,
                               bb.splitk_elems, st, W11));
  }
  // the column panel if the status word is set, else the copy of the
  // reconstructed Y's rows below the top block into the panel's storage
  const int rc = launch_panel(s, A + i0 + i0 * lda, lda, mJ, bJ, tau, Y, ldy, pw, !forced);
  if (rc == RQ_PANEL_TOO_TALL) {
    // the column panel's workgroups cannot all be resident at this height:
    // forced, that is an enqueue error; as the fallback, a failed CholeskyQR
    // (status word set) makes the call report info = -3 instead
    if (forced) return rc;
    RQ_TRY(launch_set_word(s, c.err, 3, st));
  } else if (rc) {
    return rc;
  }
  // after the column panel: its T, and W11 = S11 R11^-1 for the sample update
  RQ_TRY(launch_fallback_tail(s, mJ, bJ, Y, ldy, tau, bb.T, st, S11, srs, scs, A + i0 + i0 * lda, lda, W11));
  return 0;
}

// C = alpha op(A) op(B) + beta C in FP64, or with `mixed` on the FP32 matrix
// cores (operands rounded to FP32, FP32 accumulation, added to FP64 C).
int gemm_prec(hipStream_t s, bool mixed, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
              const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
              double* scratch, size_t scratch_elems) {
  if (mixed) return launch_gemm_f32(s, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, scratch, scratch_elems);
  return launch_gemm(s, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, scratch, scratch_elems);
}

// Trailing update Q^T C = C - Y (T^T (Y^T C)) of C = A(i0:m, i0+bJ:n); with
// `mixed` the two products with C on the FP32 matrix cores.
int trailing_update(hipStream_t s, double* A, int64_t lda, int64_t m, int64_t n, int64_t i0, int bJ, const double* Y,
                    int64_t ldy, const BlockBufs& bb, bool mixed = false) {
  const int64_t mJ = m - i0, Nt = n - i0 - bJ;
  if (Nt <= 0) return 0;
  double* C = A + i0 + (i0 + bJ) * lda;
  const double dm = (double)mJ, dn = (double)Nt, db = (double)bJ;
  {
    ProfScope ps(PC_GEMM_YTA, s, 8.0 * (dm * dn + dm * db + db * dn), 2.0 * db * dn * dm + 2.0 * db * db * dn);
    RQ_TRY(gemm_prec(s, mixed, true, false, bJ, Nt, mJ, 1.0, Y, ldy, C, lda, 0.0, bb.zbuf, bJ, bb.splitk,
                     bb.splitk_elems));
    RQ_TRY(launch_gemm(s, true, false, bJ, Nt, bJ, 1.0, bb.T, bJ, bb.zbuf, bJ, 0.0, bb.wt, bJ, nullptr, 0));
  }
  ProfScope ps(PC_GEMM_UPDATE, s, 8.0 * (2.0 * dm * dn + dm * db + db * dn), 2.0 * dm * dn * db);
  RQ_TRY(gemm_prec(s, mixed, false, false, mJ, Nt, bJ, -1.0, Y, ldy, bb.wt, bJ, 1.0, C, lda, nullptr, 0));
  return 0;
}

// ------------------------------------------------------------------ look-ahead
// RQRCP's trailing update splits in two once W^T is known: the first bJ rows
// (R12, which the sample update needs at once) and the rows below them,
// which nothing reads until the next block's swaps.  The rows below run in
// the next block's sample-QRCP launch, on workgroups of their own beside the
// sample QRCP's (which touches only the sample): one launch on the caller's
// stream, ordered before the swaps like any other.  rq_set_lookahead(0) runs
// them right after R12 instead.  The tiles are the same either way, so the
// results are bitwise the same.
std::atomic<int> g_lookahead{1};

bool lookahead_enabled() { return g_lookahead.load(std::memory_order_relaxed) != 0; }

// Workgroups of the update beside a sample QRCP of nJ columns: every CU
// the sample QRCP leaves (one workgroup per CU; the launch clamps this to
// the places that are free).  Leaving 16 or 8 of them idle measured 0.4 and
// 0.2 ms slower per 8192 x 8192 factorization: in the first blocks the
// update is the longer of the two.
int64_t beside_update_workgroups(int64_t nJ) {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
  }
  return std::max<int64_t>(1, cus - sample_qrcp_workgroups(nJ));
}

// Trailing update with look-ahead: W^T = T^T (Y^T C) and R12 on s; the rows
// below R12 are described in `later` for the next sample QRCP's launch
// (later.M = 0: nothing left).
int trailing_update_split(hipStream_t s, double* A, int64_t lda, int64_t m, int64_t n, int64_t i0, int bJ,
                          const double* Y, int64_t ldy, const BlockBufs& bb, bool mixed, BesideUpdate& later) {
  const int64_t mJ = m - i0, Nt = n - i0 - bJ;
  double* C = A + i0 + (i0 + bJ) * lda;
  const double dm = (double)mJ, dn = (double)Nt, db = (double)bJ;
  {
    ProfScope ps(PC_GEMM_YTA, s, 8.0 * (dm * dn + dm * db + db * dn), 2.0 * db * dn * dm + 2.0 * db * db * dn);
    RQ_TRY(gemm_prec(s, mixed, true, false, bJ, Nt, mJ, 1.0, Y, ldy, C, lda, 0.0, bb.zbuf, bJ, bb.splitk,
                     bb.splitk_elems));
    RQ_TRY(launch_gemm(s, true, false, bJ, Nt, bJ, 1.0, bb.T, bJ, bb.zbuf, bJ, 0.0, bb.wt, bJ, nullptr, 0));
  }
  {
    ProfScope ps(PC_GEMM_UPDATE, s, 8.0 * (2.0 * db * dn + db * db + db * dn), 2.0 * db * dn * db);
    RQ_TRY(gemm_prec(s, mixed, false, false, bJ, Nt, bJ, -1.0, Y, ldy, bb.wt, bJ, 1.0, C, lda, nullptr, 0));
  }
  later = BesideUpdate();
  if (mJ > bJ && Nt > 0) {
    later.M = mJ - bJ; later.N = Nt; later.K = bJ;
    later.A = Y + bJ; later.lda = ldy;
    later.B = bb.wt; later.ldb = bJ;
    later.C = C + bJ; later.ldc = lda;
    later.f32 = mixed;
    later.wgs = beside_update_workgroups(Nt);
  }
  return 0;
}

// Sample update, eq. (update1): B1 = S12 - (S11 R11^-1) R12, B2 = S22, on the
// sample columns of this block (S + i0 * ls, ld ls).  W11 = S11 R11^-1 is
// already in sb.w11 (written by the panel).
int sample_update(hipStream_t s, double* A, int64_t lda, int64_t n, int64_t i0, int bJ, double* s_blk,
                  const SampleBufs& sb) {
  const int64_t Nt = n - i0 - bJ;
  if (Nt <= 0) return 0;
  const double* R12 = A + i0 + (i0 + bJ) * lda;
  const double dn = (double)Nt, db = (double)bJ;
  ProfScope ps(PC_SAMPLE_UPDATE, s, 8.0 * (3.0 * db * dn + 2.0 * db * db), 2.0 * db * db * dn);
  // S(0:bJ, bJ:) -= W11 R12
  RQ_TRY(launch_gemm(s, false, false, bJ, Nt, bJ, -1.0, sb.w11, bJ, R12, lda, 1.0, s_blk + (int64_t)bJ * sb.ls, sb.ls,
                     nullptr, 0));
  return 0;
}

// Sketch: S (l x n, ld ls) = Omega A with Omega l x m (ld ldo); rows l..ls-1
// of S are zeroed.  With scratch the product is split along m.  `prec`:
// RQ_FP64, RQ_MIXED (FP32 matrix cores) or RQ_MIXED_BF16 (BF16 matrix cores,
// Omega and A rounded to BF16, FP32 accumulation).
template <typename TA>
int sketch(hipStream_t s, int64_t m, int64_t n, const TA* A, int64_t lda, int l, const double* Omega, int64_t ldo,
           double* S, int ls, double* scratch, size_t scratch_elems, int prec) {
  const double dm = (double)m, dn = (double)n, dl = (double)l;
  ProfScope ps(PC_SKETCH, s, (double)sizeof(TA) * dm * dn + 8.0 * (dl * dm + dl * dn), 2.0 * dl * dm * dn);
  if (prec == RQ_MIXED_BF16) {
    RQ_TRY(launch_sketch_bf16(s, l, n, m, Omega, ldo, A, lda, S, ls, scratch, scratch_elems));
  } else if (prec == RQ_MIXED || !std::is_same<TA, double>::value) {
    RQ_TRY(launch_gemm_f32(s, false, false, l, n, m, 1.0, Omega, ldo, A, lda, 0.0, S, ls, scratch, scratch_elems));
  } else {
    RQ_TRY(launch_gemm(s, false, false, l, n, m, 1.0, Omega, ldo, (const double*)A, lda, 0.0, S, ls, scratch,
                       scratch_elems));
  }
  return launch_zero_rows(s, l, ls, n, S, ls);
}

// ------------------------------------------------------------------ RQRCP / QR
struct FactorWS {
  Common c;
  SampleBufs sb;
  BlockBufs bb;
  double* ybuf;  // m x b
};

void carve_factor(Carve& cv, int64_t m, int64_t n, int b, int p, bool pivoting, FactorWS& f) {
  const int64_t k = std::min(m, n);
  carve_common(cv, nblocks(k, b), f.c);
  if (pivoting) carve_sample(cv, m, n, b, b + p, f.sb);
  carve_block(cv, m, n, b, f.bb);
  f.ybuf = cv.take<double>((size_t)m * b);
}

// RQRCP (Alg. 4) when pivoting, the unpivoted blocked QR otherwise; with
// resample, RSRQRCP (Alg. 5): every block draws Omega^[J] (l x mJ, Philox key
// (seed, J)) and samples the updated trailing matrix A(i0:m, i0:n) with it,
// and there is no sample update.
int factor_impl(hipStream_t s, int64_t m, int64_t n, double* A, int64_t lda, int b, int p, uint64_t seed,
                const double* Omega, int64_t ldo, int64_t* jpvt, double* tau, void* work, size_t wbytes,
                int32_t* info, bool pivoting, bool resample, int prec, int iwork, bool allow_lookahead = true) {
  const bool mixed = prec != RQ_FP64;
  FactorWS f;
  Carve cv(work, wbytes);
  carve_factor(cv, m, n, b, p, pivoting, f);
  if (!cv.ok) return -iwork;
  const int64_t k = std::min(m, n);
  const int l = b + p;
  RQ_TRY(launch_fill(s, f.c.flags, f.c.flag_words));
  if (pivoting) RQ_TRY(launch_iota(s, n, jpvt));
  const bool ahead = pivoting && !resample && allow_lookahead && lookahead_enabled();
  BesideUpdate later;  // the previous block's rows below its R12, not yet updated
  if (pivoting && !resample) {
    const double* Om = Omega;
    int64_t ldom = ldo;
    if (!Om) {
      ProfScope ps(PC_OMEGA, s, 8.0 * l * m, 0.0);
      RQ_TRY(launch_omega(s, seed, l, m, f.sb.omega, 1, l));
      Om = f.sb.omega;
      ldom = l;
    }
    RQ_TRY(sketch(s, m, n, (const double*)A, lda, l, Om, ldom, f.sb.smp, f.sb.ls, f.bb.splitk, f.bb.splitk_elems,
                  prec));
  }
  int64_t dump_off = 0;
  for (int64_t i0 = 0, J = 0; i0 < k; ++J) {
    const int bJ = (int)std::min<int64_t>(b, k - i0);
    const int64_t mJ = m - i0, nJ = n - i0;
    double* s_blk = pivoting ? f.sb.smp + i0 * f.sb.ls : nullptr;
    if (pivoting) {
      if (resample) {
        {
          ProfScope ps(PC_OMEGA, s, 8.0 * l * mJ, 0.0);
          RQ_TRY(launch_omega(s, seed, l, mJ, f.sb.omega, 1, l, (uint64_t)J));
        }
        RQ_TRY(sketch(s, mJ, nJ, (const double*)(A + i0 + i0 * lda), lda, l, f.sb.omega, l, s_blk, f.sb.ls,
                      f.bb.splitk, f.bb.splitk_elems, RQ_FP64));
      }
      if (!resample) RQ_TRY(dump_sample(s, s_blk, f.sb.ls, l, nJ, dump_off));
      {
        // (with the previous block's rows below R12 updated in the same launch)
        ProfScope ps(PC_SAMPLE_QRCP, s, 16.0 * l * nJ, sample_qrcp_flops(l, nJ, bJ));
        RQ_TRY(launch_sample_qrcp(s, s_blk, f.sb.ls, l, nJ, bJ, f.sb.piv, f.c.info, (int)i0, sq_work(f.sb, f.c, J),
                                  later.M > 0 ? &later : nullptr));
        later = BesideUpdate();
      }
      ProfScope ps(PC_SWAP, s, 32.0 * m * bJ, 0.0);
      RQ_TRY(launch_apply_swaps(s, f.sb.piv, bJ, i0, A, lda, m, jpvt));
    }
    const bool upd = pivoting && !resample && i0 + bJ < k;
    RQ_TRY(panel_and_t(s, A, lda, m, i0, bJ, tau + i0, f.ybuf, m, f.bb, f.c, J, s_blk, 1, f.sb.ls,
                       upd ? f.sb.w11 : nullptr));
    if (upd && ahead) {
      RQ_TRY(trailing_update_split(s, A, lda, m, n, i0, bJ, f.ybuf, m, f.bb, mixed, later));
    } else {
      RQ_TRY(trailing_update(s, A, lda, m, n, i0, bJ, f.ybuf, m, f.bb, mixed));
    }
    if (upd) RQ_TRY(sample_update(s, A, lda, n, i0, bJ, s_blk, f.sb));
    i0 += bJ;
  }
  if (later.M > 0) {  // (every update is taken by the next block's sample QRCP; this ends any other loop)
    RQ_TRY(gemm_prec(s, later.f32, false, false, later.M, later.N, later.K, -1.0, later.A, later.lda, later.B,
                     later.ldb, 1.0, later.C, later.ldc, nullptr, 0));
  }
  if (info) {
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, f.c.err, f.c.info, info);
    RQ_HIP(hipGetLastError());
  }
  return 0;
}

// ------------------------------------------------------------------ TRQRCP
struct TrqWS {
  Common c;
  SampleBufs sb;
  BlockBufs bb;
  double* yall;   // m x k
  double* wt;     // k x n
  double* gk;     // b x k
  float* a32 = nullptr;  // mixed precision: FP32 copy of A (ld m), permuted with A
  int prec = RQ_FP64;    // with a32: RQ_MIXED or RQ_MIXED_BF16 (the sketch's arithmetic)
};

void carve_trq(Carve& cv, int64_t m, int64_t n, int64_t k, int b, int p, TrqWS& t) {
  carve_common(cv, nblocks(k, b), t.c);
  carve_sample(cv, m, n, b, b + p, t.sb);
  carve_block(cv, m, std::max(n, k), b, t.bb);
  t.yall = cv.take<double>((size_t)m * k);
  t.wt = cv.take<double>((size_t)k * n);
  t.gk = cv.take<double>((size_t)b * k);
}

int trqrcp_core(hipStream_t s, int64_t m, int64_t n, int64_t k, double* A, int64_t lda, int b, int p, uint64_t seed,
                const double* Omega, int64_t ldo, int64_t* jpvt, double* tau, TrqWS& t) {
  const int l = b + p;
  RQ_TRY(launch_fill(s, t.c.flags, t.c.flag_words));
  RQ_TRY(launch_fill(s, t.yall, (size_t)m * k * 2));
  RQ_TRY(launch_iota(s, n, jpvt));
  const double* Om = Omega;
  int64_t ldom = ldo;
  if (!Om) {
    ProfScope ps(PC_OMEGA, s, 8.0 * l * m, 0.0);
    RQ_TRY(launch_omega(s, seed, l, m, t.sb.omega, 1, l));
    Om = t.sb.omega;
    ldom = l;
  }
  if (t.a32)  // mixed precision: from the FP32 copy
    RQ_TRY(sketch(s, m, n, (const float*)t.a32, m, l, Om, ldom, t.sb.smp, t.sb.ls, t.bb.splitk, t.bb.splitk_elems,
                  t.prec));
  else
    RQ_TRY(sketch(s, m, n, (const double*)A, lda, l, Om, ldom, t.sb.smp, t.sb.ls, t.bb.splitk, t.bb.splitk_elems,
                  RQ_FP64));
  int64_t dump_off = 0;
  for (int64_t i0 = 0, J = 0; i0 < k; ++J) {
    const int bJ = (int)std::min<int64_t>(b, k - i0);
    const int64_t mJ = m - i0, nJ = n - i0, Nt = n - i0 - bJ;
    double* s_blk = t.sb.smp + i0 * t.sb.ls;
    RQ_TRY(dump_sample(s, s_blk, t.sb.ls, l, nJ, dump_off));
    {
      ProfScope ps(PC_SAMPLE_QRCP, s, 16.0 * l * nJ, sample_qrcp_flops(l, nJ, bJ));
      RQ_TRY(launch_sample_qrcp(s, s_blk, t.sb.ls, l, nJ, bJ, t.sb.piv, t.c.info, (int)i0, sq_work(t.sb, t.c, J)));
    }
    {
      ProfScope ps(PC_SWAP, s, 32.0 * (m + i0) * bJ, 0.0);
      RQ_TRY(launch_apply_swaps(s, t.sb.piv, bJ, i0, A, lda, m, jpvt));
      if (t.a32) RQ_TRY(launch_apply_swaps_f32(s, t.sb.piv, bJ, i0, t.a32, m, m));
      if (i0 > 0) RQ_TRY(launch_apply_swaps(s, t.sb.piv, bJ, i0, t.wt, k, i0, nullptr));
    }
    double* panel = A + i0 + i0 * lda;
    double* Y2 = t.yall + i0 + i0 * m;
    // selected columns: A_hat = A(i0:m, sel) - Y(i0:m, 0:i0) W^T(0:i0, sel)
    if (i0 > 0) {
      ProfScope ps(PC_TRQ_PRODUCTS, s, 8.0 * (2.0 * mJ * bJ + mJ * i0 + i0 * bJ), 2.0 * mJ * bJ * i0);
      RQ_TRY(launch_gemm(s, false, false, mJ, bJ, i0, -1.0, t.yall + i0, m, t.wt + i0 * k, k, 1.0, panel, lda,
                         nullptr, 0));
    }
    const bool upd = i0 + bJ < k;
    RQ_TRY(panel_and_t(s, A, lda, m, i0, bJ, tau + i0, Y2, m, t.bb, t.c, J, s_blk, 1, t.sb.ls,
                       upd ? t.sb.w11 : nullptr));
    if (Nt > 0) {
      double* Atr = A + i0 + (i0 + bJ) * lda;
      double* wt_tr = t.wt + (i0 + bJ) * k;
      // Z = Y2^T A(i0:m, trail) - (Y2^T Y1) W1^T(:, trail)
      {
        ProfScope ps(PC_GEMM_YTA, s, 8.0 * ((double)mJ * Nt + (double)mJ * bJ + (double)bJ * Nt),
                     2.0 * bJ * (double)Nt * mJ);
        if (t.a32)  // mixed precision: from the FP32 copy on the FP32 matrix cores
          RQ_TRY(launch_gemm_f32(s, true, false, bJ, Nt, mJ, 1.0, Y2, m, t.a32 + i0 + (i0 + bJ) * m, m, 0.0,
                                 t.bb.zbuf, bJ, t.bb.splitk, t.bb.splitk_elems));
        else
          RQ_TRY(launch_gemm(s, true, false, bJ, Nt, mJ, 1.0, Y2, m, Atr, lda, 0.0, t.bb.zbuf, bJ, t.bb.splitk,
                             t.bb.splitk_elems));
      }
      ProfScope ps(PC_TRQ_PRODUCTS, s, 8.0 * ((double)mJ * (bJ + i0) + 2.0 * (i0 + bJ) * Nt + 3.0 * bJ * Nt),
                   2.0 * bJ * ((double)i0 * mJ + 2.0 * i0 * Nt + (double)bJ * Nt + (double)bJ * Nt));
      if (i0 > 0) {
        RQ_TRY(launch_gemm(s, true, false, bJ, i0, mJ, 1.0, Y2, m, t.yall + i0, m, 0.0, t.gk, bJ, t.bb.splitk,
                           t.bb.splitk_elems));
        RQ_TRY(launch_gemm(s, false, false, bJ, Nt, i0, -1.0, t.gk, bJ, wt_tr, k, 1.0, t.bb.zbuf, bJ, nullptr, 0));
      }
      // W2^T = T2^T Z
      RQ_TRY(launch_gemm(s, true, false, bJ, Nt, bJ, 1.0, t.bb.T, bJ, t.bb.zbuf, bJ, 0.0, wt_tr + i0, k, nullptr, 0));
      // new rows of R: A(i0:i0+bJ, trail) -= Y(i0:i0+bJ, 0:i0+bJ) W^T(0:i0+bJ, trail)
      RQ_TRY(launch_gemm(s, false, false, bJ, Nt, i0 + bJ, -1.0, t.yall + i0, m, wt_tr, k, 1.0, Atr, lda, nullptr,
                         0));
    }
    if (upd) RQ_TRY(sample_update(s, A, lda, n, i0, bJ, s_blk, t.sb));
    i0 += bJ;
  }
  return 0;
}

// ------------------------------------------------------------------ QR + explicit Q (TUXV)
struct QrWS {
  Common c;
  BlockBufs bb;
  double* yall;   // rows x kq (explicit reflectors)
  double* tall;   // nblk * b * b
  double* z2;     // b x kq
};

void carve_qr(Carve& cv, int64_t rows, int64_t kq, int b, QrWS& q) {
  carve_common(cv, nblocks(kq, b), q.c);
  carve_block(cv, rows, kq, b, q.bb);
  q.yall = cv.take<double>((size_t)rows * kq);
  q.tall = cv.take<double>((size_t)nblocks(kq, b) * b * b);
  q.z2 = cv.take<double>((size_t)b * kq);
}

// Blocked Householder QR of the rows x kq matrix M (ld ldm, rows >= kq); the
// explicit reflectors go to q.yall and each block's T to q.tall.
int qr_explicit(hipStream_t s, int64_t rows, int64_t kq, double* M, int64_t ldm, int b, double* tau, QrWS& q) {
  RQ_TRY(launch_fill(s, q.c.flags, q.c.flag_words));
  RQ_TRY(launch_fill(s, q.yall, (size_t)rows * kq * 2));
  for (int64_t i0 = 0, J = 0; i0 < kq; ++J) {
    const int bJ = (int)std::min<int64_t>(b, kq - i0);
    double* Y = q.yall + i0 + i0 * rows;
    RQ_TRY(panel_and_t(s, M, ldm, rows, i0, bJ, tau + i0, Y, rows, q.bb, q.c, J));
    RQ_TRY(launch_copy2d(s, bJ, bJ, q.bb.T, bJ, q.tall + (size_t)J * b * b, bJ));
    RQ_TRY(trailing_update(s, M, ldm, rows, kq, i0, bJ, Y, rows, q.bb));
    i0 += bJ;
  }
  return 0;
}

// Q(:, 0:kq) = H_0 ... H_{kq-1} [I; 0], accumulated backwards block by block.
int form_q(hipStream_t s, int64_t rows, int64_t kq, int b, QrWS& q, double* Q, int64_t ldq) {
  RQ_TRY(launch_set_identity(s, rows, kq, Q, ldq));
  const int64_t nb = nblocks(kq, b);
  for (int64_t J = nb - 1; J >= 0; --J) {
    const int64_t i0 = J * b;
    const int bJ = (int)std::min<int64_t>(b, kq - i0);
    const int64_t mJ = rows - i0, Nc = kq - i0;
    const double* Y = q.yall + i0 + i0 * rows;
    double* Qs = Q + i0 + i0 * ldq;
    const double* T = q.tall + (size_t)J * b * b;
    RQ_TRY(launch_gemm(s, true, false, bJ, Nc, mJ, 1.0, Y, rows, Qs, ldq, 0.0, q.bb.zbuf, bJ, q.bb.splitk,
                       q.bb.splitk_elems));
    RQ_TRY(launch_gemm(s, false, false, bJ, Nc, bJ, 1.0, T, bJ, q.bb.zbuf, bJ, 0.0, q.z2, bJ, nullptr, 0));
    RQ_TRY(launch_gemm(s, false, false, mJ, Nc, bJ, -1.0, Y, rows, q.z2, bJ, 1.0, Qs, ldq, nullptr, 0));
  }
  return 0;
}

// ------------------------------------------------------------------ TUXV
struct TuxvWS {
  TrqWS trq;
  QrWS qz, qu;
  double* ac;      // m x n copy of A
  int64_t* jp;     // n
  double* tk;      // k (TRQRCP tau)
  double* z0t;     // n x k
  double* tz;      // k
  double* v;       // n x k
  double* z1;      // m x k
  double* tu;      // k
  double* u1;      // m x k
  double* x;       // k x k
  double* ux;      // k x k
  double* vx;      // k x k
  double* svdtmp;  // k x k
  unsigned* svdflags;  // arrival counter and per-sweep flags of the Jacobi sweeps
  double* vperm;   // mixed precision: n x k, rows of V in the column order of A P
};

void carve_tuxv(Carve& cv, int64_t m, int64_t n, int64_t k, int b, int p, TuxvWS& t, int prec = RQ_FP64) {
  const bool mixed = prec != RQ_FP64;
  carve_trq(cv, m, n, k, b, p, t.trq);
  carve_qr(cv, n, k, b, t.qz);
  carve_qr(cv, m, k, b, t.qu);
  // one error word for every cooperative stage of the call
  t.qz.c.err = t.trq.c.err;
  t.qu.c.err = t.trq.c.err;
  t.ac = cv.take<double>((size_t)m * n);
  t.jp = cv.take<int64_t>(n);
  t.tk = cv.take<double>(k);
  t.z0t = cv.take<double>((size_t)n * k);
  t.tz = cv.take<double>(k);
  t.v = cv.take<double>((size_t)n * k);
  t.z1 = cv.take<double>((size_t)m * k);
  t.tu = cv.take<double>(k);
  t.u1 = cv.take<double>((size_t)m * k);
  t.x = cv.take<double>((size_t)k * k);
  t.ux = cv.take<double>((size_t)k * k);
  t.vx = cv.take<double>((size_t)k * k);
  t.svdtmp = cv.take<double>((size_t)k * k);
  t.svdflags = cv.take<unsigned>(128);
  t.vperm = nullptr;
  if (mixed) {
    t.trq.a32 = cv.take<float>((size_t)m * n);
    t.trq.prec = prec;
    t.vperm = cv.take<double>((size_t)n * k);
  }
}

// Alg. 7 with jmax multiply-and-factorize steps after the first LQ, then the
// SVD of the last connection matrix X: A ~ (U Ux) diag(sigma) (Vx^T V^T).
int tuxv_impl(hipStream_t s, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, int b, int p,
              uint64_t seed, const double* Omega, int64_t ldo, double* U, int64_t ldu, double* sigma, double* VT,
              int64_t ldvt, void* work, size_t wbytes, int32_t* info, int jmax, int prec, int iwork) {
  const bool mixed = prec != RQ_FP64;
  TuxvWS t;
  Carve cv(work, wbytes);
  carve_tuxv(cv, m, n, k, b, p, t, prec);
  if (!cv.ok) return -iwork;

  // TRQRCP on a copy: A itself is needed again for Z1 = A V.
  {
    // mixed precision: the FP32 copy of A is written in the same pass
    ProfScope ps(PC_TUXV_PRODUCTS, s, (mixed ? 20.0 : 16.0) * m * n, 0.0);
    if (mixed) RQ_TRY(launch_to_f32(s, m, n, A, lda, t.trq.a32, m, t.ac, m));
    else RQ_TRY(launch_copy2d(s, m, n, A, lda, t.ac, m));
  }
  RQ_TRY(trqrcp_core(s, m, n, k, t.ac, m, b, p, seed, Omega, ldo, t.jp, t.tk, t.trq));
  // Z0 = R P^T, stored transposed (n x k)
  RQ_TRY(launch_scatter_rt(s, k, n, t.ac, m, t.jp, t.z0t, n));
  // LQ of Z0 as the QR of Z0^T -> V (n x k)
  RQ_TRY(qr_explicit(s, n, k, t.z0t, n, b, t.tz, t.qz));
  RQ_TRY(form_q(s, n, k, b, t.qz, t.v, n));
  // Z1 = A V (m x k); mixed precision: (A P) (P^T V) from the permuted FP32 copy
  if (mixed) {
    ProfScope ps(PC_TUXV_PRODUCTS, s, 4.0 * m * n + 8.0 * (2.0 * n * k + (double)m * k), 2.0 * m * (double)n * k);
    RQ_TRY(launch_gather_rows(s, n, k, t.v, n, t.jp, t.vperm, n));
    RQ_TRY(launch_gemm_f32(s, false, false, m, k, n, 1.0, t.trq.a32, m, t.vperm, n, 0.0, t.z1, m, nullptr, 0));
  } else {
    ProfScope ps(PC_TUXV_PRODUCTS, s, 8.0 * ((double)m * n + (double)n * k + (double)m * k), 2.0 * m * (double)n * k);
    RQ_TRY(launch_gemm(s, false, false, m, k, n, 1.0, A, lda, t.v, n, 0.0, t.z1, m, nullptr, 0));
  }
  // QR of Z1 -> U1, X
  RQ_TRY(qr_explicit(s, m, k, t.z1, m, b, t.tu, t.qu));
  RQ_TRY(launch_triu_copy(s, k, t.z1, m, t.x, k));
  RQ_TRY(form_q(s, m, k, b, t.qu, t.u1, m));
  for (int j = 1; j < jmax;) {
    // Z = U^T A, LQ-factorized as the QR of Z^T = A^T U (n x k): V and X
    // lower triangular, A ~ U X V^T
    {
      ProfScope ps(PC_TUXV_PRODUCTS, s, 8.0 * ((double)m * n + (double)m * k + (double)n * k),
                   2.0 * m * (double)n * k);
      RQ_TRY(launch_gemm(s, true, false, n, k, m, 1.0, A, lda, t.u1, m, 0.0, t.z0t, n, nullptr, 0));
    }
    RQ_TRY(qr_explicit(s, n, k, t.z0t, n, b, t.tz, t.qz));
    RQ_TRY(launch_triu_copy(s, k, t.z0t, n, t.ux, k));
    RQ_TRY(launch_transpose(s, k, k, t.ux, k, t.x, k));
    RQ_TRY(form_q(s, n, k, b, t.qz, t.v, n));
    if (++j == jmax) break;
    // Z = A V, QR-factorized: U and X upper triangular
    {
      ProfScope ps(PC_TUXV_PRODUCTS, s, 8.0 * ((double)m * n + (double)n * k + (double)m * k),
                   2.0 * m * (double)n * k);
      RQ_TRY(launch_gemm(s, false, false, m, k, n, 1.0, A, lda, t.v, n, 0.0, t.z1, m, nullptr, 0));
    }
    RQ_TRY(qr_explicit(s, m, k, t.z1, m, b, t.tu, t.qu));
    RQ_TRY(launch_triu_copy(s, k, t.z1, m, t.x, k));
    RQ_TRY(form_q(s, m, k, b, t.qu, t.u1, m));
    ++j;
  }
  // X = Ux diag(sigma) Vx^T
  SvdWork sw;
  sw.colnorm = nullptr; sw.order = nullptr; sw.flags = t.svdflags; sw.err = t.trq.c.err; sw.tmp = t.svdtmp;
  {
    ProfScope ps(PC_SVD, s, 8.0 * 4 * k * k, 0.0);
    RQ_TRY(launch_jacobi_svd(s, (int)k, t.x, k, t.ux, k, sigma, t.vx, k, sw));
  }
  // U = U1 Ux ; VT = Vx^T V^T
  RQ_TRY(launch_gemm(s, false, false, m, k, k, 1.0, t.u1, m, t.ux, k, 0.0, U, ldu, nullptr, 0));
  RQ_TRY(launch_gemm(s, true, true, k, n, k, 1.0, t.vx, k, t.v, n, 0.0, VT, ldvt, nullptr, 0));
  if (info) {
    // merge the error words of every cooperative stage
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, t.trq.c.err, t.trq.c.info, info);
    RQ_HIP(hipGetLastError());
  }
  return 0;
}

// An empty matrix (m = 0 or n = 0): the identity permutation and info = 0;
// there is nothing else to write.
int empty_result(hipStream_t s, int64_t n, int64_t* jpvt, int32_t* info) {
  if (jpvt && n > 0) RQ_TRY(launch_iota(s, n, jpvt));
  if (info) RQ_TRY(launch_fill(s, info, 1));
  return 0;
}

// ------------------------------------------------------------------ argument checks
int check_common(int64_t m, int64_t n, int64_t lda, int b, int p, int im, int in, int ilda, int ib, int ip) {
  if (m < 0 || m > RQ_MAX_ROWS) return -im;
  if (n < 0) return -in;
  if (lda < std::max<int64_t>(1, m)) return -ilda;
  if (b < 1 || b > 64) return -ib;
  if (p < 0 || b + p > 128) return -ip;
  if (n > 65536) return -in;
  return 0;
}

// ------------------------------------------------------------------ allocation-free RQRCP
// The workspace of rq_rqrcp_noalloc: one static array per device, its device
// address looked up once per device (in host code the array's name is only
// a stand-in; kernels get the looked-up address).
static __device__ __align__(256) unsigned char scratch[RQ_NOALLOC_SCRATCH_BYTES];

int scratch_address(void** out) {
  static std::mutex mu;
  static void* addr[64] = {};
  int dev = 0;
  RQ_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return RQ_ERR_HIP_BASE + (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    RQ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return RQ_ERR_HIP_BASE + (int)hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *out = addr[dev];
  return 0;
}

}  // namespace
}  // namespace rq

using namespace rq;

extern "C" {

const char* rq_version(void) { return "rqrcp-gfx950 0.2"; }

int rq_set_lookahead(int32_t on) {
  return g_lookahead.exchange(on ? 1 : 0, std::memory_order_relaxed) != 0 ? 1 : 0;
}

int rq_set_panel_path(int32_t mode) {
  if (mode != 0 && mode != 1) return -1;
  return g_panel_mode.exchange(mode, std::memory_order_relaxed);
}

int rq_set_block_dump(double* buf, int64_t capacity) {
  if (capacity < 0) return -2;
  g_dump_cap.store(buf ? capacity : 0, std::memory_order_relaxed);
  g_dump.store(buf, std::memory_order_relaxed);
  return 0;
}

int rq_workspace_bytes(int32_t op, int64_t m, int64_t n, int64_t k, int32_t b, int32_t p, int32_t precision,
                       size_t* bytes) {
  if (!bytes) return -8;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (b < 1 || b > 64) return -5;
  if (p < 0 || b + p > 128) return -6;
  if (precision < RQ_FP64 || precision > RQ_MIXED_BF16) return -7;
  if (precision != RQ_FP64 && op != RQ_OP_RQRCP && op != RQ_OP_TRQRCP && op != RQ_OP_TUXV) return -7;
  // the limits of the entry points (RQ_OP_SVD reads only k)
  if (op != RQ_OP_SVD && m > RQ_MAX_ROWS) return -2;
  if (op != RQ_OP_SVD && n > 65536) return -3;
  const bool mixed = precision != RQ_FP64;
  size_t sz = 0;
  switch (op) {
    case RQ_OP_RQRCP:
    case RQ_OP_RSRQRCP:
    case RQ_OP_QR: {
      FactorWS f;
      Carve cv(nullptr, 0);
      carve_factor(cv, m, n, b, p, op != RQ_OP_QR, f);
      if (cv.overflowed()) return -2;
      sz = cv.off;
      break;
    }
    case RQ_OP_TRQRCP: {
      if (k < 1 || k > std::min(m, n)) return -4;
      TrqWS t;
      Carve cv(nullptr, 0);
      carve_trq(cv, m, n, k, b, p, t);
      if (mixed) t.a32 = cv.take<float>((size_t)m * n);
      if (cv.overflowed()) return -2;
      sz = cv.off;
      break;
    }
    case RQ_OP_TUXV: {
      if (k < 1 || k > std::min(m, n) || k > 1024) return -4;
      TuxvWS t;
      Carve cv(nullptr, 0);
      carve_tuxv(cv, m, n, k, b, p, t, precision);
      if (cv.overflowed()) return -2;
      sz = cv.off;
      break;
    }
    case RQ_OP_SAMPLE_QRCP: {
      // m = l (sample rows), n = sample columns, b = pivot steps
      if (m < 1 || m > 128) return -2;
      if (n < 1) return -3;
      if (b > m || b > n) return -5;
      Carve cv(nullptr, 0);
      Common c;
      carve_common(cv, 1, c);
      SampleBufs sb;
      carve_sample(cv, 0, n, b, (int)m, sb);
      sz = cv.off;
      break;
    }
    case RQ_OP_SVD: {
      if (k < 1 || k > 1024) return -4;
      sz = align_up((size_t)k * k * sizeof(double), 256) + 4096;
      break;
    }
    default:
      return -1;
  }
  *bytes = sz;
  return 0;
}

int rq_rqrcp(void* stream, int64_t m, int64_t n, double* A, int64_t lda, int32_t b, int32_t p, uint64_t seed,
             int32_t precision, int64_t* jpvt, double* tau, void* work, size_t work_bytes, int32_t* info) {
  int rc = check_common(m, n, lda, b, p, 2, 3, 5, 6, 7);
  if (rc) return rc;
  if (precision < RQ_FP64 || precision > RQ_MIXED_BF16) return -9;
  if (m == 0 || n == 0) return empty_result((hipStream_t)stream, n, jpvt, info);
  return factor_impl((hipStream_t)stream, m, n, A, lda, b, p, seed, nullptr, 0, jpvt, tau, work, work_bytes, info,
                     true, false, precision, 13);
}

int rq_rqrcp_noalloc(void* stream, int64_t m, int64_t n, double* A, int64_t lda, int32_t b, int32_t p,
                     uint64_t seed, int32_t precision, int64_t* jpvt, double* tau, int32_t* info) {
  int rc = check_common(m, n, lda, b, p, 2, 3, 5, 6, 7);
  if (rc) return rc;
  if (precision < RQ_FP64 || precision > RQ_MIXED_BF16) return -9;
  if (m == 0 || n == 0) return empty_result((hipStream_t)stream, n, jpvt, info);
  size_t need = 0;
  rc = rq_workspace_bytes(RQ_OP_RQRCP, m, n, 0, b, p, precision, &need);
  if (rc) return rc;
  if (need > RQ_NOALLOC_SCRATCH_BYTES) return RQ_ERR_SCRATCH_TOO_SMALL;
  void* work = nullptr;
  RQ_TRY(scratch_address(&work));
  // everything on the caller's stream: no second stream and no events
  return factor_impl((hipStream_t)stream, m, n, A, lda, b, p, seed, nullptr, 0, jpvt, tau, work,
                     RQ_NOALLOC_SCRATCH_BYTES, info, true, false, precision, 0, false);
}

int rq_rqrcp_omega(void* stream, int64_t m, int64_t n, double* A, int64_t lda, int32_t b, int32_t p,
                   const double* Omega, int64_t ldo, int64_t* jpvt, double* tau, void* work, size_t work_bytes,
                   int32_t* info) {
  int rc = check_common(m, n, lda, b, p, 2, 3, 5, 6, 7);
  if (rc) return rc;
  if (!Omega) return -8;
  if (ldo < b + p) return -9;
  if (m == 0 || n == 0) return empty_result((hipStream_t)stream, n, jpvt, info);
  return factor_impl((hipStream_t)stream, m, n, A, lda, b, p, 0, Omega, ldo, jpvt, tau, work, work_bytes, info, true,
                     false, RQ_FP64, 13);
}

int rq_rsrqrcp(void* stream, int64_t m, int64_t n, double* A, int64_t lda, int32_t b, int32_t p, uint64_t seed,
               int64_t* jpvt, double* tau, void* work, size_t work_bytes, int32_t* info) {
  int rc = check_common(m, n, lda, b, p, 2, 3, 5, 6, 7);
  if (rc) return rc;
  if (m == 0 || n == 0) return empty_result((hipStream_t)stream, n, jpvt, info);
  return factor_impl((hipStream_t)stream, m, n, A, lda, b, p, seed, nullptr, 0, jpvt, tau, work, work_bytes, info,
                     true, true, RQ_FP64, 12);
}

int rq_unpivoted_qr(void* stream, int64_t m, int64_t n, double* A, int64_t lda, int32_t b, double* tau, void* work,
                    size_t work_bytes, int32_t* info) {
  int rc = check_common(m, n, lda, b, 0, 2, 3, 5, 6, 6);
  if (rc) return rc;
  if (m == 0 || n == 0) return empty_result((hipStream_t)stream, 0, nullptr, info);
  return factor_impl((hipStream_t)stream, m, n, A, lda, b, 0, 0, nullptr, 0, nullptr, tau, work, work_bytes, info,
                     false, false, RQ_FP64, 9);
}

static int trqrcp_entry(hipStream_t s, int64_t m, int64_t n, int64_t k, double* A, int64_t lda, int b, int p,
                        uint64_t seed, const double* Omega, int64_t ldo, int64_t* jpvt, double* tau, void* work,
                        size_t wbytes, int32_t* info, int prec, int iwork) {
  const bool mixed = prec != RQ_FP64;
  TrqWS t;
  Carve cv(work, wbytes);
  carve_trq(cv, m, n, k, b, p, t);
  if (mixed) {
    t.a32 = cv.take<float>((size_t)m * n);
    t.prec = prec;
  }
  if (!cv.ok) return -iwork;
  if (mixed) {
    // the FP32 copy of A that the sketch and the per-block Y2^T A read
    ProfScope ps(PC_SKETCH, s, 12.0 * m * n, 0.0);
    RQ_TRY(launch_to_f32(s, m, n, A, lda, t.a32, m));
  }
  int rc = trqrcp_core(s, m, n, k, A, lda, b, p, seed, Omega, ldo, jpvt, tau, t);
  if (rc) return rc;
  if (info) {
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, t.c.err, t.c.info, info);
    RQ_HIP(hipGetLastError());
  }
  return 0;
}

int rq_trqrcp(void* stream, int64_t m, int64_t n, int64_t k, double* A, int64_t lda, int32_t b, int32_t p,
              uint64_t seed, int32_t precision, int64_t* jpvt, double* tau, void* work, size_t work_bytes,
              int32_t* info) {
  int rc = check_common(m, n, lda, b, p, 2, 3, 6, 7, 8);
  if (rc) return rc;
  if (k < 1 || k > std::min(m, n)) return -4;
  if (precision < RQ_FP64 || precision > RQ_MIXED_BF16) return -10;
  return trqrcp_entry((hipStream_t)stream, m, n, k, A, lda, b, p, seed, nullptr, 0, jpvt, tau, work, work_bytes,
                      info, precision, 14);
}

int rq_trqrcp_omega(void* stream, int64_t m, int64_t n, int64_t k, double* A, int64_t lda, int32_t b, int32_t p,
                    const double* Omega, int64_t ldo, int64_t* jpvt, double* tau, void* work, size_t work_bytes,
                    int32_t* info) {
  int rc = check_common(m, n, lda, b, p, 2, 3, 6, 7, 8);
  if (rc) return rc;
  if (k < 1 || k > std::min(m, n)) return -4;
  if (!Omega) return -9;
  if (ldo < b + p) return -10;
  return trqrcp_entry((hipStream_t)stream, m, n, k, A, lda, b, p, 0, Omega, ldo, jpvt, tau, work, work_bytes, info,
                      RQ_FP64, 14);
}

int rq_tuxv(void* stream, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, int32_t b, int32_t p,
            uint64_t seed, int32_t precision, double* U, int64_t ldu, double* sigma, double* VT, int64_t ldvt,
            void* work, size_t work_bytes, int32_t* info) {
  int rc = check_common(m, n, lda, b, p, 2, 3, 6, 7, 8);
  if (rc) return rc;
  if (k < 1 || k > std::min(m, n) || k > 1024) return -4;
  if (precision < RQ_FP64 || precision > RQ_MIXED_BF16) return -10;
  if (ldu < m) return -12;
  if (ldvt < k) return -15;
  return tuxv_impl((hipStream_t)stream, m, n, k, A, lda, b, p, seed, nullptr, 0, U, ldu, sigma, VT, ldvt, work,
                   work_bytes, info, 1, precision, 17);
}

int rq_tuxv_iter(void* stream, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, int32_t b, int32_t p,
                 uint64_t seed, int32_t jmax, double* U, int64_t ldu, double* sigma, double* VT, int64_t ldvt,
                 void* work, size_t work_bytes, int32_t* info) {
  int rc = check_common(m, n, lda, b, p, 2, 3, 6, 7, 8);
  if (rc) return rc;
  if (k < 1 || k > std::min(m, n) || k > 1024) return -4;
  if (jmax < 1 || jmax > RQ_TUXV_MAX_ITER) return -10;
  if (ldu < m) return -12;
  if (ldvt < k) return -15;
  return tuxv_impl((hipStream_t)stream, m, n, k, A, lda, b, p, seed, nullptr, 0, U, ldu, sigma, VT, ldvt, work,
                   work_bytes, info, jmax, RQ_FP64, 17);
}

int rq_tuxv_omega(void* stream, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, int32_t b, int32_t p,
                  const double* Omega, int64_t ldo, double* U, int64_t ldu, double* sigma, double* VT, int64_t ldvt,
                  void* work, size_t work_bytes, int32_t* info) {
  int rc = check_common(m, n, lda, b, p, 2, 3, 6, 7, 8);
  if (rc) return rc;
  if (k < 1 || k > std::min(m, n) || k > 1024) return -4;
  if (!Omega) return -9;
  if (ldo < b + p) return -10;
  if (ldu < m) return -12;
  if (ldvt < k) return -15;
  return tuxv_impl((hipStream_t)stream, m, n, k, A, lda, b, p, 0, Omega, ldo, U, ldu, sigma, VT, ldvt, work,
                   work_bytes, info, 1, RQ_FP64, 17);
}

int rq_omega(void* stream, uint64_t seed, int64_t l, int64_t m, double* Omega, int64_t ldo) {
  if (l < 0 || l > 65536) return -3;
  if (m < 0 || m > RQ_MAX_ROWS) return -4;
  if (!Omega && l > 0 && m > 0) return -5;
  if (ldo < std::max<int64_t>(1, l)) return -6;
  return launch_omega((hipStream_t)stream, seed, l, m, Omega, 1, ldo);
}

int rq_sketch(void* stream, int64_t m, int64_t n, const double* A, int64_t lda, int32_t l, uint64_t seed,
              int32_t precision, double* B, int64_t ldb, void* work, size_t work_bytes) {
  if (m < 0 || m > RQ_MAX_ROWS) return -2;
  if (n < 0 || n > RQ_MAX_ROWS) return -3;
  if (lda < std::max<int64_t>(1, m)) return -5;
  if (l < 1 || l > 128) return -6;
  if (precision < RQ_FP64 || precision > RQ_MIXED_BF16) return -8;
  if (ldb < l) return -10;
  Carve cv(work, work_bytes);
  const int ls = std::max(sample_rows_padded(l), (int)l);
  double* om = cv.take<double>((size_t)l * m);
  double* smp = cv.take<double>((size_t)n * ls);
  if (!cv.ok) return -12;
  // the split-K scratch of the factorizations' sketch, when the workspace has room for it
  Carve cv2 = cv;
  const size_t sce = gemm_scratch_elems(l, n, m);
  double* sc = cv2.take<double>(sce);
  if (!cv2.ok) sc = nullptr;
  if (n == 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  if (m == 0) return launch_zero_rows(s, 0, l, n, B, ldb);  // Omega A = 0
  RQ_TRY(launch_omega(s, seed, l, m, om, 1, l));
  RQ_TRY(sketch(s, m, n, A, lda, l, om, l, smp, ls, sc, sc ? sce : 0, precision));
  RQ_TRY(launch_copy2d(s, l, n, smp, ls, B, ldb));
  return 0;
}

int rq_sample_qrcp(void* stream, int32_t l, int64_t n, int32_t bsteps, double* B, int64_t ldb, int32_t* piv,
                   void* work, size_t work_bytes, int32_t* info) {
  if (l < 1 || l > 128) return -2;
  if (n < 1 || n > 65536) return -3;
  if (bsteps < 1 || bsteps > 64 || bsteps > l || bsteps > n) return -4;
  if (ldb < l) return -6;
  Carve cv(work, work_bytes);
  Common c;
  carve_common(cv, 1, c);
  SampleBufs sb;
  carve_sample(cv, 0, n, bsteps, l, sb);
  if (!cv.ok) return -9;
  hipStream_t s = (hipStream_t)stream;
  RQ_TRY(launch_fill(s, c.flags, c.flag_words));
  RQ_TRY(launch_copy2d(s, l, n, B, ldb, sb.smp, sb.ls));
  RQ_TRY(launch_zero_rows(s, l, sb.ls, n, sb.smp, sb.ls));
  RQ_TRY(launch_sample_qrcp(s, sb.smp, sb.ls, l, n, bsteps, piv, c.info, 0, sq_work(sb, c, 0)));
  RQ_TRY(launch_copy2d(s, l, n, sb.smp, sb.ls, B, ldb));
  if (info) {
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, c.err, c.info, info);
    RQ_HIP(hipGetLastError());
  }
  return 0;
}

int rq_small_svd(void* stream, int32_t k, double* X, int64_t ldx, double* U, int64_t ldu, double* sigma, double* V,
                 int64_t ldv, void* work, size_t work_bytes) {
  if (k < 1 || k > 1024) return -2;
  if (ldx < k) return -4;
  if (ldu < k) return -6;
  if (ldv < k) return -9;
  Carve cv(work, work_bytes);
  double* tmp = cv.take<double>((size_t)k * k);
  int* err = cv.take<int>(16);
  unsigned* flags = cv.take<unsigned>(128);
  if (!cv.ok) return -11;
  RQ_TRY(launch_fill((hipStream_t)stream, err, 16));
  SvdWork sw;
  sw.colnorm = nullptr; sw.order = nullptr; sw.flags = flags; sw.err = err; sw.tmp = tmp;
  return launch_jacobi_svd((hipStream_t)stream, k, X, ldx, U, ldu, sigma, V, ldv, sw);
}

}  // extern "C"
