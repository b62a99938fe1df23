// Optional per-stage timing: when enabled (rq_profile_start), each driver
// stage records a pair of HIP events on the caller's stream around its
// kernels, together with the stage's algorithmic bytes and flops.
#pragma once

#include "common.hpp"

namespace rq {

enum ProfClass {
  PC_OMEGA = 0,
  PC_SKETCH,
  PC_SAMPLE_QRCP,
  PC_SWAP,
  PC_PANEL,
  PC_TFACTOR,
  PC_GEMM_YTA,      // W^T = T^T (Y^T C): reduction over the rows of the trailing matrix
  PC_GEMM_UPDATE,   // C -= Y W^T: rank-b update of the trailing matrix
  PC_SAMPLE_UPDATE,
  PC_TRQ_PRODUCTS,  // TRQRCP selected columns, inner-product composition, new rows of R
  PC_TUXV_PRODUCTS, // TUXV: A V, explicit Q, U1 Ux, Vx^T V^T, copies
  PC_SVD,
  PC_NCLASS
};

bool prof_enabled();
void prof_begin(int cls, hipStream_t s);
void prof_end(int cls, hipStream_t s, double bytes, double flops);
// roctx range "rq:<stage>" around the host code that enqueues a stage (always
// on: a no-op unless a tracing tool, e.g. rocprofv3 --marker-trace, listens)
void prof_range_push(int cls);
void prof_range_pop();

struct ProfScope {
  int cls;
  hipStream_t s;
  double bytes, flops;
  bool on;
  ProfScope(int c, hipStream_t st, double by, double fl) : cls(c), s(st), bytes(by), flops(fl), on(prof_enabled()) {
    prof_range_push(cls);
    if (on) prof_begin(cls, s);
  }
  ~ProfScope() {
    if (on) prof_end(cls, s, bytes, flops);
    prof_range_pop();
  }
};

}  // namespace rq
