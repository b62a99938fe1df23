// Per-stage timing with HIP events, and roctx ranges (host side only).
#include <rocprofiler-sdk-roctx/roctx.h>

#include <mutex>
#include <vector>

#include "prof.hpp"
#include "rqrcp.h"

namespace rq {

namespace {

struct Rec {
  int cls;
  hipEvent_t e0, e1;
  double bytes, flops;
};

struct Agg {
  long long count = 0;
  double ms = 0.0, bytes = 0.0, flops = 0.0;
};

std::mutex g_mu;
bool g_on = false;
uint32_t g_mask = 0xFFFFFFFFu;  // classes that record events
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
std::vector<hipEvent_t> g_open;  // begin events waiting for their end, one per class
Agg g_agg[PC_NCLASS];

const char* kNames[PC_NCLASS] = {"omega",        "sketch",        "sample_qrcp",   "swap",
                                 "panel",        "tfactor",       "gemm_yta",      "gemm_update",
                                 "sample_update", "trq_products", "tuxv_products", "svd"};

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

bool prof_enabled() { return g_on; }

void prof_range_push(int cls) {
  static const char* const kRange[PC_NCLASS] = {
      "rq:omega",       "rq:sketch",        "rq:sample_qrcp",  "rq:swap",          "rq:panel",
      "rq:tfactor",     "rq:gemm_yta",      "rq:gemm_update",  "rq:sample_update", "rq:trq_products",
      "rq:tuxv_products", "rq:svd"};
  static_assert(PC_NCLASS == 12, "one range name per stage class");
  roctxRangePushA(cls >= 0 && cls < PC_NCLASS ? kRange[cls] : "rq:?");
}

void prof_range_pop() { roctxRangePop(); }

static bool selected(int cls) { return cls >= 0 && cls < 32 && ((g_mask >> cls) & 1u); }

void prof_begin(int cls, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_open.size() < PC_NCLASS) g_open.resize(PC_NCLASS, nullptr);
  if (!selected(cls)) {
    g_open[cls] = nullptr;
    return;
  }
  hipEvent_t e = get_event();
  if (e) hipEventRecord(e, s);
  g_open[cls] = e;
}

void prof_end(int cls, hipStream_t s, double bytes, double flops) {
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t e0 = (cls < (int)g_open.size()) ? g_open[cls] : nullptr;
  hipEvent_t e1 = get_event();
  if (!e0 || !e1) return;
  hipEventRecord(e1, s);
  g_recs.push_back(Rec{cls, e0, e1, bytes, flops});
  g_open[cls] = nullptr;
}

}  // namespace rq

using namespace rq;

extern "C" {

int rq_profile_start(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& a : g_agg) a = Agg();
  g_on = true;
  return 0;
}

int rq_profile_select(uint32_t class_mask) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_mask = class_mask;
  return 0;
}

int rq_profile_stop(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = false;
  for (auto& r : g_recs) {
    if (hipEventSynchronize(r.e1) != hipSuccess) return RQ_ERR_HIP_BASE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) return RQ_ERR_HIP_BASE;
    Agg& a = g_agg[r.cls];
    a.count += 1;
    a.ms += ms;
    a.bytes += r.bytes;
    a.flops += r.flops;
    g_pool.push_back(r.e0);
    g_pool.push_back(r.e1);
  }
  g_recs.clear();
  return 0;
}

int rq_profile_get(int32_t cls, int64_t* count, double* total_ms, double* bytes, double* flops) {
  if (cls < 0 || cls >= PC_NCLASS) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  const Agg& a = g_agg[cls];
  if (count) *count = a.count;
  if (total_ms) *total_ms = a.ms;
  if (bytes) *bytes = a.bytes;
  if (flops) *flops = a.flops;
  return 0;
}

const char* rq_profile_name(int32_t cls) {
  if (cls < 0 || cls >= PC_NCLASS) return "";
  return kNames[cls];
}

int32_t rq_profile_classes(void) { return PC_NCLASS; }

}  // extern "C"
