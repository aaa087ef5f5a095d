// Opt-in per-launch kernel timing with HIP events on the launch stream.
#include "profile.h"

namespace td {

thread_local Profiler* g_prof = nullptr;

const char* kclass_name(int k) {
  static const char* n[K_NCLASS] = {"conv3x3_mfma_f32", "conv1x1_mfma_f32", "groupnorm_stats", "conv_in",
                                    "conv_out_edm", "window_attention", "avgpool", "noise_philox",
                                    "blend", "laplace_decode", "linear_gaussian_step", "embedding",
                                    "conv3x3_mfma_bf16", "conv1x1_mfma_bf16", "gn_apply_bf16", "window_gather",
                                    "conv_wgrad_f32", "gn_apply_f32", "laplace_encode"};
  return (k >= 0 && k < K_NCLASS) ? n[k] : "?";
}

hipEvent_t Profiler::event() {
  if (!free_.empty()) {
    hipEvent_t e = free_.back();
    free_.pop_back();
    return e;
  }
  hipEvent_t e;
  TD_HIP(hipEventCreate(&e));
  all_.push_back(e);
  return e;
}

void Profiler::resolve() {
  if (recs_.empty()) return;
  TD_HIP(hipEventSynchronize(recs_.back().e1));
  for (Rec& r : recs_) {
    float ms = 0.f;
    TD_HIP(hipEventElapsedTime(&ms, r.e0, r.e1));
    Total& t = tot[r.cls];
    t.launches++;
    t.ms += ms;
    t.flops += r.flops;
    t.bytes += r.bytes;
    free_.push_back(r.e0);
    free_.push_back(r.e1);
  }
  recs_.clear();
}

void Profiler::reset() {
  resolve();
  for (Total& t : tot) t = Total{};
}

Profiler::~Profiler() {
  for (hipEvent_t e : all_) (void)hipEventDestroy(e);
}

void prof_begin(hipStream_t st) {
  Profiler* p = g_prof;
  if (!p) return;
  p->pending_ = p->event();
  TD_HIP(hipEventRecord(p->pending_, st));
}

void prof_end(hipStream_t st, int cls, double flops, double bytes) {
  Profiler* p = g_prof;
  if (!p || !p->pending_) return;
  hipEvent_t e1 = p->event();
  TD_HIP(hipEventRecord(e1, st));
  p->recs_.push_back(Profiler::Rec{cls, p->pending_, e1, flops, bytes});
  p->pending_ = nullptr;
}

}  // namespace td
