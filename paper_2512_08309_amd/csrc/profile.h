#pragma once
#include <vector>

#include "td_internal.h"

namespace td {

struct Profiler {
  struct Rec {
    int cls;
    hipEvent_t e0, e1;
    double flops, bytes;
  };
  struct Total {
    uint64_t launches = 0;
    double ms = 0, flops = 0, bytes = 0;
  };
  Total tot[K_NCLASS];
  std::vector<Rec> recs_;
  hipEvent_t pending_ = nullptr;
  ~Profiler();
  hipEvent_t event();
  void resolve();
  void reset();

 private:
  std::vector<hipEvent_t> free_, all_;
};

}  // namespace td
