// Per-kernel-class HIP-event timing (lobpcg_kernel_stats).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "lobpcg.h"

namespace lobpcg {

// HIP-event timing of kernel classes (roofline accounting).
class KernelTimer {
 public:
  ~KernelTimer();
  void enable(bool on);
  bool on() const { return on_; }
  // Record a start event for `kind`; returns a token for stop().
  int start(hipStream_t s);
  void stop(int token, int kind, double work, hipStream_t s);
  // Synchronise, fold finished records into the totals.
  void collect();
  lobpcg_kernel_stat totals[LOBPCG_KERNEL_KINDS] = {};

 private:
  hipEvent_t event(size_t i);
  struct Rec {
    int kind;
    int e0, e1;
    double work;
  };
  bool on_ = false;
  std::vector<hipEvent_t> pool_;
  size_t used_ = 0;
  std::vector<Rec> recs_;
};

}  // namespace lobpcg
