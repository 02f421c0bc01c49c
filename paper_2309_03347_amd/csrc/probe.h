// Optional per-kernel timing with HIP events on the launching stream.
#pragma once

#include "common.h"

namespace ttnt {

// Kernel classes timed by the probe.
enum ProbeClass { kProbeGemmNN = 0, kProbeGemmTN, kProbeGemmNT, kProbeGemmTT, kProbeArnoldi,
                  kProbeMatvec, kProbeKrylov, kProbeGemmBf16, kProbeClasses };

struct Probe {
  bool active = false;
  std::vector<hipEvent_t> ev;        // pool, pairs (start, stop)
  size_t used = 0;                   // events used in the current window
  std::vector<int> cls;              // class of each pair
  std::vector<double> flops, bytes;  // algorithmic work of each pair
  // accumulated over closed windows
  int64_t n[kProbeClasses] = {};
  double ms[kProbeClasses] = {};
  double fl[kProbeClasses] = {};
  double by[kProbeClasses] = {};
  size_t dropped = 0;
  double overhead_ms = 0.0;          // interval of an empty event bracket

  ~Probe();
  // Returns the start event to record before a launch of class c, or nullptr.
  hipEvent_t begin(hipStream_t s, int c, double flops, double bytes);
  void end(hipStream_t s);
  // Replaces the work recorded for the most recent bracket, or for bracket
  // `slot` (for launches whose work is known only after they ran).
  void amend_last(double flops, double bytes);
  int last_slot() const { return (int)used - 1; }
  void amend(int slot, double flops, double bytes);
  // Waits for the window's events and folds them into the totals.
  void close();
  void reset();
  // Measures the interval of an empty bracket (subtracted from every sample).
  void calibrate(hipStream_t s);
};

extern thread_local Probe* g_probe;

}  // namespace ttnt
