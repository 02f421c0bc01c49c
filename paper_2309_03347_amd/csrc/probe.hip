// Per-kernel timing with HIP events (diagnostic; off unless requested).
#include <algorithm>

#include "probe.h"

namespace ttnt {

thread_local Probe* g_probe = nullptr;

namespace {
constexpr size_t kPoolPairs = 1 << 15;

// Bounded device-side delay (one thread) enqueued ahead of each timed launch
// so that the start event, the kernel and the stop event are all queued while
// the GPU is busy: the event interval then holds the kernel alone, not the
// host's enqueue latency.
__global__ void hold_kernel(long long cycles) {
  const long long t0 = clock64();
  while (clock64() - t0 < cycles) __builtin_amdgcn_s_sleep(2);
}
}

Probe::~Probe() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

hipEvent_t Probe::begin(hipStream_t s, int c, double f, double b) {
  if (!active) return nullptr;
  if (ev.empty()) {
    ev.resize(2 * kPoolPairs);
    for (auto& e : ev) TT_HIP(hipEventCreate(&e));
    cls.resize(kPoolPairs);
    flops.resize(kPoolPairs);
    bytes.resize(kPoolPairs);
  }
  if (used >= kPoolPairs) {
    ++dropped;
    return nullptr;
  }
  cls[used] = c;
  flops[used] = f;
  bytes[used] = b;
  hold_kernel<<<1, 1, 0, s>>>(60000);   // ~25 us at the shader clock
  TT_HIP(hipGetLastError());
  TT_HIP(hipEventRecord(ev[2 * used], s));
  return ev[2 * used];
}

void Probe::end(hipStream_t s) {
  TT_HIP(hipEventRecord(ev[2 * used + 1], s));
  ++used;
}

void Probe::amend_last(double f, double b) {
  if (used == 0) return;
  flops[used - 1] = f;
  bytes[used - 1] = b;
}

void Probe::amend(int slot, double f, double b) {
  if (slot < 0 || (size_t)slot >= used) return;
  flops[slot] = f;
  bytes[slot] = b;
}

void Probe::calibrate(hipStream_t s) {
  // empty brackets queued behind a hold: the event pair's own interval
  if (ev.empty()) begin(s, 0, 0.0, 0.0), end(s), used = 0;
  hipEvent_t a = ev[0], b = ev[1];
  double tot = 0.0;
  const int reps = 32;
  for (int r = 0; r < reps; ++r) {
    hold_kernel<<<1, 1, 0, s>>>(60000);
    TT_HIP(hipEventRecord(a, s));
    TT_HIP(hipEventRecord(b, s));
    TT_HIP(hipEventSynchronize(b));
    float t = 0.f;
    TT_HIP(hipEventElapsedTime(&t, a, b));
    tot += t;
  }
  overhead_ms = tot / reps;
}

void Probe::close() {
  for (size_t i = 0; i < used; ++i) {
    TT_HIP(hipEventSynchronize(ev[2 * i + 1]));
    float t = 0.f;
    TT_HIP(hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]));
    t = std::max(0.f, t - (float)overhead_ms);
    n[cls[i]] += 1;
    ms[cls[i]] += t;
    fl[cls[i]] += flops[i];
    by[cls[i]] += bytes[i];
  }
  used = 0;
}

void Probe::reset() {
  used = 0;
  dropped = 0;
  for (int c = 0; c < kProbeClasses; ++c) n[c] = 0, ms[c] = fl[c] = by[c] = 0.0;
}

}  // namespace ttnt
