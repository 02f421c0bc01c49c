// Shared device/host helpers for the TT/QTT transport library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/ttnt.h"

namespace ttnt {

// Wavefront size on CDNA.
constexpr int kWave = 64;

struct HipError {
  hipError_t err;
  const char* where;
};

#define TT_HIP(call)                                              \
  do {                                                            \
    hipError_t e_ = (call);                                       \
    if (e_ != hipSuccess) throw ::ttnt::HipError{e_, #call};      \
  } while (0)

struct ArgError {
  std::string msg;
};

struct CapacityError {
  std::string msg;
};

struct NoConvError {};

#define TT_REQUIRE(cond, text)                                    \
  do {                                                            \
    if (!(cond)) throw ::ttnt::ArgError{std::string(text)};       \
  } while (0)

__host__ __device__ inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Device reductions (64-lane wavefronts).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide sum; `red` must hold blockDim.x / 64 doubles.  All threads get
// the result.  Contains two barriers.
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += red[i];
  return t;
}

// ---------------------------------------------------------------------------
// Host-side views.
// ---------------------------------------------------------------------------
struct Mat {            // row-major device matrix view
  double* p;
  int rows, cols, ld;
};

}  // namespace ttnt
