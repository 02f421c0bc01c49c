// FP64 GEMM tile shared by the standalone GEMM kernel and the persistent
// Krylov kernel.
#pragma once

#include "common.h"

namespace ttnt {

constexpr int kTileM = 64, kTileN = 64, kTileK = 16;

// One 64x64 tile (row block tm, column block tn) of C = alpha op(A) op(B) + beta C
// over k in [kb, ke), computed by 256 threads.  Each thread owns a 4x4 block
// (rows tr*4+i, columns tc+16*j, so C stores are coalesced).  With raw the
// unscaled partial sum is stored.  Row-major operands; op = transpose if flag.
// The next 16-wide K chunk is loaded into registers while the current one is
// multiplied out of LDS, so a chunk's load latency overlaps the previous
// chunk's products.
template <bool TA, bool TB>
__device__ __forceinline__ void gemm_tile(int tm, int tn, int M, int N, int kb, int ke,
                                          double alpha, const double* __restrict__ A, int lda,
                                          const double* __restrict__ B, int ldb, double beta,
                                          double* __restrict__ C, int ldc, bool raw,
                                          double (*As)[kTileM + 1], double (*Bs)[kTileN + 1]) {
  constexpr int NL = (kTileM * kTileK) / 256;      // loads per thread and operand
  static_assert((kTileK * kTileN) / 256 == NL, "square tile");
  const int m0 = tm * kTileM, n0 = tn * kTileN;
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  double ra[NL], rb[NL];
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < NL; ++t) {
      const int e = tid + t * 256;
      int mm, kk;
      if (!TA) { mm = e / kTileK; kk = e % kTileK; } else { kk = e / kTileM; mm = e % kTileM; }
      const int gm = m0 + mm, gk = k0 + kk;
      double v = 0.0;
      if (gm < M && gk < ke) v = TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
      ra[t] = v;
    }
#pragma unroll
    for (int t = 0; t < NL; ++t) {
      const int e = tid + t * 256;
      int kk, nn;
      if (!TB) { kk = e / kTileN; nn = e % kTileN; } else { nn = e / kTileK; kk = e % kTileK; }
      const int gk = k0 + kk, gn = n0 + nn;
      double v = 0.0;
      if (gk < ke && gn < N) v = TB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn];
      rb[t] = v;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int t = 0; t < NL; ++t) {
      const int e = tid + t * 256;
      if (!TA) As[e % kTileK][e / kTileK] = ra[t]; else As[e / kTileM][e % kTileM] = ra[t];
      if (!TB) Bs[e / kTileN][e % kTileN] = rb[t]; else Bs[e % kTileK][e / kTileK] = rb[t];
    }
  };
  load(kb);
  for (int k0 = kb; k0 < ke; k0 += kTileK) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + kTileK < ke) load(k0 + kTileK);
#pragma unroll
    for (int kk = 0; kk < kTileK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tr * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tc + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = m0 + tr * 4 + i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + tc + 16 * j;
      if (gn >= N) continue;
      double* c = C + (int64_t)gm * ldc + gn;
      if (raw) *c = acc[i][j];
      else *c = beta == 0.0 ? alpha * acc[i][j] : alpha * acc[i][j] + beta * *c;
    }
  }
}

}  // namespace ttnt

namespace ttnt {

// Agent-coherent load of a double written by another workgroup of the same
// launch before a grid barrier (bypasses the non-coherent caches, so the
// barrier needs no cache invalidation).
__device__ __forceinline__ double ld_coherent(const double* p) {
  const unsigned long long v = __hip_atomic_load(
      reinterpret_cast<unsigned long long*>(const_cast<double*>(p)), __ATOMIC_RELAXED,
      __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_bit_cast(double, v);
}

// Strided operand of the workgroup-level tile below: element (r, c) of the
// matrix is p[r * s0 + c * s1].
struct Strided {
  const double* p;
  int64_t s0, s1;
};

// Register-prefetched TM x TN tile (TM * TN == 4096, 256 threads, 4 x 4
// outputs each) of C = alpha A B with strided operands; the next 16-wide K
// chunk is loaded into registers while the current one is multiplied out of
// LDS.  CohB reads B with agent-coherent loads.  As holds 16 x (TM + 1)
// doubles, Bs 16 x (TN + 1).
template <int TM, int TN, bool CohB>
__device__ __forceinline__ void gemm_tile_pf(int tm, int tn, int M, int N, int K, double alpha,
                                             Strided A, Strided B, double* __restrict__ C,
                                             int64_t cm, int64_t cn, double* __restrict__ As,
                                             double* __restrict__ Bs) {
  static_assert(TM * TN == 4096, "tile must hold 4096 outputs");
  constexpr int KC = 16, NA = TM * KC / 256, NB = KC * TN / 256, CG = TN / 4;
  const int m0 = tm * TM, n0 = tn * TN;
  const int tid = threadIdx.x, tr = tid / CG, tc = tid % CG;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  double ra[NA], rb[NB];
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      const int e = tid + t * 256, mm = e / KC, kk = e % KC;
      const int gm = m0 + mm, gk = k0 + kk;
      ra[t] = (gm < M && gk < K) ? A.p[gm * A.s0 + gk * A.s1] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const int e = tid + t * 256, kk = e / TN, nn = e % TN;
      const int gk = k0 + kk, gn = n0 + nn;
      double v = 0.0;
      if (gk < K && gn < N) {
        const double* q = B.p + gk * B.s0 + gn * B.s1;
        v = CohB ? ld_coherent(q) : *q;
      }
      rb[t] = v;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      const int e = tid + t * 256;
      As[(e % KC) * (TM + 1) + e / KC] = ra[t];
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const int e = tid + t * 256;
      Bs[(e / TN) * (TN + 1) + e % TN] = rb[t];
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += KC) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + KC < K) load(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk * (TM + 1) + tr * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk * (TN + 1) + tc + CG * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = m0 + tr * 4 + i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + tc + CG * j;
      if (gn < N) C[gm * cm + gn * cn] = alpha * acc[i][j];
    }
  }
}

}  // namespace ttnt
