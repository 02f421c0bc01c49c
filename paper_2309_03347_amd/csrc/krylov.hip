// Restarted GMRES on a local system (PhiL (x) A (x) PhiR) x = f as one
// persistent cooperative kernel.
//
// The unknown x[a][i][c] is split by its left-rank index a: workgroup b owns
// the slices a in [b * spw, (b + 1) * spw) and with them a contiguous chunk of
// every Krylov vector.  With the left interface folded into the operator core
// once per solve,
//   Q_a[(i, beta'), (b, j)] = sum_beta A[beta, i, j, beta'] PhiL[a, beta, b],
// a slice of y = (PhiL (x) A (x) PhiR) v is two products that need all of v
// but nothing another workgroup computes:
//   T[(i, beta'), d] = sum_{b, j} Q_a[(i, beta'), (b, j)] v[b, j, d]    (T in LDS)
//   y[a, i, c]       = sum_{beta', d} T[(i, beta'), d] PhiR[c, beta', d]
// so the operator application runs without grid barriers (the first product
// on the matrix cores when a workgroup owns one slice).  The workgroup's
// chunk of the Krylov basis stays in LDS for the whole solve; one Arnoldi
// step (classical Gram-Schmidt, two passes) needs three grid barriers: after
// the first-pass dots, after the second-pass dots, and after the new direction
// is published with its norm.  Data crossing workgroups (the published
// direction, x, and the partial sums) is read with agent-coherent loads, so a
// barrier only writes back dirty lines and the operator stays cached.  Global
// sums are formed by every workgroup from per-workgroup partials in the same
// order, so all workgroups hold bit-equal scalars and take the same branches;
// the iteration count is bounded by max_iter.
#include <algorithm>
#include <cstdlib>
#include <atomic>
#include <mutex>

#include "gemm_tile.h"
#include "krylov.h"
#include "kernels.h"
#include "probe.h"

namespace ttnt {

namespace {

constexpr int kThreads = 256;
constexpr int kXcds = 8;         // accelerator complex dies of the MI355X (dispatch round-robin)
constexpr int kMaxRestart = 88;
// LDS staging of the GEMM tiles: A chunks up to 128 rows; B chunks up to 64
// columns, or a whole K x N right operand of up to kBFull doubles.
constexpr int kAsDoubles = 16 * (128 + 1);
constexpr int kBFull = 4096;
constexpr int kBsDoubles = kBFull;

struct SArgs {
  const double* phiL;   // [r0][RL][r0]
  const double* Ap;     // [(i, RR), (RL, j)]
  const double* phiR;   // [r1][RR][r1]
  const void* phiRw;    // phiR in the working precision (phiR itself in FP64 mode)
  int r0, RL, n, RR, r1;
  int64_t N;
  const double* f;
  double* x;
  void* W;              // N, working precision: current direction, published each step
  double* Q;            // r0 x (n RR) x (r0 n): folded operator per slice (FP64)
  void* Qw;             // the same in the working precision (Q itself in FP64 mode)
  double* Qf;           // general matrix-core form: Q_a in fragment order, qf_slice per slice
  void* Qfw;            // the same in the working precision (Qf itself in FP64 mode)
  int64_t qf_slice;
  int S;                // general matrix-core form: workgroups per slice (1 otherwise)
  double* Py;           // with S > 1: per workgroup partial products (n r1 each)
  double* Pd1;          // G x (m + 1)
  double* Pd2;          // G x (m + 1)
  double* Pn;           // G x 2
  int m, max_iter, spw, ldv;
  int ts_doubles;       // LDS room of the first product's T (doubles)
  int mfg_bc;           // general matrix-core form: beta' per sub-chunk
  double tol, eta;
  double inner_tol;     // mixed mode: an inner cycle stops at this fraction of its start residual
  unsigned* bar;        // grid barrier: count, epoch flag (+32), abort word (+48)
  long long wait_limit; // wall-clock ticks a workgroup waits at a grid barrier before giving up
  double* info;         // [iterations, converged, |g_k| / ||f||, -, gave up (1.0)]
};

// Grid barrier for a cooperative launch: the workgroup barrier makes every
// wave's stores complete in the workgroup's L2, then one thread writes the L2
// back to the agent coherence point (release at agent scope, which orders the
// whole workgroup's earlier stores) and counts in.  The last to arrive
// publishes the epoch in a flag 128 bytes past the count, on a cache line of
// its own, which the others poll: polling the count itself slowed the
// arrivals' atomics (about 0.8 us of a 3 us barrier at 36 workgroups).
// Readers of data from other workgroups use ld_coherent, which bypasses the
// non-coherent cache levels, so no acquire-side invalidation is needed and
// the operator stays cached across iterations.
//
// The wait is bounded: a workgroup that has waited `limit` wall-clock ticks
// sets the abort word (64 words past the count... 48 words, its own line) and
// leaves; every later barrier of the launch sees the word and does not wait.
// The Arnoldi loop is bounded by max_iter, so every workgroup then runs to
// its end and the launch drains; the host reports the abort as an error.
__device__ __forceinline__ void grid_sync(unsigned* ctr, unsigned& target, long long limit) {
  unsigned* flag = ctr + 32;
  unsigned* abort_w = ctr + 48;
  target += gridDim.x;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned old = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1 == target) {
      __hip_atomic_store(flag, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const long long t0 = wall_clock64();
      while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
        if (wall_clock64() - t0 > limit) {
          __hip_atomic_store(abort_w, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
  }
  __syncthreads();
}

__device__ __forceinline__ double wg_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// C = alpha A B for a workgroup-level product, tile shape chosen by N.
template <bool CohB>
__device__ __forceinline__ void wg_gemm(int M, int N, int K, double alpha, Strided A, Strided B,
                                        double* C, int64_t cm, int64_t cn, double* As,
                                        double* Bs) {
  if (N <= 32) {
    for (int t = 0; t < cdiv(M, 128); ++t)
      gemm_tile_pf<128, 32, CohB>(t, 0, M, N, K, alpha, A, B, C, cm, cn, As, Bs);
  } else {
    const int tn = cdiv(N, 64);
    for (int t = 0; t < cdiv(M, 64) * tn; ++t)
      gemm_tile_pf<64, 64, CohB>(t / tn, t % tn, M, N, K, alpha, A, B, C, cm, cn, As, Bs);
  }
  __syncthreads();
}

template <typename U>
__device__ __forceinline__ U ld_coh(const U* p);
template <>
__device__ __forceinline__ double ld_coh<double>(const double* p) {
  return ld_coherent(p);
}
template <>
__device__ __forceinline__ float ld_coh<float>(const float* p) {
  const unsigned v = __hip_atomic_load(reinterpret_cast<unsigned*>(const_cast<float*>(p)),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_bit_cast(float, v);
}

// acc[q] += sum_k t[q * K + k] pr[k] over k = part, part + P, ... < K for
// q < NI (t in LDS, pr in global memory); loads issued U at a time, enough
// in flight to cover the L2 latency of the stream.
template <int NI, typename E>
__device__ __forceinline__ void row_dots(const E* __restrict__ pr, const E* __restrict__ t, int K,
                                         int part, int P, E* acc) {
  constexpr int U = 32;
  int kb = part;
  for (; kb + P * (U - 1) < K; kb += P * U) {
    E pv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) pv[u] = pr[kb + P * u];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int q = 0; q < NI; ++q) acc[q] = fma(t[q * K + kb + P * u], pv[u], acc[q]);
    }
  }
  for (; kb < K; kb += P) {
    const E p = pr[kb];
#pragma unroll
    for (int q = 0; q < NI; ++q) acc[q] = fma(t[q * K + kb], p, acc[q]);
  }
}

// The matrix-core kernel's form of the same sums: lane `part` reads the units
// part, part + P, ... of the row (P = PC when PC > 0), a unit being W
// consecutive elements (16-byte loads when W sizeof(E) = 16: K a multiple of
// W and pr 16-byte aligned).  The stream is read in blocks of 256 bytes per
// lane (16 units of 16 bytes), double-buffered: the loads of block b + 1 are
// issued before block b is multiplied.  The blocks
// that are whole for every lane run in a loop whose trip count is the same
// in every lane and whose loads are unconditional, so the number of loads in
// flight is known on every path and each wait covers only the block in use;
// the rest of the row is one more block, its loads clamped to the row and
// its products past the end skipped.
template <int NI, int W, int PC, typename E>
__device__ __forceinline__ void row_dots_pipe(const E* __restrict__ pr, const E* __restrict__ t,
                                              int K, int part, int Pr, E* acc) {
  constexpr int U = 256 / (W * (int)sizeof(E)), G = 4;
  // a compile-time lane count turns a block's addresses into immediate
  // offsets from one base
  const int P = PC > 0 ? PC : Pr;
  typedef E V __attribute__((ext_vector_type(W)));
  const V* pu = reinterpret_cast<const V*>(pr);
  const int KU = K / W, S = P * U, span = P * (U - 1);
  const int nfull = KU - P - span >= 0 ? (KU - P - span) / S + 1 : 0;
  V pa[U], pb[U];
  auto load = [&](V* buf, int k0) {
#pragma unroll
    for (int u = 0; u < U; ++u) buf[u] = pu[k0 + P * u];
  };
  // the LDS operands of G units are read together before their products
  auto mac = [&](const V* buf, int k0) {
#pragma unroll
    for (int g = 0; g < U; g += G) {
      V tv[NI][G];
#pragma unroll
      for (int u = 0; u < G; ++u)
#pragma unroll
        for (int q = 0; q < NI; ++q)
          tv[q][u] = *reinterpret_cast<const V*>(t + q * K + (k0 + P * (g + u)) * W);
#pragma unroll
      for (int u = 0; u < G; ++u)
#pragma unroll
        for (int q = 0; q < NI; ++q)
#pragma unroll
          for (int h = 0; h < W; ++h) acc[q] = fma(tv[q][u][h], buf[g + u][h], acc[q]);
    }
  };
  int kb = part;
  if (nfull > 0) {
    load(pa, kb);
    int b = 0;
    while (b + 2 < nfull) {
      load(pb, kb + S);
      mac(pa, kb);
      load(pa, kb + 2 * S);
      mac(pb, kb + S);
      kb += 2 * S;
      b += 2;
    }
    if (b + 1 < nfull) {
      load(pb, kb + S);
      mac(pa, kb);
      mac(pb, kb + S);
      kb += 2 * S;
    } else {
      mac(pa, kb);
      kb += S;
    }
  }
  // the partial block left to this lane
  if (kb < KU) {
#pragma unroll
    for (int u = 0; u < U; ++u) pa[u] = pu[min(kb + P * u, KU - 1)];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ku = kb + P * u;
      if (ku < KU) {
#pragma unroll
        for (int q = 0; q < NI; ++q) {
          const V tv = *reinterpret_cast<const V*>(t + q * K + ku * W);
#pragma unroll
          for (int h = 0; h < W; ++h) acc[q] = fma(tv[h], pa[u][h], acc[q]);
        }
      }
    }
  }
}

// TM x TN tile of C = alpha A B with A (M x K, row-major, lda) streamed from
// global memory through As and B (Kp x Np, zero-padded, row stride Np)
// already in LDS; all operands of element type E.
template <int TM, int TN, typename E>
__device__ __forceinline__ void gemm_tile_ldsb(int tm, int tn, int M, int N, int K, E alpha,
                                               const E* __restrict__ A, int lda,
                                               const E* __restrict__ Bl, int Np,
                                               E* __restrict__ C, int ldc, E* __restrict__ As) {
  constexpr int KC = 16, NA = TM * KC / 256, CG = TN / 4;
  const int m0 = tm * TM, n0 = tn * TN;
  const int tid = threadIdx.x, tr = tid / CG, tc = tid % CG;
  E acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = E(0);
  E ra[NA];
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      const int e = tid + t * 256, mm = e / KC, kk = e % KC;
      const int gm = m0 + mm, gk = k0 + kk;
      ra[t] = (gm < M && gk < K) ? A[(int64_t)gm * lda + gk] : E(0);
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += KC) {
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      const int e = tid + t * 256;
      As[(e % KC) * (TM + 1) + e / KC] = ra[t];
    }
    __syncthreads();
    if (k0 + KC < K) load(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      E av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[kk * (TM + 1) + tr * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bl[(k0 + kk) * Np + n0 + tc + CG * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = m0 + tr * 4 + i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + tc + CG * j;
      if (gn < N) C[(int64_t)gm * ldc + gn] = alpha * acc[i][j];
    }
  }
}

// Matrix-core form of the first product when a workgroup owns one slice.
// The slice's folded operator Q_a (n RR <= 128 rows, n r0 <= 80 columns) is
// the A operand of the 16x16x4 matrix instruction (FP64, or FP32 in the
// refinement cycles), loaded straight into the fragment registers; the right
// operand v ((n r0) x r1, r1 <= 64) is staged in LDS in fragment order, one
// 64-element fragment per (k-step, n-tile), so every fragment read is 64
// consecutive elements.  Lane l of a wavefront holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; its four results are D[l / 16 + 4 r][l % 16] in FP64
// and D[4 (l / 16) + r][l % 16] in FP32 (both checked on the device).
// Wavefront w owns the m-tiles w and w + 4.
constexpr int kMfmaKS = 20;      // k-steps of 4: n r0 <= 80
constexpr int kMfmaMT = 2;       // m-tiles of 16 per wavefront
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

template <typename E>
struct MfmaOps;
template <>
struct MfmaOps<double> {
  typedef dbl4 Acc;
  static __device__ __forceinline__ Acc mma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
};
template <>
struct MfmaOps<float> {
  typedef flt4 Acc;
  static __device__ __forceinline__ Acc mma(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};

template <typename E>
struct QFrag {
  E q[kMfmaMT][kMfmaKS];
};

// Q_a (M1 x K1, row-major) into the wavefront's A fragments.
template <typename E>
__device__ __forceinline__ void load_qfrag(const E* __restrict__ Qa, int M1, int K1,
                                           QFrag<E>& f) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int mt = 0; mt < kMfmaMT; ++mt)
#pragma unroll
    for (int ks = 0; ks < kMfmaKS; ++ks) {
      const int mm = 16 * (w + 4 * mt) + (l & 15), kk = 4 * ks + (l >> 4);
      f.q[mt][ks] = (mm < M1 && kk < K1) ? Qa[(int64_t)mm * K1 + kk] : E(0);
    }
}

// Geometry of one workgroup's share, and its LDS regions (doubles first, the
// working-precision basis last).
struct Ctx {
  int G, b, tid, lane;
  int m, ldv, nr1, nr0, nRR, a0, a1, nloc, K3;
  int sub, own0;  // with S > 1: the workgroup's index within its slice, first own element
  int pslot;      // with S > 1: the workgroup's slot of partial products, sub r0 + slice
  int64_t e0;
  int TNf, Kp, Np;
  double* As;     // GEMM staging (kAsDoubles doubles of room)
  double* Bs;     // whole right operand of the first product (kBFull doubles of room)
  double* Ts;     // n RR x r1 product (FP64 room)
  double* Yd;     // ldv: FP64 residual output
  double* Hpk;    // rotated Hessenberg, column c at c (c + 1) / 2
  double* hcol;
  double* h2;
  double* cs;
  double* sn;
  double* gv;
  void* Vl;       // (m + 1) x ldv, working precision
};

// ys[i][c] = sum_k Ts[i][k] PhiR[c][k] for one slice, k < RR r1: P lanes per
// output row c, partial sums combined across the P lanes by a fixed butterfly.
template <typename E>
__device__ __forceinline__ void stage3(const SArgs& a, const Ctx& c, const E* phiRe, const E* Ts,
                                       E* ys) {
  const int tid = c.tid;
  int P = 64;
  while (P > 1 && P * a.r1 > kThreads) P >>= 1;
  const int rows = kThreads / P, part = tid % P;
  for (int c0 = 0; c0 < a.r1; c0 += rows) {
    const int cr = c0 + tid / P;
    for (int i0 = 0; i0 < a.n; i0 += 4) {
      const int ni = min(4, a.n - i0);
      E acc[4] = {E(0), E(0), E(0), E(0)};
      if (cr < a.r1) {
        const E* pr = phiRe + (int64_t)cr * c.K3;
        const E* t2 = Ts + (int64_t)i0 * c.K3;
        switch (ni) {
          case 1: row_dots<1, E>(pr, t2, c.K3, part, P, acc); break;
          case 2: row_dots<2, E>(pr, t2, c.K3, part, P, acc); break;
          case 3: row_dots<3, E>(pr, t2, c.K3, part, P, acc); break;
          default: row_dots<4, E>(pr, t2, c.K3, part, P, acc); break;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        for (int o = P >> 1; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, 64);
      if (part == 0 && cr < a.r1) {
        for (int q = 0; q < ni; ++q) ys[(i0 + q) * a.r1 + cr] = acc[q];
      }
    }
  }
  __syncthreads();
}

// The matrix-core kernels' form: every thread streams part of one row of
// PhiR, P = 256 / r1 lanes per row (any P), and the P partial sums of a row
// are added in a fixed order through LDS (red: 4 x 256 doubles).  T rows have
// length K (row i at Ts + i K) and meet the first K elements of each PhiR row
// starting at phiRe (row stride K3); with accum the sums are added to ys.
template <typename E, bool Pipe = true>
__device__ __forceinline__ void stage3_pipe(const SArgs& a, const Ctx& c, const E* phiRe, int K,
                                            const E* Ts, E* ys, bool accum) {
  constexpr int W = 16 / (int)sizeof(E);
  const int tid = c.tid;
  const int P = max(1, min(64, kThreads / a.r1)), rows = kThreads / P;
  const bool w2 = (K % W == 0) && (c.K3 % W == 0) &&
                  ((reinterpret_cast<uintptr_t>(phiRe) & 15) == 0);
  E* red = reinterpret_cast<E*>(c.As);
  for (int c0 = 0; c0 < a.r1; c0 += rows) {
    const int cr = c0 + tid / P, part = tid % P;
    for (int i0 = 0; i0 < a.n; i0 += 2) {
      const int ni = min(2, a.n - i0);
      E acc[2] = {E(0), E(0)};
      if (tid < rows * P && cr < a.r1) {
        const E* pr = phiRe + (int64_t)cr * c.K3;
        const E* t2 = Ts + (int64_t)i0 * K;
        // ranks 33-36 and 29-32 (P = 7, 8) take the pipelined stream
        if (Pipe && w2 && ni == 2 && P == 7) row_dots_pipe<2, W, 7, E>(pr, t2, K, part, P, acc);
        else if (Pipe && w2 && ni == 2 && P == 8) row_dots_pipe<2, W, 8, E>(pr, t2, K, part, P, acc);
        else if (ni == 2) row_dots<2, E>(pr, t2, K, part, P, acc);
        else row_dots<1, E>(pr, t2, K, part, P, acc);
      }
      red[tid] = acc[0];
      red[kThreads + tid] = acc[1];
      __syncthreads();
      if (tid < rows && c0 + tid < a.r1) {
        for (int q = 0; q < ni; ++q) {
          E sum = E(0);
          for (int p = 0; p < P; ++p) sum += red[q * kThreads + tid * P + p];
          E* o = ys + (i0 + q) * a.r1 + c0 + tid;
          *o = accum ? *o + sum : sum;
        }
      }
      __syncthreads();
    }
  }
}

// y (own slices) = (PhiL (x) A (x) PhiR)(alpha v) in precision E, into the LDS
// row `out`; v is read with coherent loads.  Qe and phiRe are the operator in
// precision E.  fullB: the whole right operand fits in Bs.
template <typename E>
__device__ void apply_slices(const SArgs& a, const Ctx& c, const E* Qe, const E* phiRe,
                             const E* v, E alpha, E* out, bool fullB) {
  const int tid = c.tid;
  E* As = reinterpret_cast<E*>(c.As);
  E* Bs = reinterpret_cast<E*>(c.Bs);
  E* Ts = reinterpret_cast<E*>(c.Ts);
  if (fullB) {
    // coherent loads issued eight at a time before they are stored
    constexpr int kB = 8;
    const int total = c.Kp * c.Np;
    __syncthreads();
    for (int e0 = tid; e0 < total; e0 += kB * kThreads) {
      E tmp[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int e = e0 + u * kThreads;
        E val = E(0);
        if (e < total) {
          const int k = e / c.Np, cc = e % c.Np;
          if (k < c.nr0 && cc < a.r1) val = ld_coh<E>(v + (int64_t)k * a.r1 + cc);
        }
        tmp[u] = val;
      }
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int e = e0 + u * kThreads;
        if (e < total) Bs[e] = tmp[u];
      }
    }
    __syncthreads();
  }
  for (int s = c.a0; s < c.a1; ++s) {
    const E* Qa = Qe + (int64_t)s * c.nRR * c.nr0;
    if (fullB) {
      if (c.TNf == 32) {
        for (int t = 0; t < cdiv(c.nRR, 128); ++t)
          gemm_tile_ldsb<128, 32, E>(t, 0, c.nRR, a.r1, c.nr0, alpha, Qa, c.nr0, Bs, c.Np, Ts,
                                     a.r1, As);
      } else {
        const int tn = c.Np / 64;
        for (int t = 0; t < cdiv(c.nRR, 64) * tn; ++t)
          gemm_tile_ldsb<64, 64, E>(t / tn, t % tn, c.nRR, a.r1, c.nr0, alpha, Qa, c.nr0, Bs,
                                    c.Np, Ts, a.r1, As);
      }
      __syncthreads();
    } else {
      // FP64 only (the host plan requires fullB in the mixed mode)
      wg_gemm<true>(c.nRR, a.r1, c.nr0, (double)alpha,
                    Strided{reinterpret_cast<const double*>(Qa), c.nr0, 1},
                    Strided{reinterpret_cast<const double*>(v), a.r1, 1},
                    reinterpret_cast<double*>(Ts), a.r1, 1, c.As, c.Bs);
    }
    stage3<E>(a, c, phiRe, Ts, out + (s - c.a0) * c.nr1);
  }
}

// The same product for one slice per workgroup on the matrix cores, in E:
// the A fragments of Q_a are loaded first (all in flight together, L2
// resident after the first use), v is staged into Bs in fragment order while
// they arrive, the first product goes into Ts and the second is stage3_pipe.
template <typename E>
__device__ void apply_slice_mfma(const SArgs& a, const Ctx& c, const E* Qe, const E* phiRe,
                                 const E* v, E alpha, E* out) {
  typedef MfmaOps<E> Ops;
  typedef typename Ops::Acc Acc;
  const int tid = c.tid, l = c.lane, w = tid >> 6;
  const int K1 = c.nr0, M1 = c.nRR, NT = cdiv(a.r1, 16), ksu = cdiv(K1, 4);
  E* Bs = reinterpret_cast<E*>(c.Bs);
  E* Ts = reinterpret_cast<E*>(c.Ts);
  QFrag<E> qf;
  load_qfrag<E>(Qe + (int64_t)c.a0 * M1 * K1, M1, K1, qf);
  {
    // all of a thread's coherent loads in flight together (up to 16)
    constexpr int kB = 16;
    const int total = ksu * NT * 64;
    __syncthreads();
    for (int e0 = tid; e0 < total; e0 += kB * kThreads) {
      E tmp[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int e = e0 + u * kThreads;
        E val = E(0);
        if (e < total) {
          const int frag = e >> 6, ln = e & 63, ks = frag / NT, nt = frag - ks * NT;
          const int kk = 4 * ks + (ln >> 4), j = 16 * nt + (ln & 15);
          if (kk < K1 && j < a.r1) val = ld_coh<E>(v + (int64_t)kk * a.r1 + j);
        }
        tmp[u] = val;
      }
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int e = e0 + u * kThreads;
        if (e < total) Bs[e] = tmp[u];
      }
    }
    __syncthreads();
  }
  const bool second = 16 * (w + 4) < M1;     // the wavefront's second m-tile holds rows
  for (int nt = 0; nt < NT; ++nt) {
    Acc acc0 = {E(0), E(0), E(0), E(0)}, acc1 = acc0;
#pragma unroll
    for (int ks = 0; ks < kMfmaKS; ++ks) {
      if (ks < ksu) {
        const E bv = Bs[(ks * NT + nt) * 64 + l];
        acc0 = Ops::mma(qf.q[0][ks], bv, acc0);
        if (second) acc1 = Ops::mma(qf.q[1][ks], bv, acc1);
      }
    }
    const int j = 16 * nt + (l & 15);
    if (j < a.r1) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m0 = 16 * w + Ops::row(l, r), m1 = m0 + 64;
        if (m0 < M1) Ts[m0 * a.r1 + j] = alpha * acc0[r];
        if (second && m1 < M1) Ts[m1 * a.r1 + j] = alpha * acc1[r];
      }
    }
  }
  __syncthreads();
  stage3_pipe<E>(a, c, phiRe, c.K3, Ts, out, false);
}

// The general matrix-core form's second product: y[i][c] (+)= sum_{k < K}
// T[i][k] PhiR[c][k] with T rows of length K in LDS (row i at Ts + i K) and
// PhiR rows starting at phiRe (row stride K3).  Each wavefront owns a quarter
// of the rows c and takes them in equal passes of at most kS3Rows, its lanes
// along k (16-byte loads when the rows are aligned): every load of PhiR uses
// whole cache lines, each T value read from LDS serves the pass's rows, and
// the loads of the next k position are in flight while the current ones are
// multiplied.  The 64 lanes' sums are added by butterflies at the end of the
// pass.
constexpr int kS3Rows = 8;

template <typename E, typename O>
__device__ void stage3_rows(const SArgs& a, const Ctx& c, const E* phiRe, int K, const E* Ts,
                            O* ys, bool accum) {
  constexpr int CR = kS3Rows;
  constexpr int W = 16 / (int)sizeof(E);     // elements per 16-byte load
  typedef E VW __attribute__((ext_vector_type(W)));
  const int w = c.tid >> 6, l = c.lane, n = a.n, r1 = a.r1;
  const int64_t K3 = c.K3;
  const bool vec = (K % W == 0) && (K3 % W == 0) &&
                   ((reinterpret_cast<uintptr_t>(phiRe) & 15) == 0);
  // wavefront w takes rows [w rpw, (w + 1) rpw) in equal passes of at most CR
  const int rpw = cdiv(r1, 4), np = cdiv(rpw, CR), rpp = cdiv(rpw, np);
  const int rw1 = min(r1, (w + 1) * rpw);
  for (int c0 = w * rpw; c0 < rw1; c0 += rpp) {
    const int nr = min(rpp, rw1 - c0);
    for (int i0 = 0; i0 < n; i0 += 2) {
      const bool two = i0 + 1 < n;
      double acc[CR][2];
#pragma unroll
      for (int r = 0; r < CR; ++r) acc[r][0] = acc[r][1] = 0.0;
      const E* t0 = Ts + (int64_t)i0 * K;
      const E* t1 = two ? t0 + K : t0;
      if (vec) {
        const int KW = K / W;
        const VW* ta = reinterpret_cast<const VW*>(t0);
        const VW* tb = reinterpret_cast<const VW*>(t1);
        const VW* p0 = reinterpret_cast<const VW*>(phiRe + (int64_t)c0 * K3);
        const int64_t rs = K3 / W;     // row stride in loads
        // every lane takes the same T = ceil(KW / 64) positions (the last
        // clamped to the row and counted with zero weight), so the loads are
        // unconditional and double-buffered: the next position's CR loads are
        // in flight while the current ones are multiplied
        const int T = (KW + 63) / 64;
        auto ldp = [&](VW* buf, int t) {
          const int kk = min(l + 64 * t, KW - 1);
#pragma unroll
          for (int r = 0; r < CR; ++r) buf[r] = p0[(int64_t)min(r, nr - 1) * rs + kk];
        };
        auto mac = [&](const VW* buf, int t) {
          const int kk = l + 64 * t;
          const bool ok = kk < KW;
          const VW zero = VW{};
          const VW x0 = ok ? ta[kk] : zero, x1 = ok ? tb[kk] : zero;
#pragma unroll
          for (int r = 0; r < CR; ++r)
#pragma unroll
            for (int h = 0; h < W; ++h) {
              acc[r][0] = fma((double)x0[h], (double)buf[r][h], acc[r][0]);
              acc[r][1] = fma((double)x1[h], (double)buf[r][h], acc[r][1]);
            }
        };
        VW pa[CR], pb[CR];
        ldp(pa, 0);
        int t = 0;
        for (; t + 1 < T; t += 2) {
          ldp(pb, t + 1);
          mac(pa, t);
          if (t + 2 < T) ldp(pa, t + 2);
          mac(pb, t + 1);
        }
        if (t < T) mac(pa, t);
      } else {
        for (int k = l; k < K; k += 64) {
          const E x0 = t0[k], x1 = t1[k];
#pragma unroll
          for (int r = 0; r < CR; ++r) {
            const E p = phiRe[(int64_t)(c0 + min(r, nr - 1)) * K3 + k];
            acc[r][0] = fma((double)x0, (double)p, acc[r][0]);
            acc[r][1] = fma((double)x1, (double)p, acc[r][1]);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < CR; ++r) {
        acc[r][0] = wave_sum(acc[r][0]);
        acc[r][1] = wave_sum(acc[r][1]);
      }
      if (l == 0) {
#pragma unroll
        for (int r = 0; r < CR; ++r)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            if (r < nr && (q == 0 || two)) {
              O* o = ys + (int64_t)(i0 + q) * r1 + c0 + r;
              const O v = (O)acc[r][q];
              *o = accum ? *o + v : v;
            }
          }
      }
    }
  }
  __syncthreads();
}

// General matrix-core form for one slice per workgroup, any n RR and n r0
// (n <= 4, r1 <= 96).  The slice's beta' are split into S contiguous ranges
// of q = ceil(RR / S), one per workgroup of the slice, and a range is taken in
// sub-chunks of at most bc beta'.  A sub-chunk's rows (i, beta') of Q_a are
// packed densely, row i bc + (beta' - b0), into m-tiles of 16, so each
// sub-chunk's part of the second product reads one range of every PhiR row.
// The first product of a sub-chunk runs over k in steps of KC: its rows of
// Q_a (into As, from a copy laid out in fragment order once per solve, see
// qf_reorder) and KC rows of v (into Bs) are staged in fragment order, the
// next step's values loaded into registers while the current one is
// multiplied; wavefront w owns the (m-tile, n-tile) pairs w, w + 4, ... and
// keeps their accumulators over the k steps.  The sub-chunk's T goes to Ts
// and its part of the second product is added to out.  With S > 1 out is the
// workgroup's partial product; the sum of the S partials is formed after a
// grid barrier (mfg_reduce).
constexpr int kMfgPairs = 6;     // (m-tile, n-tile) pairs per wavefront: 4 m-tiles x 6 n-tiles
constexpr int kMfgTiles = 4;     // m-tiles per sub-chunk, at most

struct MfgGeom {
  int q, rb0, rb1;     // beta' per workgroup, the workgroup's range
  int bc, MTmax;       // beta' per sub-chunk, its m-tiles at most
  int KS, KC, nkc;     // k-steps of 4 per stage, k per stage, stages
  int nsc;             // sub-chunks per range
  int64_t sc_size;     // elements of a sub-chunk's fragments over all stages
};

__host__ __device__ inline MfgGeom mfg_geom(int n, int r0, int RR, int r1, int S, int bc,
                                            int sub) {
  MfgGeom g;
  g.q = (RR + S - 1) / S;
  g.rb0 = sub * g.q < RR ? sub * g.q : RR;
  g.rb1 = g.rb0 + g.q < RR ? g.rb0 + g.q : RR;
  g.bc = bc;
  g.MTmax = (n * bc + 15) / 16;
  const int nt = (r1 + 15) / 16;
  // the sub-chunk's A fragments and v's fragments each fit 2048 elements
  // (eight per thread) per stage
  int ks = 32 / g.MTmax;
  if (32 / nt < ks) ks = 32 / nt;
  if (ks > 16) ks = 16;
  g.KS = ks;
  g.KC = 4 * ks;
  g.nkc = (n * r0 + g.KC - 1) / g.KC;
  g.nsc = (g.q + bc - 1) / bc;
  g.sc_size = (int64_t)g.MTmax * 16 * g.nkc * g.KC;
  return g;
}

// Q_a (row-major, n RR x K1) into the general matrix-core form's order: for
// each of the workgroup's sub-chunks and each k step of KC, the sub-chunk's
// fragments (m-tile, k-step) of 64 lanes, lane l holding A[l % 16][l / 16] of
// its fragment, zero past the rows and columns; sub-chunk j of workgroup sub
// starts at (sub nsc + j) sc_size.  Once per solve, each workgroup for its own
// range.
template <typename E>
__device__ void qf_reorder(const SArgs& a, int sub, const double* Qa, E* Qs) {
  const int K1 = a.n * a.r0, RR = a.RR, n = a.n;
  const MfgGeom g = mfg_geom(n, a.r0, RR, a.r1, a.S, a.mfg_bc, sub);
  for (int j = 0; j < g.nsc; ++j) {
    const int b0 = g.rb0 + j * g.bc;
    if (b0 >= g.rb1) break;
    const int bc = min(g.bc, g.rb1 - b0), rows = n * bc;
    const int na = cdiv(rows, 16) * g.KS * 64;
    E* Qj = Qs + (int64_t)(sub * g.nsc + j) * g.sc_size;
    for (int64_t f = threadIdx.x; f < (int64_t)g.nkc * na; f += kThreads) {
      const int st = (int)(f / na), e = (int)(f - (int64_t)st * na);
      const int frag = e >> 6, ln = e & 63, mt = frag / g.KS, ks = frag - mt * g.KS;
      const int rho = 16 * mt + (ln & 15), kk = st * g.KC + 4 * ks + (ln >> 4);
      E val = E(0);
      if (rho < rows && kk < K1) {
        const int i = rho / bc, bp = rho - i * bc;
        val = (E)Qa[(int64_t)(i * RR + b0 + bp) * K1 + kk];
      }
      Qj[f] = val;
    }
  }
  __syncthreads();
}

template <typename E, typename O>
__device__ void apply_slice_mfg(const SArgs& a, const Ctx& c, const E* Qfe, const E* phiRe,
                                const E* v, E alpha, O* out) {
  typedef MfmaOps<E> Ops;
  typedef typename Ops::Acc Acc;
  const int tid = c.tid, l = c.lane, w = tid >> 6;
  const int K1 = c.nr0, RR = a.RR, n = a.n, r1 = a.r1;
  const int NT = cdiv(r1, 16);
  const MfgGeom g = mfg_geom(n, a.r0, RR, r1, a.S, a.mfg_bc, c.sub);
  const int KC = g.KC, KS = g.KS;
  E* As = reinterpret_cast<E*>(c.As);
  E* Bs = reinterpret_cast<E*>(c.Bs);
  E* Ts = reinterpret_cast<E*>(c.Ts);
  const E* Qs = Qfe + (int64_t)c.a0 * a.qf_slice;
  // staging: A (MT m-tiles x KS k-steps fragments) and B (KS x NT fragments),
  // at most 8 + 8 elements per thread and stage
  constexpr int kSA = 8, kSB = 8;
  if (g.rb0 >= g.rb1) {
    // no beta' for this workgroup: its partial product is zero
    for (int e = tid; e < n * r1; e += kThreads) out[e] = O(0);
    __syncthreads();
  }
  for (int j = 0; j < g.nsc; ++j) {
    const int b0 = g.rb0 + j * g.bc;
    if (b0 >= g.rb1) break;
    const int bc = min(g.bc, g.rb1 - b0);     // beta' of the sub-chunk, for every i
    const int rows = n * bc;
    const int MT = cdiv(rows, 16);
    const int npairs = MT * NT;
    const int na = MT * KS * 64, nbv = KS * NT * 64;
    E ra[kSA], rb[kSB];
    const E* Qc = Qs + (int64_t)(c.sub * g.nsc + j) * g.sc_size;
    auto load = [&](int K0) {
      const E* Qk = Qc + (int64_t)(K0 / KC) * na;
#pragma unroll
      for (int u = 0; u < kSA; ++u) {
        const int e = tid + u * kThreads;
        ra[u] = e < na ? Qk[e] : E(0);
      }
#pragma unroll
      for (int u = 0; u < kSB; ++u) {
        const int e = tid + u * kThreads;
        E val = E(0);
        if (e < nbv) {
          const int frag = e >> 6, ln = e & 63, ks = frag / NT, nt = frag - ks * NT;
          const int kk = K0 + 4 * ks + (ln >> 4), jj = 16 * nt + (ln & 15);
          if (kk < K1 && jj < r1) val = ld_coh<E>(v + (int64_t)kk * r1 + jj);
        }
        rb[u] = val;
      }
    };
    Acc acc[kMfgPairs];
#pragma unroll
    for (int q = 0; q < kMfgPairs; ++q) acc[q] = {E(0), E(0), E(0), E(0)};
    load(0);
    for (int K0 = 0; K0 < K1; K0 += KC) {
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kSA; ++u) {
        const int e = tid + u * kThreads;
        if (e < na) As[e] = ra[u];
      }
#pragma unroll
      for (int u = 0; u < kSB; ++u) {
        const int e = tid + u * kThreads;
        if (e < nbv) Bs[e] = rb[u];
      }
      __syncthreads();
      if (K0 + KC < K1) load(K0 + KC);
#pragma unroll
      for (int q = 0; q < kMfgPairs; ++q) {
        const int pr = w + 4 * q;
        if (pr < npairs) {
          const int mt = pr / NT, nt = pr - mt * NT;
          for (int ks = 0; ks < KS; ++ks)
            acc[q] = Ops::mma(As[(mt * KS + ks) * 64 + l], Bs[(ks * NT + nt) * 64 + l], acc[q]);
        }
      }
    }
    // the sub-chunk's T, row i bc + (beta' - b0): Ts[rho r1 + d]
#pragma unroll
    for (int qq = 0; qq < kMfgPairs; ++qq) {
      const int pr = w + 4 * qq;
      if (pr < npairs) {
        const int mt = pr / NT, nt = pr - mt * NT;
        const int col = 16 * nt + (l & 15);
        if (col < r1) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int rho = 16 * mt + Ops::row(l, r);
            if (rho < rows) Ts[(int64_t)rho * r1 + col] = alpha * acc[qq][r];
          }
        }
      }
    }
    __syncthreads();
    stage3_rows<E, O>(a, c, phiRe + (int64_t)b0 * r1, bc * r1, Ts, out, j > 0);
  }
}

// out[e] = sum over the slice's S partial products of element own0 + e, for
// the workgroup's own elements, in a fixed order (coherent loads; with S > 1
// called after the grid barrier that follows the partial products, with S =
// 1 it copies the workgroup's own product).
template <typename O>
__device__ void mfg_reduce(const SArgs& a, const Ctx& c, O* out) {
  const double* P = a.Py + (int64_t)c.a0 * c.nr1 + c.own0;
  for (int e = c.tid; e < c.nloc; e += kThreads) {
    double acc = 0.0;
    for (int q = 0; q < a.S; ++q) acc += ld_coherent(P + (int64_t)q * a.r0 * c.nr1 + e);
    out[e] = (O)acc;
  }
  __syncthreads();
}

// The solve.  T is the working precision of the Krylov iterations; restart
// residuals r = f - A x and x itself are always FP64.  With T = float each
// restart cycle is one step of iterative refinement: the cycle solves
// A d = r in FP32 to inner_tol (or to the global target) and x += d in FP64.
// MF selects the operator application: 0 the vector-FMA form (any slices per
// workgroup), 1 the register-resident matrix-core form (one slice, n RR <= 128,
// n r0 <= 80), 2 the general matrix-core form (one slice, chunked).
template <typename T, int MF>
__global__ __launch_bounds__(kThreads) void gmres_slices_kernel(SArgs a) {
  extern __shared__ __attribute__((aligned(16))) double lds[];   // 16-byte reads of Ts
  __shared__ double red[4];
  __shared__ double bcast[4];
  constexpr bool kMixed = sizeof(T) < sizeof(double);
  Ctx c;
  c.G = gridDim.x;
  c.b = blockIdx.x;
  c.tid = threadIdx.x;
  c.lane = c.tid & 63;
  c.m = a.m;
  c.ldv = a.ldv;
  c.nr1 = a.n * a.r1;
  c.nr0 = a.n * a.r0;
  c.nRR = a.n * a.RR;
  if (a.S > 1) {
    // S workgroups per slice, each owning a contiguous part of the slice's
    // n r1 elements.  Workgroups are dispatched round-robin over the XCDs
    // (b % kXcds); numbered XCD-major, the ones that take the same beta'
    // range (same sub) share few XCDs, so their part of PhiR stays in those
    // L2s.  (Only the speed depends on the dispatch order.)
    const int x = c.b % kXcds, base = x * (c.G / kXcds) + min(x, c.G % kXcds);
    const int L = base + c.b / kXcds;
    const int q = cdiv(c.nr1, a.S);
    c.sub = L / a.r0;
    c.a0 = L - c.sub * a.r0;
    c.a1 = c.a0 + 1;
    c.pslot = L;
    c.own0 = min(c.nr1, c.sub * q);
    c.nloc = min(c.nr1, c.own0 + q) - c.own0;
    c.e0 = (int64_t)c.a0 * c.nr1 + c.own0;
  } else {
    c.a0 = min(a.r0, c.b * a.spw);
    c.a1 = min(a.r0, c.a0 + a.spw);
    c.sub = 0;
    c.own0 = 0;
    c.pslot = c.b;
    c.nloc = (c.a1 - c.a0) * c.nr1;
    c.e0 = (int64_t)c.a0 * c.nr1;
  }
  c.K3 = a.RR * a.r1;
  c.TNf = a.r1 <= 32 ? 32 : 64;
  c.Kp = cdiv(c.nr0, 16) * 16;
  c.Np = cdiv(a.r1, c.TNf) * c.TNf;
  c.As = lds;
  c.Bs = c.As + kAsDoubles;
  c.Ts = c.Bs + kBsDoubles;
  c.Yd = c.Ts + a.ts_doubles;
  c.Hpk = c.Yd + c.ldv;
  c.hcol = c.Hpk + c.m * (c.m + 1) / 2;
  c.h2 = c.hcol + (c.m + 2);
  c.cs = c.h2 + (c.m + 2);
  c.sn = c.cs + (c.m + 2);
  c.gv = c.sn + (c.m + 2);
  c.Vl = c.gv + (c.m + 2);
  const int G = c.G, b = c.b, tid = c.tid, lane = c.lane, m = c.m, ldv = c.ldv;
  const int nloc = c.nloc;
  const int64_t e0 = c.e0;
  double* Hpk = c.Hpk;
  double* hcol = c.hcol;
  double* h2 = c.h2;
  double* cs = c.cs;
  double* sn = c.sn;
  double* gv = c.gv;
  T* Vl = reinterpret_cast<T*>(c.Vl);
  T* W = reinterpret_cast<T*>(a.W);
  const T* Qw = reinterpret_cast<const T*>(a.Qw);
  const T* phiRw = reinterpret_cast<const T*>(a.phiRw);
  const bool fullB64 = (int64_t)c.Kp * c.Np <= kBFull;
  const bool fullBw = (int64_t)c.Kp * c.Np * sizeof(T) <= (int64_t)kBFull * sizeof(double);
  unsigned target = 0;

  // Q_a for the own slices (once per solve; read back by this workgroup only)
  for (int s = c.a0; s < c.a1; ++s) {
    double* Qa = a.Q + (int64_t)s * c.nRR * c.nr0;
    if (MF == 2 && a.S > 1) {
      // only the rows (i, beta') of the workgroup's own beta' range
      const MfgGeom g = mfg_geom(a.n, a.r0, a.RR, a.r1, a.S, a.mfg_bc, c.sub);
      if (g.rb1 > g.rb0) {
        for (int i = 0; i < a.n; ++i) {
          const int64_t row0 = (int64_t)i * a.RR + g.rb0;
          for (int j = 0; j < a.n; ++j)
            wg_gemm<false>(g.rb1 - g.rb0, a.r0, a.RL, 1.0,
                           Strided{a.Ap + row0 * a.RL * a.n + j, (int64_t)a.RL * a.n, a.n},
                           Strided{a.phiL + (int64_t)s * a.RL * a.r0, a.r0, 1},
                           Qa + row0 * c.nr0 + j, c.nr0, a.n, c.As, c.Bs);
        }
      }
    } else {
      for (int j = 0; j < a.n; ++j)
        wg_gemm<false>(c.nRR, a.r0, a.RL, 1.0, Strided{a.Ap + j, (int64_t)a.RL * a.n, a.n},
                       Strided{a.phiL + (int64_t)s * a.RL * a.r0, a.r0, 1}, Qa + j, c.nr0,
                       a.n, c.As, c.Bs);
    }
    if (kMixed && MF != 2) {
      T* Qt = reinterpret_cast<T*>(a.Qw) + (int64_t)s * c.nRR * c.nr0;
      for (int e = tid; e < c.nRR * c.nr0; e += kThreads) Qt[e] = (T)Qa[e];
      __syncthreads();
    }
    if constexpr (MF == 2) {
      qf_reorder<double>(a, c.sub, Qa, a.Qf + (int64_t)s * a.qf_slice);
      if (kMixed)
        qf_reorder<T>(a, c.sub, Qa, reinterpret_cast<T*>(a.Qfw) + (int64_t)s * a.qf_slice);
    }
  }

  // Partial dots of w with V_0..V_j over the chunk (gs lanes per vector, FP64 sums).
  auto dots = [&](int j, const T* w, double* out) {
    int gs = 64;
    while (gs > 1 && (j + 1) * gs > kThreads) gs >>= 1;
    const int per = kThreads / gs;
    for (int i0 = 0; i0 <= j; i0 += per) {
      const int i = i0 + tid / gs, p = tid % gs;
      double acc = 0.0;
      if (i <= j) {
        const T* vi = Vl + (int64_t)i * ldv;
        for (int e = p; e < nloc; e += gs) acc = fma((double)vi[e], (double)w[e], acc);
      }
      for (int o = gs >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if (p == 0 && i <= j) out[i] = acc;
    }
  };
  // dst[i] = sum over workgroups q of P[q][i], i <= j: gs lanes per i, each
  // summing every gs-th workgroup with its loads issued together, then a
  // fixed butterfly; the same order in every workgroup.
  auto gather = [&](const double* P, int j, double* dst) {
    int gs = 64;
    while (gs > 1 && (j + 1) * gs > kThreads) gs >>= 1;
    const int per = kThreads / gs;
    for (int i0 = 0; i0 <= j; i0 += per) {
      const int i = i0 + tid / gs, p = tid % gs;
      double acc = 0.0;
      if (i <= j) {
        constexpr int U = 8;
        for (int q0 = p; q0 < G; q0 += gs * U) {
          double v[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int q = q0 + gs * u;
            v[u] = q < G ? ld_coherent(P + (int64_t)q * (m + 1) + i) : 0.0;
          }
#pragma unroll
          for (int u = 0; u < U; ++u) acc += v[u];
        }
      }
      for (int o = gs >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if (p == 0 && i <= j) dst[i] = acc;
    }
    __syncthreads();
  };
  // sum over workgroups of Pn[2 q + k] by wave 0 (fixed order), into bcast[2 + k]
  auto gather_pn = [&](int k) {
    if (tid < 64) {
      double acc = 0.0;
      for (int q = lane; q < G; q += 64) acc += ld_coherent(a.Pn + 2 * q + k);
      acc = wave_sum(acc);
      if (lane == 0) bcast[2 + k] = acc;
    }
  };
  // w -= sum_i h[i] Vl_i over the chunk (FP64 arithmetic); returns this
  // thread's ||w||^2 share
  auto orth = [&](T* w, int j, const double* h) {
    double nn = 0.0;
    for (int e = tid; e < nloc; e += kThreads) {
      double s0 = (double)w[e], s1 = 0.0;
      int i = 0;
      for (; i + 1 <= j; i += 2) {
        s0 -= h[i] * (double)Vl[(int64_t)i * ldv + e];
        s1 -= h[i + 1] * (double)Vl[(int64_t)(i + 1) * ldv + e];
      }
      if (i <= j) s0 -= h[i] * (double)Vl[(int64_t)i * ldv + e];
      const T r = (T)(s0 + s1);
      w[e] = r;
      nn = fma((double)r, (double)r, nn);
    }
    return nn;
  };

  int total = 0;
  bool conv = false;
  double fnorm = 0.0, tgt = -1.0, res_est = 0.0;
  while (true) {
    // r = f - A x in FP64 (x and the FP64 operator); r is rounded into Vl_0
    // and W (unnormalised).  ||r||^2 and ||f||^2.
    if constexpr (MF == 1)
      apply_slice_mfma<double>(a, c, a.Q, a.phiR, a.x, 1.0, c.Yd);
    else if constexpr (MF == 2) {
      // the product (or this workgroup's partial of it) goes through Py
      apply_slice_mfg<double, double>(a, c, a.Qf, a.phiR, a.x, 1.0,
                                      a.Py + (int64_t)c.pslot * c.nr1);
      if (a.S > 1) grid_sync(a.bar, target, a.wait_limit);
      mfg_reduce<double>(a, c, c.Yd);
    }
    else
      apply_slices<double>(a, c, a.Q, a.phiR, a.x, 1.0, c.Yd, fullB64);
    double rr = 0.0, ff = 0.0;
    for (int e = tid; e < nloc; e += kThreads) {
      const double fe = a.f[e0 + e];
      const double r = fe - c.Yd[e];
      Vl[e] = (T)r;
      W[e0 + e] = (T)r;
      rr = fma(r, r, rr);
      ff = fma(fe, fe, ff);
    }
    rr = wg_sum(rr, red);
    ff = wg_sum(ff, red);
    if (tid == 0) {
      a.Pn[2 * b] = rr;
      a.Pn[2 * b + 1] = ff;
    }
    grid_sync(a.bar, target, a.wait_limit);
    gather_pn(0);
    __syncthreads();
    gather_pn(1);
    __syncthreads();
    const double beta = sqrt(bcast[2]);
    if (tgt < 0.0) {
      fnorm = sqrt(bcast[3]);
      tgt = fmax(a.tol * fnorm, a.eta * beta);
    }
    if (fnorm == 0.0) {
      for (int e = tid; e < nloc; e += kThreads) a.x[e0 + e] = 0.0;
      conv = true;
      res_est = 0.0;
      break;
    }
    res_est = beta;
    if (beta <= tgt || total >= a.max_iter) {
      conv = beta <= tgt;
      break;
    }
    // an FP32 cycle only needs to reduce its own residual by inner_tol
    const double cycle_tgt = kMixed ? fmax(tgt, a.inner_tol * beta) : tgt;
    for (int i = tid; i < m + 2; i += kThreads) gv[i] = i == 0 ? beta : 0.0;
    __syncthreads();
    double nu = beta;
    int j = 0;
    while (true) {
      T* w = Vl + (int64_t)(j + 1) * ldv;
      if constexpr (MF == 1)
        apply_slice_mfma<T>(a, c, Qw, phiRw, W, (T)(1.0 / nu), w);
      else if constexpr (MF == 2) {
        apply_slice_mfg<T, double>(a, c, reinterpret_cast<const T*>(a.Qfw), phiRw, W,
                                   (T)(1.0 / nu), a.Py + (int64_t)c.pslot * c.nr1);
        if (a.S > 1) grid_sync(a.bar, target, a.wait_limit);
        mfg_reduce<T>(a, c, w);
      }
      else
        apply_slices<T>(a, c, Qw, phiRw, W, (T)(1.0 / nu), w, fullBw);
      // normalise V_j (its norm is known now), first-pass dots
      {
        const double inv = 1.0 / nu;
        T* vj = Vl + (int64_t)j * ldv;
        for (int e = tid; e < nloc; e += kThreads) vj[e] = (T)((double)vj[e] * inv);
        __syncthreads();
        dots(j, w, a.Pd1 + (int64_t)b * (m + 1));
      }
      grid_sync(a.bar, target, a.wait_limit);
      gather(a.Pd1, j, hcol);
      orth(w, j, hcol);
      __syncthreads();
      dots(j, w, a.Pd2 + (int64_t)b * (m + 1));
      grid_sync(a.bar, target, a.wait_limit);
      gather(a.Pd2, j, h2);
      {
        double nn = orth(w, j, h2);
        for (int i = tid; i <= j; i += kThreads) hcol[i] += h2[i];
        for (int e = tid; e < nloc; e += kThreads) W[e0 + e] = w[e];
        nn = wg_sum(nn, red);
        if (tid == 0) a.Pn[2 * b] = nn;
      }
      grid_sync(a.bar, target, a.wait_limit);
      gather_pn(0);
      __syncthreads();
      // norm, Hessenberg column, Givens rotation (every workgroup, same order)
      if (tid == 0) {
        const double nrm = sqrt(bcast[2]);
        for (int i = 0; i < j; ++i) {
          const double t = cs[i] * hcol[i] + sn[i] * hcol[i + 1];
          hcol[i + 1] = -sn[i] * hcol[i] + cs[i] * hcol[i + 1];
          hcol[i] = t;
        }
        const double p = hcol[j], q = nrm;
        const double rho = sqrt(p * p + q * q);
        const double cc = rho > 0.0 ? p / rho : 1.0, sg = rho > 0.0 ? q / rho : 0.0;
        cs[j] = cc;
        sn[j] = sg;
        hcol[j] = rho;
        gv[j + 1] = -sg * gv[j];
        gv[j] = cc * gv[j];
        double* col = Hpk + j * (j + 1) / 2;
        for (int i = 0; i <= j; ++i) col[i] = hcol[i];
        bcast[0] = nrm;
        bcast[1] = fabs(gv[j + 1]);
      }
      __syncthreads();
      nu = bcast[0];
      res_est = bcast[1];
      ++j;
      ++total;
      if (res_est <= cycle_tgt) {
        // FP64: the estimate is trusted.  Mixed: the next FP64 residual decides.
        conv = !kMixed;
        break;
      }
      if (j >= m || total >= a.max_iter || !(nu > 0.0)) break;
    }
    // y = R^{-1} g by one wave (lanes hold rows r and r + 64), then x += V y
    if (tid < 64) {
      double g0 = lane < j ? gv[lane] : 0.0;
      double g1 = lane + 64 < j ? gv[lane + 64] : 0.0;
      for (int i = j - 1; i >= 0; --i) {
        const double gi = __shfl(i < 64 ? g0 : g1, i & 63, 64);
        const double* col = Hpk + i * (i + 1) / 2;
        const double d = col[i];
        const double yi = d != 0.0 ? gi / d : 0.0;
        if (lane == 0) h2[i] = yi;
        if (lane < i) g0 -= col[lane] * yi;
        if (lane + 64 < i) g1 -= col[lane + 64] * yi;
      }
    }
    __syncthreads();
    for (int e = tid; e < nloc; e += kThreads) {
      double acc = a.x[e0 + e];
      for (int i = 0; i < j; ++i) acc = fma(h2[i], (double)Vl[(int64_t)i * ldv + e], acc);
      a.x[e0 + e] = acc;
    }
    if (conv || total >= a.max_iter) break;
    grid_sync(a.bar, target, a.wait_limit);
  }
  if (b == 0 && tid == 0) {
    a.info[0] = (double)total;
    a.info[1] = conv ? 1.0 : 0.0;
    a.info[2] = fnorm > 0.0 ? res_est / fnorm : 0.0;
  }
  // info[4] was cleared before the launch; a workgroup that saw the abort
  // word (at least the one that set it) marks the result invalid.
  if (tid == 0 && __hip_atomic_load(a.bar + 48, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
    a.info[4] = 1.0;
}

struct DevInfo {
  int cus = 0;
  int lds_max = 0;
  int wall_khz = 0;     // rate of the device's constant wall clock
};

// How long a workgroup waits at a grid barrier before it gives up (seconds;
// set by ttnt_set_grid_wait_limit, default 20 s).
std::atomic<double> g_wait_limit_s{20.0};

long long wait_limit_ticks(const DevInfo& d) {
  const double t = g_wait_limit_s.load() * (double)d.wall_khz * 1e3;
  return t >= 9.0e18 ? (long long)9e18 : (long long)t;
}

constexpr int kMaxDev = 64;
std::mutex g_dev_mu;      // device queries, kernel attributes and cooperative launches

const void* kernel_ptr(bool mixed, int mode) {
  if (mixed)
    return mode == 2   ? reinterpret_cast<const void*>(gmres_slices_kernel<float, 2>)
           : mode == 1 ? reinterpret_cast<const void*>(gmres_slices_kernel<float, 1>)
                       : reinterpret_cast<const void*>(gmres_slices_kernel<float, 0>);
  return mode == 2   ? reinterpret_cast<const void*>(gmres_slices_kernel<double, 2>)
         : mode == 1 ? reinterpret_cast<const void*>(gmres_slices_kernel<double, 1>)
                     : reinterpret_cast<const void*>(gmres_slices_kernel<double, 0>);
}

// Device properties, and the kernels' LDS attribute raised once per device
// and process.
DevInfo dev_info() {
  static DevInfo di[kMaxDev];
  static bool ready[kMaxDev] = {};
  int dev = 0;
  TT_HIP(hipGetDevice(&dev));
  TT_REQUIRE(dev >= 0 && dev < kMaxDev, "device index out of range");
  std::lock_guard<std::mutex> lock(g_dev_mu);
  if (!ready[dev]) {
    DevInfo d;
    TT_HIP(hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev));
    int coop = 0;
    TT_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    TT_REQUIRE(coop != 0, "device does not support cooperative launches");
    TT_HIP(hipDeviceGetAttribute(&d.lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    TT_HIP(hipDeviceGetAttribute(&d.wall_khz, hipDeviceAttributeWallClockRate, dev));
    TT_REQUIRE(d.wall_khz > 0, "device reports no wall-clock rate");
    for (int v = 0; v < 6; ++v)
      TT_HIP(hipFuncSetAttribute(kernel_ptr(v >= 3, v % 3),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, d.lds_max - 1024));
    di[dev] = d;
    ready[dev] = true;
  }
  return di[dev];
}

thread_local int t_cap_override = 0;

int grid_cap() {
  static const int want = [] {
    const char* e = std::getenv("TTNT_KRYLOV_GRID");
    const int v = e ? std::atoi(e) : 0;
    return v > 0 ? v : kKrylovMaxGrid;
  }();
  return t_cap_override > 0 ? std::min(want, t_cap_override) : want;
}

struct Plan {
  int G = 0, spw = 0, m = 0, ldv = 0;
  int mode = 0;          // operator application form (the kernel's MF)
  int bc = 0;            // general matrix-core form: beta' per sub-chunk
  int ts = 0;            // LDS room of T (doubles)
  int S = 1;             // general matrix-core form: workgroups per slice
  size_t lds_bytes = 0;
};

bool mfma_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("TTNT_KRYLOV_MFMA");
    return !(e && e[0] == '0');
  }();
  return on;
}

size_t lds_bytes_for(int ts, int m, int ldv, bool mixed) {
  const size_t dbl = (size_t)kAsDoubles + kBsDoubles + (size_t)ts + ldv +
                     (size_t)m * (m + 1) / 2 + 5 * (size_t)(m + 2) + 32;
  return dbl * sizeof(double) + (size_t)(m + 1) * ldv * (mixed ? sizeof(float) : sizeof(double));
}

// Workgroups per slice S and beta' per sub-chunk of the general matrix-core
// form: up to four workgroups per slice within the grid cap, each with at
// least eight beta', and sub-chunks of at most 64 rows (n bc <= 64).
void mfg_split(const KrylovShape& sh, int cap, int& S, int& bc) {
  S = std::max(1, std::min({4, cap / std::max(1, sh.r0), std::max(1, sh.RR / 8)}));
  const int q = cdiv(sh.RR, S);
  bc = std::max(1, std::min(64 / sh.n, q));
}

// Largest restart length m <= mmax (at least 2) whose LDS fits, 0 if none.
int fit_restart(int ts, int mmax, int ldv, bool mixed, size_t limit) {
  int m = mmax;
  while (m >= 2 && lds_bytes_for(ts, m, ldv, mixed) > limit) --m;
  return m >= 2 ? m : 0;
}

// Workgroups, slices per workgroup, the operator application form and the
// restart length that fits in LDS (the largest m <= restart, at least 2); G
// == 0 when nothing fits.  One slice per workgroup takes a matrix-core form:
// the register-resident one when n RR <= 128, n r0 <= 80 and the
// fragment-ordered v fits in Bs, else the general one for n <= 4, r1 <= 96
// (mfg_split).  The vector form of the mixed
// kernel also needs the whole FP32 right operand of its first product in LDS.
Plan make_plan(const KrylovShape& sh, int restart, int lds_limit_bytes, bool mixed) {
  Plan p;
  const int cap = std::max(1, grid_cap());
  p.spw = (sh.r0 + cap - 1) / cap;
  p.G = (sh.r0 + p.spw - 1) / p.spw;
  const int nloc = p.spw * sh.n * sh.r1;
  p.ldv = nloc + ((nloc % 2 == 0) ? 1 : 0);
  const size_t limit = (size_t)std::max(0, lds_limit_bytes - 1024);
  const int mmax = std::min(restart, kMaxRestart);
  const int64_t k1 = (int64_t)sh.n * sh.r0, m1 = (int64_t)sh.n * sh.RR;
  const int full_ts = (int)std::min<int64_t>(m1 * sh.r1, 1 << 30);
  if (mfma_enabled() && p.spw == 1 && m1 <= 16 * 4 * kMfmaMT && k1 <= 4 * kMfmaKS &&
      cdiv(k1, (int64_t)4) * cdiv((int64_t)sh.r1, (int64_t)16) * 64 <= kBFull) {
    p.mode = 1;
    p.ts = full_ts;
    p.m = fit_restart(p.ts, mmax, p.ldv, mixed, limit);
  } else if (mfma_enabled() && p.spw == 1 && sh.n <= 4 && sh.r1 <= 16 * kMfgPairs) {
    p.mode = 2;
    mfg_split(sh, cap, p.S, p.bc);
    p.G = sh.r0 * p.S;
    const int own = cdiv(sh.n * sh.r1, p.S);
    p.ldv = own + ((own % 2 == 0) ? 1 : 0);
    p.ts = sh.n * p.bc * sh.r1;
    p.m = fit_restart(p.ts, mmax, p.ldv, mixed, limit);
  } else {
    p.mode = 0;
    p.ts = full_ts;
    if (mixed) {
      const int TNf = sh.r1 <= 32 ? 32 : 64;
      const int64_t Kp = cdiv(k1, (int64_t)16) * 16, Np = cdiv(sh.r1, TNf) * TNf;
      if (Kp * Np * (int64_t)sizeof(float) > (int64_t)kBFull * (int64_t)sizeof(double)) {
        p.G = 0;
        return p;
      }
    }
    p.m = fit_restart(p.ts, mmax, p.ldv, mixed, limit);
  }
  if (p.m < 2) {
    p.G = 0;
    return p;
  }
  p.lds_bytes = lds_bytes_for(p.ts, p.m, p.ldv, mixed);
  return p;
}

__global__ void to_f32_kernel(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

// Doubles of the fragment-ordered Q of the general matrix-core form for this
// shape and grid cap (zero for shapes it never takes).
int64_t qf_doubles(const KrylovShape& sh, int cap) {
  if (sh.n > 4 || sh.r1 > 16 * kMfgPairs || sh.r0 > cap) return 0;
  int S = 1, bc = 1;
  mfg_split(sh, cap, S, bc);
  const MfgGeom g = mfg_geom(sh.n, sh.r0, sh.RR, sh.r1, S, bc, 0);
  return (int64_t)sh.r0 * S * g.nsc * g.sc_size;
}

}  // namespace

bool krylov_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("TTNT_KRYLOV");
    return !(e && e[0] == '0');
  }();
  return on;
}

int krylov_grid() { return grid_cap(); }

void krylov_set_thread_cap(int cap) { t_cap_override = cap > 0 ? cap : 0; }

bool krylov_fits(const KrylovShape& sh, int restart, bool mixed) {
  if (restart < 2 || sh.r0 <= 0 || sh.r1 <= 0 || sh.n <= 0 || sh.RL <= 0 || sh.RR <= 0)
    return false;
  return make_plan(sh, restart, dev_info().lds_max, mixed).G > 0;
}

size_t krylov_ws_doubles(const KrylovShape& sh, int restart, int /*grid*/) {
  const int64_t N = (int64_t)sh.r0 * sh.n * sh.r1;
  const int cap = std::max(1, grid_cap());
  const int spw = (sh.r0 + cap - 1) / cap;
  // workgroups: one per spw slices, or up to four per slice within the cap
  const int64_t G = std::max<int64_t>((sh.r0 + spw - 1) / spw,
                                      std::min<int64_t>(4 * (int64_t)sh.r0, cap));
  const int64_t m = std::min(restart, kMaxRestart);
  const int64_t nq = (int64_t)sh.r0 * sh.n * sh.RR * sh.r0 * sh.n;
  const int64_t nr = (int64_t)sh.r1 * sh.RR * sh.r1;
  int64_t need = 0;
  need += N + 32;                    // W (either precision)
  need += nq + 32;                   // Q
  need += (nq + 1) / 2 + 32;         // Q in FP32 (mixed)
  need += (nr + 1) / 2 + 32;         // PhiR in FP32 (mixed)
  const int64_t nqf = qf_doubles(sh, cap);
  need += nqf + 32;                  // Q in fragment order (general matrix-core form)
  need += (nqf + 1) / 2 + 32;        // the same in FP32 (mixed)
  need += 4 * N + 32;                // partial products of up to four workgroups per slice
  need += 2 * (G * (m + 1) + 32);    // Pd1, Pd2
  need += 2 * G + 32;                // Pn
  need += 64;                        // barrier counter
  return (size_t)need + 8 * 32;
}

bool krylov_solve(hipStream_t s, const KrylovShape& sh, const double* phiL, const double* Ap,
                  const double* phiR, const double* f, double* x, int restart, int max_iter,
                  double tol, double eta, double* ws, size_t ws_doubles, double* info,
                  int /*grid*/, bool mixed, double inner_tol) {
  TT_REQUIRE(max_iter >= 0, "Krylov solve: negative iteration limit");
  const DevInfo di = dev_info();
  const Plan p = make_plan(sh, restart, di.lds_max, mixed);
  TT_REQUIRE(p.G > 0, "Krylov solve: local system too large for the LDS-resident basis");
  TT_REQUIRE(ws_doubles >= krylov_ws_doubles(sh, restart, 0), "Krylov solve: workspace too small");
  const int64_t N = (int64_t)sh.r0 * sh.n * sh.r1;
  const int64_t nq = (int64_t)sh.r0 * sh.n * sh.RR * sh.r0 * sh.n;
  const int64_t nr = (int64_t)sh.r1 * sh.RR * sh.r1;
  double* cur = ws;
  auto take = [&](int64_t count) {
    double* r = cur;
    cur += (count + 31) / 32 * 32;
    return r;
  };
  SArgs a;
  a.phiL = phiL;
  a.Ap = Ap;
  a.phiR = phiR;
  a.r0 = sh.r0;
  a.RL = sh.RL;
  a.n = sh.n;
  a.RR = sh.RR;
  a.r1 = sh.r1;
  a.N = N;
  a.f = f;
  a.x = x;
  a.W = take(N);
  a.Q = take(nq);
  float* q32 = reinterpret_cast<float*>(take((nq + 1) / 2));
  float* r32 = reinterpret_cast<float*>(take((nr + 1) / 2));
  a.Qw = mixed ? static_cast<void*>(q32) : static_cast<void*>(a.Q);
  const int64_t nqf = qf_doubles(sh, std::max(1, grid_cap()));
  a.Qf = take(nqf);
  float* qf32 = reinterpret_cast<float*>(take((nqf + 1) / 2));
  a.Qfw = mixed ? static_cast<void*>(qf32) : static_cast<void*>(a.Qf);
  a.qf_slice = 0;
  a.S = p.S;
  a.Py = take(4 * N);
  TT_REQUIRE((int64_t)p.G * sh.n * sh.r1 <= 4 * N, "Krylov solve: partial products overflow");
  if (p.mode == 2) {
    const MfgGeom g = mfg_geom(sh.n, sh.r0, sh.RR, sh.r1, p.S, p.bc, 0);
    a.qf_slice = (int64_t)p.S * g.nsc * g.sc_size;
    TT_REQUIRE(a.qf_slice * sh.r0 <= nqf, "Krylov solve: fragment-ordered operator overflow");
  }
  a.phiRw = mixed ? static_cast<const void*>(r32) : static_cast<const void*>(phiR);
  a.Pd1 = take((int64_t)p.G * (p.m + 1));
  a.Pd2 = take((int64_t)p.G * (p.m + 1));
  a.Pn = take(2 * (int64_t)p.G);
  double* barslot = take(32);   // the count, and 128 bytes on the epoch flag
  a.bar = reinterpret_cast<unsigned*>(barslot);
  a.m = p.m;
  a.max_iter = max_iter;
  a.spw = p.spw;
  a.ldv = p.ldv;
  a.ts_doubles = p.ts;
  a.mfg_bc = p.bc;
  a.tol = tol;
  a.eta = eta;
  a.inner_tol = inner_tol;
  a.wait_limit = wait_limit_ticks(di);
  a.info = info;
  TT_REQUIRE((size_t)(cur - ws) <= ws_doubles, "Krylov solve: workspace layout overflow");

  int per_cu = 0;
  TT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel_ptr(mixed, p.mode),
                                                      kThreads, p.lds_bytes));
  TT_REQUIRE((int64_t)per_cu * di.cus >= p.G, "Krylov solve: grid exceeds co-resident capacity");

  if (mixed) {
    ++g_launches;
    to_f32_kernel<<<(int)std::min<int64_t>(1024, (nr + 255) / 256), 256, 0, s>>>(phiR, r32, nr);
    TT_HIP(hipGetLastError());
  }
  fill(s, barslot, 32, 0.0);   // count, epoch flag, abort word
  fill(s, info + 4, 1, 0.0);
  ++g_launches;
  hipEvent_t pe = nullptr;
  if (g_probe) pe = g_probe->begin(s, kProbeKrylov, 0.0, 0.0);   // work amended after the run
  void* args[] = {&a};
  {
    std::lock_guard<std::mutex> lock(g_dev_mu);
    TT_HIP(hipLaunchCooperativeKernel(kernel_ptr(mixed, p.mode), dim3(p.G), dim3(kThreads), args,
                                      p.lds_bytes, s));
  }
  if (pe) g_probe->end(s);
  return pe != nullptr;
}

void krylov_set_wait_limit(double seconds) { g_wait_limit_s.store(seconds); }

int krylov_restart(const KrylovShape& sh, int restart, bool mixed) {
  const Plan p = make_plan(sh, restart, dev_info().lds_max, mixed);
  return p.G > 0 ? p.m : 0;
}

}  // namespace ttnt
