// Low-precision contractions: batched GEMM on the BF16 or FP16 matrix cores
// with FP32 accumulation (the bulk products of the mixed-precision local
// solves; the paper's contractions are the TT-matrix core products of
// Section 2.2).
//
// Operands live in FP64 and are rounded when a tile is staged into LDS;
// products accumulate in FP32 on v_mfma_f32_16x16x32_{bf16,f16} and the
// result is written in FP64.
//
// BF16 keeps the FP32 exponent range, so its operands are cast as they are;
// the relative error of each product is that of two BF16 roundings (2^-8
// each).  FP16 has three more mantissa bits but a range of 2^-24 .. 65504, so
// each operand is scaled before the cast: every row of A and every column of B
// is divided, within each 32-deep k block, by the power of two just above its
// largest magnitude (so the block's entries lie in (-1, 1) and the scaling
// itself is exact), and each block's FP32 partial product is multiplied back
// by the two scales as it is added to the accumulator.  The relative error of
// a product is then that of two FP16 roundings (2^-11 each), plus an absolute
// 2^-25 of the block scale for entries that fall below FP16's normal range
// (smaller than 2^-14 of their block's largest).  The product of a row's and
// a column's scale is formed in FP32, like the accumulator, so results (and
// block maxima) are held to FP32's range, as with BF16.  Callers use either
// form only inside iterative refinement, whose residuals are FP64.
#include <algorithm>
#include <cmath>

#include "kernels.h"
#include "probe.h"

namespace ttnt {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int LT = 64;     // output tile (LT x LT per workgroup of 256 threads)
constexpr int LK = 32;     // k-step of the matrix instruction
constexpr int LP = LK + 8; // LDS row pitch in 16-bit elements (80 bytes: 16-byte aligned rows)
// FP16 block scales are powers of two held in FP32: exponents -126 .. 127
constexpr int kScaleLo = -126, kScaleHi = 127;

template <bool F16> struct LowpT;
template <> struct LowpT<false> {
  typedef __bf16 T;
  typedef bf16x8 V;
  static __device__ f32x4 mma(V a, V b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct LowpT<true> {
  typedef _Float16 T;
  typedef f16x8 V;
  static __device__ f32x4 mma(V a, V b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// Largest magnitude over the lanes l ^ m1, l ^ m2 (the four lanes holding one
// row or column of a k block); returns the block's power-of-two scale.
__device__ inline double block_scale(double mx, int m1, int m2) {
  mx = fmax(mx, __shfl_xor(mx, m1));
  mx = fmax(mx, __shfl_xor(mx, m2));
  int e = 0;
  if (mx > 0.0) (void)frexp(mx, &e);      // mx = f 2^e, f in [0.5, 1)
  e = min(max(e, kScaleLo), kScaleHi);
  return ldexp(1.0, e);
}

// C[b] = alpha op(A[b]) op(B[b]) + beta C[b] for rows [64 by, ...) and columns
// [64 bx, ...), k in [kb, ke).  Wavefront w owns the 32 x 32 sub-tile
// (32 (w / 2), 32 (w % 2)): 2 x 2 matrix-instruction tiles of 16 x 16.  Lane l
// holds A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16] (e < 8) and
// receives D[4 (l / 16) + r][l % 16] (r < 4).
//
// Staging: each thread loads 8 consecutive k of one row of op(A) and of one
// column of op(B).  With FP16 the four threads of a row (column) sit in one
// wavefront, at lanes l ^ 1, l ^ 2 when the 8 k are contiguous in memory and
// at lanes l ^ 16, l ^ 32 when they are strided (16 rows of one k per 16 lanes,
// still 128-byte coalesced), so the block maximum is a two-step shuffle.
template <bool TA, bool TB, bool F16>
__global__ __launch_bounds__(256) void gemm_lowp_kernel(int M, int N, int K, double alpha,
                                                        const double* __restrict__ A, int lda,
                                                        int64_t sA, const double* __restrict__ B,
                                                        int ldb, int64_t sB, double beta,
                                                        double* __restrict__ C, int ldc,
                                                        int64_t sC, int nsplit, int kchunk,
                                                        int batch) {
  typedef typename LowpT<F16>::T HT;
  typedef typename LowpT<F16>::V HV;
  __shared__ __attribute__((aligned(16))) HT As[LT * LP];   // [row][k]
  __shared__ __attribute__((aligned(16))) HT Bs[LT * LP];   // [col][k]
  __shared__ __attribute__((aligned(16))) float Sa[LT];     // FP16: row scales of the k block
  __shared__ __attribute__((aligned(16))) float Sb[LT];     // FP16: column scales
  const int64_t bz = blockIdx.z % batch;
  const int split = blockIdx.z / batch;
  const int kb = split * kchunk;
  const int ke = min(K, kb + kchunk);
  const int m0 = blockIdx.y * LT, n0 = blockIdx.x * LT;
  const double* Ab = A + bz * sA;
  const double* Bb = B + bz * sB;
  double* Cb;
  int ldo = ldc;
  if (nsplit > 1) {
    Cb = C + ((int64_t)split * batch + bz) * M * N;
    ldo = N;
  } else {
    Cb = C + bz * sC;
  }
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  // staging coordinates: contiguous k (quad of lanes per row) or strided k
  const int qrow = tid >> 2, qk = (tid & 3) * 8;
  const int srow = F16 ? (tid & 15) + 16 * w : (tid & 63);
  const int sk = F16 ? ((tid >> 4) & 3) * 8 : w * 8;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = kb; k0 < ke; k0 += LK) {
    // stage op(A) rows and op(B) columns, 8 consecutive k per thread
    {
      double va[8], vb[8];
      const int ar = TA ? srow : qrow, ak = TA ? sk : qk;
      const int bc = TB ? qrow : srow, bk = TB ? qk : sk;
      const int gm = m0 + ar, gn = n0 + bc;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int gk = k0 + ak + e;
        va[e] = (gm < M && gk < ke) ? (TA ? Ab[(int64_t)gk * lda + gm] : Ab[(int64_t)gm * lda + gk])
                                    : 0.0;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int gk = k0 + bk + e;
        vb[e] = (gn < N && gk < ke) ? (TB ? Bb[(int64_t)gn * ldb + gk] : Bb[(int64_t)gk * ldb + gn])
                                    : 0.0;
      }
      double ia = 1.0, ib = 1.0;
      if (F16) {
        double ma = 0.0, mb = 0.0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          ma = fmax(ma, fabs(va[e]));
          mb = fmax(mb, fabs(vb[e]));
        }
        const double sa = TA ? block_scale(ma, 16, 32) : block_scale(ma, 1, 2);
        const double sb = TB ? block_scale(mb, 1, 2) : block_scale(mb, 16, 32);
        ia = 1.0 / sa;   // powers of two: exact
        ib = 1.0 / sb;
        if (ak == 0) Sa[ar] = (float)sa;
        if (bk == 0) Sb[bc] = (float)sb;
      }
      HV ha, hb;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        ha[e] = (HT)(float)(va[e] * ia);
        hb[e] = (HT)(float)(vb[e] * ib);
      }
      *reinterpret_cast<HV*>(&As[ar * LP + ak]) = ha;
      *reinterpret_cast<HV*>(&Bs[bc * LP + bk]) = hb;
    }
    __syncthreads();
    HV fa[2], fb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      fa[i] = *reinterpret_cast<const HV*>(&As[(32 * wr + 16 * i + (l & 15)) * LP + 8 * (l >> 4)]);
      fb[i] = *reinterpret_cast<const HV*>(&Bs[(32 * wc + 16 * i + (l & 15)) * LP + 8 * (l >> 4)]);
    }
    if (F16) {
      f32x4 ra[2];
      float rb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ra[i] = *reinterpret_cast<const f32x4*>(&Sa[32 * wr + 16 * i + 4 * (l >> 4)]);
        rb[i] = Sb[32 * wc + 16 * i + (l & 15)];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const f32x4 t = LowpT<F16>::mma(fa[i], fb[j], f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[i][j][r] += (ra[i][r] * rb[j]) * t[r];
        }
    } else {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = LowpT<F16>::mma(fa[i], fb[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + 32 * wr + 16 * i + 4 * (l >> 4) + r;
        const int gn = n0 + 32 * wc + 16 * j + (l & 15);
        if (gm < M && gn < N) {
          double* c = Cb + (int64_t)gm * ldo + gn;
          const double v = (double)acc[i][j][r];
          if (nsplit > 1)
            *c = v;
          else
            *c = beta == 0.0 ? alpha * v : alpha * v + beta * *c;
        }
      }
}

template <bool F16>
void launch_lowp(dim3 grid, hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
                 const double* A, int lda, int64_t sA, const double* B, int ldb, int64_t sB,
                 double beta, double* out, int ldc, int64_t sC, int nsplit, int kchunk,
                 int batch) {
  if (!ta && !tb)
    gemm_lowp_kernel<false, false, F16><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, out, ldc, sC, nsplit, kchunk, batch);
  else if (ta && !tb)
    gemm_lowp_kernel<true, false, F16><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, out, ldc, sC, nsplit, kchunk, batch);
  else if (!ta && tb)
    gemm_lowp_kernel<false, true, F16><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, out, ldc, sC, nsplit, kchunk, batch);
  else
    gemm_lowp_kernel<true, true, F16><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, out, ldc, sC, nsplit, kchunk, batch);
}

void gemm_lowp(bool f16, hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
               const double* A, int lda, int64_t sA, const double* B, int ldb, int64_t sB,
               double beta, double* C, int ldc, int64_t sC, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0) {
    gemm(s, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch);
    return;
  }
  // few output tiles and a long K: split K, reduce the FP64 partials in order
  const int64_t tiles = (int64_t)cdiv(N, LT) * cdiv(M, LT) * batch;
  int nsplit = 1;
  if (g_splitk_buf && tiles < 256 && K >= 8 * LK) {
    nsplit = (int)std::min<int64_t>({(int64_t)cdiv(K, 4 * LK), 512 / tiles + 1, 64});
    while (nsplit > 1 && (size_t)nsplit * batch * M * N > g_splitk_cap) --nsplit;
    if ((int64_t)nsplit * batch > 65535) nsplit = 1;
  }
  int kchunk = K;
  if (nsplit > 1) {
    kchunk = cdiv(cdiv(K, nsplit), LK) * LK;
    nsplit = cdiv(K, kchunk);
  }
  double* out = nsplit > 1 ? g_splitk_buf : C;
  dim3 grid(cdiv(N, LT), cdiv(M, LT), batch * nsplit);
  TT_REQUIRE(grid.y <= 65535 && grid.z <= 65535, "low-precision gemm grid too large");
  ++g_launches;
  hipEvent_t pe = nullptr;
  if (g_probe) {
    const double fl = 2.0 * M * N * (double)K * batch;
    const double by = 8.0 * batch * ((double)M * K + (double)K * N + (double)M * N * (beta != 0.0 ? 2 : 1));
    pe = g_probe->begin(s, kProbeGemmBf16, fl, by);
  }
  if (f16)
    launch_lowp<true>(grid, s, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, out, ldc, sC, nsplit, kchunk, batch);
  else
    launch_lowp<false>(grid, s, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, out, ldc, sC, nsplit, kchunk, batch);
  TT_HIP(hipGetLastError());
  if (pe) g_probe->end(s);
  if (nsplit > 1) splitk_reduce(s, g_splitk_buf, nsplit, batch, M, N, alpha, beta, C, ldc, sC);
}

}  // namespace

void gemm_bf16(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
               const double* A, int lda, int64_t sA, const double* B, int ldb, int64_t sB,
               double beta, double* C, int ldc, int64_t sC, int batch) {
  gemm_lowp(false, s, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch);
}

void gemm_f16(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
              const double* A, int lda, int64_t sA, const double* B, int ldb, int64_t sB,
              double beta, double* C, int ldc, int64_t sC, int batch) {
  gemm_lowp(true, s, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch);
}

}  // namespace ttnt
