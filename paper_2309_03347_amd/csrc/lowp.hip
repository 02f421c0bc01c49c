// Low-precision contractions: batched GEMM on the BF16 matrix cores with FP32
// accumulation (the bulk products of the mixed-precision local solves; the
// paper's contractions are the TT-matrix core products of Section 2.2).
//
// Operands live in FP64 and are rounded to BF16 when a tile is staged into
// LDS; products accumulate in FP32 on v_mfma_f32_16x16x32_bf16 and the result
// is written in FP64.  BF16 keeps the FP32 exponent range, so no operand
// scaling is needed to stay in range; the relative error of each product is
// that of two BF16 roundings (2^-8 each).  Callers use it only inside
// iterative refinement, whose residuals are FP64.
#include <algorithm>

#include "kernels.h"
#include "probe.h"

namespace ttnt {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int LT = 64;     // output tile (LT x LT per workgroup of 256 threads)
constexpr int LK = 32;     // k-step of the matrix instruction
constexpr int LP = LK + 8; // LDS row pitch in BF16 elements (80 bytes: 16-byte aligned rows)

// C[b] = alpha op(A[b]) op(B[b]) + beta C[b] for rows [64 by, ...) and columns
// [64 bx, ...), k in [kb, ke).  Wavefront w owns the 32 x 32 sub-tile
// (32 (w / 2), 32 (w % 2)): 2 x 2 matrix-instruction tiles of 16 x 16.  Lane l
// holds A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16] (e < 8) and
// receives D[4 (l / 16) + r][l % 16] (r < 4).
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, double alpha,
                                                        const double* __restrict__ A, int lda,
                                                        int64_t sA, const double* __restrict__ B,
                                                        int ldb, int64_t sB, double beta,
                                                        double* __restrict__ C, int ldc,
                                                        int64_t sC, int nsplit, int kchunk,
                                                        int batch) {
  __shared__ __attribute__((aligned(16))) __bf16 As[LT * LP];   // [row][k]
  __shared__ __attribute__((aligned(16))) __bf16 Bs[LT * LP];   // [col][k]
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
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = kb; k0 < ke; k0 += LK) {
    // stage op(A) rows and op(B) columns, 8 consecutive k per thread
    {
      bf16x8 va, vb;
      if (!TA) {
        const int row = tid >> 2, kq = (tid & 3) * 8;
        const int gm = m0 + row;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int gk = k0 + kq + e;
          va[e] = (__bf16)(float)((gm < M && gk < ke) ? Ab[(int64_t)gm * lda + gk] : 0.0);
        }
        *reinterpret_cast<bf16x8*>(&As[row * LP + kq]) = va;
      } else {
        const int row = tid & 63, kq = (tid >> 6) * 8;
        const int gm = m0 + row;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int gk = k0 + kq + e;
          va[e] = (__bf16)(float)((gm < M && gk < ke) ? Ab[(int64_t)gk * lda + gm] : 0.0);
        }
        *reinterpret_cast<bf16x8*>(&As[row * LP + kq]) = va;
      }
      if (!TB) {
        const int col = tid & 63, kq = (tid >> 6) * 8;
        const int gn = n0 + col;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int gk = k0 + kq + e;
          vb[e] = (__bf16)(float)((gn < N && gk < ke) ? Bb[(int64_t)gk * ldb + gn] : 0.0);
        }
        *reinterpret_cast<bf16x8*>(&Bs[col * LP + kq]) = vb;
      } else {
        const int col = tid >> 2, kq = (tid & 3) * 8;
        const int gn = n0 + col;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int gk = k0 + kq + e;
          vb[e] = (__bf16)(float)((gn < N && gk < ke) ? Bb[(int64_t)gn * ldb + gk] : 0.0);
        }
        *reinterpret_cast<bf16x8*>(&Bs[col * LP + kq]) = vb;
      }
    }
    __syncthreads();
    bf16x8 fa[2], fb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      fa[i] = *reinterpret_cast<const bf16x8*>(&As[(32 * wr + 16 * i + (l & 15)) * LP + 8 * (l >> 4)]);
      fb[i] = *reinterpret_cast<const bf16x8*>(&Bs[(32 * wc + 16 * i + (l & 15)) * LP + 8 * (l >> 4)]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
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

}  // namespace

void gemm_bf16(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
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
  TT_REQUIRE(grid.y <= 65535 && grid.z <= 65535, "bf16 gemm grid too large");
  ++g_launches;
  hipEvent_t pe = nullptr;
  if (g_probe) {
    const double fl = 2.0 * M * N * (double)K * batch;
    const double by = 8.0 * batch * ((double)M * K + (double)K * N + (double)M * N * (beta != 0.0 ? 2 : 1));
    pe = g_probe->begin(s, kProbeGemmBf16, fl, by);
  }
  if (!ta && !tb)
    gemm_bf16_kernel<false, false><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, out, ldc, sC, nsplit, kchunk, batch);
  else if (ta && !tb)
    gemm_bf16_kernel<true, false><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, out, ldc, sC, nsplit, kchunk, batch);
  else if (!ta && tb)
    gemm_bf16_kernel<false, true><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, out, ldc, sC, nsplit, kchunk, batch);
  else
    gemm_bf16_kernel<true, true><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, out, ldc, sC, nsplit, kchunk, batch);
  TT_HIP(hipGetLastError());
  if (pe) g_probe->end(s);
  if (nsplit > 1) splitk_reduce(s, g_splitk_buf, nsplit, batch, M, N, alpha, beta, C, ldc, sC);
}

}  // namespace ttnt
