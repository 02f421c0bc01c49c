// Dense FP64 building blocks: batched GEMM, copies, reductions.
#include <algorithm>

#include "gemm_tile.h"
#include "kernels.h"
#include "probe.h"

namespace ttnt {

thread_local int64_t g_launches = 0;
thread_local double* g_splitk_buf = nullptr;
thread_local size_t g_splitk_cap = 0;
thread_local double* g_fact_buf = nullptr;
thread_local size_t g_fact_cap = 0;

namespace {

constexpr int BM = kTileM, BN = kTileN, BK = kTileK, GT = 256;

template <bool TA, bool TB>
__global__ __launch_bounds__(GT) void gemm_kernel(int M, int N, int K, double alpha,
                                                  const double* __restrict__ A, int lda,
                                                  int64_t sA, const double* __restrict__ B,
                                                  int ldb, int64_t sB, double beta,
                                                  double* __restrict__ C, int ldc, int64_t sC,
                                                  int nsplit, int kchunk, int batch) {
  __shared__ double As[kTileK][kTileM + 1];
  __shared__ double Bs[kTileK][kTileN + 1];
  const int64_t bz = blockIdx.z % batch;
  const int split = blockIdx.z / batch;
  const int kb = split * kchunk;
  const int ke = min(K, kb + kchunk);
  double* Cb;
  if (nsplit > 1) {
    Cb = C + ((int64_t)split * batch + bz) * M * N;
    ldc = N;
  } else {
    Cb = C + bz * sC;
  }
  gemm_tile<TA, TB>(blockIdx.y, blockIdx.x, M, N, kb, ke, alpha, A + bz * sA, lda, B + bz * sB,
                    ldb, beta, Cb, ldc, nsplit > 1, As, Bs);
}

// C[b][m][n] = alpha * sum_s P[s][b][m][n] + beta * C[b][m][n]  (fixed order in s)
__global__ void splitk_reduce_kernel(const double* __restrict__ P, int nsplit, int batch, int M,
                                     int N, double alpha, double beta, double* __restrict__ C,
                                     int ldc, int64_t sC) {
  const int64_t per = (int64_t)M * N;
  const int64_t total = per * batch;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / per, r = e % per;
    const int m = (int)(r / N), n = (int)(r % N);
    double acc = 0.0;
    for (int s = 0; s < nsplit; ++s) acc += P[((int64_t)s * batch + b) * per + r];
    double* c = C + b * sC + (int64_t)m * ldc + n;
    *c = beta == 0.0 ? alpha * acc : alpha * acc + beta * *c;
  }
}

__global__ void transpose_kernel(const double* __restrict__ src, int rows, int cols, int lds,
                                 double* __restrict__ dst, int ldd) {
  __shared__ double tile[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 32 x 8
  for (int y = ty; y < 32; y += 8) {
    const int r = r0 + y, c = c0 + tx;
    tile[y][tx] = (r < rows && c < cols) ? src[(int64_t)r * lds + c] : 0.0;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int c = c0 + y, r = r0 + tx;
    if (c < cols && r < rows) dst[(int64_t)c * ldd + r] = tile[tx][y];
  }
}

__global__ void copy2d_kernel(const double* __restrict__ src, int rows, int cols, int lds,
                              double* __restrict__ dst, int ldd) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / cols), c = (int)(e % cols);
    dst[(int64_t)r * ldd + c] = src[(int64_t)r * lds + c];
  }
}

__global__ void fill_kernel(double* dst, int64_t n, double v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = v;
}

__global__ void axpby_kernel(int64_t n, double a, const double* __restrict__ x, double b,
                             const double* __restrict__ c, double* __restrict__ y) {
  const double bb = c ? b / *c : b;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    y[e] = a * x[e] + bb * y[e];
}

__global__ __launch_bounds__(1024) void sumsq_kernel(const double* __restrict__ x, int64_t n,
                                                     double* out) {
  __shared__ double red[16];
  double v = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) v = fma(x[e], x[e], v);
  v = block_sum(v, red);
  if (threadIdx.x == 0) *out = v;
}

__global__ void scale_inv_sqrt_kernel(double* x, int64_t n, const double* ss) {
  const double f = 1.0 / sqrt(*ss);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] *= f;
}

int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

void gemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
          int lda, int64_t sA, const double* B, int ldb, int64_t sB, double beta, double* C,
          int ldc, int64_t sC, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0) {
    // C = beta * C
    for (int b = 0; b < batch; ++b) {
      if (beta == 0.0) {
        for (int r = 0; r < M; ++r) fill(s, C + b * sC + (int64_t)r * ldc, N, 0.0);
      } else {
        for (int r = 0; r < M; ++r)
          axpby(s, N, 0.0, C + b * sC + (int64_t)r * ldc, beta, C + b * sC + (int64_t)r * ldc);
      }
    }
    return;
  }
  // Few output tiles and a long K: split K over workgroups into a scratch
  // buffer and reduce in a second, deterministic pass.
  const int64_t tiles = (int64_t)cdiv(N, BN) * cdiv(M, BM) * batch;
  int nsplit = 1;
  if (g_splitk_buf && tiles < 128 && K >= 4 * BK * 8) {
    nsplit = (int)std::min<int64_t>({(int64_t)cdiv(K, BK * 8), 256 / tiles + 1, 64});
    while (nsplit > 1 && (size_t)nsplit * batch * M * N > g_splitk_cap) --nsplit;
    if ((int64_t)nsplit * batch > 65535) nsplit = 1;
  }
  int kchunk = K;
  if (nsplit > 1) {
    kchunk = cdiv(cdiv(K, nsplit), BK) * BK;
    nsplit = cdiv(K, kchunk);
  }
  double* out = nsplit > 1 ? g_splitk_buf : C;
  dim3 grid(cdiv(N, BN), cdiv(M, BM), batch * nsplit);
  TT_REQUIRE(grid.y <= 65535 && grid.z <= 65535, "gemm grid too large");
  ++g_launches;
  hipEvent_t pe = nullptr;
  if (g_probe) {
    const double fl = 2.0 * M * N * (double)K * batch;
    const double by = 8.0 * batch * ((double)M * K + (double)K * N + (double)M * N * (beta != 0.0 ? 2 : 1));
    pe = g_probe->begin(s, (ta ? 1 : 0) + (tb ? 2 : 0), fl, by);
  }
  if (!ta && !tb)
    gemm_kernel<false, false><<<grid, GT, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, out, ldc, sC, nsplit, kchunk, batch);
  else if (ta && !tb)
    gemm_kernel<true, false><<<grid, GT, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, out, ldc, sC, nsplit, kchunk, batch);
  else if (!ta && tb)
    gemm_kernel<false, true><<<grid, GT, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, out, ldc, sC, nsplit, kchunk, batch);
  else
    gemm_kernel<true, true><<<grid, GT, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, out, ldc, sC, nsplit, kchunk, batch);
  TT_HIP(hipGetLastError());
  if (pe) g_probe->end(s);
  if (nsplit > 1) {
    ++g_launches;
    splitk_reduce_kernel<<<grid_for((int64_t)M * N * batch, 256), 256, 0, s>>>(
        g_splitk_buf, nsplit, batch, M, N, alpha, beta, C, ldc, sC);
    TT_HIP(hipGetLastError());
  }
}

void splitk_reduce(hipStream_t s, const double* P, int nsplit, int batch, int M, int N,
                   double alpha, double beta, double* C, int ldc, int64_t sC) {
  ++g_launches;
  splitk_reduce_kernel<<<grid_for((int64_t)M * N * batch, 256), 256, 0, s>>>(
      P, nsplit, batch, M, N, alpha, beta, C, ldc, sC);
  TT_HIP(hipGetLastError());
}

void transpose(hipStream_t s, const double* src, int rows, int cols, int lds, double* dst,
               int ldd) {
  if (rows <= 0 || cols <= 0) return;
  dim3 grid(cdiv(cols, 32), cdiv(rows, 32));
  TT_REQUIRE(grid.y <= 65535, "transpose grid too large");
  ++g_launches;
  transpose_kernel<<<grid, 256, 0, s>>>(src, rows, cols, lds, dst, ldd);
  TT_HIP(hipGetLastError());
}

void copy2d(hipStream_t s, const double* src, int rows, int cols, int lds, double* dst, int ldd) {
  if (rows <= 0 || cols <= 0) return;
  ++g_launches;
  copy2d_kernel<<<grid_for((int64_t)rows * cols, 256), 256, 0, s>>>(src, rows, cols, lds, dst, ldd);
  TT_HIP(hipGetLastError());
}

void copy(hipStream_t s, const double* src, double* dst, int64_t n) {
  if (n <= 0 || src == dst) return;
  ++g_launches;
  TT_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, s));
}

void fill(hipStream_t s, double* dst, int64_t n, double v) {
  if (n <= 0) return;
  ++g_launches;
  fill_kernel<<<grid_for(n, 256), 256, 0, s>>>(dst, n, v);
  TT_HIP(hipGetLastError());
}

void axpby(hipStream_t s, int64_t n, double a, const double* x, double b, double* y) {
  if (n <= 0) return;
  ++g_launches;
  axpby_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, a, x, b, nullptr, y);
  TT_HIP(hipGetLastError());
}

void axpby_div(hipStream_t s, int64_t n, double a, const double* x, double b, const double* c,
               double* y) {
  if (n <= 0) return;
  ++g_launches;
  axpby_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, a, x, b, c, y);
  TT_HIP(hipGetLastError());
}

void sumsq(hipStream_t s, const double* x, int64_t n, double* out) {
  ++g_launches;
  sumsq_kernel<<<1, 1024, 0, s>>>(x, n, out);
  TT_HIP(hipGetLastError());
}

void scale_inv_sqrt(hipStream_t s, double* x, int64_t n, const double* ss) {
  if (n <= 0) return;
  ++g_launches;
  scale_inv_sqrt_kernel<<<grid_for(n, 256), 256, 0, s>>>(x, n, ss);
  TT_HIP(hipGetLastError());
}

}  // namespace ttnt
