// Small dense factorizations used by TT rounding and the alternating solve.
// Each runs in one workgroup of 1024 threads (16 wavefronts) on global memory
// (the matrices are small and stay in cache).
#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace ttnt {
namespace {

constexpr int WG = 1024;
// Dynamic LDS budget of the single-workgroup factorizations (doubles).
constexpr int kLdsDoubles = 8000;

// Householder QR: A (m x n) -> Q (m x k), R (k x n), k = min(m, n), diag(R) >= 0.
__global__ __launch_bounds__(WG) void qr_kernel(double* __restrict__ Ag, int m, int n, int ldag,
                                                double* __restrict__ Qg, int ldqg,
                                                double* __restrict__ R, int ldr,
                                                double* __restrict__ tau, int use_lds) {
  __shared__ double red[WG / 64];
  extern __shared__ double sm[];
  const int k = min(m, n);
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wid = tid >> 6, nw = nt >> 6;
  // working copies: in LDS when they fit, else the caller's buffers
  double* A = Ag;
  double* Q = Qg;
  int lda = ldag, ldq = ldqg;
  if (use_lds) {
    A = sm;
    Q = sm + m * n;
    lda = n;
    ldq = k;
    for (int e = tid; e < m * n; e += nt) A[e] = Ag[(int64_t)(e / n) * ldag + e % n];
    __syncthreads();
  }
  for (int j = 0; j < k; ++j) {
    double v = 0.0;
    for (int i = j + 1 + tid; i < m; i += nt) {
      const double a = A[(int64_t)i * lda + j];
      v = fma(a, a, v);
    }
    const double nrm2 = block_sum(v, red);
    const double alpha = A[(int64_t)j * lda + j];
    double t = 0.0, beta = alpha, inv = 0.0;
    if (nrm2 > 0.0) {
      const double sigma = sqrt(alpha * alpha + nrm2);
      beta = alpha >= 0.0 ? -sigma : sigma;
      t = (beta - alpha) / beta;
      inv = 1.0 / (alpha - beta);
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < m; i += nt) A[(int64_t)i * lda + j] *= inv;
    if (tid == 0) {
      A[(int64_t)j * lda + j] = beta;
      tau[j] = t;
    }
    __syncthreads();
    if (t != 0.0) {
      for (int c = j + 1 + wid; c < n; c += nw) {
        double w = 0.0;
        for (int i = j + 1 + lane; i < m; i += 64)
          w = fma(A[(int64_t)i * lda + j], A[(int64_t)i * lda + c], w);
        w = wave_sum(w);
        const double ajc = A[(int64_t)j * lda + c];
        w = t * (w + ajc);
        for (int i = j + 1 + lane; i < m; i += 64) A[(int64_t)i * lda + c] -= w * A[(int64_t)i * lda + j];
        if (lane == 0) A[(int64_t)j * lda + c] = ajc - w;
      }
    }
    __syncthreads();
  }
  // Q = H_0 ... H_{k-1} [I_k; 0]
  for (int64_t e = tid; e < (int64_t)m * k; e += nt) {
    const int i = (int)(e / k), c = (int)(e % k);
    Q[(int64_t)i * ldq + c] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    const double t = tau[j];
    if (t != 0.0) {
      for (int c = j + wid; c < k; c += nw) {
        double w = 0.0;
        for (int i = j + 1 + lane; i < m; i += 64)
          w = fma(A[(int64_t)i * lda + j], Q[(int64_t)i * ldq + c], w);
        w = wave_sum(w);
        const double qjc = Q[(int64_t)j * ldq + c];
        w = t * (w + qjc);
        for (int i = j + 1 + lane; i < m; i += 64) Q[(int64_t)i * ldq + c] -= w * A[(int64_t)i * lda + j];
        if (lane == 0) Q[(int64_t)j * ldq + c] = qjc - w;
      }
    }
    __syncthreads();
  }
  // sign gauge: diag(R) >= 0
  for (int j = tid; j < k; j += nt) tau[j] = A[(int64_t)j * lda + j] < 0.0 ? -1.0 : 1.0;
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)k * n; e += nt) {
    const int i = (int)(e / n), c = (int)(e % n);
    R[(int64_t)i * ldr + c] = c >= i ? tau[i] * A[(int64_t)i * lda + c] : 0.0;
  }
  for (int64_t e = tid; e < (int64_t)m * k; e += nt) {
    const int i = (int)(e / k), c = (int)(e % k);
    Q[(int64_t)i * ldq + c] *= tau[c];
  }
  if (use_lds) {
    __syncthreads();
    for (int e = tid; e < m * k; e += nt) Qg[(int64_t)(e / k) * ldqg + e % k] = Q[e];
  }
}

__device__ __forceinline__ int rr_player(int pos, int round, int np) {
  return pos == 0 ? 0 : 1 + (pos - 1 + round) % (np - 1);
}

// One-sided Jacobi SVD.  work: Gt [n][m], Vt [n][n], sig [n], rank [n].
__global__ __launch_bounds__(WG) void svd_kernel(const double* __restrict__ G, int m, int n,
                                                 int ldg, double* __restrict__ U, int ldu,
                                                 double* __restrict__ S,
                                                 double* __restrict__ V, int ldv,
                                                 double* __restrict__ work, int use_lds) {
  __shared__ int s_rot;
  extern __shared__ double sm[];
  double* Gt = use_lds ? sm : work;
  double* Vt = Gt + (int64_t)n * m;
  double* sig = Vt + (int64_t)n * n;
  double* rk = sig + n;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wid = tid >> 6, nw = nt >> 6;
  for (int64_t e = tid; e < (int64_t)n * m; e += nt) {
    const int p = (int)(e / m), i = (int)(e % m);
    Gt[e] = G[(int64_t)i * ldg + p];
  }
  for (int64_t e = tid; e < (int64_t)n * n; e += nt) Vt[e] = (e / n == e % n) ? 1.0 : 0.0;
  const int np = n + (n & 1);
  const double eps = 1e-15;
  for (int sweep = 0; sweep < 60 && np > 1; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int round = 0; round < np - 1; ++round) {
      for (int pi = wid; pi < np / 2; pi += nw) {
        int p = rr_player(pi, round, np), q = rr_player(np - 1 - pi, round, np);
        if (p >= n || q >= n) continue;
        if (p > q) { const int tq = p; p = q; q = tq; }
        double* gp = Gt + (int64_t)p * m;
        double* gq = Gt + (int64_t)q * m;
        double a = 0.0, b = 0.0, g = 0.0;
        for (int i = lane; i < m; i += 64) {
          const double x = gp[i], y = gq[i];
          a = fma(x, x, a);
          b = fma(y, y, b);
          g = fma(x, y, g);
        }
        a = wave_sum(a);
        b = wave_sum(b);
        g = wave_sum(g);
        if (g != 0.0 && fabs(g) > eps * sqrt(a * b)) {
          const double zeta = (b - a) / (2.0 * g);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
          for (int i = lane; i < m; i += 64) {
            const double x = gp[i], y = gq[i];
            gp[i] = c * x - s * y;
            gq[i] = s * x + c * y;
          }
          double* vp = Vt + (int64_t)p * n;
          double* vq = Vt + (int64_t)q * n;
          for (int i = lane; i < n; i += 64) {
            const double x = vp[i], y = vq[i];
            vp[i] = c * x - s * y;
            vq[i] = s * x + c * y;
          }
          if (lane == 0) atomicAdd(&s_rot, 1);
        }
      }
      __syncthreads();
    }
    if (s_rot == 0) break;
    __syncthreads();
  }
  __syncthreads();
  for (int p = wid; p < n; p += nw) {
    double a = 0.0;
    for (int i = lane; i < m; i += 64) a = fma(Gt[(int64_t)p * m + i], Gt[(int64_t)p * m + i], a);
    a = wave_sum(a);
    if (lane == 0) sig[p] = sqrt(a);
  }
  __syncthreads();
  for (int p = tid; p < n; p += nt) {
    int r = 0;
    const double sp = sig[p];
    for (int q = 0; q < n; ++q) r += (sig[q] > sp) || (sig[q] == sp && q < p);
    rk[p] = (double)r;
  }
  __syncthreads();
  for (int p = wid; p < n; p += nw) {
    const int j = (int)rk[p];
    const double sp = sig[p];
    const double* gp = Gt + (int64_t)p * m;
    const double* vp = Vt + (int64_t)p * n;
    // gauge: largest-magnitude entry of the left vector positive (right vector if sp == 0)
    double best = -1.0, sgn = 1.0;
    if (sp > 0.0) {
      for (int i = lane; i < m; i += 64) {
        const double x = fabs(gp[i]);
        if (x > best) { best = x; sgn = gp[i] < 0.0 ? -1.0 : 1.0; }
      }
    } else {
      for (int i = lane; i < n; i += 64) {
        const double x = fabs(vp[i]);
        if (x > best) { best = x; sgn = vp[i] < 0.0 ? -1.0 : 1.0; }
      }
    }
    // wave argmax (first lane wins ties by max then lowest lane)
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const double os = __shfl_xor(sgn, o, 64);
      const int ol = lane ^ o;
      if (ob > best || (ob == best && ol < lane)) { best = ob; sgn = os; }
    }
    sgn = __shfl(sgn, 0, 64);
    const double inv = sp > 0.0 ? sgn / sp : 0.0;
    for (int i = lane; i < m; i += 64) U[(int64_t)i * ldu + j] = gp[i] * inv;
    for (int i = lane; i < n; i += 64) V[(int64_t)i * ldv + j] = vp[i] * sgn;
    if (lane == 0) S[j] = sp;
  }
}

__global__ void trunc_rank_kernel(const double* __restrict__ S, int n, double tol, double dm1,
                                  const double* normsq, int rmax, int* rank, double* discard) {
  if (threadIdx.x != 0) return;
  double tot = 0.0;
  for (int i = 0; i < n; ++i) tot += S[i] * S[i];
  const double ref = normsq ? *normsq : tot;
  const double delta2 = tol * tol * ref / dm1;
  double tail = 0.0;
  int r = n;
  while (r > 1) {
    const double t = tail + S[r - 1] * S[r - 1];
    if (t > delta2) break;
    tail = t;
    --r;
  }
  rank[1] = r > rmax ? 1 : 0;     // the cap decided the rank
  if (r > rmax) r = rmax;
  double disc = 0.0;
  for (int i = r; i < n; ++i) disc += S[i] * S[i];
  *rank = r;
  if (discard) *discard += disc;
}

// Dense LU with partial pivoting and solve, in place (A N x N, b length N).
__global__ __launch_bounds__(WG) void lu_solve_kernel(double* __restrict__ Ag, int N, int ldag,
                                                      double* __restrict__ bg, int use_lds) {
  extern __shared__ double sm[];
  Ag += (int64_t)blockIdx.x * N * ldag;
  bg += (int64_t)blockIdx.x * N;
  double* A = Ag;
  double* b = bg;
  int lda = ldag;
  if (use_lds) {
    A = sm;
    b = sm + N * N;
    lda = N;
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) A[e] = Ag[(int64_t)(e / N) * ldag + e % N];
    for (int e = threadIdx.x; e < N; e += blockDim.x) b[e] = bg[e];
    __syncthreads();
  }
  __shared__ double sval[WG / 64];
  __shared__ int sidx[WG / 64];
  __shared__ int s_piv;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wid = tid >> 6, nw = nt >> 6;
  for (int j = 0; j < N; ++j) {
    double best = -1.0;
    int bi = j;
    for (int i = j + tid; i < N; i += nt) {
      const double x = fabs(A[(int64_t)i * lda + j]);
      if (x > best) { best = x; bi = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) { sval[wid] = best; sidx[wid] = bi; }
    __syncthreads();
    if (tid == 0) {
      double bb = -1.0;
      int ii = j;
      for (int w = 0; w < nw; ++w)
        if (sval[w] > bb || (sval[w] == bb && sidx[w] < ii)) { bb = sval[w]; ii = sidx[w]; }
      s_piv = ii;
    }
    __syncthreads();
    const int p = s_piv;
    if (p != j) {
      for (int c = tid; c < N; c += nt) {
        const double t = A[(int64_t)j * lda + c];
        A[(int64_t)j * lda + c] = A[(int64_t)p * lda + c];
        A[(int64_t)p * lda + c] = t;
      }
      if (tid == 0) { const double t = b[j]; b[j] = b[p]; b[p] = t; }
    }
    __syncthreads();
    const double piv = A[(int64_t)j * lda + j];
    const double ipiv = piv != 0.0 ? 1.0 / piv : 0.0;
    for (int i = j + 1 + tid; i < N; i += nt) A[(int64_t)i * lda + j] *= ipiv;
    __syncthreads();
    const int rows = N - j - 1;
    const double bj = b[j];
    for (int i = j + 1 + wid; i < N; i += nw) {
      const double l = A[(int64_t)i * lda + j];
      if (l != 0.0) {
        for (int c = j + 1 + lane; c < N; c += 64) A[(int64_t)i * lda + c] -= l * A[(int64_t)j * lda + c];
        if (lane == 0) b[i] -= l * bj;
      }
    }
    (void)rows;
    __syncthreads();
  }
  for (int i = N - 1; i >= 0; --i) {
    if (tid == 0) {
      const double d = A[(int64_t)i * lda + i];
      b[i] = d != 0.0 ? b[i] / d : 0.0;
    }
    __syncthreads();
    const double xi = b[i];
    for (int r = tid; r < i; r += nt) b[r] -= A[(int64_t)r * lda + i] * xi;
    __syncthreads();
  }
  if (use_lds)
    for (int e = tid; e < N; e += nt) bg[e] = b[e];
}

}  // namespace

void qr(hipStream_t s, double* A, int m, int n, int lda, double* Q, int ldq, double* R, int ldr,
        double* tau) {
  if (m <= 0 || n <= 0) return;
  ++g_launches;
  const bool lds = (int64_t)m * n + (int64_t)m * std::min(m, n) <= kLdsDoubles;
  qr_kernel<<<1, WG, lds ? (size_t)((int64_t)m * n + (int64_t)m * std::min(m, n)) * 8 : 0, s>>>(
      A, m, n, lda, Q, ldq, R, ldr, tau, lds ? 1 : 0);
  TT_HIP(hipGetLastError());
}

size_t svd_work_doubles(int m, int n) { return (size_t)n * m + (size_t)n * n + 2 * (size_t)n; }

void svd(hipStream_t s, double* G, int m, int n, int ldg, double* U, int ldu, double* S,
         double* V, int ldv, double* work) {
  if (m <= 0 || n <= 0) return;
  TT_REQUIRE(m >= n, "svd expects m >= n");
  ++g_launches;
  const size_t need = svd_work_doubles(m, n);
  const bool lds = need <= (size_t)kLdsDoubles;
  svd_kernel<<<1, WG, lds ? need * 8 : 0, s>>>(G, m, n, ldg, U, ldu, S, V, ldv, work, lds ? 1 : 0);
  TT_HIP(hipGetLastError());
}

void trunc_rank(hipStream_t s, const double* S, int n, double tol, double dm1,
                const double* normsq, int rmax, int* rank, double* discard) {
  ++g_launches;
  trunc_rank_kernel<<<1, 64, 0, s>>>(S, n, tol, dm1, normsq, rmax, rank, discard);
  TT_HIP(hipGetLastError());
}

void lu_solve(hipStream_t s, double* A, int N, int lda, double* b, int batch) {
  if (N <= 0 || batch <= 0) return;
  ++g_launches;
  const bool lds = (int64_t)N * N + N <= kLdsDoubles;
  lu_solve_kernel<<<batch, WG, lds ? (size_t)((int64_t)N * N + N) * 8 : 0, s>>>(A, N, lda, b,
                                                                                 lds ? 1 : 0);
  TT_HIP(hipGetLastError());
}

}  // namespace ttnt
