// Small dense factorizations used by TT rounding and the alternating solve.
// Each runs in one workgroup of 1024 threads (16 wavefronts) on global memory
// (the matrices are small and stay in cache).
#include <algorithm>
#include <cmath>
#include <mutex>
#include <utility>

#include "kernels.h"

namespace ttnt {
namespace {

constexpr int WG = 1024;

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

// Sign gauge of a thin SVD's left factor: column j of U (m rows, row stride
// ldu) gets its largest-magnitude entry positive (the lowest row on ties), and
// column j of V (nv rows, row stride ldv) is flipped with it.  One workgroup
// of 256 threads per column.
__global__ __launch_bounds__(256) void col_gauge_kernel(double* __restrict__ U, int m, int ldu,
                                                        double* __restrict__ V, int nv, int ldv) {
  __shared__ double sb[4], ss[4];
  __shared__ int si[4];
  const int j = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double best = -1.0, sgn = 1.0;
  int bi = 0x7fffffff;
  for (int i = tid; i < m; i += 256) {
    const double x = U[(int64_t)i * ldu + j];
    if (fabs(x) > best) { best = fabs(x); sgn = x < 0.0 ? -1.0 : 1.0; bi = i; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const double os = __shfl_xor(sgn, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ob > best || (ob == best && oi < bi)) { best = ob; sgn = os; bi = oi; }
  }
  if (lane == 0) { sb[w] = best; ss[w] = sgn; si[w] = bi; }
  __syncthreads();
  double b = sb[0], g = ss[0];
  int ib = si[0];
  for (int q = 1; q < 4; ++q)
    if (sb[q] > b || (sb[q] == b && si[q] < ib)) { b = sb[q]; g = ss[q]; ib = si[q]; }
  if (g < 0.0) {
    for (int i = tid; i < m; i += 256) U[(int64_t)i * ldu + j] = -U[(int64_t)i * ldu + j];
    for (int e = tid; e < nv; e += 256) V[(int64_t)e * ldv + j] = -V[(int64_t)e * ldv + j];
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

// Odd leading dimension for LDS-resident matrices: lanes walking different
// rows (or columns) at the same index hit different banks.
__host__ __device__ __forceinline__ int odd_ld(int m) { return m | 1; }

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
    lda = odd_ld(N);
    A = sm;
    b = sm + N * lda;
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) A[(e / N) * lda + e % N] = Ag[(int64_t)(e / N) * ldag + e % N];
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

// Blocked right-looking LU with partial pivoting and solve, for systems whose
// matrix stays in global memory.  Per panel of kLuNB columns: the panel
// (rows k0..N-1) is factored in LDS, its row interchanges are applied to the
// columns on its right and to b, the block row of U is formed by forward
// substitution with the panel's unit lower triangle, and the trailing matrix
// takes one rank-kLuNB update, so it is read and written once per panel
// instead of once per column.  b is eliminated along, and the back
// substitution runs by blocks of kLuNB rows (row-wise, coalesced dot
// products, then the block's triangle).  The pivot rule (largest magnitude,
// lowest row on ties) and the zero-pivot convention are those of
// lu_solve_kernel.
constexpr int kLuNB = 16, kLuP = kLuNB + 1, kLuUC = 64;

size_t lu_blocked_lds_doubles(int N) {
  return (size_t)N * kLuP + (size_t)kLuNB * kLuUC + (size_t)N + 8;
}

__global__ __launch_bounds__(WG) void lu_blocked_kernel(double* __restrict__ Ag, int N, int lda,
                                                        double* __restrict__ bg) {
  extern __shared__ double sm[];
  double* A = Ag + (int64_t)blockIdx.x * N * lda;
  double* bo = bg + (int64_t)blockIdx.x * N;
  double* Pr = sm;                            // panel: rows k0..N-1, kLuNB columns, pitch kLuP
  double* Us = Pr + (size_t)N * kLuP;         // kLuNB x kLuUC chunk of the U block row
  double* xs = Us + kLuNB * kLuUC;            // b, eliminated along; then x
  __shared__ double sval[WG / 64];
  __shared__ int sidx[WG / 64];
  __shared__ int piv[kLuNB];
  constexpr int NW = WG / 64;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int e = tid; e < N; e += WG) xs[e] = bo[e];
  for (int k0 = 0; k0 < N; k0 += kLuNB) {
    const int nb = min(kLuNB, N - k0), R = N - k0, C0 = k0 + nb;
    __syncthreads();
    for (int e = tid; e < R * nb; e += WG) {
      const int r = e / nb, c = e - r * nb;
      Pr[r * kLuP + c] = A[(int64_t)(k0 + r) * lda + k0 + c];
    }
    __syncthreads();
    // factor the panel (rows relative to k0)
    for (int j = 0; j < nb; ++j) {
      double best = -1.0;
      int bi = j;
      for (int i = j + tid; i < R; i += WG) {
        const double x = fabs(Pr[i * kLuP + j]);
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
        for (int w = 0; w < NW; ++w)
          if (sval[w] > bb || (sval[w] == bb && sidx[w] < ii)) { bb = sval[w]; ii = sidx[w]; }
        piv[j] = ii;
      }
      __syncthreads();
      const int p = piv[j];
      if (p != j && tid < nb) {
        const double t = Pr[j * kLuP + tid];
        Pr[j * kLuP + tid] = Pr[p * kLuP + tid];
        Pr[p * kLuP + tid] = t;
      }
      __syncthreads();
      const double d = Pr[j * kLuP + j];
      const double id = d != 0.0 ? 1.0 / d : 0.0;
      for (int i = j + 1 + tid; i < R; i += WG) {
        const double l = Pr[i * kLuP + j] * id;
        Pr[i * kLuP + j] = l;
        for (int c = j + 1; c < nb; ++c) Pr[i * kLuP + c] -= l * Pr[j * kLuP + c];
      }
      __syncthreads();
    }
    for (int e = tid; e < R * nb; e += WG) {
      const int r = e / nb, c = e - r * nb;
      A[(int64_t)(k0 + r) * lda + k0 + c] = Pr[r * kLuP + c];
    }
    // interchanges on the columns right of the panel (each thread its own
    // columns, in pivot order), then the block row of U by forward
    // substitution with the unit lower triangle of the panel
    for (int c = C0 + tid; c < N; c += WG) {
      double u[kLuNB];
#pragma unroll
      for (int t = 0; t < kLuNB; ++t) u[t] = 0.0;
      for (int j = 0; j < nb; ++j) {
        const int p = piv[j];
        if (p != j) {
          const double t = A[(int64_t)(k0 + j) * lda + c];
          A[(int64_t)(k0 + j) * lda + c] = A[(int64_t)(k0 + p) * lda + c];
          A[(int64_t)(k0 + p) * lda + c] = t;
        }
      }
#pragma unroll
      for (int t = 0; t < kLuNB; ++t)
        if (t < nb) u[t] = A[(int64_t)(k0 + t) * lda + c];
#pragma unroll
      for (int t = 1; t < kLuNB; ++t)
#pragma unroll
        for (int q = 0; q < t; ++q)
          if (t < nb) u[t] -= Pr[t * kLuP + q] * u[q];
#pragma unroll
      for (int t = 1; t < kLuNB; ++t)
        if (t < nb) A[(int64_t)(k0 + t) * lda + c] = u[t];
    }
    if (tid == 0) {
      for (int j = 0; j < nb; ++j) {
        const int p = piv[j];
        if (p != j) {
          const double t = xs[k0 + j];
          xs[k0 + j] = xs[k0 + p];
          xs[k0 + p] = t;
        }
      }
      for (int t = 1; t < nb; ++t) {
        double v = xs[k0 + t];
        for (int q = 0; q < t; ++q) v -= Pr[t * kLuP + q] * xs[k0 + q];
        xs[k0 + t] = v;
      }
    }
    __syncthreads();
    // trailing update A22 -= L21 U12 by chunks of kLuUC columns: lane = column,
    // wavefront = every NW-th row, four rows in flight per wavefront
    for (int cc = C0; cc < N; cc += kLuUC) {
      const int cw = min(kLuUC, N - cc);
      for (int e = tid; e < kLuNB * kLuUC; e += WG) {
        const int t = e / kLuUC, cl = e - t * kLuUC;
        Us[e] = (t < nb && cl < cw) ? A[(int64_t)(k0 + t) * lda + cc + cl] : 0.0;
      }
      __syncthreads();
      if (lane < cw) {
        double uv[kLuNB];
#pragma unroll
        for (int t = 0; t < kLuNB; ++t) uv[t] = Us[t * kLuUC + lane];
        double* col = A + cc + lane;
        int r = nb + wid;
        for (; r + 3 * NW < R; r += 4 * NW) {
          double v[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) v[q] = col[(int64_t)(k0 + r + q * NW) * lda];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double* lr = Pr + (r + q * NW) * kLuP;
#pragma unroll
            for (int t = 0; t < kLuNB; ++t) v[q] -= lr[t] * uv[t];
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) col[(int64_t)(k0 + r + q * NW) * lda] = v[q];
        }
        for (; r < R; r += NW) {
          const double* lr = Pr + r * kLuP;
          double v = col[(int64_t)(k0 + r) * lda];
#pragma unroll
          for (int t = 0; t < kLuNB; ++t) v -= lr[t] * uv[t];
          col[(int64_t)(k0 + r) * lda] = v;
        }
      }
      __syncthreads();
    }
    // the same update of b (uv of columns beyond nb are zero above; here the
    // panel's unused columns are never read)
    for (int r = nb + tid; r < R; r += WG) {
      const double* lr = Pr + r * kLuP;
      double v = xs[k0 + r];
      for (int t = 0; t < nb; ++t) v -= lr[t] * xs[k0 + t];
      xs[k0 + r] = v;
    }
  }
  __syncthreads();
  // back substitution by blocks of kLuNB rows, from the bottom
  for (int i0 = ((N - 1) / kLuNB) * kLuNB; i0 >= 0; i0 -= kLuNB) {
    const int nb = min(kLuNB, N - i0), c1 = i0 + nb;
    for (int ii = wid; ii < nb; ii += NW) {
      const int i = i0 + ii;
      const double* row = A + (int64_t)i * lda;
      double acc = 0.0;
      for (int c = c1 + lane; c < N; c += 64) acc = fma(row[c], xs[c], acc);
      acc = wave_sum(acc);
      if (lane == 0) xs[i] -= acc;
    }
    __syncthreads();
    if (tid == 0) {
      for (int ii = nb - 1; ii >= 0; --ii) {
        const int i = i0 + ii;
        const double* row = A + (int64_t)i * lda;
        double v = xs[i];
        for (int c = i + 1; c < c1; ++c) v -= row[c] * xs[c];
        const double d = row[i];
        xs[i] = d != 0.0 ? v / d : 0.0;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < N; e += WG) bo[e] = xs[e];
}

// ---------------------------------------------------------------------------
// LDS-resident factorizations, one workgroup of 256 threads (4 wavefronts).
// Matrices are held column-major with an odd leading dimension so that lanes
// walking different columns at the same row hit different banks.
// ---------------------------------------------------------------------------
constexpr int WS = 256;

// One DPP lane exchange of a double (two 32-bit moves).
template <int Ctrl>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int l2 = __builtin_amdgcn_update_dpp(0, lo, Ctrl, 0xF, 0xF, false);
  const int h2 = __builtin_amdgcn_update_dpp(0, hi, Ctrl, 0xF, 0xF, false);
  return __hiloint2double(h2, l2);
}

// 1/x and 1/sqrt(x) from the hardware approximations refined by two Newton
// steps each (x finite, nonzero; x > 0 for the square root), accurate to the
// last bits for the rotation parameters of the Jacobi sweeps.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  double e = fma(-h * y, y, 0.5);
  y = fma(y, e, y);
  e = fma(-h * y, y, 0.5);
  return fma(y, e, y);
}

// Sum over the 64 lanes of a wavefront, returned to every lane: four DPP
// exchanges within each row of 16 lanes, two row broadcasts that gather the
// row sums into the last row (row_mask picks the rows that add), and a read
// of lane 63.  About a third of the latency of six cross-lane shuffles.
template <int Ctrl, int RowMask>
__device__ __forceinline__ double dpp_bcast(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), Ctrl, RowMask, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), Ctrl, RowMask, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_move<0xB1>(v);              // quad_perm [1, 0, 3, 2]
  v += dpp_move<0x4E>(v);              // quad_perm [2, 3, 0, 1]
  v += dpp_move<0x141>(v);             // row_half_mirror
  v += dpp_move<0x140>(v);             // row_mirror
  v += dpp_bcast<0x142, 0xA>(v);       // row_bcast:15 into rows 1 and 3
  v += dpp_bcast<0x143, 0xC>(v);       // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// sum_{r in [r0, r1)} x[r] y[r] + init, LDS operands loaded eight at a time.
__device__ __forceinline__ double seg_dot(const double* x, const double* y, int r0, int r1,
                                          double init) {
  double p[4] = {init, 0.0, 0.0, 0.0};
  int r = r0;
  for (; r + 8 <= r1; r += 8) {
    double a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[u] = x[r + u];
      b[u] = y[r + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) p[u & 3] = fma(a[u], b[u], p[u & 3]);
  }
  for (; r < r1; ++r) p[0] = fma(x[r], y[r], p[0]);
  return (p[0] + p[1]) + (p[2] + p[3]);
}

// y[r] += alpha x[r] for r in [r0, r1), eight rows at a time.
__device__ __forceinline__ void seg_axpy(double alpha, const double* x, double* y, int r0,
                                         int r1) {
  int r = r0;
  for (; r + 8 <= r1; r += 8) {
    double a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[u] = x[r + u];
      b[u] = y[r + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) y[r + u] = fma(alpha, a[u], b[u]);
  }
  for (; r < r1; ++r) y[r] = fma(alpha, x[r], y[r]);
}

// Rows of the four wavefronts: wavefront w owns the fixed block
// [w B, (w + 1) B), B = ceil(m / 4), of every column for the whole
// factorization, so a wavefront only ever reads rows it wrote itself and the
// workgroup barriers are needed only where partial sums cross wavefronts.
// Step j works on the rows below j: [max(j + 1, w B), min(m, (w + 1) B)).
__device__ __forceinline__ void row_block(int j, int m, int w, int& r0, int& r1) {
  const int B = (m + 3) / 4;
  r0 = max(j + 1, w * B);
  r1 = min(m, (w + 1) * B);
}

// Householder QR of the column-major m x n matrix A (leading dimension ld):
// the upper triangle receives R, the part below the diagonal the reflector
// vectors (unit leading entry implicit), tau[j] the factors of
// H_j = I - tau_j v_j v_j^T.  pw is LDS scratch of 8 (n + 1) + 4 doubles: the
// norm partials, and the column-dot partials in two halves used on
// alternate steps.  Two workgroup barriers per column.
__device__ void hh_qr(double* A, int m, int n, int ld, double* tau, double* pw) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int k = min(m, n), B = (m + 3) / 4;
  double* pn = pw + 8 * (n + 1);
  for (int j = 0; j < k; ++j) {
    double* aj = A + (int64_t)j * ld;
    double* pd = pw + (j & 1) * 4 * (n + 1);
    const bool diag = j >= w * B && j < (w + 1) * B;    // this wavefront holds row j
    int r0, r1;
    row_block(j, m, w, r0, r1);
    double s = 0.0;
    for (int r = r0 + lane; r < r1; r += 64) s = fma(aj[r], aj[r], s);
    s = wave_sum_dpp(s);
    if (lane == 0) pn[w] = s;
    __syncthreads();
    const double nrm2 = (pn[0] + pn[1]) + (pn[2] + pn[3]);
    const double alpha = aj[j];
    double t = 0.0, beta = alpha, inv = 0.0;
    if (nrm2 > 0.0) {
      // sigma = sqrt(alpha^2 + |x|^2) and the two quotients from the hardware
      // reciprocal square root and reciprocal, each refined by Newton steps
      const double s2 = fma(alpha, alpha, nrm2);
      const double sigma = s2 * rsq_nr(s2);
      beta = alpha >= 0.0 ? -sigma : sigma;
      t = (beta - alpha) * rcp_nr(beta);
      inv = rcp_nr(alpha - beta);
    }
    for (int r = r0 + lane; r < r1; r += 64) aj[r] *= inv;
    // partial w_c over this wavefront's rows (the implicit 1 of v_j meets row j)
    for (int c = j + 1 + lane; c < n; c += 64) {
      const double* ac = A + (int64_t)c * ld;
      pd[w * (n + 1) + c] = seg_dot(aj, ac, r0, r1, diag ? ac[j] : 0.0);
    }
    __syncthreads();
    if (t != 0.0) {
      for (int c = j + 1 + lane; c < n; c += 64) {
        double* ac = A + (int64_t)c * ld;
        const double wc = t * ((pd[c] + pd[(n + 1) + c]) +
                               (pd[2 * (n + 1) + c] + pd[3 * (n + 1) + c]));
        seg_axpy(-wc, aj, ac, r0, r1);
        if (diag) ac[j] -= wc;
      }
    }
    if (diag && lane == 0) {
      aj[j] = beta;
      tau[j] = t;
    }
  }
  __syncthreads();
}

// Q = H_0 ... H_{k-1} [I; 0] in place of the reflectors (columns 0..k-1),
// backwards, one workgroup barrier per column.  Rows above the diagonal of
// column c are only written by the later steps j < c (as -w_c); they are
// never read before, so they need no zeroing.  pw as in hh_qr.
__device__ void hh_form_q(double* A, int m, int n, int ld, const double* tau, double* pw) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int k = min(m, n), B = (m + 3) / 4;
  for (int j = k - 1; j >= 0; --j) {
    double* aj = A + (int64_t)j * ld;
    double* pd = pw + (j & 1) * 4 * (n + 1);
    const double t = tau[j];
    const bool diag = j >= w * B && j < (w + 1) * B;
    int r0, r1;
    row_block(j, m, w, r0, r1);
    // row j of the columns c > j is still zero here: only rows below j count
    for (int c = j + 1 + lane; c < k; c += 64) {
      const double* ac = A + (int64_t)c * ld;
      pd[w * (n + 1) + c] = seg_dot(aj, ac, r0, r1, 0.0);
    }
    __syncthreads();
    for (int c = j + 1 + lane; c < k; c += 64) {
      double* ac = A + (int64_t)c * ld;
      const double wc = t != 0.0 ? t * ((pd[c] + pd[(n + 1) + c]) +
                                        (pd[2 * (n + 1) + c] + pd[3 * (n + 1) + c]))
                                 : 0.0;
      if (wc != 0.0) seg_axpy(-wc, aj, ac, r0, r1);
      if (diag) ac[j] = -wc;
    }
    // column j of Q: (1 - t) e_j - t v_j
    for (int r = r0 + lane; r < r1; r += 64) aj[r] *= -t;
    if (diag && lane == 0) aj[j] = 1.0 - t;
  }
  __syncthreads();
}

// QR with diag(R) >= 0: Q (m x k), R (k x n), k = min(m, n); A row-major.
// Element (i, c) of the input is Ag[i ars + c acs] and element (i, c) of Q
// is written to Qg[i qrs + c qcs], so a transposed operand or result needs no
// separate transpose (the input is fully read into LDS before Q is written,
// so Qg may overlap Ag).  Workgroup b factors rows [b mb, min(m, (b + 1) mb))
// on its own, its R at R + b rbs (one workgroup: mb = m).
__global__ __launch_bounds__(WS) void qr_lds_kernel(const double* Ag, int m, int n, int64_t ars,
                                                    int64_t acs, double* Qg, int64_t qrs,
                                                    int64_t qcs, double* __restrict__ R, int ldr,
                                                    int mb, int64_t rbs) {
  extern __shared__ double sm[];
  {
    const int64_t r0 = (int64_t)blockIdx.x * mb;
    Ag += r0 * ars;
    Qg += r0 * qrs;
    R += blockIdx.x * rbs;
    m = min(mb, m - (int)r0);
  }
  const int ld = odd_ld(m), k = min(m, n), tid = threadIdx.x;
  double* A = sm;
  double* tau = A + (int64_t)ld * n;
  double* sg = tau + k;
  double* pw = sg + k;
  const bool rfast = ars == 1;   // walk the index whose stride is 1 fastest
  for (int e = tid; e < m * n; e += WS) {
    const int i = rfast ? e % m : e / n, c = rfast ? e / m : e % n;
    A[(int64_t)c * ld + i] = Ag[(int64_t)i * ars + (int64_t)c * acs];
  }
  __syncthreads();
  hh_qr(A, m, n, ld, tau, pw);
  for (int i = tid; i < k; i += WS) sg[i] = A[(int64_t)i * ld + i] < 0.0 ? -1.0 : 1.0;
  __syncthreads();
  for (int e = tid; e < k * n; e += WS) {
    const int i = e / n, c = e % n;
    R[(int64_t)i * ldr + c] = c >= i ? sg[i] * A[(int64_t)c * ld + i] : 0.0;
  }
  __syncthreads();
  hh_form_q(A, m, n, ld, tau, pw);
  const bool qfast = qrs == 1;
  for (int e = tid; e < m * k; e += WS) {
    const int i = qfast ? e % m : e / k, c = qfast ? e / m : e % k;
    Qg[(int64_t)i * qrs + (int64_t)c * qcs] = sg[c] * A[(int64_t)c * ld + i];
  }
}


// ---------------------------------------------------------------------------
// Register-resident Gauss-Jordan solve for systems up to a few hundred
// unknowns (the n blocks of a mode-diagonal core, small dense local systems).
// ---------------------------------------------------------------------------

// Pivot candidates are compared as (|x| bits, key): for non-negative doubles
// the IEEE bit patterns order like the values, and key = 2 row + sign breaks
// ties toward the lower row.  kGjNone (no candidate) loses to every row.
constexpr int kGjNone = 0x7fffffff;

__device__ __forceinline__ bool gj_better(uint64_t ob, int ok, uint64_t b, int k) {
  return (ob > b) | ((ob == b) & (ok < k));
}

template <int CTRL>
__device__ __forceinline__ void gj_combine(uint64_t& bits, int& key) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)bits, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(bits >> 32), CTRL, 0xF, 0xF, false);
  const int ok = __builtin_amdgcn_update_dpp(0, key, CTRL, 0xF, 0xF, false);
  const uint64_t ob = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
  const bool t = gj_better(ob, ok, bits, key);
  bits = t ? ob : bits;
  key = t ? ok : key;
}

// Pivot search of one column by its sixteen owners, which form one DPP row
// of a wavefront: the largest magnitude among rows not yet pivotal, the lowest
// row on ties.  Writes the step's multipliers (zero for the pivot row), its
// pivot row and its pivot value.
template <int R>
__device__ __forceinline__ void gj_pivot(const double (&col)[R], unsigned used, int ti, int j,
                                         double* __restrict__ mult, int* __restrict__ sp,
                                         double* __restrict__ pval, int* __restrict__ prow) {
  uint64_t bits = 0;
  int key = kGjNone;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const uint64_t xb = (uint64_t)__double_as_longlong(col[u]) & 0x7fffffffffffffffull;
    const int xk = 2 * (ti + 16 * u) + (col[u] < 0.0 ? 1 : 0);
    const bool t = !((used >> u) & 1u) & gj_better(xb, xk, bits, key);
    bits = t ? xb : bits;
    key = t ? xk : key;
  }
  gj_combine<0xB1>(bits, key);   // quad_perm [1,0,3,2]
  gj_combine<0x4E>(bits, key);   // quad_perm [2,3,0,1]
  gj_combine<0x141>(bits, key);  // row_half_mirror
  gj_combine<0x140>(bits, key);  // row_mirror
  const int p = key >> 1;
  const double mag = __longlong_as_double((long long)bits);
  const double piv = (key & 1) ? -mag : mag;
  const double ip = piv != 0.0 ? rcp_nr(piv) : 0.0;
#pragma unroll
  for (int u = 0; u < R; ++u) mult[ti + 16 * u] = ti + 16 * u == p ? 0.0 : col[u] * ip;
  if (ti == 0) {
    *sp = p;
    pval[j] = piv;
    prow[j] = p;
  }
}

// Gauss-Jordan elimination with partial pivoting of the augmented matrix
// [A | b], one workgroup of 16 TC threads per system.  Thread (tc, ti) =
// (tid / 16, tid % 16) holds rows i = ti + 16 u (u < R) and columns
// c = tc + TC v of [A | b], b being column N: the column blocks v < C in
// registers and the next CE blocks in LDS (each thread's own slots, laid out
// so that a wavefront's accesses are consecutive).  N <= 16 R and
// N + 1 <= TC (C + CE).  Rows are not exchanged: column j is eliminated from
// every row but its pivot row p_j, so after N steps x_j = b'(p_j) / a(p_j, j).
// A zero pivot leaves x_j = 0, as the LU kernel does.
//
// One workgroup barrier per column: the column's sixteen owners (one DPP row)
// find the pivot and publish it with the multipliers; every thread then takes
// the pivot row's entries of its own columns from lane p % 16 of its own
// sixteen-lane group (a cross-lane read, no LDS round trip) and applies the
// rank-one update to its block.  The multipliers and the pivot index are
// double-buffered by step parity, so the next owners can write while slower
// wavefronts still read.
template <int R, int C, int TC, int CE = 0>
__global__ __launch_bounds__(16 * TC) void gj_solve_kernel(const double* __restrict__ Ag, int N,
                                                           int ldag, double* __restrict__ bg) {
  constexpr int NT = 16 * TC;
  __shared__ double mult[2][16 * R];
  __shared__ double pval[16 * R], bfin[16 * R];
  __shared__ int prow[16 * R];
  __shared__ int sp[2];
  extern __shared__ __attribute__((aligned(16))) double gj_lds[];  // CE R NT doubles
  const int tid = threadIdx.x, ti = tid & 15, tc = tid >> 4, gbase = tid & 48;
  Ag += (int64_t)blockIdx.x * N * ldag;
  bg += (int64_t)blockIdx.x * N;
  auto ext = [&](int ve, int u) -> double& { return gj_lds[(ve * R + u) * NT + tid]; };
  auto entry = [&](int i, int c) {
    return i < N ? (c < N ? Ag[(int64_t)i * ldag + c] : (c == N ? bg[i] : 0.0)) : 0.0;
  };
  double a[R][C];
  unsigned used = 0;  // bit u: row ti + 16 u is a pivot row already, or padding
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int i = ti + 16 * u;
    if (i >= N) used |= 1u << u;
#pragma unroll
    for (int v = 0; v < C; ++v) a[u][v] = entry(i, tc + TC * v);
#pragma unroll
    for (int ve = 0; ve < CE; ++ve) ext(ve, u) = entry(i, tc + TC * (C + ve));
  }
  // Column blocks v0 = 0 .. C+CE-1 are expanded at compile time, so the pivot
  // column's registers have fixed indices; the TC columns of a block run as a
  // loop.
  auto block = [&](auto v0_c) {
    constexpr int v0 = decltype(v0_c)::value;
    for (int jc = 0; jc < TC; ++jc) {
      const int j = TC * v0 + jc;
      if (j >= N) return;
      const int par = j & 1;
      if (tc == jc) {
        double col[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
          if constexpr (v0 < C) col[u] = a[u][v0];
          else col[u] = ext(v0 - C, u);
        }
        gj_pivot<R>(col, used, ti, j, mult[par], &sp[par], pval, prow);
      }
      __syncthreads();
      const int p = __builtin_amdgcn_readfirstlane(sp[par]);
      if (ti == (p & 15)) used |= 1u << (p >> 4);
      double l[R];
#pragma unroll
      for (int u = 0; u < R; ++u) l[u] = mult[par][ti + 16 * u];
      // the pivot row's entries of this thread's columns sit with lane p % 16
      // of its group; one uniform branch per row block keeps register indices
      // fixed
      double rw[C] = {}, rwe[CE > 0 ? CE : 1] = {};
      const int src = gbase | (p & 15), up = p >> 4;
      [&]<int... Us>(std::integer_sequence<int, Us...>) {
        (
            [&] {
              if (up == Us) {
#pragma unroll
                for (int v = 0; v < C; ++v) rw[v] = __shfl(a[Us][v], src, 64);
#pragma unroll
                for (int ve = 0; ve < CE; ++ve) rwe[ve] = __shfl(ext(ve, Us), src, 64);
              }
            }(),
            ...);
      }(std::make_integer_sequence<int, R>{});
#pragma unroll
      for (int u = 0; u < R; ++u) {
#pragma unroll
        for (int v = 0; v < C; ++v) a[u][v] = fma(-l[u], rw[v], a[u][v]);
#pragma unroll
        for (int ve = 0; ve < CE; ++ve) ext(ve, u) = fma(-l[u], rwe[ve], ext(ve, u));
      }
      if (tc == jc) {
        // the eliminated column is exactly zero outside the pivot row
#pragma unroll
        for (int u = 0; u < R; ++u)
          if (ti + 16 * u != p) {
            if constexpr (v0 < C) a[u][v0] = 0.0;
            else ext(v0 - C, u) = 0.0;
          }
      }
    }
  };
  [&]<int... Vs>(std::integer_sequence<int, Vs...>) {
    (block(std::integral_constant<int, Vs>{}), ...);
  }(std::make_integer_sequence<int, C + CE>{});
  const int vb = N / TC, tb = N % TC;
  if (tc == tb) {
#pragma unroll
    for (int v = 0; v < C; ++v)
      if (v == vb)
#pragma unroll
        for (int u = 0; u < R; ++u) bfin[ti + 16 * u] = a[u][v];
#pragma unroll
    for (int ve = 0; ve < CE; ++ve)
      if (C + ve == vb)
#pragma unroll
        for (int u = 0; u < R; ++u) bfin[ti + 16 * u] = ext(ve, u);
  }
  __syncthreads();
  for (int j = tid; j < N; j += NT) {
    const double d = pval[j];
    bg[j] = d != 0.0 ? bfin[prow[j]] / d : 0.0;
  }
}

// The Gauss-Jordan instantiation with two of its eight column blocks in LDS
// (systems of 193 to 240 unknowns) and its dynamic LDS bytes.
constexpr int kGjExtR = 15, kGjExtC = 6, kGjExtTC = 32, kGjExtCE = 2;
constexpr size_t kGjExtLds = (size_t)kGjExtCE * kGjExtR * 16 * kGjExtTC * sizeof(double);

// Sum over aligned groups of LP lanes.  Every exchange pairs lanes by an
// involution (xor 1, xor 2, mirror within 8, mirror within 16, then xor 16
// and xor 32), so all lanes of a group hold the bit-identical sum.
template <int LP>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (LP >= 2) v += dpp_move<0xB1>(v);     // quad_perm [1, 0, 3, 2]
  if constexpr (LP >= 4) v += dpp_move<0x4E>(v);     // quad_perm [2, 3, 0, 1]
  if constexpr (LP >= 8) v += dpp_move<0x141>(v);    // row_half_mirror
  if constexpr (LP >= 16) v += dpp_move<0x140>(v);   // row_mirror
  if constexpr (LP >= 32) v += __shfl_xor(v, 16, 64);
  if constexpr (LP >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// Thin SVD G = U S V^T (m >= n), G row-major.  Householder QR G = Q R, then
// one-sided Jacobi on R^T: R^T W = Y with orthogonal columns, so that
// U = Q W and V = Y diag(1 / |Y_j|).  Singular values sorted descending;
// each column of U has its largest-magnitude entry positive.  LP lanes serve
// one Jacobi pair (the largest power of two with LP (n + 1) / 2 <= 256).
// Element (i, c) of G is Gg[i grs + c gcs]; U(i, j) goes to U[i urs + j ucs]
// and V(e, j) to V[e vrs + j vcs], so transposed operands and results need no
// separate transposes.
template <int LP>
__global__ __launch_bounds__(WS) void svd_lds_kernel(const double* __restrict__ Gg, int m, int n,
                                                     int64_t grs, int64_t gcs,
                                                     double* __restrict__ U, int64_t urs,
                                                     int64_t ucs, double* __restrict__ S,
                                                     double* __restrict__ V, int64_t vrs,
                                                     int64_t vcs) {
  extern __shared__ double sm[];
  __shared__ int s_rot, s_big;
  __shared__ double s_fro;
  const int ld = odd_ld(m), ldn = odd_ld(n), tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double* A = sm;                               // ld x n
  double* Y = A + (int64_t)ld * n;              // ldn x n
  double* Wm = Y + (int64_t)ldn * n;            // ldn x n
  double* tau = Wm + (int64_t)ldn * n;          // n
  double* sig = tau + n;                        // n
  double* rk = sig + n;                         // n
  double* pw = rk + n;                          // 8 (n + 1) + 4
  const bool rfast = grs == 1;
  for (int e = tid; e < m * n; e += WS) {
    const int i = rfast ? e % m : e / n, c = rfast ? e / m : e % n;
    A[(int64_t)c * ld + i] = Gg[(int64_t)i * grs + (int64_t)c * gcs];
  }
  __syncthreads();
  hh_qr(A, m, n, ld, tau, pw);
  // Y = R^T (column c of Y is row c of R), W = I
  for (int e = tid; e < n * n; e += WS) {
    const int c = e / n, r = e % n;
    Y[(int64_t)c * ldn + r] = c <= r ? A[(int64_t)r * ld + c] : 0.0;
    Wm[(int64_t)c * ldn + r] = c == r ? 1.0 : 0.0;
  }
  __syncthreads();
  hh_form_q(A, m, n, ld, tau, pw);
  // Frobenius norm of R: columns whose norm is below eps * ||G||_F are zero
  if (w == 0) {
    double f = 0.0;
    for (int e = lane; e < n * n; e += 64) {
      const double x = Y[(int64_t)(e / n) * ldn + e % n];
      f = fma(x, x, f);
    }
    f = wave_sum(f);
    if (lane == 0) s_fro = f;
  }
  __syncthreads();
  const double sfmin = s_fro * (2.3e-16 * 2.3e-16);
  const double tol = 1e-15;
  const int np = n + (n & 1), npair = np / 2;
  constexpr int Lp = LP;
  const int g = tid / Lp, l = tid % Lp;
  for (int sweep = 0; sweep < 60 && np > 1; ++sweep) {
    if (tid == 0) {
      s_rot = 0;
      s_big = 0;
    }
    __syncthreads();
    // Round-robin tournament: position 0 holds player 0 and position k > 0
    // holds player 1 + (k - 1 + round) mod (np - 1).  This group plays
    // positions g and np - 1 - g; both offsets advance by one per round.
    int cp = g - 1, cq = np - 2 - g;
    for (int round = 0; round < np - 1; ++round) {
      int p = 0, q = 0;
      bool valid = false;
      if (g < npair) {
        p = g == 0 ? 0 : 1 + cp;
        q = 1 + cq;
        if (p > q) { const int tq = p; p = q; q = tq; }
        valid = q < n;
      }
      cp = cp + 1 == np - 1 ? 0 : cp + 1;
      cq = cq + 1 == np - 1 ? 0 : cq + 1;
      double a = 0.0, b = 0.0, gg = 0.0;
      double* yp = Y + (int64_t)p * ldn;
      double* yq = Y + (int64_t)q * ldn;
      if (valid) {
        // four of the lane's entries loaded ahead of their products (the
        // sums keep their order)
        int e = l;
        for (; e + 3 * Lp < n; e += 4 * Lp) {
          double x[4], y[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            x[u] = yp[e + u * Lp];
            y[u] = yq[e + u * Lp];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            a = fma(x[u], x[u], a);
            b = fma(y[u], y[u], b);
            gg = fma(x[u], y[u], gg);
          }
        }
        for (; e < n; e += Lp) {
          const double x = yp[e], y = yq[e];
          a = fma(x, x, a);
          b = fma(y, y, b);
          gg = fma(x, y, gg);
        }
      }
      a = group_sum<LP>(a);
      b = group_sum<LP>(b);
      gg = group_sum<LP>(gg);
      // |g| > tol sqrt(a b) tested as g (g / a) > tol^2 b (no overflow: g^2 <= a b);
      // the conditions are combined without short-circuit branches
      const bool ok = valid & (a > sfmin) & (b > sfmin) & (gg != 0.0);
      const double ga = ok ? gg * rcp_nr(a) : 0.0;
      if (ok & (ga * gg > tol * tol * b)) {
        // a rotation above 1e-10 (relative) keeps the sweeps going
        if (l == 0 && ga * gg > 1e-20 * b) s_big = 1;
        const double zeta = (b - a) * 0.5 * rcp_nr(gg);
        const double az = fabs(zeta);
        double t;
        if (az > 1e150) {
          t = 0.5 * rcp_nr(zeta);
        } else {
          const double z2 = fma(zeta, zeta, 1.0);
          t = (zeta >= 0.0 ? 1.0 : -1.0) * rcp_nr(az + z2 * rsq_nr(z2));
        }
        const double c = rsq_nr(fma(t, t, 1.0)), sn = c * t;
        double* wp = Wm + (int64_t)p * ldn;
        double* wq = Wm + (int64_t)q * ldn;
        int e = l;
        for (; e + 3 * Lp < n; e += 4 * Lp) {
          double x[4], y[4], u4[4], v4[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            x[u] = yp[e + u * Lp];
            y[u] = yq[e + u * Lp];
            u4[u] = wp[e + u * Lp];
            v4[u] = wq[e + u * Lp];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            yp[e + u * Lp] = c * x[u] - sn * y[u];
            yq[e + u * Lp] = sn * x[u] + c * y[u];
            wp[e + u * Lp] = c * u4[u] - sn * v4[u];
            wq[e + u * Lp] = sn * u4[u] + c * v4[u];
          }
        }
        for (; e < n; e += Lp) {
          const double x = yp[e], y = yq[e];
          yp[e] = c * x - sn * y;
          yq[e] = sn * x + c * y;
          const double u = wp[e], v = wq[e];
          wp[e] = c * u - sn * v;
          wq[e] = sn * u + c * v;
        }
        if (l == 0) s_rot = 1;
      }
      __syncthreads();
    }
    const int rot = s_rot, big = s_big;
    __syncthreads();
    // Jacobi sweeps converge quadratically: after a sweep whose rotations were
    // all below 1e-10, the next one's would be below the 1e-15 threshold
    if (rot == 0 || big == 0) break;
  }
  // singular values and their descending order
  for (int c = w; c < n; c += 4) {
    double a = 0.0;
    for (int e = lane; e < n; e += 64) a = fma(Y[(int64_t)c * ldn + e], Y[(int64_t)c * ldn + e], a);
    a = wave_sum(a);
    if (lane == 0) sig[c] = sqrt(a);
  }
  __syncthreads();
  for (int p = tid; p < n; p += WS) {
    int r = 0;
    const double sp = sig[p];
    for (int q = 0; q < n; ++q) r += (sig[q] > sp) || (sig[q] == sp && q < p);
    rk[p] = (double)r;
  }
  __syncthreads();
  // U(:, j) = Q W(:, j) with the sign gauge, V(:, j) = Y(:, j) / sigma_j
  for (int c = w; c < n; c += 4) {
    const int j = (int)rk[c];
    const double sp = sig[c];
    const double* wc = Wm + (int64_t)c * ldn;
    double uv[4];
    double best = -1.0, sgn = 1.0;
    int bi = 0x7fffffff;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = lane + 64 * t;
      double acc = 0.0;
      if (i < m)
        for (int kk = 0; kk < n; ++kk) acc = fma(A[(int64_t)kk * ld + i], wc[kk], acc);
      uv[t] = acc;
      if (i < m && fabs(acc) > best) { best = fabs(acc); sgn = acc < 0.0 ? -1.0 : 1.0; bi = i; }
    }
    for (int i0 = 256; i0 < m; i0 += 64) {
      const int i = i0 + lane;
      if (i < m) {
        double acc = 0.0;
        for (int kk = 0; kk < n; ++kk) acc = fma(A[(int64_t)kk * ld + i], wc[kk], acc);
        if (fabs(acc) > best) { best = fabs(acc); sgn = acc < 0.0 ? -1.0 : 1.0; bi = i; }
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const double os = __shfl_xor(sgn, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; sgn = os; bi = oi; }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = lane + 64 * t;
      if (i < m) U[(int64_t)i * urs + (int64_t)j * ucs] = sgn * uv[t];
    }
    for (int i0 = 256; i0 < m; i0 += 64) {
      const int i = i0 + lane;
      if (i < m) {
        double acc = 0.0;
        for (int kk = 0; kk < n; ++kk) acc = fma(A[(int64_t)kk * ld + i], wc[kk], acc);
        U[(int64_t)i * urs + (int64_t)j * ucs] = sgn * acc;
      }
    }
    const double inv = sp > 0.0 ? sgn / sp : 0.0;
    for (int e = lane; e < n; e += 64) V[(int64_t)e * vrs + (int64_t)j * vcs] = Y[(int64_t)c * ldn + e] * inv;
    if (lane == 0) S[j] = sp;
  }
}

size_t qr_lds_doubles(int m, int n) {
  return (size_t)odd_ld(m) * n + 2 * (size_t)std::min(m, n) + 8 * ((size_t)n + 1) + 12;
}
size_t svd_lds_doubles(int m, int n) {
  return (size_t)odd_ld(m) * n + 2 * (size_t)odd_ld(n) * n + 3 * (size_t)n +
         8 * ((size_t)n + 1) + 12;
}

// Largest dynamic LDS allocation of one workgroup on the current device
// (bytes).  The kernels' attributes are raised once per device and process.
int lds_limit() {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static int lim[kMaxDev] = {};
  int d = 0;
  TT_HIP(hipGetDevice(&d));
  TT_REQUIRE(d >= 0 && d < kMaxDev, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (lim[d] == 0) {
    int v = 0;
    TT_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, d));
    v -= 1024;
    TT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(qr_lds_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, v));
    for (const void* k : {reinterpret_cast<const void*>(svd_lds_kernel<4>),
                          reinterpret_cast<const void*>(svd_lds_kernel<8>),
                          reinterpret_cast<const void*>(svd_lds_kernel<16>),
                          reinterpret_cast<const void*>(svd_lds_kernel<32>),
                          reinterpret_cast<const void*>(svd_lds_kernel<64>)})
      TT_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, v));
    TT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(lu_solve_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, v));
    TT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(qr_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, v));
    TT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(svd_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, v));
    TT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(lu_blocked_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, v));
    TT_HIP(hipFuncSetAttribute(
        reinterpret_cast<const void*>(gj_solve_kernel<kGjExtR, kGjExtC, kGjExtTC, kGjExtCE>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)std::min<size_t>(kGjExtLds, v)));
    lim[d] = v;
  }
  return lim[d];
}

}  // namespace

bool qr_t(hipStream_t s, const double* A, int m, int n, int64_t ars, int64_t acs, double* Q,
          int64_t qrs, int64_t qcs, double* R, int ldr) {
  if (m <= 0 || n <= 0) return true;
  if (qr_lds_doubles(m, n) * 8 > (size_t)lds_limit()) return false;
  ++g_launches;
  qr_lds_kernel<<<1, WS, qr_lds_doubles(m, n) * 8, s>>>(A, m, n, ars, acs, Q, qrs, qcs, R, ldr,
                                                        m, 0);
  TT_HIP(hipGetLastError());
  return true;
}

namespace {
// Tall factorizations whose matrix does not fit in LDS, by a tree of row
// blocks (TSQR).  Level 0 splits A (m x n) into nb_0 blocks of at least n
// rows, each factored in LDS by a workgroup of its own (Q_b written over the
// block, R_b into a stack of nb_0 n x n factors); level i + 1 does the same to
// level i's stack, until a stack fits in LDS and is factored whole (or no
// longer shrinks and is factored in global memory), S = Q_top R.  Then Q = diag(Q_b of level 0) diag(Q_b of level 1) .. Q_top,
// formed top-down by one batched GEMM per level.  Every factorization is
// Householder QR with diag(R) >= 0, so Q and R are those of one Householder
// QR of A up to rounding.
constexpr int kTallMaxLevels = 8;

struct TallPlan {
  int levels = 0;                          // row-block levels below the top
  int rows[kTallMaxLevels + 1] = {};       // rows split at each level, rows[levels] at the top
  int nb[kTallMaxLevels] = {}, mb[kTallMaxLevels] = {}, last[kTallMaxLevels] = {};
  bool top_lds = true;                     // the top stack fits in LDS (else global-memory QR)
};

// lds_doubles: one workgroup's LDS, in doubles.  Levels are added while a
// split into blocks of at least n rows that fit in LDS still shrinks the
// stack; a top that does not fit in LDS (two stacked R factors of n > 98
// columns already exceed 160 KiB) is factored by the global-memory QR, on
// nb n rows instead of m.
bool tall_plan(int m, int n, size_t lds_doubles, TallPlan& p) {
  if (n < 1 || m <= n) return false;
  auto fits = [&](int rows) { return qr_lds_doubles(rows, n) <= lds_doubles; };
  if (fits(m) || !fits(n + 1)) return false;
  int mmax = n + 1;
  while (mmax < m && fits(mmax + 1)) ++mmax;
  int rows = m;
  p.levels = 0;
  while (!fits(rows) && p.levels < kTallMaxLevels) {
    const int nb = cdiv(rows, mmax), mb = cdiv(rows, nb), last = rows - (nb - 1) * mb;
    if (nb < 2 || last < n || (int64_t)nb * n >= rows) break;
    const int L = p.levels;
    p.rows[L] = rows;
    p.nb[L] = nb;
    p.mb[L] = mb;
    p.last[L] = last;
    rows = nb * n;
    ++p.levels;
  }
  if (p.levels == 0) return false;
  p.rows[p.levels] = rows;
  p.top_lds = fits(rows);
  return true;
}

// Scratch of the tree: the R stacks of every level, Q_top, the global QR's
// n scale factors, and two buffers for the partial products of levels
// 1 .. levels - 1.
size_t tall_scratch(const TallPlan& p, int n) {
  const size_t nn = (size_t)n * n;
  size_t need = (size_t)p.rows[p.levels] * n + n;
  size_t pp = 0;
  for (int i = 0; i < p.levels; ++i) {
    need += (size_t)p.nb[i] * nn;
    if (i >= 1) pp = std::max(pp, (size_t)p.rows[i] * n);
  }
  return need + 2 * pp;
}

bool overlaps(const double* a, int64_t na, const double* b, int64_t nb) {
  return a < b + nb && b < a + na;
}

// The one-workgroup factorizations outside the LDS-resident forms: working
// copies in LDS when they fit in it, else in global memory.
void qr_global(hipStream_t s, double* A, int m, int n, int lda, double* Q, int ldq, double* R,
               int ldr, double* tau) {
  ++g_launches;
  const bool lds =
      ((int64_t)m * n + (int64_t)m * std::min(m, n)) * 8 <= (int64_t)lds_limit();
  qr_kernel<<<1, WG, lds ? (size_t)((int64_t)m * n + (int64_t)m * std::min(m, n)) * 8 : 0, s>>>(
      A, m, n, lda, Q, ldq, R, ldr, tau, lds ? 1 : 0);
  TT_HIP(hipGetLastError());
}

size_t svd_kernel_doubles(int m, int n) {
  return (size_t)n * m + (size_t)n * n + 2 * (size_t)n;
}

void svd_global(hipStream_t s, double* G, int m, int n, int ldg, double* U, int ldu, double* S,
                double* V, int ldv, double* work) {
  ++g_launches;
  const size_t need = svd_kernel_doubles(m, n);
  const bool lds = need * 8 <= (size_t)lds_limit();
  svd_kernel<<<1, WG, lds ? need * 8 : 0, s>>>(G, m, n, ldg, U, ldu, S, V, ldv, work, lds ? 1 : 0);
  TT_HIP(hipGetLastError());
}

// Level i: Q_b over the blocks of A in place, R_b at Rs + b n n.
void tall_blocks(hipStream_t s, double* A, int n, int lda, const TallPlan& p, int i,
                 double* Rs) {
  ++g_launches;
  qr_lds_kernel<<<p.nb[i], WS, qr_lds_doubles(p.mb[i], n) * 8, s>>>(
      A, p.rows[i], n, lda, 1, A, lda, 1, Rs, n, p.mb[i], (int64_t)n * n);
  TT_HIP(hipGetLastError());
}

// Level i: C_b = A_b W_b for every row block (W_b at W + b n n, n x n).
void tall_apply(hipStream_t s, const double* A, int n, int lda, const TallPlan& p, int i,
                const double* W, double* C, int ldc) {
  const int mb = p.mb[i], nb = p.nb[i];
  const int full = p.last[i] == mb ? nb : nb - 1;
  gemm(s, false, false, mb, n, n, 1.0, A, lda, (int64_t)mb * lda, W, n, (int64_t)n * n, 0.0, C,
       ldc, (int64_t)mb * ldc, full);
  if (full < nb) {
    const int64_t r0 = (int64_t)full * mb;
    gemm(s, false, false, p.last[i], n, n, 1.0, A + r0 * lda, lda, 0, W + (int64_t)full * n * n,
         n, 0, 0.0, C + r0 * ldc, ldc, 0);
  }
}

// The tree QR with a plan and its scratch (tall_scratch doubles); A is
// overwritten, Q must not overlap A.
void tall_qr(hipStream_t s, double* A, int m, int n, int lda, double* Q, int ldq, double* R,
             int ldr, const TallPlan& p, double* ws) {
  const int L = p.levels;
  double* S[kTallMaxLevels];
  double* cur = ws;
  for (int i = 0; i < L; ++i) {
    S[i] = cur;
    cur += (size_t)p.nb[i] * n * n;
  }
  double* Qtop = cur;
  cur += (size_t)p.rows[L] * n;
  double* tau = cur;
  cur += n;
  size_t pp = 0;
  for (int i = 1; i < L; ++i) pp = std::max(pp, (size_t)p.rows[i] * n);
  double* P[2] = {cur, cur + pp};
  double* Ai = A;
  int ldi = lda;
  for (int i = 0; i < L; ++i) {
    tall_blocks(s, Ai, n, ldi, p, i, S[i]);
    Ai = S[i];
    ldi = n;
  }
  if (p.top_lds)
    TT_REQUIRE(qr_t(s, Ai, p.rows[L], n, n, 1, Qtop, n, 1, R, ldr), "top R stack exceeds LDS");
  else
    qr_global(s, Ai, p.rows[L], n, n, Qtop, n, R, ldr, tau);
  const double* W = Qtop;
  for (int i = L - 1; i >= 0; --i) {
    const double* Ab = i == 0 ? A : S[i - 1];
    double* out = i == 0 ? Q : P[i & 1];
    tall_apply(s, Ab, n, i == 0 ? lda : n, p, i, W, out, i == 0 ? ldq : n);
    W = out;
  }
  (void)m;
}

bool svd_lds_ok(int m, int n) {
  const int npair = (n + 1) / 2;
  int lp = 64;
  while (lp > 4 && npair * lp > WS) lp >>= 1;
  return npair * lp <= WS && svd_lds_doubles(m, n) * 8 <= (size_t)lds_limit();
}

// QR of a tall A by the row-block tree; false (nothing launched) when the
// plan does not apply, the scratch is short or Q overlaps A.
bool qr_tall(hipStream_t s, double* A, int m, int n, int lda, double* Q, int ldq, double* R,
             int ldr, double* ws, size_t ws_doubles) {
  TallPlan p;
  if (!ws || !tall_plan(m, n, (size_t)lds_limit() / 8, p)) return false;
  if (tall_scratch(p, n) > ws_doubles) return false;
  if (overlaps(A, (int64_t)(m - 1) * lda + n, Q, (int64_t)(m - 1) * ldq + n)) return false;
  tall_qr(s, A, m, n, lda, Q, ldq, R, ldr, p, ws);
  return true;
}

// Thin SVD of a tall G: G = Q R by the tree (Q into scratch), R = U_R S V^T in
// LDS, U = Q U_R, then the sign gauge of U (V flipped with it).
bool svd_tall(hipStream_t s, double* G, int m, int n, int ldg, double* U, int ldu, double* S,
              double* V, int ldv, double* ws, size_t ws_doubles) {
  TallPlan p;
  if (!ws || !tall_plan(m, n, (size_t)lds_limit() / 8, p)) return false;
  const size_t nn = (size_t)n * n;
  const bool r_lds = svd_lds_ok(n, n);
  const size_t tree = tall_scratch(p, n);
  if ((size_t)m * n + 2 * nn + std::max(tree, r_lds ? 0 : svd_kernel_doubles(n, n)) > ws_doubles)
    return false;
  if (overlaps(G, (int64_t)(m - 1) * ldg + n, U, (int64_t)(m - 1) * ldu + n)) return false;
  double* Qf = ws;
  double* Rf = Qf + (size_t)m * n;
  double* UR = Rf + nn;
  double* rest = UR + nn;
  tall_qr(s, G, m, n, ldg, Qf, n, Rf, n, p, rest);
  // the n x n SVD of R: in LDS, else in global memory (its scratch reuses the tree's)
  if (r_lds)
    TT_REQUIRE(svd_t(s, Rf, n, n, n, 1, UR, n, 1, S, V, ldv, 1), "R factor exceeds LDS");
  else
    svd_global(s, Rf, n, n, n, UR, n, S, V, ldv, rest);
  gemm(s, false, false, m, n, n, 1.0, Qf, n, 0, UR, n, 0, 0.0, U, ldu, 0);
  ++g_launches;
  col_gauge_kernel<<<n, 256, 0, s>>>(U, m, ldu, V, n, ldv);
  TT_HIP(hipGetLastError());
  return true;
}
}  // namespace

size_t tall_qr_doubles(int m, int n) {
  TallPlan p;
  return tall_plan(m, n, kTallLdsDoubles, p) ? tall_scratch(p, n) : 0;
}

void qr(hipStream_t s, double* A, int m, int n, int lda, double* Q, int ldq, double* R, int ldr,
        double* tau) {
  if (m <= 0 || n <= 0) return;
  if (qr_t(s, A, m, n, lda, 1, Q, ldq, 1, R, ldr)) return;
  if (qr_tall(s, A, m, n, lda, Q, ldq, R, ldr, g_fact_buf, g_fact_cap)) return;
  qr_global(s, A, m, n, lda, Q, ldq, R, ldr, tau);
}

// The global-memory SVD's scratch, and at least the row-block tree's: Q
// (m n), R and U_R, then the tree or the n x n global SVD of R.
size_t svd_work_doubles(int m, int n) {
  const size_t tall = tall_qr_doubles(m, n);
  const size_t tree =
      tall ? (size_t)m * n + 2 * (size_t)n * n + std::max(tall, svd_kernel_doubles(n, n)) : 0;
  return std::max(svd_kernel_doubles(m, n), tree);
}

bool svd_t(hipStream_t s, const double* G, int m, int n, int64_t gr, int64_t gc, double* U,
           int64_t ur, int64_t uc, double* S, double* V, int64_t vr, int64_t vc) {
  if (m <= 0 || n <= 0) return true;
  TT_REQUIRE(m >= n, "svd expects m >= n");
  // lanes per Jacobi pair: the largest power of two (at most 64) that lets
  // all (n + 1) / 2 pairs of a round run at once in 256 threads
  const int npair = (n + 1) / 2;
  int lp = 64;
  while (lp > 4 && npair * lp > WS) lp >>= 1;
  if (npair * lp > WS || svd_lds_doubles(m, n) * 8 > (size_t)lds_limit()) return false;
  ++g_launches;
  const size_t lds = svd_lds_doubles(m, n) * 8;
  switch (lp) {
    case 64: svd_lds_kernel<64><<<1, WS, lds, s>>>(G, m, n, gr, gc, U, ur, uc, S, V, vr, vc); break;
    case 32: svd_lds_kernel<32><<<1, WS, lds, s>>>(G, m, n, gr, gc, U, ur, uc, S, V, vr, vc); break;
    case 16: svd_lds_kernel<16><<<1, WS, lds, s>>>(G, m, n, gr, gc, U, ur, uc, S, V, vr, vc); break;
    case 8: svd_lds_kernel<8><<<1, WS, lds, s>>>(G, m, n, gr, gc, U, ur, uc, S, V, vr, vc); break;
    default: svd_lds_kernel<4><<<1, WS, lds, s>>>(G, m, n, gr, gc, U, ur, uc, S, V, vr, vc); break;
  }
  TT_HIP(hipGetLastError());
  return true;
}

void svd(hipStream_t s, double* G, int m, int n, int ldg, double* U, int ldu, double* S,
         double* V, int ldv, double* work) {
  if (m <= 0 || n <= 0) return;
  TT_REQUIRE(m >= n, "svd expects m >= n");
  if (svd_t(s, G, m, n, ldg, 1, U, ldu, 1, S, V, ldv, 1)) return;
  if (svd_tall(s, G, m, n, ldg, U, ldu, S, V, ldv, work, svd_work_doubles(m, n))) return;
  svd_global(s, G, m, n, ldg, U, ldu, S, V, ldv, work);
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
  // One workgroup per system.  Gauss-Jordan up to 240 unknowns, with the
  // augmented matrix in registers (up to 192) or in registers and LDS; larger
  // systems use the LU kernel (in LDS up to 141 unknowns), blocked by panels
  // beyond that while a panel fits LDS (about 1,000 unknowns).
  if (N <= 64) {
    gj_solve_kernel<4, 3, 32><<<batch, 512, 0, s>>>(A, N, lda, b);
  } else if (N <= 112) {
    gj_solve_kernel<7, 4, 32><<<batch, 512, 0, s>>>(A, N, lda, b);
  } else if (N <= 144) {
    gj_solve_kernel<9, 5, 32><<<batch, 512, 0, s>>>(A, N, lda, b);
  } else if (N <= 192) {
    gj_solve_kernel<12, 7, 32><<<batch, 512, 0, s>>>(A, N, lda, b);
  } else if (N <= 16 * kGjExtR && kGjExtLds <= (size_t)lds_limit()) {
    gj_solve_kernel<kGjExtR, kGjExtC, kGjExtTC, kGjExtCE>
        <<<batch, 16 * kGjExtTC, kGjExtLds, s>>>(A, N, lda, b);
  } else {
    const size_t need = ((size_t)N * odd_ld(N) + N) * 8;
    const bool lds = need <= (size_t)lds_limit();
    const size_t need_blk = lu_blocked_lds_doubles(N) * 8;
    if (!lds && need_blk <= (size_t)lds_limit())
      lu_blocked_kernel<<<batch, WG, need_blk, s>>>(A, N, lda, b);
    else
      lu_solve_kernel<<<batch, WG, lds ? need : 0, s>>>(A, N, lda, b, lds ? 1 : 0);
  }
  TT_HIP(hipGetLastError());
}

}  // namespace ttnt
