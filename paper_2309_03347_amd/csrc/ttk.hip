// Tensor-train kernels: core matvec, operator-core permutation, dense local
// matrix, Krylov (Arnoldi) step, small vector helpers.
#include "kernels.h"
#include "ttk.h"
#include "probe.h"

#include <algorithm>

namespace ttnt {
namespace {

int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

// Y[(b*r0 + a), i, (b'*r1 + a')] = sum_j A[b, i, j, b'] X[a, j, a']
__global__ __launch_bounds__(256) void core_matvec_kernel(const double* __restrict__ A, int R0,
                                                          int m, int n, int R1,
                                                          const double* __restrict__ X, int r0,
                                                          int r1, double* __restrict__ Y) {
  const int64_t C = (int64_t)R1 * r1;
  const int64_t total = (int64_t)R0 * r0 * m * C;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = e % C;
    const int64_t t = e / C;
    const int i = (int)(t % m);
    const int64_t row = t / m;
    const int b = (int)(row / r0), a = (int)(row % r0);
    const int bp = (int)(col / r1), ap = (int)(col % r1);
    const double* Ab = A + (((int64_t)b * m + i) * n) * R1 + bp;
    const double* Xa = X + ((int64_t)a * n) * r1 + ap;
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc = fma(Ab[(int64_t)j * R1], Xa[(int64_t)j * r1], acc);
    Y[e] = acc;
  }
}

// Ap[(i*RR + b'), (b*n + j)] = A[b, i, j, b']
__global__ void permute_op_kernel(const double* __restrict__ A, int RL, int m, int n, int RR,
                                  double* __restrict__ Ap) {
  const int64_t total = (int64_t)RL * m * n * RR;
  const int64_t cols = (int64_t)RL * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / cols, col = e % cols;
    const int i = (int)(row / RR), bp = (int)(row % RR);
    const int b = (int)(col / n), j = (int)(col % n);
    Ap[e] = A[(((int64_t)b * m + i) * n + j) * RR + bp];
  }
}

// M[(a,i,c), (a2,j,c2)] = sum_b PhiL[a, b, a2] P[(b,i,j), c, c2]
__global__ void local_matrix_kernel(const double* __restrict__ phiL, int ra, int RL,
                                    const double* __restrict__ P, int m, int n, int rc,
                                    double* __restrict__ M) {
  const int64_t N = (int64_t)ra * n * rc;
  const int64_t total = (int64_t)ra * m * rc * N;
  const int64_t rc2 = (int64_t)rc * rc;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / N, col = e % N;
    const int c = (int)(row % rc);
    const int i = (int)((row / rc) % m);
    const int a = (int)(row / ((int64_t)rc * m));
    const int c2 = (int)(col % rc);
    const int j = (int)((col / rc) % n);
    const int a2 = (int)(col / ((int64_t)rc * n));
    double acc = 0.0;
    for (int b = 0; b < RL; ++b)
      acc = fma(phiL[((int64_t)a * RL + b) * ra + a2],
                P[(((int64_t)b * m + i) * n + j) * rc2 + (int64_t)c * rc + c2], acc);
    M[e] = acc;
  }
}

// Mode-diagonal core applied to a contracted operand (the middle stage of a
// local product or interface update when A[b, i, j, b'] = delta_ij Hd[b, i, b']):
//   out[a][i][b'][c] = sum_b Hd[b][i][b'] in[a][b][i][c]
__global__ __launch_bounds__(256) void mode_mix_kernel(const double* __restrict__ in, int ra,
                                                       int RL, int n, int rc,
                                                       const double* __restrict__ Hd, int RR,
                                                       double* __restrict__ out) {
  const int64_t total = (int64_t)ra * n * RR * rc;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % rc);
    const int bp = (int)((e / rc) % RR);
    const int i = (int)((e / ((int64_t)rc * RR)) % n);
    const int a = (int)(e / ((int64_t)rc * RR * n));
    const double* x = in + ((int64_t)a * RL * n + i) * rc + c;
    const double* h = Hd + (int64_t)i * RR + bp;
    double acc = 0.0;
    for (int b = 0; b < RL; ++b) acc = fma(h[(int64_t)b * n * RR], x[(int64_t)b * n * rc], acc);
    out[e] = acc;
  }
}

// The transposed use (right interfaces):
//   out[a][b][i][c] = sum_b' Hd[b][i][b'] in[a][i][b'][c]
__global__ __launch_bounds__(256) void mode_mix_t_kernel(const double* __restrict__ in, int ra,
                                                         int n, int RR, int rc,
                                                         const double* __restrict__ Hd, int RL,
                                                         double* __restrict__ out) {
  const int64_t total = (int64_t)ra * RL * n * rc;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % rc);
    const int i = (int)((e / rc) % n);
    const int b = (int)((e / ((int64_t)rc * n)) % RL);
    const int a = (int)(e / ((int64_t)rc * n * RL));
    const double* x = in + (((int64_t)a * n + i) * RR) * rc + c;
    const double* h = Hd + ((int64_t)b * n + i) * RR;
    double acc = 0.0;
    for (int bp = 0; bp < RR; ++bp) acc = fma(h[bp], x[(int64_t)bp * rc], acc);
    out[e] = acc;
  }
}

// Weighted sum over the mode: u[a][c] = sum_j w[j] v[a][j][c]
__global__ __launch_bounds__(256) void mode_contract_kernel(const double* __restrict__ v, int ra,
                                                            int n, int rc,
                                                            const double* __restrict__ w,
                                                            double* __restrict__ u) {
  const int64_t total = (int64_t)ra * rc;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % rc);
    const int a = (int)(e / rc);
    const double* x = v + (int64_t)a * n * rc + c;
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc = fma(w[j], x[(int64_t)j * rc], acc);
    u[e] = acc;
  }
}

// Row factor of a core whose columns are multiples of one column j0
// (A[b, i, j, b'] = a[b, i, b'] w_j with w_j0 = 1), as a GEMM operand:
//   Arp[(i*RR + b'), b] = A[b, i, j0, b']
__global__ void rank1_rows_kernel(const double* __restrict__ A, int RL, int n, int RR, int j0,
                                  double* __restrict__ Arp) {
  const int64_t total = (int64_t)n * RR * RL;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e % RL);
    const int bp = (int)((e / RL) % RR);
    const int i = (int)(e / ((int64_t)RL * RR));
    Arp[e] = A[(((int64_t)b * n + i) * n + j0) * RR + bp];
  }
}

// Diagonal of an operator core: Hd[b][i][b'] = A[b, i, i, b']
__global__ void op_diag_kernel(const double* __restrict__ A, int RL, int n, int RR,
                               double* __restrict__ Hd) {
  const int64_t total = (int64_t)RL * n * RR;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int bp = (int)(e % RR);
    const int i = (int)((e / RR) % n);
    const int b = (int)(e / ((int64_t)RR * n));
    Hd[e] = A[(((int64_t)b * n + i) * n + i) * RR + bp];
  }
}

// Block-diagonal local matrices of a mode-diagonal core:
// M[i][(a,c), (a2,c2)] = sum_b PhiL[a, b, a2] P[(b,i)][c][c2]
__global__ void local_matrix_diag_kernel(const double* __restrict__ phiL, int ra, int RL,
                                         const double* __restrict__ P, int n, int rc,
                                         double* __restrict__ M) {
  const int64_t B = (int64_t)ra * rc;
  const int64_t total = (int64_t)n * B * B;
  const int64_t rc2 = (int64_t)rc * rc;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = e % B, row = (e / B) % B;
    const int i = (int)(e / (B * B));
    const int a = (int)(row / rc), c = (int)(row % rc);
    const int a2 = (int)(col / rc), c2 = (int)(col % rc);
    double acc = 0.0;
    for (int b = 0; b < RL; ++b)
      acc = fma(phiL[((int64_t)a * RL + b) * ra + a2],
                P[((int64_t)b * n + i) * rc2 + (int64_t)c * rc + c2], acc);
    M[e] = acc;
  }
}

// [a][i][c] <-> [i][a][c]
__global__ void swap_mode_kernel(const double* __restrict__ src, int ra, int n, int rc,
                                 double* __restrict__ dst, int to_blocks) {
  const int64_t total = (int64_t)ra * n * rc;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % rc);
    const int i = (int)((e / rc) % n);
    const int a = (int)(e / ((int64_t)rc * n));
    const int64_t blk = ((int64_t)i * ra + a) * rc + c;
    if (to_blocks) dst[blk] = src[e]; else dst[e] = src[blk];
  }
}

__global__ void scale_cols_kernel(double* __restrict__ X, int rows, int cols, int ld,
                                  const double* __restrict__ s) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / cols), c = (int)(e % cols);
    X[(int64_t)r * ld + c] *= s[c];
  }
}

// GMRES Arnoldi step (one workgroup): V rows are Krylov vectors of length N.
// On entry V[j+1] holds w = A V[j].  CGS2 against V[0..j]; H column j
// (stored Hc[j*(ldh) + i]); Givens update of g; writes |g[j+1]| to *res.
__global__ __launch_bounds__(1024) void arnoldi_kernel(double* __restrict__ V, int64_t N, int j,
                                                       double* __restrict__ Hc, int ldh,
                                                       double* __restrict__ cs,
                                                       double* __restrict__ sn,
                                                       double* __restrict__ g,
                                                       double* __restrict__ res) {
  __shared__ double red[16];
  __shared__ double h[1024];
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wid = tid >> 6, nw = nt >> 6;
  double* w = V + (int64_t)(j + 1) * N;
  double* hcol = Hc + (int64_t)j * ldh;
  for (int i = tid; i <= j + 1; i += nt) h[i] = 0.0;
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    for (int i = wid; i <= j; i += nw) {
      const double* vi = V + (int64_t)i * N;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int64_t e = lane;
      for (; e + 192 < N; e += 256) {
        a0 = fma(vi[e], w[e], a0);
        a1 = fma(vi[e + 64], w[e + 64], a1);
        a2 = fma(vi[e + 128], w[e + 128], a2);
        a3 = fma(vi[e + 192], w[e + 192], a3);
      }
      for (; e < N; e += 64) a0 = fma(vi[e], w[e], a0);
      const double acc = wave_sum((a0 + a1) + (a2 + a3));
      if (lane == 0) h[512 + i] = acc;
    }
    __syncthreads();
    for (int64_t e = tid; e < N; e += nt) {
      double a0 = w[e], a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int i = 0;
      for (; i + 3 <= j; i += 4) {
        a0 -= h[512 + i] * V[(int64_t)i * N + e];
        a1 -= h[513 + i] * V[(int64_t)(i + 1) * N + e];
        a2 -= h[514 + i] * V[(int64_t)(i + 2) * N + e];
        a3 -= h[515 + i] * V[(int64_t)(i + 3) * N + e];
      }
      for (; i <= j; ++i) a0 -= h[512 + i] * V[(int64_t)i * N + e];
      w[e] = (a0 + a1) + (a2 + a3);
    }
    for (int i = tid; i <= j; i += nt) h[i] += h[512 + i];
    __syncthreads();
  }
  // stage the previous rotations in LDS (the serial update below reads them)
  __shared__ double rc[512], rs[512];
  for (int i = tid; i < j; i += nt) {
    rc[i] = cs[i];
    rs[i] = sn[i];
  }
  double v = 0.0;
  for (int64_t e = tid; e < N; e += nt) v = fma(w[e], w[e], v);
  const double nrm = sqrt(block_sum(v, red));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int64_t e = tid; e < N; e += nt) w[e] *= inv;
  if (tid == 0) {
    h[j + 1] = nrm;
    for (int i = 0; i < j; ++i) {
      const double t = rc[i] * h[i] + rs[i] * h[i + 1];
      h[i + 1] = -rs[i] * h[i] + rc[i] * h[i + 1];
      h[i] = t;
    }
    const double a = h[j], b = h[j + 1];
    const double rr = sqrt(a * a + b * b);
    const double c = rr > 0.0 ? a / rr : 1.0, s = rr > 0.0 ? b / rr : 0.0;
    cs[j] = c;
    sn[j] = s;
    h[j] = rr;
    h[j + 1] = 0.0;
    g[j + 1] = -s * g[j];
    g[j] = c * g[j];
    for (int i = 0; i <= j; ++i) hcol[i] = h[i];
    *res = fabs(g[j + 1]);
  }
}

// ---- multi-workgroup Arnoldi step (CGS2), four launches ----
// Workgroup b owns elements [b*chunk, min(N, (b+1)*chunk)); chunk is a
// multiple of 64 so every lane of a wavefront has at most chunk/64 elements.
// Partials: P1[b][i], P2[b][i] (dots of the two passes), P3[b] (norm^2),
// hacc[i] (the accumulated Hessenberg column).

__device__ __forceinline__ void chunk_dots(const double* __restrict__ V, const double* __restrict__ w,
                                           int64_t N, int j, int64_t e0, int64_t e1,
                                           double* __restrict__ out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i = wid; i <= j; i += nw) {
    const double* vi = V + (int64_t)i * N;
    double acc = 0.0;
    for (int64_t e = e0 + lane; e < e1; e += 64) acc = fma(vi[e], w[e], acc);
    acc = wave_sum(acc);
    if (lane == 0) out[i] = acc;
  }
}

__global__ __launch_bounds__(256) void arn_dots_kernel(const double* __restrict__ V, int64_t N,
                                                       int j, int64_t chunk,
                                                       double* __restrict__ P1) {
  const int b = blockIdx.x;
  const int64_t e0 = b * chunk, e1 = min(N, e0 + chunk);
  chunk_dots(V, V + (int64_t)(j + 1) * N, N, j, e0, e1, P1 + (int64_t)b * (j + 1));
}

// h = sum_b Pin[b][:];  w -= V^T h on this chunk;  then either the next dots
// (Pout != null) or the partial norm^2 (P3).  Workgroup 0 accumulates h into hacc.
__global__ __launch_bounds__(256) void arn_update_kernel(double* __restrict__ V, int64_t N, int j,
                                                         int64_t chunk, int G,
                                                         const double* __restrict__ Pin,
                                                         double* __restrict__ Pout,
                                                         double* __restrict__ P3,
                                                         double* __restrict__ hacc, int first) {
  __shared__ double h[128];
  __shared__ double red[4];
  const int b = blockIdx.x, tid = threadIdx.x;
  for (int i = tid; i <= j; i += 256) {
    double s = 0.0;
    for (int q = 0; q < G; ++q) s += Pin[(int64_t)q * (j + 1) + i];
    h[i] = s;
    if (b == 0) hacc[i] = first ? s : hacc[i] + s;
  }
  __syncthreads();
  double* w = V + (int64_t)(j + 1) * N;
  const int64_t e0 = b * chunk, e1 = min(N, e0 + chunk);
  double nn = 0.0;
  for (int64_t e = e0 + tid; e < e1; e += 256) {
    double a0 = w[e], a1 = 0.0;
    int i = 0;
    for (; i + 1 <= j; i += 2) {
      a0 -= h[i] * V[(int64_t)i * N + e];
      a1 -= h[i + 1] * V[(int64_t)(i + 1) * N + e];
    }
    if (i <= j) a0 -= h[i] * V[(int64_t)i * N + e];
    const double r = a0 + a1;
    w[e] = r;
    nn = fma(r, r, nn);
  }
  __syncthreads();
  if (Pout) {
    chunk_dots(V, w, N, j, e0, e1, Pout + (int64_t)b * (j + 1));
  } else {
    nn = wave_sum(nn);
    if ((tid & 63) == 0) red[tid >> 6] = nn;
    __syncthreads();
    if (tid == 0) P3[b] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

__global__ __launch_bounds__(256) void arn_finish_kernel(double* __restrict__ V, int64_t N, int j,
                                                         int64_t chunk, int G,
                                                         const double* __restrict__ P3,
                                                         const double* __restrict__ hacc,
                                                         double* __restrict__ Hc, int ldh,
                                                         double* __restrict__ cs,
                                                         double* __restrict__ sn,
                                                         double* __restrict__ g,
                                                         double* __restrict__ res) {
  __shared__ double snrm;
  const int b = blockIdx.x, tid = threadIdx.x;
  if (tid == 0) {
    double s = 0.0;
    for (int q = 0; q < G; ++q) s += P3[q];
    snrm = sqrt(s);
  }
  __syncthreads();
  const double nrm = snrm;
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  double* w = V + (int64_t)(j + 1) * N;
  const int64_t e0 = b * chunk, e1 = min(N, e0 + chunk);
  for (int64_t e = e0 + tid; e < e1; e += 256) w[e] *= inv;
  if (b == 0 && tid == 0) {
    double h[130];
    for (int i = 0; i <= j; ++i) h[i] = hacc[i];
    h[j + 1] = nrm;
    for (int i = 0; i < j; ++i) {
      const double t = cs[i] * h[i] + sn[i] * h[i + 1];
      h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
      h[i] = t;
    }
    const double a = h[j], bb = h[j + 1];
    const double rr = sqrt(a * a + bb * bb);
    const double c = rr > 0.0 ? a / rr : 1.0, s = rr > 0.0 ? bb / rr : 0.0;
    cs[j] = c;
    sn[j] = s;
    h[j] = rr;
    g[j + 1] = -s * g[j];
    g[j] = c * g[j];
    double* hcol = Hc + (int64_t)j * ldh;
    for (int i = 0; i <= j; ++i) hcol[i] = h[i];
    res[j] = fabs(g[j + 1]);
  }
}

// Solve the k x k upper-triangular least-squares system and update x += V^T y.
__global__ __launch_bounds__(1024) void gmres_update_kernel(const double* __restrict__ V,
                                                            int64_t N, int k,
                                                            const double* __restrict__ Hc,
                                                            int ldh, const double* __restrict__ g,
                                                            double* __restrict__ x) {
  __shared__ double y[128];
  __shared__ double gs[128];
  extern __shared__ double Hs[];      // k x k upper triangle, column-major like Hc
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int c = e / k, i = e % k;
    Hs[e] = i <= c ? Hc[(int64_t)c * ldh + i] : 0.0;
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) gs[i] = g[i];
  __syncthreads();
  // column-oriented back substitution: one division, then a parallel update
  for (int i = k - 1; i >= 0; --i) {
    if (threadIdx.x == 0) {
      const double d = Hs[i * k + i];
      y[i] = d != 0.0 ? gs[i] / d : 0.0;
    }
    __syncthreads();
    const double yi = y[i];
    for (int r = threadIdx.x; r < i; r += blockDim.x) gs[r] -= Hs[i * k + r] * yi;
    __syncthreads();
  }
  for (int64_t e = threadIdx.x; e < N; e += blockDim.x) {
    double acc = x[e];
    for (int i = 0; i < k; ++i) acc = fma(y[i], V[(int64_t)i * N + e], acc);
    x[e] = acc;
  }
}

// r = f - r ; beta = ||r|| ; V0 = r / beta ; g = [beta, 0, ...] ; out[0] = beta, out[1] = ||f||
__global__ __launch_bounds__(1024) void gmres_start_kernel(const double* __restrict__ f,
                                                           double* __restrict__ r, int64_t N,
                                                           double* __restrict__ V0,
                                                           double* __restrict__ g, int gl,
                                                           double* __restrict__ out) {
  __shared__ double red[16];
  double a = 0.0, b = 0.0;
  for (int64_t e = threadIdx.x; e < N; e += blockDim.x) {
    const double t = f[e] - r[e];
    r[e] = t;
    a = fma(t, t, a);
    b = fma(f[e], f[e], b);
  }
  const double beta = sqrt(block_sum(a, red));
  const double fn = sqrt(block_sum(b, red));
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int64_t e = threadIdx.x; e < N; e += blockDim.x) V0[e] = r[e] * inv;
  for (int i = threadIdx.x; i < gl; i += blockDim.x) g[i] = (i == 0) ? beta : 0.0;
  if (threadIdx.x == 0) {
    out[0] = beta;
    out[1] = fn;
  }
}

// out[idx] = ||y - f|| / ||f||  (residual indicator of the current core)
__global__ __launch_bounds__(1024) void rel_res_kernel(const double* __restrict__ y,
                                                       const double* __restrict__ f, int64_t N,
                                                       double* __restrict__ out) {
  __shared__ double red[16];
  double a = 0.0, b = 0.0;
  for (int64_t e = threadIdx.x; e < N; e += blockDim.x) {
    const double t = y[e] - f[e];
    a = fma(t, t, a);
    b = fma(f[e], f[e], b);
  }
  a = block_sum(a, red);
  b = block_sum(b, red);
  if (threadIdx.x == 0) *out = b > 0.0 ? sqrt(a / b) : (a > 0.0 ? INFINITY : 0.0);
}

// k_new = k * num / den ; outputs on device: kinfo[0] = k_new, kinfo[1] = k_old.
__global__ void k_update_kernel(double* kval, const double* num, const double* den,
                                double* kinfo) {
  if (threadIdx.x == 0) {
    const double k = *kval;
    const double kn = k * (*num) / (*den);
    kinfo[0] = kn;
    kinfo[1] = k;
    *kval = kn;
  }
}

// den_next = num / sqrt(nrm2)
__global__ void scale_ratio_kernel(const double* num, const double* nrm2, double* out) {
  if (threadIdx.x == 0) *out = *num / sqrt(*nrm2);
}

}  // namespace

void tt_core_matvec(hipStream_t s, const double* A, int R0, int m, int n, int R1,
                    const double* X, int r0, int r1, double* Y) {
  const int64_t total = (int64_t)R0 * r0 * m * R1 * r1;
  if (total <= 0) return;
  ++g_launches;
  hipEvent_t pe = nullptr;
  if (g_probe) {
    const double fl = 2.0 * (double)total * n;
    const double by = 8.0 * ((double)total + (double)R0 * m * n * R1 + (double)r0 * n * r1);
    pe = g_probe->begin(s, kProbeMatvec, fl, by);
  }
  core_matvec_kernel<<<grid_for(total, 256), 256, 0, s>>>(A, R0, m, n, R1, X, r0, r1, Y);
  TT_HIP(hipGetLastError());
  if (pe) g_probe->end(s);
}

void permute_op(hipStream_t s, const double* A, int RL, int m, int n, int RR, double* Ap) {
  const int64_t total = (int64_t)RL * m * n * RR;
  if (total <= 0) return;
  ++g_launches;
  permute_op_kernel<<<grid_for(total, 256), 256, 0, s>>>(A, RL, m, n, RR, Ap);
  TT_HIP(hipGetLastError());
}

void local_matrix(hipStream_t s, const double* phiL, int ra, int RL, const double* P, int m,
                  int n, int rc, double* M) {
  const int64_t total = (int64_t)ra * m * rc * ra * n * rc;
  if (total <= 0) return;
  ++g_launches;
  local_matrix_kernel<<<grid_for(total, 256), 256, 0, s>>>(phiL, ra, RL, P, m, n, rc, M);
  TT_HIP(hipGetLastError());
}

void mode_mix(hipStream_t s, const double* in, int ra, int RL, int n, int rc, const double* Hd,
              int RR, double* out) {
  const int64_t total = (int64_t)ra * n * RR * rc;
  if (total <= 0) return;
  ++g_launches;
  mode_mix_kernel<<<grid_for(total, 256), 256, 0, s>>>(in, ra, RL, n, rc, Hd, RR, out);
  TT_HIP(hipGetLastError());
}

void mode_mix_t(hipStream_t s, const double* in, int ra, int n, int RR, int rc, const double* Hd,
                int RL, double* out) {
  const int64_t total = (int64_t)ra * RL * n * rc;
  if (total <= 0) return;
  ++g_launches;
  mode_mix_t_kernel<<<grid_for(total, 256), 256, 0, s>>>(in, ra, n, RR, rc, Hd, RL, out);
  TT_HIP(hipGetLastError());
}

void mode_contract(hipStream_t s, const double* v, int ra, int n, int rc, const double* w,
                   double* u) {
  const int64_t total = (int64_t)ra * rc;
  if (total <= 0) return;
  ++g_launches;
  mode_contract_kernel<<<grid_for(total, 256), 256, 0, s>>>(v, ra, n, rc, w, u);
  TT_HIP(hipGetLastError());
}

void rank1_rows(hipStream_t s, const double* A, int RL, int n, int RR, int j0, double* Arp) {
  const int64_t total = (int64_t)n * RR * RL;
  if (total <= 0) return;
  ++g_launches;
  rank1_rows_kernel<<<grid_for(total, 256), 256, 0, s>>>(A, RL, n, RR, j0, Arp);
  TT_HIP(hipGetLastError());
}

void op_diag(hipStream_t s, const double* A, int RL, int n, int RR, double* Hd) {
  ++g_launches;
  op_diag_kernel<<<grid_for((int64_t)RL * n * RR, 256), 256, 0, s>>>(A, RL, n, RR, Hd);
  TT_HIP(hipGetLastError());
}

void local_matrix_diag(hipStream_t s, const double* phiL, int ra, int RL, const double* P, int n,
                       int rc, double* M) {
  const int64_t total = (int64_t)n * ra * rc * ra * rc;
  ++g_launches;
  local_matrix_diag_kernel<<<grid_for(total, 256), 256, 0, s>>>(phiL, ra, RL, P, n, rc, M);
  TT_HIP(hipGetLastError());
}

void swap_mode(hipStream_t s, const double* src, int ra, int n, int rc, double* dst,
               bool to_blocks) {
  ++g_launches;
  swap_mode_kernel<<<grid_for((int64_t)ra * n * rc, 256), 256, 0, s>>>(src, ra, n, rc, dst,
                                                                       to_blocks ? 1 : 0);
  TT_HIP(hipGetLastError());
}

void scale_cols(hipStream_t s, double* X, int rows, int cols, int ld, const double* sv) {
  if (rows <= 0 || cols <= 0) return;
  ++g_launches;
  scale_cols_kernel<<<grid_for((int64_t)rows * cols, 256), 256, 0, s>>>(X, rows, cols, ld, sv);
  TT_HIP(hipGetLastError());
}

void arnoldi(hipStream_t s, double* V, int64_t N, int j, double* Hc, int ldh, double* cs,
             double* sn, double* g, double* res) {
  TT_REQUIRE(j + 2 <= 512, "Krylov dimension too large");
  ++g_launches;
  hipEvent_t pe = nullptr;
  if (g_probe) {
    // two classical Gram-Schmidt passes: dots and updates over j+1 vectors
    const double fl = 8.0 * (double)N * (j + 1) + 3.0 * N;
    const double by = 8.0 * (double)N * (2.0 * (j + 1) + 4.0);
    pe = g_probe->begin(s, kProbeArnoldi, fl, by);
  }
  arnoldi_kernel<<<1, 1024, 0, s>>>(V, N, j, Hc, ldh, cs, sn, g, res);
  TT_HIP(hipGetLastError());
  if (pe) g_probe->end(s);
}

namespace {
int64_t arn_chunk(int64_t N) {
  const int64_t per = (N + 127) / 128;                 // at most 128 workgroups
  return std::max<int64_t>(64, (per + 63) / 64 * 64);
}
}  // namespace

size_t arnoldi_mwg_doubles(int64_t N, int m) {
  const int64_t G = (N + arn_chunk(N) - 1) / arn_chunk(N);
  return (size_t)(2 * G * (m + 1) + G + m + 8);
}

void arnoldi_mwg(hipStream_t s, double* V, int64_t N, int j, double* Hc, int ldh, double* cs,
                 double* sn, double* g, double* res, double* work) {
  TT_REQUIRE(j + 2 <= 128, "Krylov dimension too large for the multi-workgroup step");
  const int64_t chunk = arn_chunk(N);
  const int G = (int)((N + chunk - 1) / chunk);
  double* P1 = work;
  double* P2 = P1 + (int64_t)G * (j + 1);
  double* P3 = P2 + (int64_t)G * (j + 1);
  double* hacc = P3 + G;
  hipEvent_t pe = nullptr;
  if (g_probe) {
    const double fl = 8.0 * (double)N * (j + 1) + 3.0 * N;
    const double by = 8.0 * (double)N * (2.0 * (j + 1) + 4.0);
    pe = g_probe->begin(s, kProbeArnoldi, fl, by);
  }
  g_launches += 4;
  arn_dots_kernel<<<G, 256, 0, s>>>(V, N, j, chunk, P1);
  arn_update_kernel<<<G, 256, 0, s>>>(V, N, j, chunk, G, P1, P2, nullptr, hacc, 1);
  arn_update_kernel<<<G, 256, 0, s>>>(V, N, j, chunk, G, P2, nullptr, P3, hacc, 0);
  arn_finish_kernel<<<G, 256, 0, s>>>(V, N, j, chunk, G, P3, hacc, Hc, ldh, cs, sn, g, res);
  TT_HIP(hipGetLastError());
  if (pe) g_probe->end(s);
}

void gmres_update(hipStream_t s, const double* V, int64_t N, int k, const double* Hc, int ldh,
                  const double* g, double* x) {
  if (k <= 0) return;
  TT_REQUIRE(k <= 88, "Krylov dimension above the LDS budget of the update");
  ++g_launches;
  gmres_update_kernel<<<1, 1024, (size_t)k * k * 8, s>>>(V, N, k, Hc, ldh, g, x);
  TT_HIP(hipGetLastError());
}

void gmres_start(hipStream_t s, const double* f, double* r, int64_t N, double* V0, double* g,
                 int gl, double* out) {
  ++g_launches;
  gmres_start_kernel<<<1, 1024, 0, s>>>(f, r, N, V0, g, gl, out);
  TT_HIP(hipGetLastError());
}

void rel_res(hipStream_t s, const double* y, const double* f, int64_t N, double* out) {
  ++g_launches;
  rel_res_kernel<<<1, 1024, 0, s>>>(y, f, N, out);
  TT_HIP(hipGetLastError());
}

void k_update(hipStream_t s, double* kval, const double* num, const double* den, double* kinfo) {
  ++g_launches;
  k_update_kernel<<<1, 64, 0, s>>>(kval, num, den, kinfo);
  TT_HIP(hipGetLastError());
}

void scale_ratio(hipStream_t s, const double* num, const double* nrm2, double* out) {
  ++g_launches;
  scale_ratio_kernel<<<1, 64, 0, s>>>(num, nrm2, out);
  TT_HIP(hipGetLastError());
}

}  // namespace ttnt
