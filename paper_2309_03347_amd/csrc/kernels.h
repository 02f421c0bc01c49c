// Internal host-side launchers (all enqueue on `s`; none synchronize).
#pragma once

#include "common.h"

namespace ttnt {

// Launch counter (diagnostic: kernels issued since last reset).
extern thread_local int64_t g_launches;
// Scratch for split-K partial products (set by the caller that owns it; null
// disables the split).  Capacity in doubles.
extern thread_local double* g_splitk_buf;
extern thread_local size_t g_splitk_cap;
// Scratch of the tall QR by a tree of row blocks (qr), set like the split-K
// buffer by the caller that owns it; null, or shorter than the shape needs
// (tall_qr_doubles), leaves tall matrices that do not fit in LDS to the
// one-workgroup global-memory QR.  Capacity in doubles.
extern thread_local double* g_fact_buf;
extern thread_local size_t g_fact_cap;
// LDS a workgroup may use on gfx950, in doubles: 160 KiB less the 1 KiB kept
// for static arrays (the dynamic LDS limit the factorization kernels get)
constexpr size_t kTallLdsDoubles = (160 * 1024 - 1024) / 8;
constexpr size_t kFactDoubles = 2 * kTallLdsDoubles + 1024;   // the least a caller provides
// Scratch of the row-block QR of an m x n matrix planned for kTallLdsDoubles
// of LDS (0: the shape fits in LDS or has no row-block plan).
size_t tall_qr_doubles(int m, int n);
// Points g_fact_buf at a buffer for the lifetime of the object.
struct FactScope {
  double* prev_buf;
  size_t prev_cap;
  FactScope(double* p, size_t cap) : prev_buf(g_fact_buf), prev_cap(g_fact_cap) {
    g_fact_buf = p;
    g_fact_cap = cap;
  }
  ~FactScope() {
    g_fact_buf = prev_buf;
    g_fact_cap = prev_cap;
  }
};

// C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b]; row-major, op = transpose if flag.
// op(A) is M x K, op(B) is K x N.
void gemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
          int lda, int64_t sA, const double* B, int ldb, int64_t sB, double beta, double* C,
          int ldc, int64_t sC, int batch = 1);

// The same product on the BF16 matrix cores: operands rounded to BF16 as they
// are staged, FP32 accumulation, FP64 result (lowp.hip).
void gemm_bf16(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
               const double* A, int lda, int64_t sA, const double* B, int ldb, int64_t sB,
               double beta, double* C, int ldc, int64_t sC, int batch = 1);
// The same product on the FP16 matrix cores: each row of op(A) and column of
// op(B) scaled by a power of two per 32-deep k block before the cast, FP32
// accumulation with the scales multiplied back, FP64 result (lowp.hip).
void gemm_f16(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
              const double* A, int lda, int64_t sA, const double* B, int ldb, int64_t sB,
              double beta, double* C, int ldc, int64_t sC, int batch = 1);
// C[b][m][n] = alpha * sum_s P[s][b][m][n] + beta * C[b][m][n], s in order (split-K partials
// of nsplit x batch dense M x N blocks).
void splitk_reduce(hipStream_t s, const double* P, int nsplit, int batch, int M, int N,
                   double alpha, double beta, double* C, int ldc, int64_t sC);

// dst[j][i] = src[i][j] for an rows x cols source (row-major, leading dims given).
void transpose(hipStream_t s, const double* src, int rows, int cols, int lds, double* dst,
               int ldd);
// dst[i][j] = src[i][j] (rows x cols).
void copy2d(hipStream_t s, const double* src, int rows, int cols, int lds, double* dst, int ldd);
void copy(hipStream_t s, const double* src, double* dst, int64_t n);
void fill(hipStream_t s, double* dst, int64_t n, double v);
// y = a * x + b * y
void axpby(hipStream_t s, int64_t n, double a, const double* x, double b, double* y);
// y = a * x + (b / *c) * y   (c device scalar; used for 1/k scaling)
void axpby_div(hipStream_t s, int64_t n, double a, const double* x, double b, const double* c,
               double* y);
// out = sum x^2 (device scalar), single launch.
void sumsq(hipStream_t s, const double* x, int64_t n, double* out);
// x *= 1/sqrt(*ss)  (ss device scalar holding a sum of squares)
void scale_inv_sqrt(hipStream_t s, double* x, int64_t n, const double* ss);

// ---- dense factorizations (one workgroup each) ----
// Householder QR of A (m x n, lda), overwritten.  Q (m x k, ldq) and R (k x n, ldr),
// k = min(m, n), with diag(R) >= 0.  A is destroyed.
void qr(hipStream_t s, double* A, int m, int n, int lda, double* Q, int ldq, double* R, int ldr,
        double* tau);
// One-sided Jacobi SVD of G (m x n, m >= n), destroyed.  U (m x n), S (n), V (n x n)
// row-major, singular values descending; each column of U has its largest-magnitude
// entry positive (V flipped to match).
void svd(hipStream_t s, double* G, int m, int n, int ldg, double* U, int ldu, double* S,
         double* V, int ldv, double* work);
size_t svd_work_doubles(int m, int n);
// The LDS-resident QR and SVD with strided operands: element (i, c) of the
// input at A[i ars + c acs] (G[i gr + c gc]), Q(i, c) written to
// Q[i qrs + c qcs], U(i, j) to U[i ur + j uc], V(e, j) to V[e vr + j vc]; a
// transposed operand or result then needs no transpose launch.  The input is
// read before any output is written (Q may overlap A).  Return false, having
// launched nothing, when the matrix does not fit in LDS.
bool qr_t(hipStream_t s, const double* A, int m, int n, int64_t ars, int64_t acs, double* Q,
          int64_t qrs, int64_t qcs, double* R, int ldr);
bool svd_t(hipStream_t s, const double* G, int m, int n, int64_t gr, int64_t gc, double* U,
           int64_t ur, int64_t uc, double* S, double* V, int64_t vr, int64_t vc);
// Truncation rank: smallest r with sqrt(sum_{i>=r} S_i^2) <= delta, where
// delta = tol * sqrt(*normsq) / sqrt(dm1) (or tol * ||S|| when normsq == NULL);
// r capped to [1, rmax]; writes rank[0] (device int), rank[1] = 1 if rmax bound, and adds the discarded
// sum of squares to *discard (device, may be NULL).
void trunc_rank(hipStream_t s, const double* S, int n, double tol, double dm1,
                const double* normsq, int rmax, int* rank, double* discard);
// Dense LU with partial pivoting of A (N x N, lda; destroyed) and solve A x = b in place.
// batch > 1: matrices at A + i*N*lda and right-hand sides at b + i*N, one workgroup each.
void lu_solve(hipStream_t s, double* A, int N, int lda, double* b, int batch = 1);

// ---- TT kernels ----
void tt_core_matvec(hipStream_t s, const double* A, int R0, int m, int n, int R1,
                    const double* X, int r0, int r1, double* Y);

}  // namespace ttnt
