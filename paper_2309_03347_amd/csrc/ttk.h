// Launchers of the tensor-train kernels (ttk.hip).
#pragma once

#include "common.h"

namespace ttnt {

// Ap[(i*RR + b'), (b*n + j)] = A[b, i, j, b']   (operator core as a GEMM operand)
void permute_op(hipStream_t s, const double* A, int RL, int m, int n, int RR, double* Ap);
// Dense local matrix from PhiL [ra][RL][ra] and P[(b,i,j)][c][c2]
void local_matrix(hipStream_t s, const double* phiL, int ra, int RL, const double* P, int m,
                  int n, int rc, double* M);
void scale_cols(hipStream_t s, double* X, int rows, int cols, int ld, const double* sv);
// Hd[b][i][b'] = A[b, i, i, b']
void op_diag(hipStream_t s, const double* A, int RL, int n, int RR, double* Hd);
// Mode-diagonal core (A[b,i,j,b'] = delta_ij Hd[b,i,b']) in a contraction:
//   out[a][i][b'][c] = sum_b Hd[b][i][b'] in[a][b][i][c]
void mode_mix(hipStream_t s, const double* in, int ra, int RL, int n, int rc, const double* Hd,
              int RR, double* out);
//   out[a][b][i][c] = sum_b' Hd[b][i][b'] in[a][i][b'][c]
void mode_mix_t(hipStream_t s, const double* in, int ra, int n, int RR, int rc, const double* Hd,
                int RL, double* out);
// u[a][c] = sum_j w[j] v[a][j][c]
void mode_contract(hipStream_t s, const double* v, int ra, int n, int rc, const double* w,
                   double* u);
// Arp[(i*RR + b'), b] = A[b, i, j0, b'] (row factor of a core with proportional columns)
void rank1_rows(hipStream_t s, const double* A, int RL, int n, int RR, int j0, double* Arp);
// n block matrices M[i] ((ra rc) x (ra rc)) of a mode-diagonal local operator
void local_matrix_diag(hipStream_t s, const double* phiL, int ra, int RL, const double* P, int n,
                       int rc, double* M);
// [a][i][c] -> [i][a][c] (to_blocks) or back
void swap_mode(hipStream_t s, const double* src, int ra, int n, int rc, double* dst,
               bool to_blocks);
void arnoldi(hipStream_t s, double* V, int64_t N, int j, double* Hc, int ldh, double* cs,
             double* sn, double* g, double* res);
// Multi-workgroup Arnoldi step (CGS2 in four launches); res[j] = |g[j+1]|.
size_t arnoldi_mwg_doubles(int64_t N, int m);
void arnoldi_mwg(hipStream_t s, double* V, int64_t N, int j, double* Hc, int ldh, double* cs,
                 double* sn, double* g, double* res, double* work);
void gmres_update(hipStream_t s, const double* V, int64_t N, int k, const double* Hc, int ldh,
                  const double* g, double* x);
void gmres_start(hipStream_t s, const double* f, double* r, int64_t N, double* V0, double* g,
                 int gl, double* out);
void rel_res(hipStream_t s, const double* y, const double* f, int64_t N, double* out);
void k_update(hipStream_t s, double* kval, const double* num, const double* den, double* kinfo);
void scale_ratio(hipStream_t s, const double* num, const double* nrm2, double* out);

}  // namespace ttnt
