// TT algorithms on the device: exact matvec, rounding (QR sweep + truncated
// SVD sweep), dot product, right orthogonalization, local operator
// application and local solves.
#include <algorithm>
#include <cmath>

#include "engine.h"
#include "krylov.h"
#include "kernels.h"
#include "ttk.h"
#include "probe.h"

namespace ttnt {

TTv view(const tt_vec* v) {
  TTv t;
  t.d = v->d;
  t.n.assign(v->n, v->n + v->d);
  t.r.assign(v->r, v->r + v->d + 1);
  t.rcap.assign(v->rcap, v->rcap + v->d + 1);
  t.data = v->data;
  t.off.assign(v->off, v->off + v->d);
  return t;
}

TTm view(const tt_mat* m) {
  TTm t;
  t.d = m->d;
  t.m.assign(m->m, m->m + m->d);
  t.n.assign(m->n, m->n + m->d);
  t.R.assign(m->R, m->R + m->d + 1);
  t.data = m->data;
  t.off.assign(m->off, m->off + m->d);
  return t;
}

void matvec(hipStream_t s, const TTm& A, const TTv& x, TTv& y) {
  for (int k = 0; k < A.d; ++k)
    tt_core_matvec(s, A.core(k), A.R[k], A.m[k], A.n[k], A.R[k + 1], x.core(k), x.r[k],
                   x.r[k + 1], y.core(k));
  for (int k = 0; k <= A.d; ++k) y.r[k] = A.R[k] * x.r[k];
}

// ---------------------------------------------------------------------------
// Thin SVD of a rows x cols matrix W (ld = cols): Lft (rows x p, ld p),
// S (p), RtT (p x cols, ld cols) with p = min(rows, cols).
// ---------------------------------------------------------------------------
namespace {

struct SvdScratch {
  double *G, *U, *V, *work;
};

size_t thin_svd_doubles(int64_t rows, int64_t cols) {
  const int64_t M = std::max(rows, cols), p = std::min(rows, cols);
  return (size_t)(M * p) /*G*/ + (size_t)(M * p) /*U*/ + (size_t)(p * p) /*V*/ +
         svd_work_doubles((int)M, (int)p);
}

SvdScratch carve_svd(Bump& ws, int64_t rows, int64_t cols) {
  const int64_t M = std::max(rows, cols), p = std::min(rows, cols);
  SvdScratch sc;
  sc.G = ws.d(M * p);
  sc.U = ws.d(M * p);
  sc.V = ws.d(p * p);
  sc.work = ws.d(svd_work_doubles((int)M, (int)p));
  return sc;
}

int thin_svd(hipStream_t s, const double* W, int rows, int cols, double* Lft, double* S,
             double* RtT, const SvdScratch& sc) {
  if (rows >= cols) {
    const int p = cols;
    // V^T written straight into RtT (p x cols)
    if (svd_t(s, W, rows, cols, cols, 1, Lft, p, 1, S, RtT, 1, cols)) return p;
    svd(s, const_cast<double*>(W), rows, cols, cols, Lft, p, S, sc.V, p, sc.work);
    transpose(s, sc.V, p, p, p, RtT, cols);
    return p;
  }
  const int p = rows;
  // the SVD of W^T (cols x rows) read through strides, its U^T written into RtT
  if (svd_t(s, W, cols, rows, 1, cols, RtT, 1, cols, S, Lft, p, 1)) return p;
  transpose(s, W, rows, cols, cols, sc.G, rows);               // G = W^T (cols x rows)
  svd(s, sc.G, cols, rows, rows, sc.U, rows, S, Lft, p, sc.work);  // U: cols x rows
  transpose(s, sc.U, cols, rows, rows, RtT, cols);             // RtT = U^T (rows x cols)
  return p;
}

int64_t max_core(const TTv& x) {
  int64_t mx = 1;
  for (int k = 0; k < x.d; ++k) mx = std::max(mx, x.size(k));
  return mx;
}

int max_dim(const TTv& x) {
  int mx = 1;
  for (int k = 0; k < x.d; ++k) mx = std::max(mx, std::max(x.r[k] * x.n[k], x.r[k + 1]));
  for (int k = 0; k < x.d; ++k) mx = std::max(mx, std::max(x.r[k], x.n[k] * x.r[k + 1]));
  return mx;
}

}  // namespace

size_t fact_doubles_for(const TTv& x) {
  size_t f = kFactDoubles;
  for (int k = 0; k < x.d; ++k) {
    const int64_t left = (int64_t)x.r[k] * x.n[k], right = (int64_t)x.n[k] * x.r[k + 1];
    if (left <= INT32_MAX) f = std::max(f, tall_qr_doubles((int)left, x.r[k + 1]));
    if (right <= INT32_MAX) f = std::max(f, tall_qr_doubles((int)right, x.r[k]));
  }
  return f;
}

size_t round_ws_bytes(const TTv& x) {
  Bump b;
  const int64_t mc = max_core(x);
  const int md = max_dim(x);
  b.d(mc);        // W
  b.d(mc);        // R
  b.d(md);        // tau
  b.d(mc);        // tmp
  b.d(mc);        // Lft
  b.d(mc);        // RtT
  b.d(md);        // S
  size_t svd_need = 0;
  for (int k = 0; k < x.d; ++k)
    svd_need = std::max(svd_need, thin_svd_doubles(x.r[k], (int64_t)x.n[k] * x.r[k + 1]));
  b.d(svd_need + 512);
  b.d(4);         // scalars
  b.i(4);
  b.d(fact_doubles_for(x));   // tall-QR scratch of the API calls (g_fact_buf)
  return b.used + 4096;
}

namespace {
// Event and pinned scratch for blocking calls made by one host thread, kept
// until release_thread_resources() (or the end of the process).
struct BlockingCtx {
  SyncSlot slot;
  HostBuf hb{nullptr, nullptr};
};
thread_local BlockingCtx* t_blocking = nullptr;
BlockingCtx& blocking_ctx() {
  if (!t_blocking) {
    auto* n = new BlockingCtx();
    TT_HIP(hipEventCreateWithFlags(&n->slot.ev, hipEventDisableTiming));
    void* p = nullptr;
    TT_HIP(hipHostMalloc(&p, 256, hipHostMallocDefault));
    n->hb.i = static_cast<int*>(p);
    n->hb.d = reinterpret_cast<double*>(static_cast<char*>(p) + 64);
    t_blocking = n;
  }
  return *t_blocking;
}
}  // namespace

void release_thread_resources() {
  if (!t_blocking) return;
  if (t_blocking->slot.ev) (void)hipEventDestroy(t_blocking->slot.ev);
  if (t_blocking->hb.i) (void)hipHostFree(t_blocking->hb.i);
  delete t_blocking;
  t_blocking = nullptr;
}

void round_tt(hipStream_t s, TTv& x, double tol, int rmax, double* rel_err, Bump& ws) {
  BlockingCtx& c = blocking_ctx();
  Co t = round_tt_co(s, x, tol, rmax, rel_err, ws, c.slot, c.hb);
  run_blocking(t, c.slot);
}

Co round_tt_co(hipStream_t s, TTv& x, double tol, int rmax, double* rel_err, Bump& ws,
               SyncSlot& slot, HostBuf hb, bool left_orth) {
  const int d = x.d;
  const int64_t mc = max_core(x);
  const int md = max_dim(x);
  double* W = ws.d(mc);
  double* R = ws.d(mc);
  double* tau = ws.d(md);
  double* tmp = ws.d(mc);
  double* Lft = ws.d(mc);
  double* RtT = ws.d(mc);
  double* S = ws.d(md);
  size_t svd_need = 0;
  for (int k = 0; k < d; ++k)
    svd_need = std::max(svd_need, thin_svd_doubles(x.r[k], (int64_t)x.n[k] * x.r[k + 1]));
  Bump sub;
  sub.base = (char*)ws.d(svd_need + 512);
  sub.cap = (svd_need + 512) * sizeof(double);
  double* scal = ws.d(4);
  int* irank = ws.i(4);
  double* nrm2 = scal;
  double* disc = scal + 1;
  if (d == 1) {
    if (rel_err) *rel_err = 0.0;
    co_return;
  }
  // left-to-right Householder QR sweep
  for (int k = 0; k < d - 1 && !left_orth; ++k) {
    const int rows = x.r[k] * x.n[k], cols = x.r[k + 1];
    const int q = std::min(rows, cols);
    copy(s, x.core(k), W, (int64_t)rows * cols);
    qr(s, W, rows, cols, cols, x.core(k), q, R, cols, tau);
    const int n2 = x.n[k + 1] * x.r[k + 2];
    gemm(s, false, false, q, n2, cols, 1.0, R, cols, 0, x.core(k + 1), n2, 0, 0.0, tmp, n2, 0);
    copy(s, tmp, x.core(k + 1), (int64_t)q * n2);
    x.r[k + 1] = q;
  }
  sumsq(s, x.core(d - 1), x.size(d - 1), nrm2);
  fill(s, disc, 1, 0.0);
  // right-to-left truncated SVD sweep
  for (int k = d - 1; k >= 1; --k) {
    const int rows = x.r[k], cols = x.n[k] * x.r[k + 1];
    sub.used = 0;
    SvdScratch sc = carve_svd(sub, rows, cols);
    const int p = thin_svd(s, x.core(k), rows, cols, Lft, S, RtT, sc);
    trunc_rank(s, S, p, tol, (double)(d - 1), nrm2, rmax, irank, disc);
    TT_HIP(hipMemcpyAsync(hb.i, irank, sizeof(int), hipMemcpyDeviceToHost, s));
    co_await Sync{&slot, s};
    const int rk = hb.i[0];
    copy(s, RtT, x.core(k), (int64_t)rk * cols);
    const int prow = x.r[k - 1] * x.n[k - 1];
    gemm(s, false, false, prow, rk, rows, 1.0, x.core(k - 1), rows, 0, Lft, p, 0, 0.0, tmp, rk, 0);
    scale_cols(s, tmp, prow, rk, rk, S);
    copy(s, tmp, x.core(k - 1), (int64_t)prow * rk);
    x.r[k] = rk;
  }
  if (rel_err) {
    TT_HIP(hipMemcpyAsync(hb.d, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    co_await Sync{&slot, s};
    *rel_err = hb.d[0] > 0.0 ? std::sqrt(hb.d[1] / hb.d[0]) : 0.0;
  }
}

size_t dot_ws_bytes(const TTv& a, const TTv& b) {
  int64_t mx = 1;
  for (int k = 0; k <= a.d; ++k) mx = std::max(mx, (int64_t)a.r[k] * b.r[k]);
  int64_t mt = 1;
  for (int k = 0; k < a.d; ++k) mt = std::max(mt, (int64_t)a.r[k] * a.n[k] * b.r[k + 1]);
  Bump bb;
  bb.d(mx);
  bb.d(mx);
  bb.d(mt);
  return bb.used + 1024;
}

void dot_tt(hipStream_t s, const TTv& a, const TTv& b, double* out, Bump& ws) {
  int64_t mx = 1;
  for (int k = 0; k <= a.d; ++k) mx = std::max(mx, (int64_t)a.r[k] * b.r[k]);
  int64_t mt = 1;
  for (int k = 0; k < a.d; ++k) mt = std::max(mt, (int64_t)a.r[k] * a.n[k] * b.r[k + 1]);
  double* v0 = ws.d(mx);
  double* v1 = ws.d(mx);
  double* T = ws.d(mt);
  fill(s, v0, 1, 1.0);
  for (int k = 0; k < a.d; ++k) {
    const int ra = a.r[k], rb = b.r[k], n = a.n[k], ra1 = a.r[k + 1], rb1 = b.r[k + 1];
    // T[(a, i), b'] = sum_b v[a][b] B_k[b][(i, b')]
    gemm(s, false, false, ra, n * rb1, rb, 1.0, v0, rb, 0, b.core(k), n * rb1, 0, 0.0, T, n * rb1, 0);
    // v'[a', b'] = sum_{(a,i)} A_k[(a,i)][a'] T[(a,i)][b']
    gemm(s, true, false, ra1, rb1, ra * n, 1.0, a.core(k), ra1, 0, T, rb1, 0, 0.0, v1, rb1, 0);
    std::swap(v0, v1);
  }
  copy(s, v0, out, 1);
}

void orth_right(hipStream_t s, TTv& x, Bump& ws) {
  const int d = x.d;
  const int64_t mc = max_core(x);
  const int md = max_dim(x);
  double* Wt = ws.d(mc);
  double* Q = ws.d(mc);
  double* R = ws.d(mc);
  double* tau = ws.d(md);
  double* tmp = ws.d(mc);
  for (int k = d - 1; k >= 1; --k) {
    const int rows = x.r[k], cols = x.n[k] * x.r[k + 1];
    const int q = std::min(rows, cols);
    // QR of core k^T (cols x rows); core k = Q^T (q x cols), written in place
    if (!qr_t(s, x.core(k), cols, rows, 1, cols, x.core(k), 1, cols, R, rows)) {
      transpose(s, x.core(k), rows, cols, cols, Wt, rows);      // cols x rows
      qr(s, Wt, cols, rows, rows, Q, q, R, rows, tau);           // Q: cols x q, R: q x rows
      transpose(s, Q, cols, q, q, x.core(k), cols);              // core k = Q^T (q x cols)
    }
    const int prow = x.r[k - 1] * x.n[k - 1];
    gemm(s, false, true, prow, q, rows, 1.0, x.core(k - 1), rows, 0, R, rows, 0, 0.0, tmp, q, 0);
    copy(s, tmp, x.core(k - 1), (int64_t)prow * q);
    x.r[k] = q;
  }
}

// ---------------------------------------------------------------------------
// Local operator and local solve
// ---------------------------------------------------------------------------
namespace {
typedef void (*GemmFn)(hipStream_t, bool, bool, int, int, int, double, const double*, int,
                       int64_t, const double*, int, int64_t, double, double*, int, int64_t, int);

void local_apply_with(GemmFn mm, hipStream_t s, const LocalOp& o, const double* v, double* y,
                      double alpha, double beta, double* T1, double* T2) {
  if (o.form.kind == 2) {
    // proportional columns: the mode of v is summed with w first
    // u[b2, d'] = sum_j w_j v[b2, j, d'] (held in T2 until T2 is rewritten)
    mode_contract(s, v, o.rb, o.n, o.rd, o.form.w, T2);
    // T1[(a, b), d'] = sum_{b2} PhiL[(a, b), b2] u[b2, d']
    mm(s, false, false, o.ra * o.RL, o.rd, o.rb, 1.0, o.phiL, o.rb, 0, T2, o.rd, 0, 0.0, T1,
         o.rd, 0, 1);
    // T2[a][(i, b'), d'] = sum_b Arp[(i, b'), b] T1[a][b, d']
    mm(s, false, false, o.m * o.RR, o.rd, o.RL, 1.0, o.form.Arp, o.RL, 0, T1, o.rd,
         (int64_t)o.RL * o.rd, 0.0, T2, o.rd, (int64_t)o.m * o.RR * o.rd, o.ra);
  } else {
    // T1[(a, b), (j, d')] = sum_{b2} PhiL[(a, b), b2] v[b2, (j, d')]
    mm(s, false, false, o.ra * o.RL, o.n * o.rd, o.rb, 1.0, o.phiL, o.rb, 0, v, o.n * o.rd, 0,
         0.0, T1, o.n * o.rd, 0, 1);
    if (o.form.kind == 1) {
      // diagonal in the mode: T2[a][i][b'][d'] = sum_b Hd[b, i, b'] T1[a][b][i][d']
      mode_mix(s, T1, o.ra, o.RL, o.n, o.rd, o.form.Hd, o.RR, T2);
    } else {
      // T2[a][(i, b'), d'] = sum_{(b, j)} Ap[(i, b'), (b, j)] T1[a][(b, j), d']
      mm(s, false, false, o.m * o.RR, o.rd, o.RL * o.n, 1.0, o.Ap, o.RL * o.n, 0, T1, o.rd,
           (int64_t)o.RL * o.n * o.rd, 0.0, T2, o.rd, (int64_t)o.m * o.RR * o.rd, o.ra);
    }
  }
  // y[(a, i), c] = sum_{(b', d')} T2[(a, i), (b', d')] PhiR[c, (b', d')]
  mm(s, false, true, o.ra * o.m, o.rc, o.RR * o.rd, alpha, T2, o.RR * o.rd, 0, o.phiR,
       o.RR * o.rd, 0, beta, y, o.rc, 0, 1);
}
}  // namespace

void local_apply(hipStream_t s, const LocalOp& o, const double* v, double* y, double alpha,
                 double beta, double* T1, double* T2) {
  local_apply_with(gemm, s, o, v, y, alpha, beta, T1, T2);
}

void local_apply_lp(hipStream_t s, const LocalOp& o, const double* v, double* y, double alpha,
                    double beta, double* T1, double* T2, bool f16) {
  local_apply_with(f16 ? gemm_f16 : gemm_bf16, s, o, v, y, alpha, beta, T1, T2);
}

static int pick_method(const LocalOp& op, const LocalSolveOpts& o) {
  const int64_t N = (int64_t)op.ra * op.n * op.rc;
  if (o.method != 0) return o.method;
  if (N <= o.direct_max) return 1;
  if (op.diag && (int64_t)op.ra * op.rc <= o.block_max) return 3;
  return 2;
}

size_t local_solve_ws_doubles(const LocalOp& op, const LocalSolveOpts& o) {
  const int64_t N = (int64_t)op.ra * op.n * op.rc;
  const int64_t t1 = (int64_t)op.ra * op.RL * op.n * op.rd;
  const int64_t t2 = (int64_t)op.ra * op.m * op.RR * op.rd;
  int64_t need = 0;
  need += t1 + t2 + 64;
  const int method = pick_method(op, o);
  if (method == 3) {
    const int64_t B = (int64_t)op.ra * op.rc;
    need += (int64_t)op.RL * op.n * op.RR + (int64_t)op.RL * op.n * op.rc * op.rc + op.n * B * B +
            N + 256;
  } else if (method == 1) {
    need += N * N + (int64_t)op.RL * op.m * op.n * op.rc * op.rc + 64;
  } else {
    const int m = std::max(2, std::min(o.restart, 88));
    need += (int64_t)(m + 1) * N + N + (int64_t)(m + 1) * (m + 1) + 4 * (m + 2) + 64 +
            (int64_t)arnoldi_mwg_doubles(N, m);
    const KrylovShape sh{op.ra, op.RL, op.n, op.RR, op.rc};
    if (method == 2 && krylov_enabled())
      need = std::max<int64_t>(need, t1 + t2 + 64 + 64 + krylov_ws_doubles(sh, m, krylov_grid()));
  }
  need += N + 16;
  return (size_t)need + 1024;
}

void throw_barrier_abort() {
  throw HipError{hipErrorLaunchTimeOut,
                 "persistent GMRES: a workgroup gave up waiting at a grid barrier"};
}

void krylov_probe_amend(const LocalOp& op, int restart, int iterations, int slot, bool mixed) {
  if (!g_probe || slot < 0) return;
  const KrylovShape sh{op.ra, op.RL, op.n, op.RR, op.rc};
  const int m = krylov_restart(sh, std::max(2, std::min(restart, 88)), mixed);
  if (m <= 0) return;
  const int64_t N = (int64_t)op.ra * op.n * op.rc;
  // one operator application per Arnoldi step and per restart residual, and
  // the two Gram-Schmidt passes over j + 1 vectors
  const int64_t T = iterations;
  const int64_t full = T / m, rem = T % m;
  const double sumj = (double)full * m * (m + 1) / 2 + (double)rem * (rem + 1) / 2;
  const int64_t applies = T + std::max<int64_t>(1, (T + m - 1) / m);
  const double fa = 2.0 * ((double)op.ra * op.RL * op.n * op.rd * op.rb +
                           (double)op.ra * op.m * op.RR * op.RL * op.n * op.rd +
                           (double)op.ra * op.m * op.rc * op.RR * op.rd);
  const double ba = 8.0 * ((double)op.ra * op.RL * op.rb + (double)op.m * op.RR * op.RL * op.n +
                           (double)op.rc * op.RR * op.rd + 2.0 * N);
  const double fl = applies * fa + 8.0 * N * sumj + 6.0 * N * T;
  const double by = applies * ba + 8.0 * N * (2.0 * sumj + 4.0 * T);
  g_probe->amend(slot, fl, by);
}

LocalSolveResult local_solve(hipStream_t s, const LocalOp& op, const double* f, double* x,
                             const LocalSolveOpts& o, Bump& ws, bool final_res,
                             double* defer_info) {
  LocalSolveResult res;
  const int64_t N = (int64_t)op.ra * op.n * op.rc;
  TT_REQUIRE(op.ra == op.rb && op.rc == op.rd && op.m == op.n, "local system must be square");
  double* T1 = ws.d((int64_t)op.ra * op.RL * op.n * op.rd + 16);
  double* T2 = ws.d((int64_t)op.ra * op.m * op.RR * op.rd + 16);
  double* scal = ws.d(8);
  const int method = pick_method(op, o);
  if (method == 3) {
    // mode-diagonal core: n independent (ra rc) x (ra rc) systems
    res.method = 3;
    const int B = op.ra * op.rc;
    double* Hd = ws.d((int64_t)op.RL * op.n * op.RR);
    double* P = ws.d((int64_t)op.RL * op.n * op.rc * op.rc);
    double* M = ws.d((int64_t)op.n * B * B);
    double* b = ws.d(N);
    op_diag(s, op.A, op.RL, op.n, op.RR, Hd);
    // P[(b,i)][c][c2] = sum_b' Hd[(b,i), b'] PhiR[c][b'][c2]
    gemm(s, false, false, op.RL * op.n, op.rc, op.RR, 1.0, Hd, op.RR, 0, op.phiR, op.rc,
         (int64_t)op.RR * op.rc, 0.0, P, op.rc * op.rc, op.rc, op.rc);
    local_matrix_diag(s, op.phiL, op.ra, op.RL, P, op.n, op.rc, M);
    swap_mode(s, f, op.ra, op.n, op.rc, b, true);
    lu_solve(s, M, B, B, b, op.n);
    swap_mode(s, b, op.ra, op.n, op.rc, x, false);
  } else if (method == 1) {
    res.method = 1;
    double* M = ws.d(N * N);
    double* P = ws.d((int64_t)op.RL * op.m * op.n * op.rc * op.rc);
    // P[(b,i,j)][c][c2] = sum_b' A[(b,i,j), b'] PhiR[c][b'][c2]
    gemm(s, false, false, op.RL * op.m * op.n, op.rc, op.RR, 1.0, op.A, op.RR, 0, op.phiR, op.rc,
         (int64_t)op.RR * op.rc, 0.0, P, op.rc * op.rc, op.rc, op.rc);
    local_matrix(s, op.phiL, op.ra, op.RL, P, op.m, op.n, op.rc, M);
    copy(s, f, x, N);
    lu_solve(s, M, (int)N, (int)N, x);
  } else if (method == 2 && krylov_enabled() && o.persistent &&
             krylov_fits(KrylovShape{op.ra, op.RL, op.n, op.RR, op.rc},
                         std::max(2, std::min(o.restart, 88)))) {
    res.method = 2;
    const int m = std::max(2, std::min(o.restart, 88));
    const KrylovShape sh{op.ra, op.RL, op.n, op.RR, op.rc};
    const bool mixed = o.mixed && krylov_fits(sh, m, true);
    res.mixed = mixed;
    const int grid = krylov_grid();
    const size_t kw = krylov_ws_doubles(sh, m, grid);
    double* kws = ws.d(kw);
    const bool probed = krylov_solve(s, sh, op.phiL, op.Ap, op.phiR, f, x, m, o.max_iter, o.tol,
                                     o.eta, kws, kw, scal, grid, mixed, o.inner_tol);
    const int slot = probed ? g_probe->last_slot() : -1;
    if (o.dev_info) {
      copy(s, scal, o.dev_info, 5);
    } else if (defer_info && !final_res) {
      TT_HIP(hipMemcpyAsync(defer_info, scal, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
      res.deferred = true;
      res.probe_slot = slot;
    } else {
      double info[5];
      TT_HIP(hipMemcpyAsync(info, scal, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
      TT_HIP(hipStreamSynchronize(s));
      if (info[4] != 0.0) throw_barrier_abort();
      res.iterations = (int)info[0];
      res.converged = info[1] != 0.0;
      krylov_probe_amend(op, o.restart, res.iterations, slot, mixed);
    }
  } else {
    if (o.dev_info)
      throw ArgError{"asynchronous step: a local system outside the persistent GMRES kernel "
                     "(multi-launch GMRES needs the host between launches)"};
    res.method = method;
    const int m = std::max(2, std::min(o.restart, 88));
    double* V = ws.d((int64_t)(m + 1) * N);
    double* r = ws.d(N);
    double* Hc = ws.d((int64_t)(m + 1) * (m + 1));
    double* cs = ws.d(m + 2);
    double* sn = ws.d(m + 2);
    double* g = ws.d(m + 2);
    double* resv = ws.d(m + 2);
    double* awork = ws.d(arnoldi_mwg_doubles(N, m));
    double host[2];
    int total = 0;
    bool conv = false;
    double fnorm = 0.0;
    double target = -1.0;
    while (true) {
      local_apply(s, op, x, r, 1.0, 0.0, T1, T2);
      gmres_start(s, f, r, N, V, g, m + 2, scal);
      TT_HIP(hipMemcpyAsync(host, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      TT_HIP(hipStreamSynchronize(s));
      fnorm = host[1];
      if (fnorm == 0.0) {
        fill(s, x, N, 0.0);
        conv = true;
        break;
      }
      if (target < 0.0) target = std::max(o.tol * fnorm, o.eta * host[0]);
      if (host[0] <= target || total >= o.max_iter) {
        conv = host[0] <= target;
        break;
      }
      // With lowp each restart cycle is one step of iterative refinement: the
      // cycle's products run on the BF16 matrix cores and it ends once its own
      // residual estimate fell by inner_tol_lp; the FP64 residual of the next
      // restart decides convergence.
      const double cycle_tgt = o.lowp ? std::max(target, o.inner_tol_lp * host[0]) : target;
      bool cycle_done = false;
      // Arnoldi steps; the residual estimates are read back every kCheck
      // steps and the solution uses the first step that met the target.
      constexpr int kCheck = 4;
      int j = 0;
      while (j < m && total < o.max_iter && !cycle_done) {
        const int j0 = j;
        for (int q = 0; q < kCheck && j < m && total < o.max_iter; ++q, ++j, ++total) {
          if (o.lowp)
            local_apply_lp(s, op, V + (int64_t)j * N, V + (int64_t)(j + 1) * N, 1.0, 0.0, T1, T2,
                           o.lowp == 3);
          else
            local_apply(s, op, V + (int64_t)j * N, V + (int64_t)(j + 1) * N, 1.0, 0.0, T1, T2);
          arnoldi_mwg(s, V, N, j, Hc, m + 1, cs, sn, g, resv, awork);
        }
        double est[kCheck];
        TT_HIP(hipMemcpyAsync(est, resv + j0, (j - j0) * sizeof(double), hipMemcpyDeviceToHost, s));
        TT_HIP(hipStreamSynchronize(s));
        for (int q = 0; q < j - j0; ++q)
          if (est[q] <= cycle_tgt) {
            total -= (j - j0) - (q + 1);
            j = j0 + q + 1;
            cycle_done = true;
            break;
          }
      }
      if (cycle_done && !o.lowp) conv = true;
      gmres_update(s, V, N, j, Hc, m + 1, g, x);
      if (conv || (total >= o.max_iter && !o.lowp)) break;
    }
    res.iterations = total;
    res.converged = conv;
  }
  if (final_res) {
    double* y = ws.d(N);
    local_apply(s, op, x, y, 1.0, 0.0, T1, T2);
    rel_res(s, y, f, N, scal + 3);
    double h = 0.0;
    TT_HIP(hipMemcpyAsync(&h, scal + 3, sizeof(double), hipMemcpyDeviceToHost, s));
    TT_HIP(hipStreamSynchronize(s));
    res.rel_res = h;
    if (res.method == 2 || res.method == 4) res.converged = h <= o.tol * 10.0 || res.converged;
  }
  return res;
}

}  // namespace ttnt
