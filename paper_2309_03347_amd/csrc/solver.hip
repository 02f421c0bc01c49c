// Power-iteration solver: AMEn solve of H psi+ = (S + F/k) psi, rounding,
// eigenvalue update (eq. TT_k_eff_fixed_points).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "engine.h"
#include "kernels.h"
#include "solver.h"
#include "probe.h"
#include "ttk.h"

namespace ttnt {
namespace {

int64_t sat_mul(int64_t a, int64_t b) {
  const int64_t lim = (int64_t)1 << 40;
  const int64_t p = a * b;
  return p > lim ? lim : p;
}

// Left interface at bond k+1 from bond k:
// out[a2, b1, c2] = sum PhiL[a, b, c] Y[a, i, a2] A[b, i, j, b1] X[c, j, c2]
void iface_left(hipStream_t s, const double* phiL, const double* Y, int ry0, int ry1,
                const double* Ap, int RL, int m, int n, int RR, const double* X, int rx0,
                int rx1, double* out, double* T1, double* T2, const ModeForm& f = ModeForm{}) {
  if (f.kind == 2) {
    // u[c, c2] = sum_j w_j X[c, j, c2]; T1[(a, b), c2] = PhiL u;
    // T2[a][(i, b1), c2] = sum_b Arp[(i, b1), b] T1[a][b, c2]
    mode_contract(s, X, rx0, n, rx1, f.w, T2);
    gemm(s, false, false, ry0 * RL, rx1, rx0, 1.0, phiL, rx0, 0, T2, rx1, 0, 0.0, T1, rx1, 0);
    gemm(s, false, false, m * RR, rx1, RL, 1.0, f.Arp, RL, 0, T1, rx1, (int64_t)RL * rx1, 0.0, T2,
         rx1, (int64_t)m * RR * rx1, ry0);
  } else {
    gemm(s, false, false, ry0 * RL, n * rx1, rx0, 1.0, phiL, rx0, 0, X, n * rx1, 0, 0.0, T1,
         n * rx1, 0);
    if (f.kind == 1)
      mode_mix(s, T1, ry0, RL, n, rx1, f.Hd, RR, T2);
    else
      gemm(s, false, false, m * RR, rx1, RL * n, 1.0, Ap, RL * n, 0, T1, rx1,
           (int64_t)RL * n * rx1, 0.0, T2, rx1, (int64_t)m * RR * rx1, ry0);
  }
  gemm(s, true, false, ry1, RR * rx1, ry0 * m, 1.0, Y, ry1, 0, T2, RR * rx1, 0, 0.0, out,
       RR * rx1, 0);
}

// Right interface at bond k from bond k+1:
// out[a, b, c] = sum Y[a, i, a2] A[b, i, j, b1] X[c, j, c2] PhiR[a2, b1, c2]
void iface_right(hipStream_t s, const double* phiR, const double* Y, int ry0, int ry1,
                 const double* Ap, int RL, int m, int n, int RR, const double* X, int rx0,
                 int rx1, double* out, double* T1, double* T2, const ModeForm& f = ModeForm{}) {
  gemm(s, false, false, ry0 * m, RR * rx1, ry1, 1.0, Y, ry1, 0, phiR, RR * rx1, 0, 0.0, T1,
       RR * rx1, 0);
  if (f.kind == 2) {
    // T2[a][b, c2] = sum_{(i, b1)} Arp[(i, b1), b] T1[a][(i, b1), c2];
    // out[(a, b), c] = sum_c2 T2[(a, b), c2] u[c, c2], u[c, c2] = sum_j w_j X[c, j, c2]
    gemm(s, true, false, RL, rx1, m * RR, 1.0, f.Arp, RL, 0, T1, rx1, (int64_t)m * RR * rx1, 0.0,
         T2, rx1, (int64_t)RL * rx1, ry0);
    mode_contract(s, X, rx0, n, rx1, f.w, T1);
    gemm(s, false, true, ry0 * RL, rx0, rx1, 1.0, T2, rx1, 0, T1, rx1, 0, 0.0, out, rx0, 0);
    return;
  }
  if (f.kind == 1)
    mode_mix_t(s, T1, ry0, n, RR, rx1, f.Hd, RL, T2);
  else
    gemm(s, true, false, RL * n, rx1, m * RR, 1.0, Ap, RL * n, 0, T1, rx1, (int64_t)m * RR * rx1,
         0.0, T2, rx1, (int64_t)RL * n * rx1, ry0);
  gemm(s, false, true, ry0 * RL, rx0, n * rx1, 1.0, T2, n * rx1, 0, X, n * rx1, 0, 0.0, out,
       rx0, 0);
}

uint64_t lcg(uint64_t& st) {
  st = st * 6364136223846793005ULL + 1442695040888963407ULL;
  return st >> 11;
}

}  // namespace

// ---------------------------------------------------------------------------
// Planning: the same routine sizes (dry run) and carves the device memory.
// ---------------------------------------------------------------------------
void Solver::plan(Bump& b) {
  const int dd = d;
  // operators: H, SF (with core 0 replaced by A0), identity, F0, permuted cores
  Hc = b.d(H.total());
  SFc = b.d(SF.total());
  F0 = b.d(SF.size(0));
  A0 = b.d(SF.size(0));
  Ic = b.d(Id.total());
  ApH.assign(dd, nullptr);
  ApA.assign(dd, nullptr);
  ApI.assign(dd, nullptr);
  for (int k = 0; k < dd; ++k) {
    ApH[k] = b.d(H.size(k));
    ApA[k] = b.d(SF.size(k));
    ApI[k] = b.d(Id.size(k));
  }
  HdH.assign(dd, nullptr);
  ArpSF.assign(dd, nullptr);
  wSF.assign(dd, nullptr);
  for (int k = 0; k < dd; ++k) {
    if (Hdiag[k]) HdH[k] = b.d((int64_t)H.R[k] * n[k] * H.R[k + 1]);
    if (sf_rank1[k]) {
      ArpSF[k] = b.d((int64_t)n[k] * SF.R[k + 1] * SF.R[k]);
      wSF[k] = b.d(n[k]);
    }
  }
  // TT vectors
  auto carve_vec = [&](TTv& v, const std::vector<int>& cap) {
    v.d = dd;
    v.n = n;
    v.rcap = cap;
    if ((int)v.r.size() != dd + 1) v.r.assign(dd + 1, 1);
    v.off.assign(dd, 0);
    int64_t tot = 0;
    for (int k = 0; k < dd; ++k) {
      v.off[k] = tot;
      tot += (int64_t)cap[k] * n[k] * cap[k + 1];
    }
    v.data = b.d(tot + 8);
  };
  carve_vec(psi, capPsi);
  carve_vec(X, capX);
  carve_vec(Z, zr);
  carve_vec(cF, capCF);
  if (rhs_mode == 1) carve_vec(B, capB);
  // interfaces
  auto carve_if = [&](std::vector<double*>& L, std::vector<double*>& R,
                      const std::vector<int>& bra, const std::vector<int>& op,
                      const std::vector<int>& ket) {
    L.assign(dd + 1, nullptr);
    R.assign(dd + 1, nullptr);
    for (int k = 0; k <= dd; ++k) {
      const int64_t sz = (int64_t)bra[k] * op[k] * ket[k] + 1;
      L[k] = b.d(sz);
      R[k] = b.d(sz);
    }
  };
  carve_if(LXH, RXH, capX, RH, capX);
  carve_if(LXA, RXA, capX, Rop, capV);
  carve_if(LZH, RZH, zr, RH, capX);
  carve_if(LZA, RZA, zr, Rop, capV);
  // scratch
  int64_t tmax = 16, coreX = 16, dimX = 16;
  for (int k = 0; k < dd; ++k) {
    const int64_t lcap = std::max(capX[k], zr[k]);
    const int64_t rcap = std::max({capX[k + 1], capV[k + 1], zr[k + 1]});
    const int64_t rop = std::max({RH[k], RH[k + 1], Rop[k], Rop[k + 1]});
    tmax = std::max(tmax, lcap * n[k] * rcap * rop);
    coreX = std::max(coreX, (int64_t)capX[k] * n[k] * capX[k + 1]);
    dimX = std::max(dimX, (int64_t)std::max(capX[k] * n[k], capX[k + 1] + kick));
  }
  T1 = b.d(tmax);
  T2 = b.d(tmax);
  fvec = b.d(coreX);
  xloc = b.d(coreX);
  yvec = b.d(coreX);
  crz = b.d(coreX + dimX * (kick + 1));
  zc = b.d(coreX + dimX * (kick + 1));
  U2 = b.d(coreX + dimX * (kick + 1));
  U2w = b.d(coreX + dimX * (kick + 1));
  Lft = b.d(coreX + dimX);
  RtT = b.d(coreX + dimX);
  Sv = b.d(dimX + 8);
  Rb = b.d(coreX + dimX * (kick + 1));
  tau = b.d(dimX + kick + 8);
  tmp = b.d(coreX + dimX * (kick + 1));
  int64_t svdn = 16;
  for (int k = 0; k < dd; ++k) {
    const int64_t rows = (int64_t)capX[k] * n[k], cols = capX[k + 1];
    const int64_t M = std::max(rows, cols), p = std::min(rows, cols);
    svdn = std::max(svdn, (int64_t)(2 * M * p + p * p + svd_work_doubles((int)M, (int)p)));
  }
  svdw = b.d(svdn + 512);
  svd_cap = (size_t)(svdn + 512) * sizeof(double);
  // local solve scratch: the larger of the LU and GMRES needs at capacity
  int64_t lsn = 16;
  for (int k = 0; k < dd; ++k) {
    LocalOp op{};
    op.ra = op.rb = capX[k];
    op.rc = op.rd = capX[k + 1];
    op.RL = RH[k];
    op.RR = RH[k + 1];
    op.m = op.n = n[k];
    LocalSolveOpts o2 = lso;
    const int64_t N = (int64_t)op.ra * op.n * op.rc;
    o2.method = 2;
    lsn = std::max(lsn, (int64_t)local_solve_ws_doubles(op, o2));
    if (Hdiag[k]) {
      const int64_t Bm = std::min<int64_t>((int64_t)op.ra * op.rc, lso.block_max);
      const int64_t t = (int64_t)op.ra * std::max(op.RL, op.RR) * n[k] * op.rd;
      lsn = std::max(lsn, 2 * t + (int64_t)op.RL * n[k] * op.RR +
                              (int64_t)op.RL * n[k] * op.rc * op.rc + (int64_t)n[k] * Bm * Bm + N +
                              4096);
    }
    if (lso.method != 2) {
      // largest dense system that can occur at this core
      o2.method = 1;
      LocalOp lo = op;
      if (N > lso.direct_max && lso.method == 0) {
        // LU only for N <= direct_max: bound rc by direct_max / (ra n) and ra by direct_max / n
        const int64_t dm = lso.direct_max;
        lo.ra = lo.rb = (int)std::min<int64_t>(op.ra, std::max<int64_t>(1, dm / n[k]));
        lo.rc = lo.rd = (int)std::min<int64_t>(op.rc, std::max<int64_t>(1, dm / n[k]));
        const int64_t Nl = std::min<int64_t>(N, dm);
        int64_t need = (int64_t)local_solve_ws_doubles(lo, o2);
        need = std::max(need, Nl * Nl + (int64_t)op.RL * n[k] * n[k] * lo.rc * lo.rc +
                                  (int64_t)lo.ra * op.RL * n[k] * lo.rc * 2 + Nl + 4096);
        lsn = std::max(lsn, need);
      } else {
        lsn = std::max(lsn, (int64_t)local_solve_ws_doubles(op, o2));
      }
    }
  }
  lsw = b.d(lsn + 64);
  ls_cap = (size_t)(lsn + 64) * sizeof(double);
  // rounding / dot / orthogonalization scratch
  {
    TTv t;
    t.d = dd;
    t.n = n;
    t.r = capX;
    size_t need = round_ws_bytes(t);
    if (rhs_mode == 1) {
      TTv tb;
      tb.d = dd;
      tb.n = n;
      tb.r = capB;
      need = std::max(need, round_ws_bytes(tb));
    }
    TTv tz;
    tz.d = dd;
    tz.n = n;
    tz.r = capCF;
    need = std::max(need, dot_ws_bytes(tz, t));
    rw = (char*)b.take(need + 4096);
    rw_cap = need + 4096;
  }
  splitk = b.d(kSplitK);
  {
    // the QR shapes of every TT the solver factors, at capacity
    factw_cap = kFactDoubles;
    for (const std::vector<int>* cap : {&capPsi, &capX, &zr, &capV}) {
      TTv t;
      t.d = dd;
      t.n = n;
      t.r = *cap;
      factw_cap = std::max(factw_cap, fact_doubles_for(t));
    }
    factw = b.d(factw_cap);
  }
  scal = b.d(64);
  resarr = b.d(dd + 8);
  kry_dev = b.d(5 * (int64_t)dd + 8);
  irank = b.i(16);
}

Solver::~Solver() {
  if (mem && owns_mem) (void)hipFree(mem);
  if (slot.ev) (void)hipEventDestroy(slot.ev);
  if (hostmem) (void)hipHostFree(hostmem);
}

void Solver::enter() {
  g_splitk_buf = splitk;
  g_splitk_cap = kSplitK;
  g_fact_buf = factw;
  g_fact_cap = factw_cap;
  g_probe = probe.active ? &probe : nullptr;
  g_launches = launch_acc;
}

void Solver::leave() {
  launch_acc = g_launches;
  g_splitk_buf = nullptr;
  g_splitk_cap = 0;
  g_fact_buf = nullptr;
  g_fact_cap = 0;
  g_probe = nullptr;
}

void Solver::create(const tt_problem* p, const tt_solver_opts* o, void* ext, size_t ext_bytes,
                    size_t* size_only) {
  TT_REQUIRE(p && o, "null problem or options");
  H = view(&p->H);
  SF = view(&p->SF);
  const TTv cf_in = view(&p->cF);
  const TTv psi_in = view(&p->psi0);
  d = H.d;
  TT_REQUIRE(d >= 1 && SF.d == d && cf_in.d == d && psi_in.d == d, "core counts differ");
  n = H.n;
  for (int k = 0; k < d; ++k) {
    TT_REQUIRE(H.m[k] == n[k] && SF.m[k] == n[k] && SF.n[k] == n[k], "operators must be square");
    TT_REQUIRE(cf_in.n[k] == n[k] && psi_in.n[k] == n[k], "vector modes differ");
  }
  TT_REQUIRE(H.R[0] == 1 && H.R[d] == 1 && SF.R[0] == 1 && SF.R[d] == 1, "boundary ranks");
  TT_REQUIRE(p->F_core0 != nullptr, "F_core0 is required");
  TT_REQUIRE(p->k0 > 0.0, "k0 must be positive");
  tol = o->tol;
  rmax = o->rmax;
  kick = o->kick;
  max_sweeps = o->max_sweeps;
  rhs_mode = o->rhs_mode;
  rhs_rmax = o->rhs_rmax > 0 ? o->rhs_rmax : (1 << 30);
  TT_REQUIRE(tol > 0.0 && rmax >= 1 && kick >= 1 && max_sweeps >= 1, "bad solver options");
  TT_REQUIRE(rhs_mode == 0 || rhs_mode == 1, "rhs_mode must be 0 or 1");
  lso.method = 0;
  lso.tol = o->local_tol > 0.0 ? o->local_tol : tol / std::sqrt((double)d);
  lso.max_iter = o->gmres_max_iter > 0 ? o->gmres_max_iter : 1000;
  lso.restart = o->gmres_restart > 0 ? o->gmres_restart : 80;
  lso.direct_max = o->direct_max >= 0 ? o->direct_max : 256;
  lso.eta = 0.0;
  TT_REQUIRE(o->precision >= 0 && o->precision <= 3, "precision must be 0, 1, 2 or 3");
  TT_REQUIRE(o->min_sweeps >= 0 && o->cap_eta >= 0.0 && o->cap_eta < 1.0 && o->stall >= 0.0 &&
                 o->stall <= 1.0,
             "bad sweep-stopping options");
  if (o->min_sweeps > 0) min_sweeps = o->min_sweeps;
  if (o->cap_eta > 0.0) cap_eta = o->cap_eta;
  if (o->stall > 0.0) stall = o->stall;
  lso.mixed = o->precision >= 1;
  lso.lowp = o->precision >= 2 ? o->precision : 0;
  TT_REQUIRE(o->krylov_path == 0 || o->krylov_path == 1, "krylov_path must be 0 or 1");
  lso.persistent = o->krylov_path == 0;
  // identity operator (explicit mode right-hand side)
  Id.d = d;
  Id.m = n;
  Id.n = n;
  Id.R.assign(d + 1, 1);
  // capacities
  std::vector<int64_t> pl(d + 1, 1), pr(d + 1, 1);
  for (int k = 0; k < d; ++k) pl[k + 1] = sat_mul(pl[k], n[k]);
  for (int k = d - 1; k >= 0; --k) pr[k] = sat_mul(pr[k + 1], n[k]);
  capPsi.assign(d + 1, 1);
  capX.assign(d + 1, 1);
  zr.assign(d + 1, 1);
  capB.assign(d + 1, 1);
  capV.assign(d + 1, 1);
  capCF = cf_in.r;
  RH = H.R;
  for (int k = 1; k < d; ++k) {
    capPsi[k] = (int)std::min<int64_t>({(int64_t)rmax, pl[k], pr[k]});
    capPsi[k] = std::max(capPsi[k], psi_in.r[k]);
    capX[k] = (int)std::min<int64_t>((int64_t)std::max(rmax, psi_in.r[k]) + kick, pl[k]);
    zr[k] = (int)std::min<int64_t>({(int64_t)kick, pl[k], pr[k]});
    capB[k] = SF.R[k] * capPsi[k];
    capV[k] = rhs_mode == 0 ? capPsi[k]
                            : (int)std::min<int64_t>({(int64_t)rhs_rmax, pl[k], pr[k],
                                                      (int64_t)capB[k]});
  }
  Rop = rhs_mode == 0 ? SF.R : Id.R;
  // mode-diagonal cores of H (the transport operator does not couple groups
  // or directions): their local systems split into independent blocks.  A
  // core counts as diagonal when its off-diagonal entries are at rounding
  // level (below 1e-13 of its largest entry), as compressed operator cores
  // are; the block solve then drops them.
  Hdiag.assign(d, false);
  for (int k = 0; k < d; ++k) {
    if (n[k] <= 2) continue;
    std::vector<double> h(H.size(k));
    TT_HIP(hipMemcpy(h.data(), H.core(k), h.size() * sizeof(double), hipMemcpyDeviceToHost));
    double amax = 0.0;
    for (double v : h) amax = std::max(amax, std::fabs(v));
    const double cut = 1e-13 * amax;
    bool diag = true;
    for (int b = 0; b < H.R[k] && diag; ++b)
      for (int i = 0; i < n[k] && diag; ++i)
        for (int j = 0; j < n[k] && diag; ++j)
          if (i != j)
            for (int c = 0; c < H.R[k + 1]; ++c)
              if (std::fabs(h[(((int64_t)b * n[k] + i) * n[k] + j) * H.R[k + 1] + c]) > cut) {
                diag = false;
                break;
              }
    Hdiag[k] = diag;
  }
  // cores of S + F/k whose columns (in the mode) are multiples of one column:
  // the angular integral sums every direction with the quadrature weights, so
  // A[b, i, j, b'] = a[b, i, b'] w_j.  Core 0 is rebuilt each step as
  // SF_0 + F_0 / k, so there both parts must share the weights.
  sf_rank1.assign(d, 0);
  sf_j0.assign(d, -1);
  sf_w.assign(d, std::vector<double>());
  auto col_form = [&](const std::vector<double>& a, int R0, int nn, int R1, int& j0,
                      std::vector<double>& w) {
    auto at = [&](int b, int i, int j, int c) {
      return a[(((int64_t)b * nn + i) * nn + j) * R1 + c];
    };
    double amax = 0.0, best = -1.0;
    for (double v : a) amax = std::max(amax, std::fabs(v));
    if (amax == 0.0) return false;
    for (int j = 0; j < nn; ++j) {
      double t = 0.0;
      for (int b = 0; b < R0; ++b)
        for (int i = 0; i < nn; ++i)
          for (int c = 0; c < R1; ++c) t += at(b, i, j, c) * at(b, i, j, c);
      if (t > best) { best = t; j0 = j; }
    }
    w.assign(nn, 0.0);
    for (int j = 0; j < nn; ++j) {
      double t = 0.0;
      for (int b = 0; b < R0; ++b)
        for (int i = 0; i < nn; ++i)
          for (int c = 0; c < R1; ++c) t += at(b, i, j, c) * at(b, i, j0, c);
      w[j] = t / best;
    }
    const double cut = 1e-13 * amax;
    for (int b = 0; b < R0; ++b)
      for (int i = 0; i < nn; ++i)
        for (int j = 0; j < nn; ++j)
          for (int c = 0; c < R1; ++c)
            if (std::fabs(at(b, i, j, c) - at(b, i, j0, c) * w[j]) > cut) return false;
    return true;
  };
  for (int k = 0; k < d && rhs_mode == 0; ++k) {
    if (n[k] <= 2) continue;
    std::vector<double> a(SF.size(k));
    TT_HIP(hipMemcpy(a.data(), SF.core(k), a.size() * sizeof(double), hipMemcpyDeviceToHost));
    int j0 = -1;
    std::vector<double> w;
    bool ok = col_form(a, SF.R[k], n[k], SF.R[k + 1], j0, w);
    if (ok && k == 0) {
      // the F part with the same weights (and reference column)
      std::vector<double> f(SF.size(0));
      TT_HIP(hipMemcpy(f.data(), p->F_core0, f.size() * sizeof(double), hipMemcpyDeviceToHost));
      int jf = -1;
      std::vector<double> wf;
      if (!col_form(f, SF.R[0], n[0], SF.R[1], jf, wf)) ok = false;
      if (ok) {
        double fmax = 0.0;
        for (double v : f) fmax = std::max(fmax, std::fabs(v));
        for (int b = 0; b < SF.R[0] && ok; ++b)
          for (int i = 0; i < n[0] && ok; ++i)
            for (int j = 0; j < n[0] && ok; ++j)
              for (int c = 0; c < SF.R[1]; ++c) {
                const double fij = f[(((int64_t)b * n[0] + i) * n[0] + j) * SF.R[1] + c];
                const double fi0 = f[(((int64_t)b * n[0] + i) * n[0] + j0) * SF.R[1] + c];
                if (std::fabs(fij - fi0 * w[j]) > 1e-13 * fmax) { ok = false; break; }
              }
      }
    }
    if (ok) {
      sf_rank1[k] = 1;
      sf_j0[k] = j0;
      sf_w[k] = w;
    }
  }
  // dry run, allocate, carve
  Bump dry;
  plan(dry);
  mem_bytes = dry.used + 4096;
  if (size_only) {
    *size_only = mem_bytes;
    return;
  }
  if (ext) {
    if (ext_bytes < mem_bytes)
      throw CapacityError{"solver workspace smaller than tt_solver_workspace_size"};
    TT_REQUIRE((reinterpret_cast<uintptr_t>(ext) & 255) == 0,
               "solver workspace must be 256-byte aligned");
    mem = ext;
    owns_mem = false;
  } else {
    TT_HIP(hipMalloc(&mem, mem_bytes));
  }
  TT_HIP(hipEventCreateWithFlags(&slot.ev, hipEventDisableTiming));
  TT_HIP(hipHostMalloc(&hostmem, (size_t)(6 * d + 32) * sizeof(double), hipHostMallocDefault));
  h_res = static_cast<double*>(hostmem);
  h_k = h_res + d;
  h_kry = h_k + 2;
  hb.d = h_kry + 5 * d;
  hb.i = reinterpret_cast<int*>(hb.d + 8);
  kry_pending.assign(d, 0);
  kry_slot.assign(d, -1);
  kry_op.assign(d, LocalOp{});
  kry_mixed.assign(d, 0);
  Bump real;
  real.base = (char*)mem;
  real.cap = mem_bytes;
  plan(real);
  hipStream_t s = nullptr;
  // operator copies
  TTm Hsrc = H, SFsrc = SF;
  auto copy_mat = [&](const TTm& src, double* dst, TTm& out) {
    int64_t off = 0;
    out = src;
    for (int k = 0; k < d; ++k) {
      copy(s, src.core(k), dst + off, src.size(k));
      out.off[k] = off;
      off += src.size(k);
    }
    out.data = dst;
  };
  copy_mat(Hsrc, Hc, H);
  copy_mat(SFsrc, SFc, SF);
  copy(s, p->F_core0, F0, SF.size(0));
  {
    std::vector<double> hid;
    int64_t off = 0;
    Id.off.assign(d, 0);
    for (int k = 0; k < d; ++k) {
      Id.off[k] = off;
      for (int i = 0; i < n[k]; ++i)
        for (int j = 0; j < n[k]; ++j) hid.push_back(i == j ? 1.0 : 0.0);
      off += (int64_t)n[k] * n[k];
    }
    TT_HIP(hipMemcpy(Ic, hid.data(), hid.size() * sizeof(double), hipMemcpyHostToDevice));
    Id.data = Ic;
  }
  for (int k = 0; k < d; ++k) {
    permute_op(s, H.core(k), H.R[k], n[k], n[k], H.R[k + 1], ApH[k]);
    permute_op(s, SF.core(k), SF.R[k], n[k], n[k], SF.R[k + 1], ApA[k]);
    permute_op(s, Id.core(k), 1, n[k], n[k], 1, ApI[k]);
  }
  // A(k) view: core 0 -> A0, others -> SF
  Ak = SF;
  Ak.off[0] = A0 - SF.data;
  formH.assign(d, ModeForm{});
  formSF.assign(d, ModeForm{});
  formId.assign(d, ModeForm{});
  for (int k = 0; k < d; ++k) {
    if (Hdiag[k]) {
      op_diag(s, H.core(k), H.R[k], n[k], H.R[k + 1], HdH[k]);
      formH[k].kind = 1;
      formH[k].Hd = HdH[k];
    }
    if (sf_rank1[k]) {
      TT_HIP(hipMemcpy(wSF[k], sf_w[k].data(), n[k] * sizeof(double), hipMemcpyHostToDevice));
      // core 0's row factor is taken from SF_0 + F_0 / k at every step
      if (k > 0) rank1_rows(s, SF.core(k), SF.R[k], n[k], SF.R[k + 1], sf_j0[k], ArpSF[k]);
      formSF[k].kind = 2;
      formSF[k].Arp = ArpSF[k];
      formSF[k].w = wSF[k];
    }
  }

  // vectors
  for (int k = 0; k < d; ++k) copy(s, cf_in.core(k), cF.core(k), cf_in.size(k));
  cF.r = cf_in.r;
  for (int k = 0; k < d; ++k) copy(s, psi_in.core(k), psi.core(k), psi_in.size(k));
  psi.r = psi_in.r;
  // random Z (fixed seed), unit interface at the chain ends
  {
    uint64_t st = 0x9E3779B97F4A7C15ULL;
    for (int k = 0; k < d; ++k) {
      const int64_t sz = (int64_t)zr[k] * n[k] * zr[k + 1];
      std::vector<double> h(sz);
      for (auto& v : h) v = ((double)(lcg(st) & 0xFFFFFF) / (double)0xFFFFFF) - 0.5;
      TT_HIP(hipMemcpy(Z.core(k), h.data(), sz * sizeof(double), hipMemcpyHostToDevice));
    }
    Z.r = zr;
    for (auto* v : {&LXH, &LXA, &LZH, &LZA}) fill(s, (*v)[0], 1, 1.0);
    for (auto* v : {&RXH, &RXA, &RZH, &RZA}) fill(s, (*v)[d], 1, 1.0);
  }
  // k and the normalized start vector
  TT_HIP(hipMemcpy(scal + KVAL, &p->k0, sizeof(double), hipMemcpyHostToDevice));
  k_host = p->k0;
  {
    Bump w;
    w.base = rw;
    w.cap = rw_cap;
    orth_right(s, psi, w);
    sumsq(s, psi.core(0), psi.size(0), scal + NRM2);
    if (!product_only) scale_inv_sqrt(s, psi.core(0), psi.size(0), scal + NRM2);
    w.used = 0;
    dot_tt(s, cF, psi, scal + DEN, w);
  }
  TT_HIP(hipDeviceSynchronize());
}

Co Solver::sweep_core_co(hipStream_t s, int k, const TTv& V, const TTm& Aop,
                         const std::vector<double*>& ApOp, const std::vector<ModeForm>& fOp,
                         StepStats& st) {
  const int rk = X.r[k], rk1 = X.r[k + 1], nk = n[k];
  const int vk = V.r[k], vk1 = V.r[k + 1];
  LocalOp xh{LXH[k], rk, RH[k], rk, ApH[k], H.core(k), nk, nk, RH[k + 1], RXH[k + 1], rk1, rk1,
             (bool)Hdiag[k]};
  LocalOp xa{LXA[k], rk, Rop[k], vk, ApOp[k], Aop.core(k), nk, nk, Rop[k + 1], RXA[k + 1], rk1, vk1};
  xh.form = formH[k];
  xa.form = fOp[k];
  const int64_t N = (int64_t)rk * nk * rk1;
  local_apply(s, xa, V.core(k), fvec, 1.0, 0.0, T1, T2);
  local_apply(s, xh, X.core(k), yvec, 1.0, 0.0, T1, T2);
  rel_res(s, yvec, fvec, N, resarr + k);
  copy(s, X.core(k), xloc, N);
  Bump lw;
  lw.base = (char*)lsw;
  lw.cap = ls_cap;
  // When the rank cap binds, the truncation error exceeds tol, so local
  // solves only need to reduce their residual by a fixed factor.
  LocalSolveOpts lo = lso;
  if (cap_bound) lo.eta = cap_eta;
  LocalSolveResult lr = local_solve(s, xh, fvec, xloc, lo, lw, false, h_kry + 5 * k);
  if (lr.deferred) {
    // iterations are read at the end of the sweep
    kry_pending[k] = 1;
    kry_slot[k] = lr.probe_slot;
    kry_op[k] = xh;
    kry_mixed[k] = lr.mixed ? 1 : 0;
  } else {
    st.local_iters += lr.iterations;
  }
  if (k == d - 1) {
    copy(s, xloc, X.core(k), N);
    co_return;
  }
  // truncated SVD of the solved core, (r_k n_k) x r_{k+1}
  const int rows = rk * nk, cols = rk1;
  Bump sw;
  sw.base = (char*)svdw;
  sw.cap = svd_cap;
  const int64_t M = std::max(rows, cols), pp = std::min(rows, cols);
  double* sG = sw.d(M * pp);
  double* sU = sw.d(M * pp);
  double* sV = sw.d(pp * pp);
  double* sWk = sw.d(svd_work_doubles((int)M, (int)pp));
  int p;
  if (rows >= cols) {
    p = cols;
    if (!svd_t(s, xloc, rows, cols, cols, 1, Lft, p, 1, Sv, RtT, 1, cols)) {
      svd(s, xloc, rows, cols, cols, Lft, p, Sv, sV, p, sWk);
      transpose(s, sV, p, p, p, RtT, cols);
    }
  } else {
    p = rows;
    if (!svd_t(s, xloc, cols, rows, 1, cols, RtT, 1, cols, Sv, Lft, p, 1)) {
      transpose(s, xloc, rows, cols, cols, sG, rows);
      svd(s, sG, cols, rows, rows, sU, rows, Sv, Lft, p, sWk);
      transpose(s, sU, cols, rows, rows, RtT, cols);
    }
  }
  trunc_rank(s, Sv, p, tol, (double)d, nullptr, rmax, irank, nullptr);
  TT_HIP(hipMemcpyAsync(hb.i, irank, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  co_await Sync{&slot, s};
  const int rt = hb.i[0];
  if (hb.i[1]) st.cap_hit = true;
  const int kz = Z.r[k + 1];
  const int w = rt + kz;
  // U2 = [u | crz]
  copy2d(s, Lft, rows, rt, p, U2, w);
  // xtr = u diag(S) v^T  (uses Lft scaled in place)
  scale_cols(s, Lft, rows, rt, p, Sv);
  gemm(s, false, false, rows, cols, rt, 1.0, Lft, p, 0, RtT, cols, 0, 0.0, yvec, cols, 0);
  // enrichment: residual projected with X on the left and Z on the right
  LocalOp za{LXA[k], rk, Rop[k], vk, ApOp[k], Aop.core(k), nk, nk, Rop[k + 1], RZA[k + 1], kz, vk1};
  LocalOp zh{LXH[k], rk, RH[k], rk, ApH[k], H.core(k), nk, nk, RH[k + 1], RZH[k + 1], kz, rk1};
  za.form = fOp[k];
  zh.form = formH[k];
  local_apply(s, za, V.core(k), crz, 1.0, 0.0, T1, T2);
  local_apply(s, zh, yvec, crz, -1.0, 1.0, T1, T2);
  copy2d(s, crz, rows, kz, kz, U2 + rt, w);
  const int q = std::min(rows, w);
  if (q > X.rcap[k + 1]) throw CapacityError{"enriched rank exceeds capacity"};
  qr(s, U2, rows, w, w, X.core(k), q, Rb, w, tau);
  // next core: (R[:, :rt] diag(S) v^T) X_{k+1}
  scale_cols(s, Rb, q, rt, w, Sv);
  gemm(s, false, false, q, cols, rt, 1.0, Rb, w, 0, RtT, cols, 0, 0.0, U2w, cols, 0);
  const int n2 = n[k + 1] * X.r[k + 2];
  gemm(s, false, false, q, n2, cols, 1.0, U2w, cols, 0, X.core(k + 1), n2, 0, 0.0, tmp, n2, 0);
  copy(s, tmp, X.core(k + 1), (int64_t)q * n2);
  // Z core update: residual projected with Z on both sides
  const int zk = Z.r[k];
  LocalOp zza{LZA[k], zk, Rop[k], vk, ApOp[k], Aop.core(k), nk, nk, Rop[k + 1], RZA[k + 1], kz, vk1};
  LocalOp zzh{LZH[k], zk, RH[k], rk, ApH[k], H.core(k), nk, nk, RH[k + 1], RZH[k + 1], kz, rk1};
  zza.form = fOp[k];
  zzh.form = formH[k];
  local_apply(s, zza, V.core(k), zc, 1.0, 0.0, T1, T2);
  local_apply(s, zzh, yvec, zc, -1.0, 1.0, T1, T2);
  qr(s, zc, zk * nk, kz, kz, Z.core(k), kz, U2w, kz, tau);
  X.r[k + 1] = q;
  // left interfaces at bond k+1
  iface_left(s, LXH[k], X.core(k), rk, q, ApH[k], RH[k], nk, nk, RH[k + 1], X.core(k), rk, q,
             LXH[k + 1], T1, T2, formH[k]);
  iface_left(s, LXA[k], X.core(k), rk, q, ApOp[k], Rop[k], nk, nk, Rop[k + 1], V.core(k), vk,
             vk1, LXA[k + 1], T1, T2, fOp[k]);
  iface_left(s, LZH[k], Z.core(k), zk, kz, ApH[k], RH[k], nk, nk, RH[k + 1], X.core(k), rk, q,
             LZH[k + 1], T1, T2, formH[k]);
  iface_left(s, LZA[k], Z.core(k), zk, kz, ApOp[k], Rop[k], nk, nk, Rop[k + 1], V.core(k), vk,
             vk1, LZA[k + 1], T1, T2, fOp[k]);
}

namespace {

// tt_step_info of the asynchronous step, formed on the device: k and k_prev
// from the k update, the largest local residual seen before a solve in the
// last sweep, the GMRES iterations summed from the per-core infos, and the
// status (TT_E_HIP when a persistent solve gave up at a grid barrier,
// TT_E_NUMERIC on a non-finite k or residual, TT_E_NOCONV when the last
// sweep's largest residual is above tol).
__global__ void step_info_kernel(const double* kinfo, const double* res, const double* kry, int d,
                                 double tol, int sweeps, int max_rank, tt_step_info* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double mr = 0.0;
  bool finite = true;
  long long iters = 0;
  bool gave_up = false;
  for (int k = 0; k < d; ++k) {
    const double r = res[k];
    if (!(r == r) || isinf(r)) finite = false;
    mr = fmax(mr, r);
    iters += (long long)kry[5 * k];
    if (kry[5 * k + 4] != 0.0) gave_up = true;
  }
  tt_step_info v;
  v.k = kinfo[0];
  v.k_prev = kinfo[1];
  v.dk = fabs(kinfo[0] - kinfo[1]);
  v.max_local_res = mr;
  v.trunc_err = 0.0;
  v.sweeps = sweeps;
  v.max_rank = max_rank;
  v.local_iters = (int32_t)iters;
  if (!(v.k == v.k) || isinf(v.k)) finite = false;
  v.status = gave_up ? TT_E_HIP : (!finite ? TT_E_NUMERIC : (mr < tol ? TT_OK : TT_E_NOCONV));
  *out = v;
}

}  // namespace

void Solver::sweep_core_async(hipStream_t s, int k, const LocalSolveOpts& lo) {
  const int rk = X.r[k], rk1 = X.r[k + 1], nk = n[k];
  const int vk = psi.r[k], vk1 = psi.r[k + 1];
  LocalOp xh{LXH[k], rk, RH[k], rk, ApH[k], H.core(k), nk, nk, RH[k + 1], RXH[k + 1], rk1, rk1,
             (bool)Hdiag[k]};
  LocalOp xa{LXA[k], rk, Rop[k], vk, ApA[k], Ak.core(k), nk, nk, Rop[k + 1], RXA[k + 1], rk1, vk1};
  xh.form = formH[k];
  xa.form = formSF[k];
  const int64_t N = (int64_t)rk * nk * rk1;
  local_apply(s, xa, psi.core(k), fvec, 1.0, 0.0, T1, T2);
  local_apply(s, xh, X.core(k), yvec, 1.0, 0.0, T1, T2);
  rel_res(s, yvec, fvec, N, resarr + k);
  copy(s, X.core(k), xloc, N);
  Bump lw;
  lw.base = (char*)lsw;
  lw.cap = ls_cap;
  LocalSolveOpts o = lo;
  o.dev_info = kry_dev + 5 * k;
  local_solve(s, xh, fvec, xloc, o, lw, false, nullptr);
  if (k == d - 1) {
    copy(s, xloc, X.core(k), N);
    return;
  }
  // one-site split: QR of the solved core, (r_k n_k) x r_{k+1}; R moves into
  // core k + 1
  const int rows = rk * nk, q = std::min(rows, rk1);
  qr(s, xloc, rows, rk1, rk1, X.core(k), q, Rb, rk1, tau);
  const int n2 = n[k + 1] * X.r[k + 2];
  gemm(s, false, false, q, n2, rk1, 1.0, Rb, rk1, 0, X.core(k + 1), n2, 0, 0.0, tmp, n2, 0);
  copy(s, tmp, X.core(k + 1), (int64_t)q * n2);
  X.r[k + 1] = q;
  iface_left(s, LXH[k], X.core(k), rk, q, ApH[k], RH[k], nk, nk, RH[k + 1], X.core(k), rk, q,
             LXH[k + 1], T1, T2, formH[k]);
  iface_left(s, LXA[k], X.core(k), rk, q, ApA[k], Rop[k], nk, nk, Rop[k + 1], psi.core(k), vk,
             vk1, LXA[k + 1], T1, T2, formSF[k]);
}

void Solver::step_async(hipStream_t s, int sweeps, tt_step_info* device_info) {
  TT_REQUIRE(rhs_mode == 0 && !product_only,
             "the asynchronous step needs the projected right-hand side of a k solve");
  TT_REQUIRE(!probe.active, "the asynchronous step runs without the kernel probe");
  if (sweeps <= 0) sweeps = max_sweeps;
  enter();
  try {
    g_launches = 0;
    // A(k) core 0 = SF_0 + F_0 / k (k read on the device)
    copy(s, F0, A0, SF.size(0));
    axpby_div(s, SF.size(0), 1.0, SF.core(0), 1.0, scal + KVAL, A0);
    permute_op(s, A0, SF.R[0], n[0], n[0], SF.R[1], ApA[0]);
    if (formSF[0].kind == 2) rank1_rows(s, A0, SF.R[0], n[0], SF.R[1], sf_j0[0], ArpSF[0]);
    fill(s, kry_dev, 5 * (int64_t)d, 0.0);
    LocalSolveOpts lo = lso;
    lo.eta = 0.0;
    Bump w;
    w.base = rw;
    w.cap = rw_cap;
    X.r = psi.r;
    for (int k = 0; k < d; ++k) copy(s, psi.core(k), X.core(k), psi.size(k));
    for (int sw = 0; sw < sweeps; ++sw) {
      // right-orthonormal cores 1..d-1, then the right interfaces
      w.used = 0;
      orth_right(s, X, w);
      for (int k = d - 1; k >= 1; --k) {
        iface_right(s, RXH[k + 1], X.core(k), X.r[k], X.r[k + 1], ApH[k], RH[k], n[k], n[k],
                    RH[k + 1], X.core(k), X.r[k], X.r[k + 1], RXH[k], T1, T2, formH[k]);
        iface_right(s, RXA[k + 1], X.core(k), X.r[k], X.r[k + 1], ApA[k], Rop[k], n[k], n[k],
                    Rop[k + 1], psi.core(k), psi.r[k], psi.r[k + 1], RXA[k], T1, T2, formSF[k]);
      }
      for (int k = 0; k < d; ++k) sweep_core_async(s, k, lo);
    }
    // psi <- X, right-orthonormal in cores 1..d-1 as every step leaves it (so
    // the norm is core 0's), then the k update and the unit-norm scaling
    psi.r = X.r;
    for (int k = 0; k < d; ++k) copy(s, X.core(k), psi.core(k), X.size(k));
    w.used = 0;
    orth_right(s, psi, w);
    w.used = 0;
    dot_tt(s, cF, psi, scal + NUM, w);
    k_update(s, scal + KVAL, scal + NUM, scal + DEN, scal + KINFO);
    sumsq(s, psi.core(0), psi.size(0), scal + NRM2);
    scale_inv_sqrt(s, psi.core(0), psi.size(0), scal + NRM2);
    scale_ratio(s, scal + NUM, scal + NRM2, scal + DEN);
    int mr = 0;
    for (int v : psi.r) mr = std::max(mr, v);
    ++g_launches;
    step_info_kernel<<<1, 64, 0, s>>>(scal + KINFO, resarr, kry_dev, d, tol, sweeps, mr,
                                      device_info);
    TT_HIP(hipGetLastError());
    last_launches = g_launches;
  } catch (...) {
    leave();
    throw;
  }
  leave();
}

double Solver::step_cost() const {
  // local operator applications dominate: n r^3 R + n^2 r^2 R^2 per core
  double c = 0.0;
  for (int k = 0; k < d; ++k) {
    const double r = std::max(psi.r[k], psi.r[k + 1]), R = std::max(RH[k], RH[k + 1]);
    c += n[k] * r * r * r * R + (double)n[k] * n[k] * r * r * R * R;
  }
  return c;
}

void Solver::step(hipStream_t s, tt_step_info* info) {
  enter();
  try {
    Co t = step_co(s, info);
    run_blocking(t, slot);
  } catch (...) {
    leave();
    throw;
  }
  leave();
}

Co Solver::step_co(hipStream_t s, tt_step_info* info) {
  g_launches = 0;
  std::fill(kry_pending.begin(), kry_pending.end(), 0);
  if (probe.active && probe.overhead_ms == 0.0) probe.calibrate(s);
  StepStats st;
  // A(k) core 0 = SF_0 + F_0 / k
  copy(s, F0, A0, SF.size(0));
  axpby_div(s, SF.size(0), 1.0, SF.core(0), 1.0, scal + KVAL, A0);
  permute_op(s, A0, SF.R[0], n[0], n[0], SF.R[1], ApA[0]);
  if (formSF[0].kind == 2) rank1_rows(s, A0, SF.R[0], n[0], SF.R[1], sf_j0[0], ArpSF[0]);
  Bump w;
  w.base = rw;
  w.cap = rw_cap;
  const TTv* V = &psi;
  const TTm* Aop = &Ak;
  const std::vector<double*>* ApOp = &ApA;
  const std::vector<ModeForm>* fOp = &formSF;
  if (rhs_mode == 1) {
    matvec(s, Ak, psi, B);
    w.used = 0;
    co_await round_tt_co(s, B, tol, rhs_rmax, nullptr, w, slot, hb);
    V = &B;
    Aop = &Id;
    ApOp = &ApI;
    fOp = &formId;
  }
  // warm start X = psi
  X.r = psi.r;
  for (int k = 0; k < d; ++k) copy(s, psi.core(k), X.core(k), psi.size(k));
  double max_res = 0.0, prev_res = 1e300;
  int sweeps = 0;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    st.cap_hit = false;
    w.used = 0;
    // psi (hence X at the first sweep) is right-orthonormal in cores 1..d-1:
    // it is orthogonalized at creation and left so by every step's rounding
    if (sw > 0) orth_right(s, X, w);
    w.used = 0;
    orth_right(s, Z, w);
    for (int k = d - 1; k >= 1; --k) {
      iface_right(s, RXH[k + 1], X.core(k), X.r[k], X.r[k + 1], ApH[k], RH[k], n[k], n[k],
                  RH[k + 1], X.core(k), X.r[k], X.r[k + 1], RXH[k], T1, T2, formH[k]);
      iface_right(s, RXA[k + 1], X.core(k), X.r[k], X.r[k + 1], (*ApOp)[k], Rop[k], n[k], n[k],
                  Rop[k + 1], V->core(k), V->r[k], V->r[k + 1], RXA[k], T1, T2, (*fOp)[k]);
      iface_right(s, RZH[k + 1], Z.core(k), Z.r[k], Z.r[k + 1], ApH[k], RH[k], n[k], n[k],
                  RH[k + 1], X.core(k), X.r[k], X.r[k + 1], RZH[k], T1, T2, formH[k]);
      iface_right(s, RZA[k + 1], Z.core(k), Z.r[k], Z.r[k + 1], (*ApOp)[k], Rop[k], n[k], n[k],
                  Rop[k + 1], V->core(k), V->r[k], V->r[k + 1], RZA[k], T1, T2, (*fOp)[k]);
    }
    for (int k = 0; k < d; ++k) co_await sweep_core_co(s, k, *V, *Aop, *ApOp, *fOp, st);
    TT_HIP(hipMemcpyAsync(h_res, resarr, d * sizeof(double), hipMemcpyDeviceToHost, s));
    co_await Sync{&slot, s};
    max_res = 0.0;
    for (int k = 0; k < d; ++k) max_res = std::max(max_res, h_res[k]);
    for (int k = 0; k < d; ++k) {
      if (!kry_pending[k]) continue;
      if (h_kry[5 * k + 4] != 0.0) throw_barrier_abort();
      const int it = (int)h_kry[5 * k];
      st.local_iters += it;
      krylov_probe_amend(kry_op[k], lso.restart, it, kry_slot[k], kry_mixed[k] != 0);
      kry_pending[k] = 0;
    }
    ++sweeps;
    if (!(max_res == max_res)) throw NumericError{};
    if (max_res < tol) break;
    cap_bound = st.cap_hit;
    // stagnation: the rank cap bound and the residual no longer falls
    if (st.cap_hit && sweeps >= min_sweeps && max_res > stall * prev_res) break;
    prev_res = max_res;
  }
  // compress the solution and update k
  double trunc = 0.0;
  w.used = 0;
  // the left-to-right sweep left cores 0..d-2 orthonormal (QR of each split)
  co_await round_tt_co(s, X, tol, rmax, &trunc, w, slot, hb, true);
  if (product_only) {
    // the rounded product replaces psi as it is (no k update, no scaling)
    psi.r = X.r;
    for (int k = 0; k < d; ++k) copy(s, X.core(k), psi.core(k), X.size(k));
    co_await Sync{&slot, s};
    if (probe.active) probe.close();
    if (info) {
      *info = tt_step_info{};
      info->max_local_res = max_res;
      info->trunc_err = trunc;
      info->sweeps = sweeps;
      int mr = 0;
      for (int v : psi.r) mr = std::max(mr, v);
      info->max_rank = mr;
      info->local_iters = st.local_iters;
      info->status = max_res < tol ? TT_OK : TT_E_NOCONV;
    }
    last_launches = g_launches;
    co_return;
  }
  w.used = 0;
  dot_tt(s, cF, X, scal + NUM, w);
  k_update(s, scal + KVAL, scal + NUM, scal + DEN, scal + KINFO);
  sumsq(s, X.core(0), X.size(0), scal + NRM2);
  scale_inv_sqrt(s, X.core(0), X.size(0), scal + NRM2);
  scale_ratio(s, scal + NUM, scal + NRM2, scal + DEN);
  psi.r = X.r;
  for (int k = 0; k < d; ++k) copy(s, X.core(k), psi.core(k), X.size(k));
  TT_HIP(hipMemcpyAsync(h_k, scal + KINFO, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  co_await Sync{&slot, s};
  const double kinfo[2] = {h_k[0], h_k[1]};
  k_host = kinfo[0];
  if (probe.active) probe.close();
  if (info) {
    info->k = kinfo[0];
    info->k_prev = kinfo[1];
    info->dk = std::fabs(kinfo[0] - kinfo[1]);
    info->max_local_res = max_res;
    info->trunc_err = trunc;
    info->sweeps = sweeps;
    int mr = 0;
    for (int v : psi.r) mr = std::max(mr, v);
    info->max_rank = mr;
    info->local_iters = st.local_iters;
    info->status = max_res < tol ? TT_OK : TT_E_NOCONV;
  }
  if (!(kinfo[0] == kinfo[0]) || !std::isfinite(kinfo[0])) throw NumericError{};
  last_launches = g_launches;
}

}  // namespace ttnt
