// extern "C" entry points of libttnt.so (declared in include/ttnt.h).
#include <algorithm>
#include <optional>
#include <thread>
#include <cmath>
#include <exception>
#include <mutex>
#include <string>

#include "engine.h"
#include "krylov.h"
#include "kernels.h"
#include "solver.h"
#include "ttk.h"

using namespace ttnt;

struct tt_solver_s {
  Solver impl;
};

namespace {

thread_local std::string g_err;

template <class F>
tt_status guard(F&& f) {
  try {
    f();
    return TT_OK;
  } catch (const CapacityError& e) {
    g_err = e.msg;
    return TT_E_CAPACITY;
  } catch (const ArgError& e) {
    g_err = e.msg;
    return TT_E_ARG;
  } catch (const HipError& e) {
    g_err = std::string("HIP error '") + hipGetErrorString(e.err) + "' in " + e.where;
    return TT_E_HIP;
  } catch (const NoConvError&) {
    g_err = "iteration limit reached before the tolerance";
    return TT_E_NOCONV;
  } catch (const NumericError&) {
    g_err = "non-finite value detected";
    return TT_E_NUMERIC;
  } catch (const std::exception& e) {
    g_err = e.what();
    return TT_E_ARG;
  } catch (...) {
    g_err = "unknown failure";
    return TT_E_ARG;
  }
}

void check_vec(const tt_vec* v, const char* name) {
  const std::string nm(name);
  TT_REQUIRE(v != nullptr, nm + " is NULL");
  TT_REQUIRE(v->d >= 1, nm + ": d must be >= 1");
  TT_REQUIRE(v->n && v->r && v->rcap && v->off && v->data, nm + ": NULL field");
  TT_REQUIRE(v->r[0] == 1 && v->r[v->d] == 1, nm + ": boundary ranks must be 1");
  for (int k = 0; k < v->d; ++k) TT_REQUIRE(v->n[k] >= 1, nm + ": mode size < 1");
  for (int k = 0; k <= v->d; ++k) {
    TT_REQUIRE(v->r[k] >= 1, nm + ": rank < 1");
    TT_REQUIRE(v->rcap[k] >= v->r[k], nm + ": rank exceeds its capacity");
  }
}

void check_mat(const tt_mat* m, const char* name) {
  const std::string nm(name);
  TT_REQUIRE(m != nullptr, nm + " is NULL");
  TT_REQUIRE(m->d >= 1, nm + ": d must be >= 1");
  TT_REQUIRE(m->m && m->n && m->R && m->off && m->data, nm + ": NULL field");
  TT_REQUIRE(m->R[0] == 1 && m->R[m->d] == 1, nm + ": boundary ranks must be 1");
  for (int k = 0; k < m->d; ++k) TT_REQUIRE(m->m[k] >= 1 && m->n[k] >= 1, nm + ": mode size < 1");
  for (int k = 0; k <= m->d; ++k) TT_REQUIRE(m->R[k] >= 1, nm + ": rank < 1");
}

LocalOp local_op_from(const tt_local* sys) {
  LocalOp op{};
  op.phiL = sys->phiL;
  op.ra = op.rb = sys->ra;
  op.RL = sys->RL;
  op.A = sys->A;
  op.m = sys->m;
  op.n = sys->n;
  op.RR = sys->RR;
  op.phiR = sys->phiR;
  op.rc = op.rd = sys->rc;
  return op;
}

LocalSolveOpts solve_opts_from(const tt_solve_opts* o) {
  LocalSolveOpts so;
  if (o) {
    so.method = o->method;
    so.tol = o->tol > 0 ? o->tol : 1e-12;
    so.max_iter = o->max_iter > 0 ? o->max_iter : 1000;
    so.restart = o->restart > 0 ? o->restart : 80;
    so.direct_max = o->direct_max >= 0 ? o->direct_max : 256;
    TT_REQUIRE(o->precision >= 0 && o->precision <= 3, "precision must be 0, 1, 2 or 3");
    so.mixed = o->precision >= 1;
    so.lowp = o->precision >= 2 ? o->precision : 0;
  }
  return so;
}

void local_solve_impl(const tt_local* sys, double* x, const tt_solve_opts* opts,
                      tt_solve_info* info, void* ws, size_t ws_bytes, hipStream_t s) {
  TT_REQUIRE(sys && x && ws, "NULL system, x or workspace");
  TT_REQUIRE(sys->phiL && sys->A && sys->phiR && sys->f, "NULL field in system");
  TT_REQUIRE(sys->ra >= 1 && sys->RL >= 1 && sys->m >= 1 && sys->n >= 1 && sys->RR >= 1 &&
                 sys->rc >= 1,
             "dimensions must be >= 1");
  TT_REQUIRE(sys->m == sys->n, "local operator must be square (m == n)");
  LocalSolveOpts so = solve_opts_from(opts);
  TT_REQUIRE(so.method >= 0 && so.method <= 4, "method must be 0, 1, 2, 3 or 4");
  if (ws_bytes < tt_local_solve_workspace(sys, opts))
    throw CapacityError{"workspace smaller than tt_local_solve_workspace"};
  Bump w;
  w.base = (char*)ws;
  w.cap = ws_bytes;
  double* Ap = w.d((size_t)sys->RL * sys->m * sys->n * sys->RR);
  permute_op(s, sys->A, sys->RL, sys->m, sys->n, sys->RR, Ap);
  LocalOp op = local_op_from(sys);
  op.Ap = Ap;
  op.diag = so.method == 3;
  LocalSolveResult r = local_solve(s, op, sys->f, x, so, w, true);
  if (info) {
    info->iterations = r.iterations;
    info->method_used = r.method;
    info->rel_res = r.rel_res;
  }
  if (!std::isfinite(r.rel_res)) throw NumericError{};
  if (!r.converged) throw NoConvError{};
}

// Static scratch of the allocation-free local solve.  Each device holds its
// own copy for the life of the process; its address there is looked up once
// per device (the array's name is not a device address in host code).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
__device__ __align__(256) char scratch[kNoAllocScratchBytes];

void* noalloc_scratch() {
  constexpr int kMaxDev = 64;
  static void* ptr[kMaxDev] = {};
  static std::mutex mu;
  int dev = 0;
  TT_HIP(hipGetDevice(&dev));
  TT_REQUIRE(dev >= 0 && dev < kMaxDev, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    TT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    TT_REQUIRE(p != nullptr, "static scratch has no device address");
    ptr[dev] = p;
  }
  return ptr[dev];
}

}  // namespace

extern "C" {

int32_t ttnt_version(void) { return 10000; }

const char* tt_last_error(void) { return g_err.c_str(); }

tt_status tt_matvec(const tt_mat* A, const tt_vec* x, tt_vec* y, tt_stream stream) {
  return guard([&] {
    check_mat(A, "A");
    check_vec(x, "x");
    TT_REQUIRE(y && y->n && y->r && y->rcap && y->off && y->data, "y: NULL field");
    TT_REQUIRE(A->d == x->d && y->d == A->d, "core counts differ");
    for (int k = 0; k < A->d; ++k) {
      TT_REQUIRE(A->n[k] == x->n[k], "A column modes differ from x modes");
      TT_REQUIRE(y->n[k] == A->m[k], "y modes differ from A row modes");
    }
    for (int k = 0; k <= A->d; ++k)
      if (y->rcap[k] < A->R[k] * x->r[k]) throw CapacityError{"y capacity below R_k * r_k"};
    TTm a = view(A);
    TTv xv = view(x);
    TTv yv;
    yv.d = y->d;
    yv.n.assign(y->n, y->n + y->d);
    yv.r.assign(y->d + 1, 1);
    yv.rcap.assign(y->rcap, y->rcap + y->d + 1);
    yv.data = y->data;
    yv.off.assign(y->off, y->off + y->d);
    matvec((hipStream_t)stream, a, xv, yv);
    for (int k = 0; k <= A->d; ++k) y->r[k] = yv.r[k];
  });
}

size_t tt_round_workspace(const tt_vec* x) {
  if (!x || x->d < 1 || !x->r || !x->n) return 0;
  TTv t;
  t.d = x->d;
  t.n.assign(x->n, x->n + x->d);
  t.r.assign(x->r, x->r + x->d + 1);
  return round_ws_bytes(t);
}

tt_status tt_round(tt_vec* x, double tol, int32_t rmax, double* rel_err, void* ws,
                   size_t ws_bytes, tt_stream stream) {
  return guard([&] {
    check_vec(x, "x");
    TT_REQUIRE(tol >= 0.0 && std::isfinite(tol), "tol must be finite and >= 0");
    TT_REQUIRE(rmax >= 1, "rmax must be >= 1");
    TT_REQUIRE(ws != nullptr, "workspace is NULL");
    TTv t = view(x);
    if (ws_bytes < round_ws_bytes(t)) throw CapacityError{"workspace smaller than tt_round_workspace"};
    Bump b;
    b.base = (char*)ws;
    b.cap = ws_bytes;
    const size_t fact = fact_doubles_for(t);
    FactScope fs(b.d(fact), fact);
    round_tt((hipStream_t)stream, t, tol, rmax, rel_err, b);
    TT_HIP(hipStreamSynchronize((hipStream_t)stream));
    for (int k = 0; k <= x->d; ++k) x->r[k] = t.r[k];
  });
}

tt_status tt_orth_right(tt_vec* x, void* ws, size_t ws_bytes, tt_stream stream) {
  return guard([&] {
    check_vec(x, "x");
    TT_REQUIRE(ws != nullptr, "workspace is NULL");
    TTv t = view(x);
    if (ws_bytes < round_ws_bytes(t)) throw CapacityError{"workspace smaller than tt_round_workspace"};
    Bump b;
    b.base = (char*)ws;
    b.cap = ws_bytes;
    const size_t fact = fact_doubles_for(t);
    FactScope fs(b.d(fact), fact);
    orth_right((hipStream_t)stream, t, b);
    TT_HIP(hipStreamSynchronize((hipStream_t)stream));
    for (int k = 0; k <= x->d; ++k) x->r[k] = t.r[k];
  });
}

size_t tt_dot_workspace(const tt_vec* a, const tt_vec* b) {
  if (!a || !b || a->d < 1 || a->d != b->d) return 0;
  TTv ta, tb;
  ta.d = tb.d = a->d;
  ta.n.assign(a->n, a->n + a->d);
  ta.r.assign(a->r, a->r + a->d + 1);
  tb.n = ta.n;
  tb.r.assign(b->r, b->r + b->d + 1);
  return dot_ws_bytes(ta, tb) + 256;
}

tt_status tt_dot(const tt_vec* a, const tt_vec* b, double* result, void* ws, size_t ws_bytes,
                 tt_stream stream) {
  return guard([&] {
    check_vec(a, "a");
    check_vec(b, "b");
    TT_REQUIRE(a->d == b->d, "core counts differ");
    for (int k = 0; k < a->d; ++k) TT_REQUIRE(a->n[k] == b->n[k], "modes differ");
    TT_REQUIRE(result && ws, "NULL result or workspace");
    TTv ta = view(a), tb = view(b);
    if (ws_bytes < dot_ws_bytes(ta, tb) + 256) throw CapacityError{"workspace smaller than tt_dot_workspace"};
    Bump w;
    w.base = (char*)ws;
    w.cap = ws_bytes;
    double* out = w.d(1);
    dot_tt((hipStream_t)stream, ta, tb, out, w);
    TT_HIP(hipMemcpyAsync(result, out, sizeof(double), hipMemcpyDeviceToHost, (hipStream_t)stream));
    TT_HIP(hipStreamSynchronize((hipStream_t)stream));
  });
}

size_t tt_local_solve_workspace(const tt_local* sys, const tt_solve_opts* opts) {
  if (!sys) return 0;
  LocalOp op = local_op_from(sys);
  LocalSolveOpts so = solve_opts_from(opts);
  const size_t ap = (size_t)sys->RL * sys->m * sys->n * sys->RR;
  return (local_solve_ws_doubles(op, so) + ap + 64) * sizeof(double) + 8192;
}

size_t tt_local_apply_workspace(const tt_local* sys) {
  if (!sys) return 0;
  const size_t ap = (size_t)sys->RL * sys->m * sys->n * sys->RR;
  const size_t t1 = (size_t)sys->ra * sys->RL * sys->n * sys->rc;
  const size_t t2 = (size_t)sys->ra * sys->m * sys->RR * sys->rc;
  return (ap + t1 + t2 + 3 * 64) * sizeof(double) + 1024;
}

tt_status tt_local_apply(const tt_local* sys, const double* x, double* y, int32_t precision,
                         void* ws, size_t ws_bytes, tt_stream stream) {
  return guard([&] {
    TT_REQUIRE(sys && x && y && ws, "NULL system, x, y or workspace");
    TT_REQUIRE(sys->phiL && sys->A && sys->phiR, "NULL field in system");
    TT_REQUIRE(sys->ra >= 1 && sys->RL >= 1 && sys->m >= 1 && sys->n >= 1 && sys->RR >= 1 &&
                   sys->rc >= 1,
               "dimensions must be >= 1");
    TT_REQUIRE(precision == 0 || precision == 2 || precision == 3,
               "precision must be 0 (FP64), 2 (BF16) or 3 (FP16)");
    if (ws_bytes < tt_local_apply_workspace(sys))
      throw CapacityError{"workspace smaller than tt_local_apply_workspace"};
    hipStream_t s = (hipStream_t)stream;
    Bump w;
    w.base = (char*)ws;
    w.cap = ws_bytes;
    double* Ap = w.d((size_t)sys->RL * sys->m * sys->n * sys->RR);
    double* T1 = w.d((size_t)sys->ra * sys->RL * sys->n * sys->rc);
    double* T2 = w.d((size_t)sys->ra * sys->m * sys->RR * sys->rc);
    permute_op(s, sys->A, sys->RL, sys->m, sys->n, sys->RR, Ap);
    LocalOp op = local_op_from(sys);
    op.Ap = Ap;
    if (precision >= 2)
      local_apply_lp(s, op, x, y, 1.0, 0.0, T1, T2, precision == 3);
    else
      local_apply(s, op, x, y, 1.0, 0.0, T1, T2);
    TT_HIP(hipStreamSynchronize(s));
  });
}

tt_status tt_local_solve(const tt_local* sys, double* x, const tt_solve_opts* opts,
                         tt_solve_info* info, void* ws, size_t ws_bytes, tt_stream stream) {
  return guard([&] { local_solve_impl(sys, x, opts, info, ws, ws_bytes, (hipStream_t)stream); });
}

tt_status tt_local_solve_noalloc(const tt_local* sys, double* x, const tt_solve_opts* opts,
                                 tt_solve_info* info, tt_stream stream) {
  return guard([&] {
    TT_REQUIRE(sys != nullptr, "NULL system");
    const size_t need = tt_local_solve_workspace(sys, opts);
    if (need > kNoAllocScratchBytes)
      throw CapacityError{"system needs " + std::to_string(need) +
                          " bytes of workspace, above the static scratch of " +
                          std::to_string(kNoAllocScratchBytes)};
    local_solve_impl(sys, x, opts, info, noalloc_scratch(), kNoAllocScratchBytes,
                     (hipStream_t)stream);
  });
}

tt_status ttnt_release(void) {
  return guard([&] {
    TT_HIP(hipDeviceSynchronize());
    release_thread_resources();
  });
}

tt_status ttnt_set_grid_wait_limit(double seconds) {
  return guard([&] {
    TT_REQUIRE(seconds == seconds, "seconds is NaN");
    krylov_set_wait_limit(seconds);
  });
}

namespace {

void check_problem(const tt_problem* problem) {
  check_mat(&problem->H, "H");
  check_mat(&problem->SF, "SF");
  check_vec(&problem->cF, "cF");
  check_vec(&problem->psi0, "psi0");
}

tt_status solver_create(const tt_problem* problem, const tt_solver_opts* opts, void* ws,
                        size_t ws_bytes, tt_solver** out) {
  return guard([&] {
    TT_REQUIRE(problem && opts && out, "NULL argument");
    check_problem(problem);
    auto* s = new tt_solver_s();
    try {
      s->impl.create(problem, opts, ws, ws_bytes);
    } catch (...) {
      delete s;
      throw;
    }
    *out = s;
  });
}

}  // namespace

tt_status tt_solver_create(const tt_problem* problem, const tt_solver_opts* opts,
                           tt_solver** out) {
  return solver_create(problem, opts, nullptr, 0, out);
}

tt_status ttnt_set_grid_cap(int32_t cap) {
  return guard([&] {
    TT_REQUIRE(cap >= 0, "cap must be >= 0");
    krylov_set_thread_cap(cap);
  });
}

tt_status tt_power_step_async(tt_solver* s, int32_t sweeps, tt_step_info* device_info,
                              tt_stream stream) {
  return guard([&] {
    TT_REQUIRE(s && device_info, "NULL argument");
    TT_REQUIRE(sweeps >= 0, "sweeps must be >= 0");
    s->impl.step_async((hipStream_t)stream, sweeps, device_info);
  });
}

tt_status tt_solver_workspace_size(const tt_problem* problem, const tt_solver_opts* opts,
                                   size_t* bytes) {
  return guard([&] {
    TT_REQUIRE(problem && opts && bytes, "NULL argument");
    check_problem(problem);
    Solver probe_only;
    probe_only.create(problem, opts, nullptr, 0, bytes);
  });
}

tt_status tt_solver_create_in(const tt_problem* problem, const tt_solver_opts* opts,
                              void* workspace, size_t workspace_bytes, tt_solver** out) {
  if (!workspace) {
    g_err = "workspace is NULL";
    return TT_E_ARG;
  }
  return solver_create(problem, opts, workspace, workspace_bytes, out);
}

tt_status tt_amen_mv(const tt_mat* A, const tt_vec* x, tt_vec* y, double tol, int32_t rmax,
                     int32_t max_sweeps, tt_step_info* info, tt_stream stream) {
  tt_status st = guard([&] {
    check_mat(A, "A");
    check_vec(x, "x");
    TT_REQUIRE(y && y->n && y->r && y->rcap && y->off && y->data, "y: NULL field");
    TT_REQUIRE(A->d == x->d && y->d == A->d, "core counts differ");
    for (int k = 0; k < A->d; ++k) {
      TT_REQUIRE(A->m[k] == A->n[k], "A must be square in every mode");
      TT_REQUIRE(A->n[k] == x->n[k] && y->n[k] == A->m[k], "modes differ");
    }
    TT_REQUIRE(tol > 0.0 && rmax >= 1 && max_sweeps >= 1, "bad tolerance, rank cap or sweeps");
    const int d = A->d;
    hipStream_t hs = (hipStream_t)stream;
    // identity operator (the "H" of the projected product) and a zero F part
    std::vector<int> ones(d + 1, 1);
    std::vector<int64_t> ioff(d, 0);
    std::vector<double> hid;
    for (int k = 0; k < d; ++k) {
      ioff[k] = (int64_t)hid.size();
      for (int i = 0; i < A->n[k]; ++i)
        for (int j = 0; j < A->n[k]; ++j) hid.push_back(i == j ? 1.0 : 0.0);
    }
    const size_t f0n = (size_t)A->R[0] * A->m[0] * A->n[0] * A->R[1];
    double* tmp = nullptr;
    TT_HIP(hipMalloc(&tmp, (hid.size() + f0n) * sizeof(double)));
    struct Free {
      double* p;
      ~Free() { if (p) (void)hipFree(p); }
    } guard_tmp{tmp};
    TT_HIP(hipMemcpy(tmp, hid.data(), hid.size() * sizeof(double), hipMemcpyHostToDevice));
    TT_HIP(hipMemset(tmp + hid.size(), 0, f0n * sizeof(double)));
    tt_problem prob{};
    prob.H = tt_mat{d, A->n, A->n, ones.data(), tmp, ioff.data()};
    prob.SF = *A;
    prob.F_core0 = tmp + hid.size();
    prob.cF = *x;
    prob.psi0 = *x;
    prob.k0 = 1.0;
    tt_solver_opts o{};
    o.tol = tol;
    o.rmax = rmax;
    o.kick = 4;
    o.max_sweeps = max_sweeps;
    o.rhs_mode = 0;
    o.gmres_restart = 40;
    o.gmres_max_iter = 200;
    o.direct_max = 256;
    Solver sv;
    sv.product_only = true;
    sv.create(&prob, &o);
    const TTv& p = sv.psi;
    sv.step(hs, info);
    for (int k = 0; k <= d; ++k)
      if (y->rcap[k] < p.r[k]) throw CapacityError{"y capacity below the ranks of the product"};
    for (int k = 0; k < d; ++k) copy(hs, p.core(k), y->data + y->off[k], p.size(k));
    for (int k = 0; k <= d; ++k) y->r[k] = p.r[k];
    TT_HIP(hipStreamSynchronize(hs));
  });
  if (st == TT_OK && info && info->status == TT_E_NOCONV) return TT_E_NOCONV;
  return st;
}

tt_status tt_power_step(tt_solver* s, tt_step_info* info, tt_stream stream) {
  tt_status st = guard([&] {
    TT_REQUIRE(s != nullptr, "NULL solver");
    s->impl.step((hipStream_t)stream, info);
  });
  if (st == TT_OK && info && info->status == TT_E_NOCONV) return TT_E_NOCONV;
  return st;
}

tt_status tt_power_step_batched(tt_solver** solvers, int32_t count, tt_step_info* infos,
                                const tt_stream* streams, int32_t nstreams) {
  std::vector<tt_status> st;
  std::vector<std::string> msg;
  tt_status top = guard([&] {
    TT_REQUIRE(count >= 0, "count must be >= 0");
    if (count == 0) return;
    TT_REQUIRE(solvers && infos && streams, "NULL argument");
    TT_REQUIRE(nstreams >= 1, "nstreams must be >= 1");
    std::vector<const tt_solver*> seen(solvers, solvers + count);
    for (const tt_solver* p : seen) TT_REQUIRE(p != nullptr, "NULL solver in the batch");
    std::sort(seen.begin(), seen.end());
    TT_REQUIRE(std::adjacent_find(seen.begin(), seen.end()) == seen.end(),
               "a solver appears twice in the batch");
    int dev = 0, cus = 0;
    TT_HIP(hipGetDevice(&dev));
    TT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int lanes = std::min<int>(nstreams, count);
    // largest estimated step cost first
    std::vector<double> cost(count);
    for (int i = 0; i < count; ++i) cost[i] = solvers[i]->impl.step_cost();
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    st.assign(count, TT_OK);
    msg.assign(count, std::string());

    // One host thread keeps up to `lanes` steps in flight, one per stream,
    // and resumes whichever step's device synchronization has completed.
    struct Lane {
      int idx = -1;
      std::optional<Co> task;
    };
    std::vector<Lane> lane(lanes);
    struct CapScope {
      explicit CapScope(int c) { krylov_set_thread_cap(c); }
      ~CapScope() { krylov_set_thread_cap(0); }
    } cap_scope(std::max(1, cus / lanes));
    auto finish = [&](int l, tt_status code) {
      const int idx = lane[l].idx;
      if (code == TT_OK && infos[idx].status == TT_E_NOCONV) code = TT_E_NOCONV;
      st[idx] = code;
      if (code != TT_OK && code != TT_E_NOCONV) msg[idx] = g_err;
      lane[l].task.reset();
      lane[l].idx = -1;
    };
    // resume lane l's task once; returns true while it is still running
    auto advance = [&](int l) {
      Solver& sv = solvers[lane[l].idx]->impl;
      bool done = false;
      const tt_status code = guard([&] {
        sv.enter();
        try {
          done = resume_task(*lane[l].task, sv.slot);
        } catch (...) {
          sv.leave();
          throw;
        }
        sv.leave();
      });
      if (code != TT_OK || done) {
        finish(l, code);
        return false;
      }
      return true;
    };
    int next = 0, running = 0;
    for (;;) {
      for (int l = 0; l < lanes && next < count; ++l) {
        if (lane[l].idx >= 0) continue;
        lane[l].idx = order[next++];
        Solver& sv = solvers[lane[l].idx]->impl;
        sv.slot.resume = nullptr;
        lane[l].task.emplace(sv.step_co((hipStream_t)streams[l], &infos[lane[l].idx]));
        ++running;
        if (!advance(l)) --running;
      }
      if (running == 0 && next >= count) break;
      bool progressed = false;
      for (int l = 0; l < lanes; ++l) {
        if (lane[l].idx < 0) continue;
        const hipError_t q = hipEventQuery(solvers[lane[l].idx]->impl.slot.ev);
        if (q == hipErrorNotReady) continue;
        progressed = true;
        if (q != hipSuccess) {
          g_err = std::string("event query failed: ") + hipGetErrorString(q);
          finish(l, TT_E_HIP);
          --running;
          continue;
        }
        if (!advance(l)) --running;
      }
      if (!progressed) std::this_thread::yield();
    }
  });
  if (top != TT_OK) return top;
  tt_status worst = TT_OK;
  for (size_t i = 0; i < st.size(); ++i) {
    const tt_status x = st[i];
    if (x != TT_OK && (worst == TT_OK || worst == TT_E_NOCONV)) {
      worst = x;
      if (x != TT_E_NOCONV) g_err = "batch instance " + std::to_string(i) + ": " + msg[i];
    }
  }
  return worst;
}

tt_status tt_solver_get_psi(tt_solver* s, tt_vec* out, tt_stream stream) {
  return guard([&] {
    TT_REQUIRE(s && out && out->n && out->r && out->rcap && out->off && out->data, "NULL argument");
    const TTv& p = s->impl.psi;
    TT_REQUIRE(out->d == p.d, "core count differs");
    for (int k = 0; k < p.d; ++k) TT_REQUIRE(out->n[k] == p.n[k], "modes differ");
    for (int k = 0; k <= p.d; ++k)
      if (out->rcap[k] < p.r[k]) throw CapacityError{"output capacity below the flux ranks"};
    for (int k = 0; k < p.d; ++k) copy((hipStream_t)stream, p.core(k), out->data + out->off[k], p.size(k));
    for (int k = 0; k <= p.d; ++k) out->r[k] = p.r[k];
    TT_HIP(hipStreamSynchronize((hipStream_t)stream));
  });
}

tt_status tt_solver_ranks(tt_solver* s, int32_t* ranks, int32_t* d) {
  return guard([&] {
    TT_REQUIRE(s && ranks && d, "NULL argument");
    *d = s->impl.d;
    for (int k = 0; k <= s->impl.d; ++k) ranks[k] = s->impl.psi.r[k];
  });
}

int64_t tt_solver_launches(tt_solver* s) { return s ? s->impl.last_launches : -1; }

tt_status tt_solver_set_probe(tt_solver* s, int32_t on) {
  return guard([&] {
    TT_REQUIRE(s != nullptr, "NULL solver");
    s->impl.probe.active = on != 0;
    s->impl.probe.reset();
  });
}

tt_status tt_solver_probe_stats(tt_solver* s, int32_t kernel_class, tt_probe_stats* out) {
  return guard([&] {
    TT_REQUIRE(s && out, "NULL argument");
    TT_REQUIRE(kernel_class >= 0 && kernel_class < kProbeClasses, "kernel_class out of range");
    const Probe& p = s->impl.probe;
    out->launches = p.n[kernel_class];
    out->total_ms = p.ms[kernel_class];
    out->flops = p.fl[kernel_class];
    out->bytes = p.by[kernel_class];
    out->dropped = (int64_t)p.dropped;
  });
}

tt_status tt_solver_destroy(tt_solver* s) {
  delete s;
  return TT_OK;
}

}  // extern "C"
