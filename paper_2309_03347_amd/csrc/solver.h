// Power-iteration solver state (one instance per tt_solver handle).
#pragma once

#include "coro.h"
#include "engine.h"
#include "probe.h"

namespace ttnt {

struct NumericError {};

struct StepStats {
  int local_iters = 0;
  bool cap_hit = false;
};

struct Solver {
  // device scalars (offsets into `scal`)
  enum { KVAL = 0, DEN = 1, NUM = 2, NRM2 = 3, KINFO = 4 };

  int d = 0;
  std::vector<int> n;
  double tol = 1e-8;
  int rmax = 32, kick = 4, max_sweeps = 10, rhs_mode = 0, rhs_rmax = 1 << 30;
  LocalSolveOpts lso;
  double k_host = 1.0;
  double stall = 0.5;          // stop sweeping when the residual falls by less than this
  double cap_eta = 1e-2;       // local residual reduction while the rank cap binds
  int min_sweeps = 2;          // sweeps before the stagnation test may stop
  bool cap_bound = false;      // the rank cap bound during the previous sweep
  // Product mode: the solver computes x <- round(A x) by the same alternating
  // sweeps with H the identity (no eigenvalue update, no normalization).
  bool product_only = false;
  std::vector<char> Hdiag;
  // structure of each core in its mode, used by the contractions: H's
  // mode-diagonal cores (kind 1), S + F/k's cores with proportional columns
  // (kind 2, the angular integral); the identity operator's are general
  std::vector<char> sf_rank1;
  std::vector<int> sf_j0;
  std::vector<std::vector<double>> sf_w;       // host copies of the column weights
  std::vector<ModeForm> formH, formSF, formId;
  std::vector<double*> HdH, ArpSF, wSF;
  int64_t last_launches = 0;
  Probe probe;

  void* mem = nullptr;
  size_t mem_bytes = 0;
  bool owns_mem = true;        // false when the caller supplied the workspace

  TTm H, SF, Id, Ak;
  double *Hc = nullptr, *SFc = nullptr, *F0 = nullptr, *A0 = nullptr, *Ic = nullptr;
  std::vector<double*> ApH, ApA, ApI;
  TTv cF, psi, X, Z, B;
  std::vector<int> capPsi, capX, zr, capB, capV, capCF, RH, Rop;
  std::vector<double*> LXH, RXH, LXA, RXA, LZH, RZH, LZA, RZA;
  double *T1 = nullptr, *T2 = nullptr, *fvec = nullptr, *xloc = nullptr, *yvec = nullptr;
  double *crz = nullptr, *zc = nullptr, *U2 = nullptr, *U2w = nullptr, *Lft = nullptr;
  double *RtT = nullptr, *Sv = nullptr, *Rb = nullptr, *tau = nullptr, *tmp = nullptr;
  double* svdw = nullptr;
  size_t svd_cap = 0;
  double* lsw = nullptr;
  size_t ls_cap = 0;
  char* rw = nullptr;
  size_t rw_cap = 0;
  static constexpr size_t kSplitK = (size_t)1 << 21;   // split-K partials (doubles)
  double* splitk = nullptr;
  double* factw = nullptr;     // tall-QR scratch (g_fact_buf while the solver runs)
  size_t factw_cap = 0;        // its doubles
  double *scal = nullptr, *resarr = nullptr;
  double* kry_dev = nullptr;   // 5 per core: persistent GMRES info of the asynchronous step
  int* irank = nullptr;

  // host synchronization of the step task: its event and pinned readbacks
  SyncSlot slot;
  void* hostmem = nullptr;
  double* h_res = nullptr;    // d local residuals
  double* h_k = nullptr;      // k, k_prev
  double* h_kry = nullptr;    // 5 per core: persistent GMRES [iterations, converged, res, -, gave up]
  HostBuf hb{nullptr, nullptr};
  std::vector<char> kry_pending;
  std::vector<int> kry_slot;
  std::vector<LocalOp> kry_op;
  std::vector<char> kry_mixed;
  int64_t launch_acc = 0;

  ~Solver();
  // Sets up the solver.  With size_only the device workspace it needs is
  // stored there and nothing is allocated or copied; with ext (ext_bytes at
  // least that size, 256-byte aligned) the caller's buffer is used instead of
  // a hipMalloc and is borrowed until destruction.
  void create(const tt_problem* p, const tt_solver_opts* o, void* ext = nullptr,
              size_t ext_bytes = 0, size_t* size_only = nullptr);
  // One power step, blocking.
  void step(hipStream_t s, tt_step_info* info);
  // One power step as a task; drive it between enter() and leave().
  Co step_co(hipStream_t s, tt_step_info* info);
  // One power step at the current ranks with no host synchronization (so a
  // stream capture can record it): max_sweeps one-site alternating sweeps
  // (QR splits, no truncation or enrichment), the k update and the
  // normalization; the step information goes to device memory.
  void step_async(hipStream_t s, int sweeps, tt_step_info* device_info);
  // Bind / release this solver's thread-local context (split-K scratch,
  // kernel probe, launch counter) around each resumption of its task.
  void enter();
  void leave();
  // Rough relative cost of one step at the current ranks (orders batches).
  double step_cost() const;

 private:
  void plan(Bump& b);
  Co sweep_core_co(hipStream_t s, int k, const TTv& V, const TTm& Aop,
                   const std::vector<double*>& ApOp, const std::vector<ModeForm>& fOp,
                   StepStats& st);
  void sweep_core_async(hipStream_t s, int k, const LocalSolveOpts& lo);
};


}  // namespace ttnt
