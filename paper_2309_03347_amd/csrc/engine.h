// Host-side orchestration of the TT algorithms (rounding, alternating solve,
// power step) on top of the device kernels.
#pragma once

#include "common.h"
#include "coro.h"

namespace ttnt {

struct TTv {
  int d = 0;
  std::vector<int> n, r, rcap;
  double* data = nullptr;
  std::vector<int64_t> off;
  double* core(int k) const { return data + off[k]; }
  int64_t size(int k) const { return (int64_t)r[k] * n[k] * r[k + 1]; }
  int64_t total() const {
    int64_t t = 0;
    for (int k = 0; k < d; ++k) t += size(k);
    return t;
  }
};

struct TTm {
  int d = 0;
  std::vector<int> m, n, R;
  const double* data = nullptr;
  std::vector<int64_t> off;
  const double* core(int k) const { return data + off[k]; }
  int64_t size(int k) const { return (int64_t)R[k] * m[k] * n[k] * R[k + 1]; }
  int64_t total() const {
    int64_t t = 0;
    for (int k = 0; k < d; ++k) t += size(k);
    return t;
  }
};

// Bump allocator over device memory; with base == nullptr it only measures.
struct Bump {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  void* take(size_t bytes) {
    const size_t at = used;
    used += (bytes + 255) & ~(size_t)255;
    if (base && used > cap) throw ArgError{"workspace too small"};
    return base ? (void*)(base + at) : nullptr;
  }
  double* d(size_t count) { return (double*)take(count * sizeof(double)); }
  int* i(size_t count) { return (int*)take(count * sizeof(int)); }
};

TTv view(const tt_vec* v);
TTm view(const tt_mat* m);

// y = A x (exact), y ranks R_k r_k.
void matvec(hipStream_t s, const TTm& A, const TTv& x, TTv& y);
// Pinned host memory for values a task reads back (at least 4 ints, 4 doubles).
struct HostBuf {
  int* i;
  double* d;
};
// In-place rounding as a task (suspends once per truncated core); writes the
// relative discarded norm to *rel_err (host) if rel_err != nullptr.  With
// left_orth the caller guarantees cores 0..d-2 are already left-orthonormal
// (for example after a left-to-right alternating sweep), and the QR sweep is
// skipped.
Co round_tt_co(hipStream_t s, TTv& x, double tol, int rmax, double* rel_err, Bump& ws,
               SyncSlot& slot, HostBuf hb, bool left_orth = false);
// Frees the calling thread's event and pinned buffer used by blocking calls
// (recreated on the next such call).
void release_thread_resources();
// Blocking form of round_tt_co (synchronizes the stream).
void round_tt(hipStream_t s, TTv& x, double tol, int rmax, double* rel_err, Bump& ws);
size_t round_ws_bytes(const TTv& x);
// Tall-QR scratch (doubles, g_fact_buf) for the QR sweeps of x's cores at its
// ranks, left (r n x r') and right (n r' x r) unfoldings; at least kFactDoubles.
size_t fact_doubles_for(const TTv& x);
// <a, b> into a device scalar `out` (no synchronization).
void dot_tt(hipStream_t s, const TTv& a, const TTv& b, double* out, Bump& ws);
size_t dot_ws_bytes(const TTv& a, const TTv& b);
// Right-orthogonalize cores 1..d-1 (R->L LQ sweep).
void orth_right(hipStream_t s, TTv& x, Bump& ws);

// Structure of an operator core in its mode (row i, column j), used to skip
// work in contractions.  kind 0: general.  kind 1: diagonal,
// A[b, i, j, b'] = delta_ij Hd[b, i, b'] (the transport operator on the energy
// and angle cores).  kind 2: proportional columns, A[b, i, j, b'] =
// a[b, i, b'] w_j (the angular integral of the scattering and fission terms),
// with Arp[(i, b'), b] = a[b, i, b'].
struct ModeForm {
  int kind = 0;
  const double* Hd = nullptr;    // kind 1: [RL][n][RR]
  const double* Arp = nullptr;   // kind 2: [(n RR)][RL]
  const double* w = nullptr;     // kind 2: [n]
};

// Local operator application y = alpha * (PhiL (x) A (x) PhiR) v + beta * y.
struct LocalOp {
  const double* phiL;  // [ra][RL][rb]
  int ra, RL, rb;
  const double* Ap;    // permuted core [(i, RR), (RL, j)]
  const double* A;     // natural core [RL][m][n][RR]
  int m, n, RR;
  const double* phiR;  // [rc][RR][rd]
  int rc, rd;
  bool diag = false;   // core is diagonal in the mode (A[b, i, j, b'] = 0 for i != j)
  ModeForm form{};     // structure used by the contractions (kind 0: none)
};
void local_apply(hipStream_t s, const LocalOp& op, const double* v, double* y, double alpha,
                 double beta, double* T1, double* T2);
// The same product with its GEMMs on the BF16 (f16 false) or block-scaled FP16
// (f16 true) matrix cores, FP32 accumulation.
void local_apply_lp(hipStream_t s, const LocalOp& op, const double* v, double* y, double alpha,
                    double beta, double* T1, double* T2, bool f16);

struct LocalSolveOpts {
  int method = 0;          // 0 auto, 1 dense LU, 2 GMRES (persistent), 3 block LU, 4 GMRES (per-stage launches)
  double tol = 1e-10;      // relative residual target
  double eta = 0.0;        // GMRES also stops at ||r|| <= eta * ||r_0|| (0: off)
  int max_iter = 400;
  int restart = 60;
  int direct_max = 256;    // auto: dense LU up to this many unknowns
  int block_max = 1024;    // auto: mode-diagonal cores solved as n blocks up to this size
  bool mixed = false;      // persistent GMRES: FP32 Arnoldi, FP64 residual refinement
  double inner_tol = 1e-5; // mixed: an FP32 cycle ends once its residual fell by this factor
  bool persistent = true;  // GMRES may use the persistent kernel (false: multi-launch only)
  int lowp = 0;            // multi-launch GMRES: operator products on the matrix cores inside
                           // each restart cycle (2 BF16, 3 block-scaled FP16; 0 off), FP64
                           // residual at every restart
  double inner_tol_lp = 1e-2;  // lowp: a cycle ends once its residual fell by this factor
  // Set for solves inside a step that must not wait for the device: a
  // persistent GMRES solve copies its 5-double info there (device to device)
  // instead of reading it back, and every path that needs the host between
  // launches (the multi-launch GMRES) is refused.
  double* dev_info = nullptr;
};
struct LocalSolveResult {
  int iterations = 0;
  int method = 0;
  double rel_res = 0.0;
  bool converged = true;
  bool deferred = false;   // iterations / convergence are in the caller's defer_info
  int probe_slot = -1;     // probe bracket of a deferred persistent solve
  bool mixed = false;      // the persistent solve ran FP32 Arnoldi cycles
};
// Scratch for a local solve of N unknowns (LU and/or GMRES).
size_t local_solve_ws_doubles(const LocalOp& op, const LocalSolveOpts& o);
// Solve (PhiL (x) A (x) PhiR) x = f; x holds the initial guess.  `final_res`
// requests the final residual (one extra apply and a synchronization).
// With defer_info (pinned host, 5 doubles) a persistent GMRES solve does not
// synchronize: [iterations, converged, residual estimate, -, gave up] land
// there once the stream reaches this point, and the result is marked deferred.
LocalSolveResult local_solve(hipStream_t s, const LocalOp& op, const double* f, double* x,
                             const LocalSolveOpts& o, Bump& ws, bool final_res,
                             double* defer_info = nullptr);
// Raises the error of a persistent solve whose workgroups gave up waiting at a
// grid barrier (reported as TT_E_HIP).
[[noreturn]] void throw_barrier_abort();
// Work of a persistent GMRES solve (for the kernel probe), once its iteration
// count is known.
void krylov_probe_amend(const LocalOp& op, int restart, int iterations, int slot,
                        bool mixed = false);

}  // namespace ttnt
