// Persistent restarted GMRES for the local systems of the alternating solver.
#pragma once

#include "common.h"

namespace ttnt {

// Local operator PhiL (x) A (x) PhiR of a square local system: PhiL is
// [r0][RL][r0], the permuted core Ap is [(i, RR), (RL, j)] with i, j < n, and
// PhiR is [r1][RR][r1]; the unknown is [r0][n][r1].
struct KrylovShape {
  int r0, RL, n, RR, r1;
};

// Largest grid of the persistent kernel (workgroups of 256 threads); each
// workgroup owns ceil(r0 / grid) left-rank slices.  TTNT_KRYLOV_GRID overrides.
constexpr int kKrylovMaxGrid = 256;

// Grid cap in use (kKrylovMaxGrid unless overridden).
int krylov_grid();
// Caps the grid of persistent solves issued by the calling host thread (0
// restores the default).  Concurrent solves on several streams keep the sum
// of their grids within the compute-unit count, so that all of them can be
// resident at once.
void krylov_set_thread_cap(int cap);
// Restart length the persistent solver uses for `restart` (smaller when the
// LDS-resident basis would not fit), 0 when the shape is not supported.
int krylov_restart(const KrylovShape& sh, int restart, bool mixed = false);
// Whether local GMRES solves use the persistent kernel (default on; the
// environment variable TTNT_KRYLOV=0 selects the multi-launch path).
bool krylov_enabled();
// True when the persistent solver handles this shape on the current device
// (queries the device).
bool krylov_fits(const KrylovShape& sh, int restart, bool mixed = false);
size_t krylov_ws_doubles(const KrylovShape& sh, int restart, int grid);
// GMRES(restart) from the initial guess in x; stops when ||r|| <= max(tol ||f||,
// eta ||r_0||) or after max_iter Arnoldi steps.  info (device, 5 doubles)
// receives [iterations, converged (0/1), final residual estimate / ||f||, -,
// gave up]: info[4] is 1.0 when a workgroup gave up waiting at a grid
// barrier (the result is then invalid), else 0.0.
// mixed: the Arnoldi iterations run in FP32 and each restart cycle is one
// step of iterative refinement on the FP64 residual (a cycle ends once its
// own residual fell by inner_tol); convergence is judged on the FP64 residual.
// One cooperative launch (plus a one-element fill of the barrier counter and,
// when mixed, an FP32 copy of PhiR).  Returns true when the launch was
// bracketed by the kernel probe.
// Seconds a workgroup of the persistent kernel waits at a grid barrier before
// it gives up (default 20; applies to launches issued afterwards).
void krylov_set_wait_limit(double seconds);
bool krylov_solve(hipStream_t s, const KrylovShape& sh, const double* phiL, const double* Ap,
                  const double* phiR, const double* f, double* x, int restart, int max_iter,
                  double tol, double eta, double* ws, size_t ws_doubles, double* info, int grid,
                  bool mixed = false, double inner_tol = 1e-5);

}  // namespace ttnt
