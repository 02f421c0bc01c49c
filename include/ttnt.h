/*
 * ttnt.h - C ABI of the MI355X tensor-train k-eigenvalue library (libttnt.so).
 *
 * The library runs, on one gfx950 GPU, the per-iteration work of the mixed
 * TT/QTT power iteration for the discretized transport eigenproblem
 *     H psi = (S + F / k) psi                          (eq. OpFormkNTE)
 * iterated as
 *     B_t      = (S + F / k_t) psi_t
 *     H psi_t+1 = B_t
 *     k_t+1    = k_t * sum(F psi_t+1) / sum(F psi_t)  (eq. TT_k_eff_fixed_points)
 * with H, S, F tensor-train (TT) matrices and psi a TT vector (Section 2.2,
 * eqs. TT-vector and TT-matrix-componentwise).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Numbers are IEEE binary64 unless a field says otherwise.
 *  - A TT vector with d cores stores core k as a dense row-major array
 *    [r_k][n_k][r_{k+1}] (last index fastest), r_0 = r_d = 1.  Core k begins
 *    at data + off[k] (element offset) and may use up to
 *    rcap[k] * n[k] * rcap[k+1] elements (its capacity slot); the core in use
 *    is packed at the start of the slot with its actual ranks r[].
 *  - A TT matrix core k is [R_k][m_k][n_k][R_{k+1}], m = row (output) mode,
 *    n = column (input) mode, packed at data + off[k].
 *  - `data` pointers are device pointers; every other pointer in a descriptor
 *    is a host pointer.  All buffers belong to the caller; entry points do
 *    not keep pointers after they return, except a tt_solver, which owns the
 *    device copies it makes at creation.
 *  - Calls are enqueued on `stream`.  Entry points that decide ranks on the
 *    device (tt_round, tt_local_solve, tt_power_step) synchronize `stream`
 *    before returning, because the chosen ranks size later launches.
 *  - Errors are returned as tt_status; nothing is thrown across the ABI.
 *    On TT_E_ARG / TT_E_CAPACITY / TT_E_DTYPE nothing is written.
 *    tt_last_error() returns a message for the last failure on this thread.
 */
#ifndef TTNT_H_
#define TTNT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tt_status;
#define TT_OK 0
#define TT_E_ARG (-1)       /* bad descriptor, shape or option */
#define TT_E_CAPACITY (-2)  /* output ranks exceed the caller's capacity */
#define TT_E_NOCONV (-3)    /* iteration limit reached; result written */
#define TT_E_NUMERIC (-4)   /* NaN or Inf detected */
#define TT_E_DTYPE (-5)     /* unsupported number type */
#define TT_E_HIP (-6)       /* HIP runtime error */

typedef struct ihipStream_t* tt_stream; /* hipStream_t; NULL = default stream */

typedef struct {
  int32_t d;             /* number of cores, >= 1 */
  const int32_t* n;      /* [d] mode sizes */
  int32_t* r;            /* [d+1] ranks; input, and output where stated */
  const int32_t* rcap;   /* [d+1] capacity ranks of the slots (rcap >= r) */
  double* data;          /* device base pointer */
  const int64_t* off;    /* [d] element offset of each core slot */
} tt_vec;

typedef struct {
  int32_t d;
  const int32_t* m;      /* [d] row (output) mode sizes */
  const int32_t* n;      /* [d] column (input) mode sizes */
  const int32_t* R;      /* [d+1] ranks, R_0 = R_d = 1 */
  const double* data;    /* device base pointer */
  const int64_t* off;    /* [d] element offset of each core */
} tt_mat;

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t ttnt_version(void);
/* Message describing the last error returned on the calling thread. */
const char* tt_last_error(void);

/*
 * tt_matvec - exact TT-matrix x TT-vector product y = A x.
 *
 * Core contraction of Oseledets' TT matrix-by-vector product (Section 2.2,
 * "Linear Operators in TT format"; the explicit exact algorithm named in
 * Section 3.3):
 *     Y_k[(b,a), i, (b',a')] = sum_j A_k[b, i, j, b'] X_k[a, j, a'],
 * so y has ranks R_k * r_k and modes m_k.  Row index (b,a) = b * r_k + a.
 * Requires A->n[k] == x->n[k] and y->n[k] == A->m[k] for every k, and
 * y->rcap[k] >= A->R[k] * x->r[k]; otherwise TT_E_ARG / TT_E_CAPACITY.
 * Writes y->r.  Asynchronous on `stream`.
 */
tt_status tt_matvec(const tt_mat* A, const tt_vec* x, tt_vec* y, tt_stream stream);

/*
 * tt_round - in-place TT rounding (rank truncation with an error bound).
 *
 * A left-to-right sweep of Householder QR factorizations (each core made
 * left-orthonormal, R pushed into the next core), then a right-to-left
 * sweep of truncated SVDs that keeps, at every bond, the fewest singular
 * values whose discarded tail has norm <= tol * ||x|| / sqrt(d-1), capped at
 * rmax.  Rank reduction after sums and products is the step named in
 * Section 2.2 ("a rank reduction step could be necessary").  Guarantees
 * ||x_in - x_out|| <= tol * ||x_in|| unless rmax binds (not an error).
 * rel_err (host, may be NULL) receives sqrt(sum of discarded sigma^2)/||x||.
 * `ws` is device workspace of at least tt_round_workspace(x) bytes.
 * Updates x->r.  Synchronizes `stream`.
 */
size_t tt_round_workspace(const tt_vec* x);
tt_status tt_round(tt_vec* x, double tol, int32_t rmax, double* rel_err, void* ws,
                   size_t ws_bytes, tt_stream stream);

/*
 * tt_orth_right - in-place right orthogonalization: a right-to-left sweep of
 * QR factorizations of the transposed unfoldings makes cores 1..d-1
 * right-orthonormal (each core's rows orthonormal over (n_k, r_{k+1})),
 * with the R factors pushed into core k-1; the tensor is unchanged (the
 * orthogonalization step of TT rounding, Section 2.2).  Ranks may shrink to
 * min(r_k, n_k r_{k+1}); x->r is updated.  `ws` at least tt_round_workspace(x)
 * bytes.  Synchronizes `stream`.
 */
tt_status tt_orth_right(tt_vec* x, void* ws, size_t ws_bytes, tt_stream stream);

/*
 * tt_dot - inner product <a, b> of two TT vectors with equal modes
 * (sequential contraction of the core pairs).  result: host double.
 * `ws` device workspace of tt_dot_workspace(a, b) bytes.  Synchronizes.
 */
size_t tt_dot_workspace(const tt_vec* a, const tt_vec* b);
tt_status tt_dot(const tt_vec* a, const tt_vec* b, double* result, void* ws, size_t ws_bytes,
                 tt_stream stream);

/*
 * tt_local_solve - the projected local linear system of the alternating
 * (ALS / AMEn) solve of A x = f for core k (Section 3.3, eq.
 * TT_min_LS_problem; Galerkin projection onto the left and right orthonormal
 * interfaces of the current iterate):
 *     sum_{b,b'} PhiL[:, b, :] (x) A_k[b, :, :, b'] (x) PhiR[:, b', :]  x_k = f_k
 * Shapes: PhiL [ra][RL][ra], A_k [RL][m][n][RR] with m == n, PhiR [rc][RR][rc],
 * f and x [ra][n][rc] (all device, row-major).  x holds the initial guess
 * on input and the solution on output.  method: 0 automatic (dense LU when
 * ra*n*rc <= direct_max, else restarted GMRES), 1 dense solve with partial
 * pivoting (register Gauss-Jordan up to 192 unknowns, LU above), 2 GMRES (one
 * persistent cooperative kernel per solve, restart length capped at 88), 3
 * mode-diagonal block solve: only the entries A_k[b, i, i, b'] are used and
 * the system splits into n dense (ra rc) x (ra rc) systems, solved as in
 * method 1 (for cores whose operator is diagonal in the mode index, such as
 * the angle core), 4 GMRES with one launch per stage of each Arnoldi step
 * (same arithmetic, for comparison).  info (host) receives iterations and the final relative
 * residual ||A x - f|| / ||f||.  Returns TT_E_NOCONV if GMRES stops at
 * max_iter above tol (x still written).  Synchronizes `stream`.
 */
typedef struct {
  int32_t ra, RL, m, n, RR, rc;
  const double* phiL;
  const double* A;
  const double* phiR;
  const double* f;
} tt_local;

typedef struct {
  int32_t method;       /* 0 auto, 1 dense, 2 GMRES (persistent), 3 mode-diagonal blocks,
                           4 GMRES (per-stage launches) */
  double tol;           /* relative residual target for GMRES */
  int32_t max_iter;     /* total GMRES iterations */
  int32_t restart;      /* Krylov dimension per cycle */
  int32_t direct_max;   /* auto: LU up to this many unknowns */
  int32_t precision;    /* GMRES: 0 FP64; 1 mixed - the persistent kernel runs FP32
                           Arnoldi cycles as iterative refinement of the FP64 residual;
                           2 as 1, and GMRES outside the persistent kernel (method 4, or
                           method 2 for systems it cannot hold) runs its operator products
                           on the BF16 matrix cores with FP32 accumulation inside each
                           restart cycle (a cycle ends at a 1e-2 reduction), with the FP64
                           residual at every restart; 3 as 2 with the products on the FP16
                           matrix cores, each operand row / column scaled by a power of two
                           per 32-deep block of the contraction before the cast (FP32
                           accumulation, the scales multiplied back); all converge in FP64
                           to tol.  Other values: TT_E_ARG */
} tt_solve_opts;

typedef struct {
  int32_t iterations;
  int32_t method_used;
  double rel_res;
} tt_solve_info;

size_t tt_local_solve_workspace(const tt_local* sys, const tt_solve_opts* opts);

/*
 * tt_local_apply - the local operator of tt_local_solve applied to a vector,
 *     y = sum_{b,b'} PhiL[:, b, :] (x) A_k[b, :, :, b'] (x) PhiR[:, b', :]  x
 * (the matrix-vector product inside the local Krylov solve, Section 3.3), as
 * three contractions: PhiL with x, the core, PhiR.  sys->f is not used.
 * precision 0: FP64; 2: the contractions on the BF16 matrix cores (operands
 * rounded to BF16, FP32 accumulation, FP64 result); 3: on the FP16 matrix
 * cores, every row of the left and column of the right operand of each
 * contraction divided, per 32-deep block of the contracted index, by the
 * power of two just above its largest magnitude before the cast (entries in
 * (-1, 1)), FP32 accumulation with the scales multiplied back, FP64 result;
 * as with BF16, operands and results are held to FP32's range.  Other values:
 * TT_E_ARG.  x [ra][n][rc] and y
 * [ra][m][rc] are device arrays; y is overwritten.  `ws` at least
 * tt_local_apply_workspace(sys) bytes.  Synchronizes `stream`.
 */
size_t tt_local_apply_workspace(const tt_local* sys);
tt_status tt_local_apply(const tt_local* sys, const double* x, double* y, int32_t precision,
                         void* ws, size_t ws_bytes, tt_stream stream);

tt_status tt_local_solve(const tt_local* sys, double* x, const tt_solve_opts* opts,
                         tt_solve_info* info, void* ws, size_t ws_bytes, tt_stream stream);

/*
 * tt_local_solve_noalloc - tt_local_solve for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same system, options, results and errors as
 * tt_local_solve, but the workspace is a static device array of 64 MiB that
 * the library holds on each GPU it runs on until the process ends; nothing is
 * allocated by the call (no hipMalloc, hipFree or allocating library
 * routine).  A system whose tt_local_solve_workspace exceeds 64 MiB returns
 * TT_E_CAPACITY with nothing written.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (different streams or threads)
 * race, so the caller serializes them.  The caller still owns sys's buffers
 * and x.  Synchronizes `stream`.
 */
tt_status tt_local_solve_noalloc(const tt_local* sys, double* x, const tt_solve_opts* opts,
                                 tt_solve_info* info, tt_stream stream);

/*
 * ttnt_set_grid_wait_limit - how long (seconds, default 20) a workgroup of a
 * persistent local solve waits at a grid barrier before it gives up.  A solve
 * whose workgroups gave up returns TT_E_HIP instead of hanging (for example
 * if a cooperative grid could not be resident at once).  Applies to launches
 * issued after the call, process-wide.  A limit <= 0 makes the first wait
 * give up (used to test the error path).  TT_E_ARG for NaN.
 */
tt_status ttnt_set_grid_wait_limit(double seconds);
/*
 * ttnt_set_grid_cap - caps the workgroups of the persistent GMRES launches
 * that the calling host thread enqueues from now on (0 restores the default,
 * 256), for callers that run several solves at once on different streams:
 * with every grid within (compute units / concurrent streams) all of them can
 * be resident together, as the grid barriers require.  The cap is recorded in
 * launches captured into graphs.  TT_E_ARG for a negative cap.
 */
tt_status ttnt_set_grid_cap(int32_t cap);

/*
 * ttnt_release - waits for the device, then frees the HIP event and pinned
 * host buffer that the blocking calls (tt_round and the other calls that read
 * ranks back) keep for the calling thread.  For an orderly teardown before
 * the process ends (every tt_solver should be destroyed first); later calls
 * recreate what they need.
 */
tt_status ttnt_release(void);

/*
 * Power-iteration solver (one call of tt_power_step = one step of
 * eq. TT_k_eff_fixed_points).
 *
 * Problem: H (transport operator), and S + F/k given as one TT matrix `SF`
 * whose cores 1..d-1 are shared by S and F and whose core 0 is the S part;
 * `F_core0` (device, the shape of SF core 0) is the F part, so that
 * core 0 of S + F/k is SF_0 + F_core0 / k.  `cF` is the TT vector F^T 1 so
 * that sum(F psi) = <cF, psi> (eq. TT_k_eff_fixed_points, last line).
 * `psi0` is the start vector and k0 the start eigenvalue.
 *
 * Each step:
 *   1. right-hand side: rhs_mode 1 forms B = tt_matvec(S + F/k, psi) and
 *      rounds it (tt_round, tol, rhs_rmax); rhs_mode 0 projects
 *      (S + F/k) psi onto the solve's interfaces core by core without
 *      forming B (the projected matrix-vector product of eq. mv_obj);
 *   2. AMEn sweeps for H psi+ = B with psi as the initial guess (Galerkin
 *      local systems by tt_local_solve, truncated SVD of each solved core,
 *      residual-based enrichment of rank `kick`), at most max_sweeps, until
 *      the largest local relative residual before a solve is below tol;
 *   3. psi+ rounded to (tol, rmax);
 *   4. k+ = k * <cF, psi+> / <cF, psi>; psi+ scaled to unit 2-norm.
 * The solver copies all problem data to device memory it allocates at
 * creation (hipMalloc happens only in tt_solver_create), or to a workspace
 * the caller owns (tt_solver_workspace_size, tt_solver_create_in).
 */
typedef struct {
  tt_mat H;
  tt_mat SF;
  const double* F_core0;
  tt_vec cF;
  tt_vec psi0;
  double k0;
} tt_problem;

typedef struct {
  double tol;            /* truncation tolerance (relative, Frobenius) */
  int32_t rmax;          /* rank cap of psi */
  int32_t kick;          /* AMEn enrichment rank */
  int32_t max_sweeps;    /* AMEn sweeps per power step */
  int32_t rhs_mode;      /* 0 projected, 1 explicit matvec + rounding */
  int32_t rhs_rmax;      /* rank cap of the explicit B */
  double local_tol;      /* relative tolerance of local solves (0: tol / sqrt(d)) */
  int32_t gmres_restart;
  int32_t gmres_max_iter;
  int32_t direct_max;    /* local systems up to this size use dense LU */
  int32_t precision;     /* local GMRES: 0 FP64, 1 mixed (FP32 Arnoldi, FP64 refinement),
                            2 mixed with BF16 matrix-core products in the multi-launch GMRES,
                            3 the same with block-scaled FP16 products
                            (as tt_solve_opts.precision); everything else in the step
                            (interfaces, QR, SVD, k) stays FP64 */
  /* Sweeping while the rank cap binds (the truncation error then exceeds
     tol, so the sweeps stop at stagnation instead of at tol): */
  int32_t min_sweeps;    /* sweeps before the stagnation test may stop (0: 2) */
  double cap_eta;        /* local solves reduce their residual by this factor (0: 1e-2) */
  double stall;          /* stop when the largest local residual falls by less than this
                            factor over a sweep (0: 0.5) */
  int32_t krylov_path;   /* local GMRES: 0 the persistent kernel where it fits, 1 always
                            the multi-launch form (one launch per stage of each step) */
} tt_solver_opts;

typedef struct {
  double k;              /* k after the step */
  double k_prev;         /* k before the step */
  double dk;             /* |k - k_prev| */
  double max_local_res;  /* largest local residual seen before a solve (last sweep) */
  double trunc_err;      /* relative truncation error of the final rounding */
  int32_t sweeps;        /* AMEn sweeps performed */
  int32_t max_rank;      /* largest rank of psi after the step */
  int32_t local_iters;   /* GMRES iterations summed over the step */
  int32_t status;        /* TT_OK, or TT_E_NOCONV if the sweep limit was hit */
} tt_step_info;

typedef struct tt_solver_s tt_solver;

tt_status tt_solver_create(const tt_problem* problem, const tt_solver_opts* opts,
                           tt_solver** out);
/*
 * tt_solver_workspace_size - device bytes the solver of `problem` and `opts`
 * needs (the working copies of H, S + F/k, psi and its interfaces, the AMEn
 * and Z trains, the local-solve and rounding scratch, all sized for the rank
 * caps).  Reads the problem's cores from device memory (synchronous);
 * allocates nothing.  TT_E_ARG on a bad descriptor or option.
 *
 * tt_solver_create_in - tt_solver_create on a caller-owned device workspace
 * of at least that many bytes, 256-byte aligned: the solver makes no device
 * allocation and borrows the workspace until tt_solver_destroy (which does
 * not free it; the caller frees it afterwards).  Its pinned host readback
 * area (6 d + 32 doubles) and one HIP event are still created.
 * TT_E_CAPACITY if workspace_bytes is smaller than the query's answer,
 * TT_E_ARG if the workspace is NULL or misaligned.
 */
tt_status tt_solver_workspace_size(const tt_problem* problem, const tt_solver_opts* opts,
                                   size_t* bytes);
/*
 * tt_power_step_async - one power step (eq. TT_k_eff_fixed_points) at psi's
 * current ranks with no host synchronization, so that a stream capture can
 * record it as a graph and replays repeat it: `sweeps` (0: opts.max_sweeps)
 * one-site alternating sweeps for H psi+ = (S + F/k) psi (each core's Galerkin system
 * solved as in tt_power_step, the solved core split by QR with R moved into
 * the next core, no truncation or enrichment), then psi+ right-orthonormal in
 * cores 1..d-1, k+ = k <cF, psi+> / <cF, psi> and the unit-norm scaling, all
 * on the device.  device_info (device memory, written by a kernel at the end
 * of the step) receives k, k_prev, dk, the largest local residual seen
 * before a solve in the last sweep, sweeps, max_rank, the GMRES iterations,
 * and status: TT_OK, TT_E_NOCONV (that residual above tol), TT_E_NUMERIC (a
 * non-finite k or residual) or TT_E_HIP (a persistent solve gave up at a
 * grid barrier).  The ranks never change, so run tt_power_step until they
 * settle first.  Requirements: rhs_mode 0, the kernel probe off, and every
 * local system on a path without host readback (dense, mode-diagonal
 * blocks, or the persistent GMRES kernel); otherwise TT_E_ARG (the stream
 * may then hold part of the step's launches).  Returns after enqueueing.
 */
tt_status tt_power_step_async(tt_solver* s, int32_t sweeps, tt_step_info* device_info,
                              tt_stream stream);
tt_status tt_solver_create_in(const tt_problem* problem, const tt_solver_opts* opts,
                              void* workspace, size_t workspace_bytes, tt_solver** out);
tt_status tt_power_step(tt_solver* s, tt_step_info* info, tt_stream stream);
/*
 * tt_amen_mv - approximate TT matrix-vector product y ~ A x with y's ranks
 * chosen by the alternating sweeps (the amen_mv route named in Section 3.3,
 * eq. mv_obj): the sweeps of tt_power_step with the identity in place of H,
 * so each local problem is the projection of A x onto the current left and
 * right orthonormal interfaces, followed by the residual enrichment and the
 * final rounding to (tol, rmax).  Unlike tt_matvec the product's ranks never
 * reach R_k r_k.  A square in every mode; x and y modes equal A's.  Writes
 * y->r; TT_E_CAPACITY if y's capacity is below the ranks found (nothing
 * written to y).  info (host, may be NULL) receives sweeps, the largest
 * local change before a sweep (max_local_res), the final truncation error
 * and the ranks; TT_E_NOCONV when max_sweeps ended the sweeps above tol (y
 * still written).  Allocates its own device scratch (like
 * tt_solver_create).  Synchronizes `stream`.
 */
tt_status tt_amen_mv(const tt_mat* A, const tt_vec* x, tt_vec* y, double tol, int32_t rmax,
                     int32_t max_sweeps, tt_step_info* info, tt_stream stream);

/*
 * tt_power_step_batched - one power step of each of `count` independent
 * solvers (for example a parameter study of many small problems; each
 * instance is the iteration of eq. TT_k_eff_fixed_points on its own data).
 * The steps run concurrently from the calling thread: up to nstreams steps
 * are in flight, one per stream, taken from the list largest estimated cost
 * first; each step runs until it needs a device value on the host, and the
 * thread resumes whichever step's stream event has completed.  Persistent
 * local solves of a step use at most (compute units / min(nstreams, count))
 * workgroups, so that the concurrent ones can all be resident.  Four streams
 * match HIP's default of four hardware queues per process; more add no
 * overlap.  infos[i]
 * receives solver i's step information.  Every solver must appear once.
 * Returns TT_OK, TT_E_NOCONV if some step hit its sweep limit, or the first
 * other error of any instance (the remaining instances still run).  Each
 * stream is synchronized before return.
 */
tt_status tt_power_step_batched(tt_solver** solvers, int32_t count, tt_step_info* infos,
                                const tt_stream* streams, int32_t nstreams);
/* Copy the current psi into the caller's TT vector (capacity checked); writes out->r. */
tt_status tt_solver_get_psi(tt_solver* s, tt_vec* out, tt_stream stream);
/* Current ranks of psi (host array of d+1) and d. */
tt_status tt_solver_ranks(tt_solver* s, int32_t* ranks, int32_t* d);
/* Number of kernel launches issued by the last tt_power_step (diagnostic). */
int64_t tt_solver_launches(tt_solver* s);
tt_status tt_solver_destroy(tt_solver* s);

/*
 * Kernel probe (measurement aid, off by default).  When on, every launch of
 * the timed kernel classes inside tt_power_step is bracketed by HIP events
 * recorded on the step's stream, and the elapsed times are accumulated with
 * the launch's algorithmic work: for a GEMM, 2 M N K flops and the bytes of
 * reading A and B once and writing C once.  Classes: 0..3 the FP64 GEMM
 * (no transpose, transposed A, transposed B, both), 4 the Krylov (Arnoldi)
 * step of the per-stage GMRES, 5 the TT core matvec, 6 a whole persistent
 * GMRES local solve (work: its operator applications and Gram-Schmidt
 * passes, counted after it ran).  set_probe resets the totals.
 */
typedef struct {
  int64_t launches;
  double total_ms;
  double flops;
  double bytes;
  int64_t dropped;       /* launches not timed because the event pool was full */
} tt_probe_stats;

tt_status tt_solver_set_probe(tt_solver* s, int32_t on);
tt_status tt_solver_probe_stats(tt_solver* s, int32_t kernel_class, tt_probe_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* TTNT_H_ */
