/*
 * kcycle.h -- C-ABI of libkcycle.so, an MI355X (gfx950) implementation of the
 * kappa-cycle multigrid method of Avnat & Yavneh, "On the recursive structure
 * of multigrid cycles", for the 2D rotated anisotropic diffusion equation.
 *
 * Problem (Section 4): -div(D grad u) = f on the unit square, u = 0 on the
 * boundary, D = R(theta) diag(1, eps) R(theta)^T, discretised with the
 * nine-point stencil table of Section 4 on an n x n interior grid
 * (h = 1/(n+1)), n = 2^L - 1.  The operator is A = S / h^2.
 *
 * Array layout (every u, f, x, y, lam argument): row-major, element (j, i) at
 * p[j * ld + i], row j along +y, column i along +x, interior points only,
 * ld >= n.  Arrays are caller-owned device memory (e.g. torch tensors).
 *
 * Hierarchy: levels l = 1..L with n_l = 2^(L-l+1) - 1 down to n_coarsest
 * (1, 3 or 7); coarse operators are Galerkin, A_{l+1} = R A_l P with bilinear
 * prolongation P and full weighting R = P^T / 4 (Section 4).
 *
 * Streams: every call is ordered on the hip stream given to kc_create.  Calls
 * that return host values (kc_solve, kc_pcg, kc_grad_params, kc_stats)
 * synchronise that stream before returning.
 *
 * Batches: a hierarchy may hold `count` independent instances of different
 * sizes, angles and anisotropies.  Every array argument is then a host array
 * of `count` device pointers and every ld / iters / relres argument a host
 * array of `count` entries.  All instances advance together, one kernel
 * launch per cycle stage (the call tree of an n-level instance is the top of
 * a deeper instance's call tree, Proposition 2).
 *
 * Errors: every function returns kc_status.  Negative values are errors (the
 * arrays keep their input values unless stated); positive values are
 * algorithmic outcomes and leave the result arrays valid.  kc_last_error()
 * gives a thread-local message for the last failing call.
 *
 * Memory: the library allocates no device memory of its own.  The caller asks
 * kc_workspace_bytes for a size and passes a device buffer of that size
 * (256-byte aligned) to kc_create; it must outlive the hierarchy.  Host-side
 * allocations (tables, graphs, pinned staging) are owned by the handle.
 * A handle is not thread-safe; use one per host thread.
 */
#ifndef KCYCLE_H
#define KCYCLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KC_OK = 0,
    KC_NOT_CONVERGED = 1,   /* maxit reached; result valid, relres filled        */
    KC_DIVERGED = 2,        /* relres grew beyond 1e3 x its initial value         */
    KC_BREAKDOWN = 3,       /* PCG: p^T A p <= 0 (indefinite preconditioner)      */
    KC_ERR_ARG = -1,        /* invalid argument (size, counter, null pointer ...) */
    KC_ERR_HIP = -2,        /* a HIP runtime call failed                          */
    KC_ERR_WORKSPACE = -3,  /* workspace missing, too small or misaligned         */
    KC_ERR_NONFINITE = -4,  /* NaN or Inf met in f or in a residual               */
    KC_ERR_STATE = -5       /* call not valid for this hierarchy (e.g. precision) */
} kc_status;

typedef enum {
    KC_F64 = 0,             /* cycles, vectors and norms in FP64                          */
    KC_F32_CYCLE = 1        /* cycles in FP32; residuals, updates, CG recurrences in FP64 */
} kc_precision;

/* one problem instance: n = 2^L - 1 points per side; n_coarsest in {1, 3, 7}
 * and n_coarsest <= n; 0 < eps; omega is the Jacobi damping factor */
typedef struct {
    int32_t n;
    int32_t n_coarsest;
    double theta;
    double eps;
} kc_problem;

#define KC_KAPPA_W INT32_MAX   /* any kappa >= L gives the W-cycle (Proposition 1) */

/* cycle parameters (Algorithm 3): counter kappa >= 1, nu1/nu2 >= 0 damped
 * Jacobi sweeps before/after the coarse-grid correction, damping omega > 0 */
typedef struct {
    int32_t kappa;
    int32_t nu1;
    int32_t nu2;
    int32_t smoother;   /* 0 = damped Jacobi with omega (default); 1 = alternating zebra line Gauss-Seidel (Section 4,
                           third and fourth solvers): relaxation r of a smoothing step solves every x-line (r even)
                           or y-line (r odd) exactly, lines of even index first, then odd.  In the fused mode
                           the levels above the coarse cutover run one kernel per operation and every call at
                           the cutover runs in the persistent kernel (line solves in LDS); in the
                           paper-structured mode every level runs one kernel per operation.  Needs n <= 16383
                           (else KC_ERR_ARG) */
    double omega;
} kc_cycle_params;

/* execution options; kc_exec_default fills the defaults */
typedef struct {
    int32_t mode;           /* 0 = fused kernels + persistent coarse subtree (default);
                               1 = one kernel per operation of Algorithm 4 ("paper-structured") */
    int32_t use_graph;      /* 1 = capture one cycle as a hipGraph and replay it (default) */
    int32_t coarse_cutover; /* levels with n <= cutover run in the persistent kernel (7..63; default 31) */
    int32_t coarse_threads; /* threads of the persistent kernel (256, 512, or 1024 with FP32 cycles; default 512) */
    int32_t poll_every;     /* cycles launched between host polls of the stop flags (default 0 = adaptive) */
    int32_t coarse_wave_n;  /* persistent-kernel levels with n <= this run on one wave (0..15; default 15) */
    int32_t small_tile_n;   /* fused grid kernels on levels whose largest n <= this use 16 x 16 tiles instead of
                               64 x 32 (0 = never; 0..4095; default 511); results do not depend on it */
    int32_t stream_n;       /* fused grid kernels on levels whose largest n >= this stream row strips through
                               registers instead of staging tiles in LDS (0 = never; default 2047); results do
                               not depend on it */
    int32_t wave_regs;      /* 1 = whole calls on the levels wave 0 runs alone (n <= coarse_wave_n) run in
                               registers (instances with n_coarsest = 1; default 1); 0 = phase by phase in LDS;
                               results do not depend on it */
    int32_t fuse_junctions; /* 1 = on levels run in 8 x 8 or 16 x 16 tiles, the post-smoothing of a call's first child and the
                               pre-smoothing of its second child (kappa >= 2) run as one kernel (default 1); results
                               do not depend on it */
    int32_t mid_tile_n;     /* fused grid kernels on levels whose largest n is above small_tile_n and <= this use
                               32 x 32 tiles (0 = never; 0..4095; default 2047); results do not depend on it */
    int32_t tiny_tile_n;    /* fused grid kernels on levels whose largest n <= this use 8 x 8 tiles (one point per
                               thread and phase; takes precedence over small_tile_n; 0 = never; 0..4095; default 255);
                               results do not depend on it */
    int32_t zebra_wave_n;   /* zebra line relaxation on levels with n >= this solves each line with half a wave (two
                               lines per wave, 32 points per chunk, many lines in flight); smaller levels use one
                               thread per line (0 = never; 0..16383; default 63); results do not depend on it */
    int32_t zebra_quad_n;   /* of those levels, the ones with n >= this solve each line with a quarter wave (four
                               lines per wave, 16 points per chunk: on the largest levels the line recurrences then
                               share fewer LDS instructions per point; 0 = never; 0..16383; default 8191); results
                               do not depend on it */
} kc_exec;

typedef struct kc_hier kc_hier;

/* defaults for kc_exec */
void kc_exec_default(kc_exec* e);

/* bytes of device workspace for `count` instances (Section 3.1: all data are
 * resident on the GPU after setup); no device work, no GPU needed */
kc_status kc_workspace_bytes(const kc_problem* probs, int32_t count, kc_precision prec, size_t* bytes);

/* build the hierarchies (fine stencil, Galerkin coarse stencils, coarsest
 * inverse) on the host and copy them into the workspace; `exec` may be NULL
 * for the defaults; `hip_stream` is a hipStream_t (NULL = default stream) */
kc_status kc_create(const kc_problem* probs, int32_t count, kc_precision prec, const kc_exec* exec,
                    void* d_workspace, size_t bytes, void* hip_stream, kc_hier** out);

kc_status kc_destroy(kc_hier* h);

/* semi-coarsening (Section 4, fifth and sixth solvers): hierarchies whose
 * levels keep the n points of a line (x) and halve the lines (y), level l
 * holding (n + 1) / 2^(l-1) - 1 lines down to a single line; linear
 * interpolation P along y, full weighting R = P^T / 2 along y, Galerkin
 * stencils R A P in units of the fine h^2; relaxation by x-line zebra (the
 * cycle parameters must give smoother = 1; every relaxation runs the lines of
 * even index, then odd, each solved exactly); the single coarsest line is
 * solved exactly by the same line elimination.  Every instance must have the
 * same n <= 16383 and n_coarsest = 1 (unused).  Levels run one kernel per
 * operation (exec.mode is set to 1; kc_set_exec refuses 0).  The other calls
 * (kc_cycle, kc_solve, kc_pcg, FP32 hierarchies, kc_apply_A, kc_grad_params)
 * work on these hierarchies as on the standard ones; kc_set_convection
 * returns KC_ERR_STATE. */
kc_status kc_workspace_bytes_semi(const kc_problem* probs, int32_t count, kc_precision prec, size_t* bytes);
kc_status kc_create_semi(const kc_problem* probs, int32_t count, kc_precision prec, const kc_exec* exec,
                         void* d_workspace, size_t bytes, void* hip_stream, kc_hier** out);

/* host-only: the stencils of every semi-coarsened level of one problem (units
 * of the fine h^2), s[9*l + 3*(b+1) + (a+1)]; no GPU needed */
kc_status kc_semi_stencils(const kc_problem* p, int32_t max_levels, int32_t* nlevels, double* stencils);

/* change execution options (drops captured graphs) */
kc_status kc_set_exec(kc_hier* h, const kc_exec* exec);

/* one kappa-cycle (Algorithm 3) on every instance: v <- cycle(v, f), FP64
 * arrays, asynchronous on the stream.  KC_ERR_STATE on an FP32 hierarchy. */
kc_status kc_cycle(kc_hier* h, double* const* d_v, const int64_t* ldv, const double* const* d_f,
                   const int64_t* ldf, const kc_cycle_params* c);

/* stand-alone solver (Section 4, first solver): u holds the initial guess and
 * receives the result.  Repeats kappa-cycles until ||f - A u_k|| / ||f|| < tol
 * (relres checked before every cycle) or maxit cycles.  FP32 hierarchies run
 * FP32 cycles inside FP64 iterative refinement.  iters[i] = cycles done,
 * relres[i] = final relative residual.  The return value is the worst
 * instance status.  Synchronises. */
kc_status kc_solve(kc_hier* h, double* const* d_u, const int64_t* ldu, const double* const* d_f,
                   const int64_t* ldf, const kc_cycle_params* c, double tol, int32_t maxit,
                   int32_t* iters, double* relres, int32_t* status);

/* conjugate gradients preconditioned by one zero-guess kappa-cycle per
 * iteration (Section 4, second solver), x_0 = 0, Fletcher-Reeves beta.  Once
 * the recurrence residual gives ||r_k|| / ||f|| < tol, the true residual
 * f - A u_k is formed in FP64 and decides: below tol the solve stops,
 * otherwise it replaces r_k and CG goes on (residual replacement), so a
 * converged instance has a true relative residual below tol.  Vectors and
 * dot products (Dot2 sums) in FP64; the cycle in FP32 on FP32 hierarchies.
 * Synchronises. */
kc_status kc_pcg(kc_hier* h, double* const* d_u, const int64_t* ldu, const double* const* d_f,
                 const int64_t* ldf, const kc_cycle_params* c, double tol, int32_t maxit,
                 int32_t* iters, double* relres, int32_t* status);

/* relative-residual history of instance `instance` in the last kc_solve or
 * kc_pcg on h: out[k] = ||r_k|| / ||f|| after k cycles (stand-alone; out[0]
 * is the initial guess) or k CG iterations (recurrence residual, or the true
 * residual where PCG formed it; out[0] = 1).
 * *count receives the number of entries recorded, min(iters + 1, 8192): the
 * first 8192 are kept, longer runs are not limited by this.  Copies
 * min(cap, *count) entries to the host buffer out (may be NULL when cap is
 * 0).  KC_ERR_STATE before any solve.  Synchronises. */
kc_status kc_residual_history(kc_hier* h, int32_t instance, double* out, int32_t cap, int32_t* count);

/* y = A x on every instance's fine level (FP64), asynchronous */
kc_status kc_apply_A(kc_hier* h, double* const* d_y, const int64_t* ldy, const double* const* d_x,
                     const int64_t* ldx);

/* parameter gradients of a scalar loss through u = A(theta, eps)^{-1} f:
 * dtheta[i] = -lam_i^T (dA/dtheta) u_i and deps[i] = -lam_i^T (dA/deps) u_i,
 * lam the adjoint solution (A is symmetric).  FP64.  Synchronises. */
kc_status kc_grad_params(kc_hier* h, const double* const* d_lam, const int64_t* ldl, const double* const* d_u,
                         const int64_t* ldu, double* dtheta, double* deps);

/* For callers that cannot allocate device memory or create a hierarchy (code
 * under graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the gradient inner products of kc_grad_params for `count` instances given
 * by probs (n, theta, eps; n_coarsest is checked but unused), without a
 * hierarchy or workspace.  lam and u are caller-owned FP64 arrays in the
 * layout above; dtheta / deps are host arrays of count entries.  The instance
 * table, per-instance state, block table and the Dot2 block partials (32 B
 * per 64 x 32 tile of every instance) live in a static device array of
 * KC_NOALLOC_SCRATCH_BYTES, one per GPU, held until the process ends; the
 * call allocates no device memory.  KC_ERR_ARG when count exceeds
 * KC_NOALLOC_MAX_INSTANCES or the tiles do not fit (one 16383^2 instance
 * does, two do not).  Runs on the current device, ordered on hip_stream
 * (NULL = default stream), and synchronises it.  Calls on one GPU share the
 * array: calls that overlap (other host threads are serialised by a lock,
 * other processes are not) race.  Results are those of kc_grad_params. */
#define KC_NOALLOC_SCRATCH_BYTES (8 << 20)
#define KC_NOALLOC_MAX_INSTANCES 64
kc_status kc_grad_params_noalloc(const kc_problem* probs, int32_t count, const double* const* d_lam,
                                 const int64_t* ldl, const double* const* d_u, const int64_t* ldu, void* hip_stream,
                                 double* dtheta, double* deps);

/* convection-diffusion (the nonsymmetric problem the conclusions propose):
 * switches every instance i to -div(D grad u) + b_i . grad u with the Section 4
 * diffusion and constant velocity b_i = (bx[i], by[i]) (host arrays of count
 * entries), the convection by first-order upwind differences; every level
 * takes the same operator at its own mesh width (rediscretisation, not
 * Galerkin).  Needs n_coarsest = 1 for every instance (else KC_ERR_ARG, nothing
 * changed); afterwards the zebra smoother is refused (KC_ERR_ARG) and kc_pcg
 * and kc_grad_params return KC_ERR_STATE (the operator is not symmetric).
 * bx = by = 0 gives the diffusion operator with rediscretised coarse levels.
 * Synchronises. */
kc_status kc_set_convection(kc_hier* h, const double* bx, const double* by);

/* host-only: the h^2-scaled 3x3 stencils of every level of one problem with
 * convection (bx, by), as kc_set_convection builds them; no GPU needed */
kc_status kc_convection_stencils(const kc_problem* p, double bx, double by, int32_t max_levels, int32_t* nlevels,
                                 double* stencils);

/* host-only: the h^2-scaled 3x3 stencils of every level of one problem,
 * s[9*l + 3*(b+1) + (a+1)] for offset (a, b) in (x, y); no GPU needed */
kc_status kc_level_stencils(const kc_problem* p, int32_t max_levels, int32_t* nlevels, double* stencils);

/* host-only: the flattened stage schedule of one cycle, as launches per cycle
 * (grid kernels, persistent-kernel launches, persistent-kernel stages);
 * no GPU needed */
kc_status kc_schedule_counts(const kc_problem* probs, int32_t count, const kc_exec* exec,
                             const kc_cycle_params* c, int64_t* grid_launches, int64_t* subtree_launches,
                             int64_t* subtree_stages);

/* instrumentation: average duration of one launch of a single schedule
 * stage, timed with hip events around `reps` back-to-back launches on the
 * hierarchy's stream, on the arrays bound by the previous driver call (run a
 * kc_solve / kc_pcg / kc_cycle first).  which:
 *   0 = fused pre-smoothing kernel of the fine level (nu1 sweeps + residual +
 *       full weighting; the stand-alone FP64 variant also sums the residual),
 *   1 = fused post-smoothing kernel of the fine level (prolong-add + nu2),
 *   2 = one persistent coarse launch (both calls below the first parent),
 *   3 = the FP64 residual pass of refinement (FP32 hierarchies),
 *   100 + d / 200 + d = the pre / post kernel of depth d (0 = finest),
 *   300 + d = the persistent launch of depth d (a pair of calls; for d = 0
 *   a single call of the whole cycle).
 * bytes receives the algorithmic bytes one launch must move (every input read
 * once, every output written once).  The instances are left finished (the
 * stop flags are set), so run a driver call again before relying on them.
 * Synchronises.  KC_ERR_STATE if the stage does not exist in this schedule. */
kc_status kc_time_stage(kc_hier* h, int32_t which, const kc_cycle_params* c, int32_t reps, double* avg_ms,
                        double* bytes);

/* instrumentation for the run-time model (Section 3.2): one warm-up cycle,
 * then `reps` kappa-cycles on (v, f) back to back (graph replays, no stop
 * test), timed with hip events on the hierarchy's stream; v is overwritten.
 * FP64 hierarchies.  Synchronises. */
kc_status kc_time_cycles(kc_hier* h, double* const* d_v, const int64_t* ldv, const double* const* d_f,
                         const int64_t* ldf, const kc_cycle_params* c, int32_t reps, double* ms_per_cycle);

/* per-launch profile of one solver iteration (driver 0 = stand-alone kc_solve,
 * 1 = kc_pcg; the same driver must have run last on h, whose arrays it keeps
 * iterating on, so they are overwritten).  Runs one warm-up iteration, then
 * repeats each launch of the iteration `reps` times back to back between two
 * hip events (its finalize step likewise), every instance kept active
 * (tolerance 0).  Writes JSON to out: iteration_ms and,
 * per kernel (compiler names, as a profiler lists them), the launches per
 * iteration, total and average ms, and the algorithmic bytes and flops per
 * launch (each input read once, each output written once); the sequence of
 * launches as [kernel, depth, ms, algorithmic bytes].  Synchronises. */
kc_status kc_profile_iteration(kc_hier* h, int32_t driver, const kc_cycle_params* c, int32_t reps, char* out,
                               size_t cap);

/* JSON summary: sizes, launches per cycle, last solve's timings */
kc_status kc_stats(const kc_hier* h, char* out, size_t cap);

const char* kc_status_string(kc_status s);
const char* kc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
