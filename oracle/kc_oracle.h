/*
 * kc_oracle.h -- reference (oracle) implementation of the kappa-cycle multigrid
 * method of Avnat & Yavneh, "On the recursive structure of multigrid cycles".
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded FP64 CPU
 * implementation written directly from the paper.  It exists to check the GPU
 * library.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product never links, imports or calls it.
 * It shares no code with the GPU library.
 *
 * Conventions (all arrays are row-major, interior points only, zero Dirichlet
 * values outside the grid):
 *   - a level with n points per side has mesh width h = 1/(n+1);
 *   - x[j*n + i] is the value at (x, y) = ((i+1)h, (j+1)h);  j runs along +y;
 *   - a 3x3 stencil s[3*(b+1) + (a+1)] is the coefficient of the neighbour at
 *     offset (a, b) in (x, y); the operator on the level is A = S / h^2
 *     (Section 4, the nine-point stencil table);
 *   - levels are numbered l = 1 (finest) .. L (coarsest), as in Algorithm 3.
 */
#ifndef KC_ORACLE_H
#define KC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAXL 16

/* status codes returned by the drivers */
#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_DIVERGED 2
#define OR_BREAKDOWN 3
#define OR_ERR_ARG (-1)
#define OR_ERR_NONFINITE (-4)

/* trace record: (op << 24) | (level << 16) | min(counter, 0xffff) */
#define OR_OP_CALL 1     /* entry into the cycle routine on a level      */
#define OR_OP_SOLVE 2    /* coarsest-level direct solve                  */
#define OR_OP_RELAX 3    /* one damped-Jacobi sweep                      */
#define OR_OP_RESID 4    /* residual computation                         */
#define OR_OP_RESTR 5    /* full-weighting restriction                   */
#define OR_OP_ZERO 6     /* coarse initial guess set to zero             */
#define OR_OP_PROL 7     /* bilinear prolongation                        */
#define OR_OP_ADD 8      /* correction added to the current estimate     */

typedef struct or_hier or_hier;

/* fine-grid nine-point stencil of Section 4 for angle theta, anisotropy eps */
void or_fine_stencil(double theta, double eps, double s[9]);
/* its partial derivatives with respect to theta and eps */
void or_fine_stencil_derivs(double theta, double eps, double dth[9], double deps[9]);

/* level operators on one grid (unscaled operator A = S/h^2, h = 1/(n+1)) */
void or_apply_stencil(int n, const double s[9], const double* x, double* y);
void or_restrict_fw(int n, const double* r, double* fc);      /* fine n -> coarse (n-1)/2 */
void or_prolong(int nc, const double* vc, double* e);         /* coarse nc -> fine 2nc+1  */
/* Galerkin coarse stencil A_c = R A P (R = full weighting, P = bilinear) */
void or_galerkin_stencil(const double s_fine[9], double s_coarse[9]);

/* hierarchy: n = fine points per side, n_coarsest in {1, 3, 7, ...} */
int or_hier_new(int n, double theta, double eps, int n_coarsest, double omega, or_hier** out);
/* the fifth / sixth solvers of Section 4: x-line zebra relaxation (two per
 * smoothing step with nu = 2), coarsening along y only (level l has n points
 * per line and (n+1)/2^(l-1) - 1 lines, down to one line, solved exactly by
 * the line elimination), Galerkin operators s_{l+1} = R s_l P with linear
 * interpolation P along y and R = P^T / 2.  Drivers and or_cycle (kind 0)
 * work on it as on a standard hierarchy; or_hier_info reports lines per level
 * and stencils in units of the fine h^2 */
int or_hier_new_semi(int n, double theta, double eps, or_hier** out);
void or_hier_free(or_hier* h);
int or_hier_info(const or_hier* h, int* nlevels, int* sizes, double* stencils);
/* y = A_1 x on the fine level */
void or_hier_apply(const or_hier* h, const double* x, double* y);

/* relaxation of every cycle, solve and CG run on h: 0 = damped Jacobi (the
 * default), 1 = alternating zebra line Gauss-Seidel (relaxation r of a
 * smoothing step along x-lines when r is even, y-lines when odd; lines of
 * even index first) */
int or_set_smoother(or_hier* h, int smoother);

/* convection-diffusion: h^2-scaled stencil of -div(D grad u) + b . grad u
 * (first-order upwind convection) on an n x n grid, and the switch of a
 * hierarchy to it (every level rediscretised at its mesh width; damped Jacobi
 * and a 1 x 1 coarsest level only, else OR_ERR_ARG; or_pcg then returns
 * OR_ERR_ARG) */
void or_convection_stencil(int n, double theta, double eps, double bx, double by, double s[9]);
int or_set_convection(or_hier* h, double bx, double by);

/* one zebra relaxation on the fine level in place (dir 0: x-lines, 1: y-lines) */
void or_zebra_relax(or_hier* h, int dir, double* v, const double* f);
/* the line-elimination tables of level `level` (1-based) for x-lines (dir 0)
 * or y-lines (dir 1): reciprocal pivots rp[q] = 1/p_q and upper multipliers
 * um[q] = up/p_q, n_l entries each, FP64 */
int or_zebra_tables(const or_hier* h, int level, int dir, double* rp, double* um);

/* Dot2 dot product of Ogita, Rump and Oishi (the form of every norm and dot
 * product the drivers take) */
double or_dot2(const double* x, const double* y, int64_t m);

/*
 * One cycle on the fine level (Algorithm 3 for kind 0, Algorithm 1 for kind 1
 * with cycle index = param, Algorithm 2 for kind 2).  v is updated in place;
 * f is the fine right-hand side.  When tr != NULL each operation is appended
 * (up to cap entries).  The return value is the number of trace records the
 * cycle produced (written or not).
 */
int64_t or_cycle(or_hier* h, int kind, int param, int nu1, int nu2,
                 double* v, const double* f, int32_t* tr, int64_t cap);
/* the same kappa-cycle run entirely in FP32 arithmetic on FP32 copies */
void or_kcycle_f32(or_hier* h, int kappa, int nu1, int nu2, float* v, const float* f);

/* stand-alone iteration: u holds the initial guess and receives the result.
 * mode 0: stop at the first k with ||f - A u_k|| / ||f|| < tol;
 * mode 1: stop at the first k with ||u_k|| / ||u_0|| < tol (f = 0 runs).
 * hist (maxit + 1 entries, may be NULL) receives the monitored ratio. */
int or_solve(or_hier* h, int kappa, int nu1, int nu2, double* u, const double* f,
             double tol, int maxit, int mode, int* iters, double* hist);

/* conjugate gradients preconditioned by one zero-guess kappa-cycle, Fletcher-
 * Reeves beta; once the recurrence residual is below tol the true residual
 * decides (stop, or replace the recurrence residual and go on).
 * precond_f32 != 0 runs the cycle in FP32 (vectors and dots stay FP64). */
int or_pcg(or_hier* h, int kappa, int nu1, int nu2, int precond_f32,
           double* u, const double* f, double tol, int maxit, int* iters, double* hist);

/* FP32 kappa-cycles inside FP64 iterative refinement (u starts at the input) */
int or_ir_solve(or_hier* h, int kappa, int nu1, int nu2, double* u, const double* f,
                double tol, int maxit, int* iters, double* hist);

/* power-of-two scale used before rounding a residual to FP32 */
double or_ir_scale(double sumsq, int64_t npoints);

/* dL/dtheta = -lam^T (dA/dtheta) u and dL/deps = -lam^T (dA/deps) u on the fine level */
void or_grad_params(const or_hier* h, double theta, double eps, const double* lam,
                    const double* u, double* dtheta, double* deps);

#ifdef __cplusplus
}
#endif
#endif
