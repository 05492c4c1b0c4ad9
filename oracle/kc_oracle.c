/*
 * kc_oracle.c -- reference (oracle) implementation of the kappa-cycle method.
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, single-threaded CPU implementation
 * written from the paper (Avnat & Yavneh, "On the recursive structure of
 * multigrid cycles").  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code with the GPU library.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fPIC -shared (the compiler
 * contracts nothing; every fused multiply-add is an explicit fma() call).
 * Arithmetic reading: inside the cycle every product that is added to or
 * subtracted from a running value is one fused multiply-add (FMAR below):
 * the nine-point and off-line stencil sums, the Jacobi update
 * v + omega/S_0 (f - A v) and both recurrences of the line elimination.
 * Products by the transfer weights (1, 1/2, 1/4) are exact, so full
 * weighting and prolongation keep plain products and sums; the dense
 * coarsest solve, the setup (Galerkin stencils, factors) and the Krylov
 * vector updates round every product and sum on its own.  The norms and
 * dot products use fma() to extract a product's exact rounding error.
 *
 * What each part follows:
 *   - fine operator: the nine-point stencil table of Section 4;
 *   - coarse operators: Galerkin A_{l+1} = R A_l P with full weighting R and
 *     bilinear prolongation P (Section 4, the Galerkin solvers; R is the
 *     adjoint of P as stated in the symmetry discussion of Section 4);
 *   - relaxation: damped Jacobi, simultaneous update (Section 4), or the
 *     alternating zebra line Gauss-Seidel of the third and fourth solvers;
 *   - cycles: Algorithm 1 (gamma-cycle), Algorithm 2 (F-cycle) and
 *     Algorithm 3 (kappa-cycle), recursion exactly as printed, including the
 *     redundant second call at the level above the coarsest (Section 1);
 *   - drivers: the stand-alone cycle and CG preconditioned by one cycle per
 *     iteration (Section 4, solvers one and two).
 */
#include "kc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t* buf;
    int64_t cap;
    int64_t len;
} or_tr;

static void tr_push(or_tr* t, int op, int level, int counter)
{
    if (!t) return;
    if (t->buf && t->len < t->cap) {
        int c = counter < 0 ? 0 : (counter > 0xffff ? 0xffff : counter);
        t->buf[t->len] = (int32_t)(((uint32_t)op << 24) | ((uint32_t)level << 16) | (uint32_t)c);
    }
    t->len++;
}

#define REAL double
#define SFX(x) x##_d
#define FMAR fma
#include "kc_oracle_levels.inc"
#undef REAL
#undef SFX
#undef FMAR

#define REAL float
#define SFX(x) x##_s
#define FMAR fmaf
#include "kc_oracle_levels.inc"
#undef REAL
#undef SFX
#undef FMAR

#define REAL double
#define SFX(x) x##_d
#define FMAR fma
#include "kc_oracle_semi.inc"
#undef REAL
#undef SFX
#undef FMAR

#define REAL float
#define SFX(x) x##_s
#define FMAR fmaf
#include "kc_oracle_semi.inc"
#undef REAL
#undef SFX
#undef FMAR

struct or_hier {
    lv_d d;          /* FP64 hierarchy (semi-coarsening: the fine level only) */
    lv_s s;          /* FP32 copy used by the FP32 cycle                */
    int semi;        /* 1: x-line zebra with semi-coarsening along y    */
    int conv;        /* 1: convection term set (nonsymmetric operator)  */
    lvs_d sd;        /* semi-coarsened levels, FP64 and FP32            */
    lvs_s ss;
    double theta, eps, omega;
    double* fine_v;  /* owned fine-level storage when no user array is bound */
    double* fine_f;
    float* fine_v32;
    float* fine_f32;
};

/* ------------------------------------------------------------------ */
/* discrete problem (Section 4)                                         */
/* ------------------------------------------------------------------ */

void or_fine_stencil(double theta, double eps, double s[9])
{
    double C = cos(theta), S = sin(theta);
    double cross = 0.5 * (1.0 - eps) * C * S;
    double we = -(C * C + eps * S * S);    /* west / east      */
    double sn = -(eps * C * C + S * S);    /* south / north    */
    s[0] = -cross; s[1] = sn;                s[2] = cross;    /* SW  S  SE */
    s[3] = we;     s[4] = 2.0 * (1.0 + eps); s[5] = we;       /* W   C  E  */
    s[6] = cross;  s[7] = sn;                s[8] = -cross;   /* NW  N  NE */
}

/* Convection-diffusion (the nonsymmetric problem the conclusions propose):
 * -div(D grad u) + b . grad u = f with the diffusion of the Section 4 table
 * and a constant velocity b = (bx, by), the convection discretised by
 * first-order upwind differences (backward along a positive velocity
 * component, forward along a negative one), which keeps the matrix an
 * M-matrix.  In h^2-scaled units the convection adds h |bx| + h |by| to the
 * centre and subtracts h max(bx, 0) from the west, h max(-bx, 0) from the
 * east, h max(by, 0) from the south and h max(-by, 0) from the north entry. */
void or_convection_stencil(int n, double theta, double eps, double bx, double by, double s[9])
{
    or_fine_stencil(theta, eps, s);
    const double h = 1.0 / (double)(n + 1);
    const double cx = h * bx, cy = h * by;
    s[4] = s[4] + (fabs(cx) + fabs(cy));
    s[3] = s[3] - fmax(cx, 0.0);
    s[5] = s[5] - fmax(-cx, 0.0);
    s[1] = s[1] - fmax(cy, 0.0);
    s[7] = s[7] - fmax(-cy, 0.0);
}

void or_fine_stencil_derivs(double theta, double eps, double dth[9], double deps[9])
{
    double C = cos(theta), S = sin(theta);
    /* d/dtheta: C' = -S, S' = C */
    double d_cross = 0.5 * (1.0 - eps) * (C * C - S * S);
    double d_we = 2.0 * (1.0 - eps) * C * S;
    double d_sn = -2.0 * (1.0 - eps) * C * S;
    dth[0] = -d_cross; dth[1] = d_sn; dth[2] = d_cross;
    dth[3] = d_we;     dth[4] = 0.0;  dth[5] = d_we;
    dth[6] = d_cross;  dth[7] = d_sn; dth[8] = -d_cross;
    /* d/deps */
    double e_cross = -0.5 * C * S;
    double e_we = -S * S;
    double e_sn = -C * C;
    deps[0] = -e_cross; deps[1] = e_sn; deps[2] = e_cross;
    deps[3] = e_we;     deps[4] = 2.0;  deps[5] = e_we;
    deps[6] = e_cross;  deps[7] = e_sn; deps[8] = -e_cross;
}

void or_apply_stencil(int n, const double s[9], const double* x, double* y)
{
    apply_d(n, s, 1.0, x, y);
}

void or_restrict_fw(int n, const double* r, double* fc) { restr_d(n, r, fc); }

void or_prolong(int nc, const double* vc, double* e) { prol_d(nc, vc, e); }

/* Galerkin coarse stencil: with A = S/h^2 on each level and h_c = 2h,
 * S_c = h_c^2 R (S/h^2) P = 4 R S P.  It is read off by applying R S P to a
 * coarse unit vector on a 5x5 coarse grid (11x11 fine), far enough from the
 * boundary that no term is cut off. */
void or_galerkin_stencil(const double sf[9], double sc[9])
{
    enum { NC = 5, NF = 11 };
    double ec[NC * NC], e[NF * NF], ae[NF * NF], rc[NC * NC];
    memset(ec, 0, sizeof ec);
    ec[2 * NC + 2] = 1.0;
    prol_d(NC, ec, e);
    apply_d(NF, sf, 1.0, e, ae);
    restr_d(NF, ae, rc);
    for (int b = -1; b <= 1; ++b)
        for (int a = -1; a <= 1; ++a)
            sc[3 * (b + 1) + (a + 1)] = 4.0 * rc[(2 + b) * NC + (2 + a)];
}

/* ------------------------------------------------------------------ */
/* hierarchy                                                            */
/* ------------------------------------------------------------------ */

static int is_pow2(long x) { return x > 0 && (x & (x - 1)) == 0; }

void or_hier_free(or_hier* h)
{
    if (!h) return;
    for (int k = 0; k < OR_MAXL; ++k) {
        if (k > 0) {
            free(h->d.v[k]); free(h->d.f[k]);
            free(h->s.v[k]); free(h->s.f[k]);
        }
        free(h->d.t[k]);
        free(h->s.t[k]);
        for (int dir = 0; dir < 2; ++dir) {
            free(h->d.zp[k][dir]); free(h->d.zu[k][dir]);
            free(h->s.zp[k][dir]); free(h->s.zu[k][dir]);
        }
    }
    for (int k = 0; k < OR_MAXL; ++k) {
        if (k > 0) {
            free(h->sd.v[k]); free(h->sd.f[k]);
            free(h->ss.v[k]); free(h->ss.f[k]);
        }
        free(h->sd.t[k]); free(h->ss.t[k]);
        free(h->sd.zp[k]); free(h->sd.zu[k]);
        free(h->ss.zp[k]); free(h->ss.zu[k]);
    }
    free(h->fine_v); free(h->fine_f); free(h->fine_v32); free(h->fine_f32);
    free(h->d.chol);
    free(h->s.chol);
    free(h);
}

int or_hier_new(int n, double theta, double eps, int n_coarsest, double omega, or_hier** out)
{
    *out = NULL;
    if (n < 1 || n_coarsest < 1 || n_coarsest > n) return OR_ERR_ARG;
    if (!is_pow2((long)n + 1) || !is_pow2((long)n_coarsest + 1)) return OR_ERR_ARG;
    int L = 1;
    while (((n + 1) >> (L - 1)) > n_coarsest + 1) ++L;
    if (L > OR_MAXL) return OR_ERR_ARG;

    or_hier* h = (or_hier*)calloc(1, sizeof(or_hier));
    if (!h) return OR_ERR_ARG;
    h->theta = theta; h->eps = eps; h->omega = omega;
    h->d.L = h->s.L = L;
    for (int k = 0; k < L; ++k) {
        int nk = ((n + 1) >> k) - 1;
        size_t m = (size_t)nk * nk;
        h->d.n[k] = h->s.n[k] = nk;
        h->d.h2inv[k] = (double)(nk + 1) * (double)(nk + 1);
        if (k == 0) or_fine_stencil(theta, eps, h->d.s[0]);
        else or_galerkin_stencil(h->d.s[k - 1], h->d.s[k]);
        h->d.wjac[k] = omega / (h->d.s[k][4] * h->d.h2inv[k]);
        h->d.t[k] = (double*)calloc(m, sizeof(double));
        h->s.t[k] = (float*)calloc(m, sizeof(float));
        if (k > 0) {
            h->d.v[k] = (double*)calloc(m, sizeof(double));
            h->d.f[k] = (double*)calloc(m, sizeof(double));
            h->s.v[k] = (float*)calloc(m, sizeof(float));
            h->s.f[k] = (float*)calloc(m, sizeof(float));
            if (!h->d.v[k] || !h->d.f[k] || !h->s.v[k] || !h->s.f[k]) { or_hier_free(h); return OR_ERR_ARG; }
        }
        if (!h->d.t[k] || !h->s.t[k]) { or_hier_free(h); return OR_ERR_ARG; }
        /* FP32 copy: every coefficient rounded once from its FP64 value */
        for (int q = 0; q < 9; ++q) h->s.s[k][q] = (float)h->d.s[k][q];
        h->s.h2inv[k] = (float)h->d.h2inv[k];
        h->s.wjac[k] = (float)h->d.wjac[k];
    }
    if (factor_coarsest_d(&h->d) != OR_OK || factor_coarsest_s(&h->s) != OR_OK) {
        or_hier_free(h);
        return OR_BREAKDOWN;
    }
    for (int k = 0; k < L; ++k)
        if (zebra_factor_d(&h->d, k) != OR_OK || zebra_factor_s(&h->s, k) != OR_OK) {
            or_hier_free(h);
            return OR_ERR_ARG;
        }
    size_t m0 = (size_t)n * n;
    h->fine_v = (double*)calloc(m0, sizeof(double));
    h->fine_f = (double*)calloc(m0, sizeof(double));
    h->fine_v32 = (float*)calloc(m0, sizeof(float));
    h->fine_f32 = (float*)calloc(m0, sizeof(float));
    if (!h->fine_v || !h->fine_f || !h->fine_v32 || !h->fine_f32) { or_hier_free(h); return OR_ERR_ARG; }
    *out = h;
    return OR_OK;
}

/* Fifth and sixth solvers of Section 4: x-line zebra relaxation, coarsening
 * along y only, Galerkin coarse operators.  The fine level (d, L = 1) carries
 * the fine operator for the drivers' residuals; the cycle runs on sd / ss. */
int or_hier_new_semi(int n, double theta, double eps, or_hier** out)
{
    *out = NULL;
    if (n < 1 || !is_pow2((long)n + 1)) return OR_ERR_ARG;
    int L = 1;
    while (((n + 1) >> (L - 1)) > 2) ++L;
    if (L > OR_MAXL) return OR_ERR_ARG;
    or_hier* h = (or_hier*)calloc(1, sizeof(or_hier));
    if (!h) return OR_ERR_ARG;
    h->semi = 1;
    h->theta = theta; h->eps = eps; h->omega = 0.0;
    h->d.L = h->s.L = 1;
    h->d.n[0] = h->s.n[0] = n;
    h->d.h2inv[0] = (double)(n + 1) * (double)(n + 1);
    or_fine_stencil(theta, eps, h->d.s[0]);
    h->d.smoother = h->s.smoother = 1;
    h->sd.L = h->ss.L = L;
    h->sd.nx = h->ss.nx = n;
    h->sd.h2inv = h->d.h2inv[0];
    h->ss.h2inv = (float)h->sd.h2inv;
    int ok = 1;
    for (int k = 0; k < L; ++k) {
        const int ny = ((n + 1) >> k) - 1;
        const size_t m = (size_t)n * ny;
        h->sd.ny[k] = h->ss.ny[k] = ny;
        if (k == 0) memcpy(h->sd.s[0], h->d.s[0], sizeof h->sd.s[0]);
        else sgalerkin_d(h->sd.s[k - 1], h->sd.s[k]);
        for (int q = 0; q < 9; ++q) h->ss.s[k][q] = (float)h->sd.s[k][q];
        h->sd.t[k] = (double*)calloc(m, sizeof(double));
        h->ss.t[k] = (float*)calloc(m, sizeof(float));
        ok = ok && h->sd.t[k] && h->ss.t[k];
        if (k > 0) {
            h->sd.v[k] = (double*)calloc(m, sizeof(double));
            h->sd.f[k] = (double*)calloc(m, sizeof(double));
            h->ss.v[k] = (float*)calloc(m, sizeof(float));
            h->ss.f[k] = (float*)calloc(m, sizeof(float));
            ok = ok && h->sd.v[k] && h->sd.f[k] && h->ss.v[k] && h->ss.f[k];
        }
        ok = ok && sfactor_d(&h->sd, k) == OR_OK && sfactor_s(&h->ss, k) == OR_OK;
    }
    const size_t m0 = (size_t)n * n;
    h->fine_v = (double*)calloc(m0, sizeof(double));
    h->fine_f = (double*)calloc(m0, sizeof(double));
    h->fine_v32 = (float*)calloc(m0, sizeof(float));
    h->fine_f32 = (float*)calloc(m0, sizeof(float));
    if (!ok || !h->fine_v || !h->fine_f || !h->fine_v32 || !h->fine_f32) { or_hier_free(h); return OR_ERR_ARG; }
    *out = h;
    return OR_OK;
}

int or_hier_info(const or_hier* h, int* nlevels, int* sizes, double* stencils)
{
    if (h->semi) {   /* sizes: lines per level; stencils in units of the fine h^2 */
        *nlevels = h->sd.L;
        for (int k = 0; k < h->sd.L; ++k) {
            if (sizes) sizes[k] = h->sd.ny[k];
            if (stencils) memcpy(stencils + 9 * k, h->sd.s[k], 9 * sizeof(double));
        }
        return OR_OK;
    }
    *nlevels = h->d.L;
    for (int k = 0; k < h->d.L; ++k) {
        if (sizes) sizes[k] = h->d.n[k];
        if (stencils) memcpy(stencils + 9 * k, h->d.s[k], 9 * sizeof(double));
    }
    return OR_OK;
}

void or_hier_apply(const or_hier* h, const double* x, double* y)
{
    apply_d(h->d.n[0], h->d.s[0], h->d.h2inv[0], x, y);
}

/* Replaces the operator by the convection-diffusion one.  Every level takes
 * the stencil above at its own mesh width (coarse operators by
 * rediscretisation): Galerkin operators R A P of the upwind operator with
 * bilinear P and full weighting R lose the M-matrix property on coarse levels
 * and the cycle diverges once h |b| is of order one there, while the
 * rediscretised upwind operators keep it.  Damped Jacobi only, and a 1 x 1
 * coarsest level (its "Cholesky factor" is the square root of a positive
 * scalar; larger coarsest matrices are no longer symmetric). */
int or_set_convection(or_hier* h, double bx, double by)
{
    if (h->semi || h->d.smoother != 0 || h->d.nc2 != 1) return OR_ERR_ARG;
    lv_d* D = &h->d;
    lv_s* F = &h->s;
    for (int k = 0; k < D->L; ++k) {
        or_convection_stencil(D->n[k], h->theta, h->eps, bx, by, D->s[k]);
        D->wjac[k] = h->omega / (D->s[k][4] * D->h2inv[k]);
        for (int q = 0; q < 9; ++q) F->s[k][q] = (float)D->s[k][q];
        F->wjac[k] = (float)D->wjac[k];
    }
    free(D->chol); D->chol = NULL;
    free(F->chol); F->chol = NULL;
    if (factor_coarsest_d(D) != OR_OK || factor_coarsest_s(F) != OR_OK) return OR_BREAKDOWN;
    h->conv = 1;
    return OR_OK;
}

int or_set_smoother(or_hier* h, int smoother)
{
    if (smoother != 0 && smoother != 1) return OR_ERR_ARG;
    if (h->conv && smoother != 0) return OR_ERR_ARG;   /* convection-diffusion: damped Jacobi only */
    if (h->semi) return smoother == 1 ? OR_OK : OR_ERR_ARG;   /* always x-line zebra */
    h->d.smoother = h->s.smoother = smoother;
    return OR_OK;
}

void or_zebra_relax(or_hier* h, int dir, double* v, const double* f)
{
    if (h->semi) {   /* one x-line relaxation of the fine level (dir ignored) */
        h->sd.v[0] = v;
        h->sd.f[0] = (double*)f;
        szebra_d(&h->sd, 0);
        h->sd.v[0] = NULL;
        h->sd.f[0] = NULL;
        return;
    }
    h->d.v[0] = v;
    h->d.f[0] = (double*)f;
    zebra_d(&h->d, 0, dir);
    h->d.v[0] = NULL;
    h->d.f[0] = NULL;
}

int or_zebra_tables(const or_hier* h, int level, int dir, double* rp, double* um)
{
    if (h->semi) {   /* x-lines only, nx entries */
        if (level < 1 || level > h->sd.L || dir != 0) return OR_ERR_ARG;
        memcpy(rp, h->sd.zp[level - 1], sizeof(double) * (size_t)h->sd.nx);
        memcpy(um, h->sd.zu[level - 1], sizeof(double) * (size_t)h->sd.nx);
        return OR_OK;
    }
    if (level < 1 || level > h->d.L || (dir != 0 && dir != 1)) return OR_ERR_ARG;
    const int k = level - 1;
    memcpy(rp, h->d.zp[k][dir], sizeof(double) * (size_t)h->d.n[k]);
    memcpy(um, h->d.zu[k][dir], sizeof(double) * (size_t)h->d.n[k]);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* cycles                                                               */
/* ------------------------------------------------------------------ */

int64_t or_cycle(or_hier* h, int kind, int param, int nu1, int nu2,
                 double* v, const double* f, int32_t* tr, int64_t cap)
{
    or_tr t = {tr, cap, 0};
    if (h->semi) {   /* only the kappa-cycle (Algorithm 3) is defined on these levels */
        if (kind != 0) return -1;
        h->sd.v[0] = v;
        h->sd.f[0] = (double*)f;
        skcycle_d(&h->sd, 1, param, nu1, nu2, &t);
        h->sd.v[0] = NULL;
        h->sd.f[0] = NULL;
        return t.len;
    }
    h->d.v[0] = v;
    h->d.f[0] = (double*)f;
    if (kind == 0) kcycle_d(&h->d, 1, param, nu1, nu2, &t);
    else if (kind == 1) gcycle_d(&h->d, 1, param, nu1, nu2, &t);
    else fcycle_d(&h->d, 1, nu1, nu2, &t);
    h->d.v[0] = NULL;
    h->d.f[0] = NULL;
    return t.len;
}

void or_kcycle_f32(or_hier* h, int kappa, int nu1, int nu2, float* v, const float* f)
{
    if (h->semi) {
        h->ss.v[0] = v;
        h->ss.f[0] = (float*)f;
        skcycle_s(&h->ss, 1, kappa, nu1, nu2, NULL);
        h->ss.v[0] = NULL;
        h->ss.f[0] = NULL;
        return;
    }
    h->s.v[0] = v;
    h->s.f[0] = (float*)f;
    kcycle_s(&h->s, 1, kappa, nu1, nu2, NULL);
    h->s.v[0] = NULL;
    h->s.f[0] = NULL;
}

/* ------------------------------------------------------------------ */
/* drivers                                                              */
/* ------------------------------------------------------------------ */

/* Norms and dot products: Dot2 of Ogita, Rump and Oishi ("Accurate sum and
 * dot product", SIAM J. Sci. Comput. 26, 2005, Algorithm 5.3).  Every product
 * is split into its rounded value and its exact rounding error (TwoProduct,
 * with an explicit fused multiply-add), the running sum is split likewise
 * (TwoSum, Knuth's six-operation form), the errors are summed in ordinary
 * floating point and added once at the end.  The result is as accurate as if
 * computed in twice the working precision and then rounded, so two
 * summation orders agree to the last bit unless the exact value lies within
 * about n u^2 (relative) of a rounding boundary. */
static void two_sum(double a, double b, double* s, double* e)
{
    const double x = a + b;
    const double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static void two_prod(double a, double b, double* p, double* e)
{
    const double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

static double dot(const double* x, const double* y, size_t m)
{
    double s = 0.0, c = 0.0;
    for (size_t k = 0; k < m; ++k) {
        double h, r, q;
        two_prod(x[k], y[k], &h, &r);
        two_sum(s, h, &s, &q);
        c = c + (q + r);
    }
    return s + c;
}

static double sumsq(const double* x, size_t m) { return dot(x, x, m); }

double or_dot2(const double* x, const double* y, int64_t m) { return dot(x, y, (size_t)m); }

/* residual of the fine FP64 problem and its squared 2-norm */
static double fine_residual(or_hier* h, const double* u, const double* f, double* r)
{
    resid_d(h->d.n[0], h->d.s[0], h->d.h2inv[0], u, f, r);
    return sumsq(r, (size_t)h->d.n[0] * h->d.n[0]);
}

int or_solve(or_hier* h, int kappa, int nu1, int nu2, double* u, const double* f,
             double tol, int maxit, int mode, int* iters, double* hist)
{
    size_t m = (size_t)h->d.n[0] * h->d.n[0];
    double* r = h->fine_f;   /* scratch: residual */
    double denom, ratio0 = 0.0;
    *iters = 0;
    if (kappa < 1 || nu1 < 0 || nu2 < 0 || maxit < 0) return OR_ERR_ARG;
    if (mode == 0) denom = sqrt(sumsq(f, m));
    else denom = sqrt(sumsq(u, m));
    if (!isfinite(denom)) return OR_ERR_NONFINITE;
    for (int k = 0;; ++k) {
        double num = (mode == 0) ? sqrt(fine_residual(h, u, f, r)) : sqrt(sumsq(u, m));
        double ratio = (denom > 0.0) ? num / denom : 0.0;
        if (hist) hist[k] = ratio;
        *iters = k;
        if (!isfinite(ratio)) return OR_ERR_NONFINITE;
        if (k == 0) ratio0 = ratio;
        if (ratio < tol) return OR_OK;
        if (ratio > 1e3 * ratio0) return OR_DIVERGED;
        if (k == maxit) return OR_NOT_CONVERGED;
        or_cycle(h, 0, kappa, nu1, nu2, u, f, NULL, 0);
    }
}

double or_ir_scale(double ss, int64_t npoints)
{
    if (!(ss > 0.0) || !isfinite(ss)) return 1.0;
    int e = ilogb(ss / (double)npoints);
    int k = (int)floor((double)e / 2.0);
    return ldexp(1.0, -k);
}

/* e = B r with B one zero-guess kappa-cycle in FP32:  the residual is scaled
 * by a power of two, rounded to FP32, cycled, and scaled back in FP64 */
static void precond_f32(or_hier* h, int kappa, int nu1, int nu2, const double* r,
                        double ss, double* z)
{
    size_t m = (size_t)h->d.n[0] * h->d.n[0];
    double sc = or_ir_scale(ss, (int64_t)m);
    for (size_t q = 0; q < m; ++q) {
        h->fine_f32[q] = (float)(sc * r[q]);
        h->fine_v32[q] = 0.0f;
    }
    or_kcycle_f32(h, kappa, nu1, nu2, h->fine_v32, h->fine_f32);
    for (size_t q = 0; q < m; ++q) z[q] = (double)h->fine_v32[q] / sc;
}

int or_ir_solve(or_hier* h, int kappa, int nu1, int nu2, double* u, const double* f,
                double tol, int maxit, int* iters, double* hist)
{
    size_t m = (size_t)h->d.n[0] * h->d.n[0];
    double* r = h->fine_f;
    double* e = h->fine_v;
    double ssf = sumsq(f, m);
    double normf = sqrt(ssf), ratio0 = 0.0;
    /* the FP32 right-hand side of refinement step k is scaled by a power of
     * two taken from the previous residual (from f for the first step) */
    double ss_prev = ssf;
    *iters = 0;
    if (kappa < 1 || nu1 < 0 || nu2 < 0 || maxit < 0) return OR_ERR_ARG;
    if (!isfinite(normf)) return OR_ERR_NONFINITE;
    for (int k = 0;; ++k) {
        double ss = fine_residual(h, u, f, r);
        double ratio = (normf > 0.0) ? sqrt(ss) / normf : 0.0;
        if (hist) hist[k] = ratio;
        *iters = k;
        if (!isfinite(ratio)) return OR_ERR_NONFINITE;
        if (k == 0) ratio0 = ratio;
        if (ratio < tol) return OR_OK;
        if (ratio > 1e3 * ratio0) return OR_DIVERGED;
        if (k == maxit) return OR_NOT_CONVERGED;
        precond_f32(h, kappa, nu1, nu2, r, ss_prev, e);
        ss_prev = ss;
        for (size_t q = 0; q < m; ++q) u[q] = u[q] + e[q];
    }
}

/* Preconditioned CG (Section 4, the second solver): x_0 = 0, r_0 = f,
 * z_k = B r_k with B one zero-guess kappa-cycle, Fletcher-Reeves
 * beta_k = (r_k . z_k) / (r_{k-1} . z_{k-1}), p_k = z_k + beta_k p_{k-1},
 * alpha_k = (r_k . z_k) / (p_k . A p_k), x_{k+1} = x_k + alpha_k p_k,
 * r_{k+1} = r_k - alpha_k A p_k.  The recurrence residual r_k drifts from the
 * true residual f - A x_k by rounding; when ||r_{k+1}|| / ||f|| falls below tol
 * the true residual is formed in FP64 and decides: below tol the iteration
 * stops, otherwise r_{k+1} is replaced by the true residual and the iteration
 * goes on (residual replacement).  hist[k] is ||r_k|| / ||f|| of the residual
 * the iteration carries after k steps (the true one where it was formed). */
int or_pcg(or_hier* h, int kappa, int nu1, int nu2, int precond_f32_flag,
           double* u, const double* f, double tol, int maxit, int* iters, double* hist)
{
    size_t m = (size_t)h->d.n[0] * h->d.n[0];
    int rc = OR_OK;
    *iters = 0;
    if (kappa < 1 || nu1 < 0 || nu2 < 0 || maxit < 0) return OR_ERR_ARG;
    if (h->conv) return OR_ERR_ARG;   /* CG needs a symmetric operator */
    double* r = (double*)malloc(m * sizeof(double));
    double* z = (double*)malloc(m * sizeof(double));
    double* p = (double*)malloc(m * sizeof(double));
    double* q = (double*)malloc(m * sizeof(double));
    if (!r || !z || !p || !q) { rc = OR_ERR_ARG; goto done; }

    /* x_0 = 0, r_0 = f */
    for (size_t k = 0; k < m; ++k) { u[k] = 0.0; r[k] = f[k]; }
    double normf = sqrt(sumsq(f, m));
    if (!isfinite(normf)) { rc = OR_ERR_NONFINITE; goto done; }
    double ssr = sumsq(r, m);
    double ratio = (normf > 0.0) ? sqrt(ssr) / normf : 0.0;
    if (hist) hist[0] = ratio;
    if (!isfinite(ratio)) { rc = OR_ERR_NONFINITE; goto done; }
    if (ratio < tol) goto done;

    double rz = 0.0;
    for (int it = 0;; ++it) {
        if (it == maxit) { rc = OR_NOT_CONVERGED; break; }
        /* z = B r */
        if (precond_f32_flag) {
            precond_f32(h, kappa, nu1, nu2, r, ssr, z);
        } else {
            memset(z, 0, m * sizeof(double));
            or_cycle(h, 0, kappa, nu1, nu2, z, r, NULL, 0);
        }
        double rz_new = dot(r, z, m);
        if (it == 0) {
            memcpy(p, z, m * sizeof(double));
        } else {
            double beta = rz_new / rz;   /* Fletcher-Reeves */
            for (size_t k = 0; k < m; ++k) p[k] = z[k] + beta * p[k];
        }
        rz = rz_new;
        apply_d(h->d.n[0], h->d.s[0], h->d.h2inv[0], p, q);
        double pq = dot(p, q, m);
        if (!(pq > 0.0) || !isfinite(pq)) { rc = isfinite(pq) ? OR_BREAKDOWN : OR_ERR_NONFINITE; break; }
        double alpha = rz / pq;
        for (size_t k = 0; k < m; ++k) {
            u[k] = u[k] + alpha * p[k];
            r[k] = r[k] - alpha * q[k];
        }
        ssr = sumsq(r, m);
        ratio = sqrt(ssr) / normf;
        *iters = it + 1;
        if (isfinite(ratio) && ratio < tol) {
            /* the recurrence says converged: the true residual decides */
            ssr = fine_residual(h, u, f, r);
            ratio = sqrt(ssr) / normf;
        }
        if (hist) hist[it + 1] = ratio;
        if (!isfinite(ratio)) { rc = OR_ERR_NONFINITE; break; }
        if (ratio < tol) break;
    }
done:
    free(r); free(z); free(p); free(q);
    return rc;
}

void or_grad_params(const or_hier* h, double theta, double eps, const double* lam,
                    const double* u, double* dtheta, double* deps)
{
    int n = h->d.n[0];
    size_t m = (size_t)n * n;
    double dth[9], de[9];
    or_fine_stencil_derivs(theta, eps, dth, de);
    double* y = (double*)malloc(m * sizeof(double));
    apply_d(n, dth, h->d.h2inv[0], u, y);
    *dtheta = -dot(lam, y, m);
    apply_d(n, de, h->d.h2inv[0], u, y);
    *deps = -dot(lam, y, m);
    free(y);
}

/* the FP32 instantiations only need the kappa-cycle */
static void (*const or_unused_fcycle_s)(lv_s*, int, int, int, or_tr*) __attribute__((unused)) = fcycle_s;
static void (*const or_unused_sgalerkin_s)(const float*, float*) __attribute__((unused)) = sgalerkin_s;
