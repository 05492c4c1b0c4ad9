// kc_internal.h -- device-visible tables and kernel launch interface shared by
// the host runtime (kc_runtime.cpp) and the HIP kernels (kc_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kc {

constexpr int MAXL = 16;          // levels per instance
constexpr int NTABLES = 1 + 4 * MAXL;   // block tables: whole fine level, fused grid per depth, per level, zebra per level,
                                        // fused post-smoothing per depth (where its strips differ from the pre-smoothing's)
constexpr int ZLDS_TABLE = 480;   // persistent-kernel LDS elements for the zebra tables of levels 1 .. 63 (4 n each)
constexpr int TX = 64;            // grid-kernel tile width  (one wave64 row)
constexpr int TY = 32;            // grid-kernel tile height
constexpr int TS = 16;            // small-level tile side of the fused kernels
constexpr int TM = 32;            // mid-level tile side of the fused kernels
constexpr int TT = 8;             // tiny tile side of the fused kernels (one point per thread and phase)
constexpr int STRIP_BLOCK_W = 216; // columns of a streaming block (4 strips of 54)
constexpr int GRID_THREADS = 256; // threads of the grid-wide kernels
constexpr int ZEBRA_QUAD_LPW = 4; // lines per wave of the zebra line kernel on its largest levels
constexpr int HIST_CAP = 8192;    // relres history entries kept per instance

// one level of one instance; arrays are row-major with leading dimension ld.
// A holds the current estimate between calls, B is the second sweep buffer,
// F the right-hand side.  Element type is double or float by precision.
struct LevelDev {
    void* A;
    void* B;
    void* F;
    int32_t n;               // lines (rows) of the level
    int32_t nx;              // points per line (columns): n, or the fine n on semi-coarsened levels
    int32_t lda, ldb, ldf;   // leading dimensions of A, B and F
    double fscale;           // F is multiplied by fscale when loaded (h^2 for a user f, else 1)
};

struct InstDev {
    int32_t L;           // number of levels
    int32_t cut;         // first depth handled by the persistent coarse kernel
    int32_t nc2;         // order of the coarsest matrix
    int32_t sub_lds;     // LDS elements used by the persistent kernel
    double s64[MAXL][9]; // h^2-scaled stencils, s[3*(b+1)+(a+1)] for offset (a, b)
    float s32[MAXL][9];
    double w64[MAXL];    // omega / s[4]
    float w32[MAXL];
    LevelDev lev[MAXL];  // cycle levels (level 0 may alias user arrays)
    const double* chol64;  // lower Cholesky factor of the coarsest matrix, nc2 x nc2 row-major (scaled system)
    const float* chol32;
    const double* zt64[MAXL];  // zebra line-solve tables of level d: reciprocal pivots, multipliers (x-lines), then (y-lines), n each
    const float* zt32[MAXL];
    int32_t lds_off[MAXL]; // persistent kernel: element offset of level d's three (n+2)^2 arrays
    int32_t ops_beg[MAXL + 1]; // persistent kernel op list of a call with counter k = 1..MAXL+1
    int32_t ops_len[MAXL + 1];
    int32_t zops_beg[MAXL + 1];  // the same for zebra relaxation (no register calls)
    int32_t zops_len[MAXL + 1];
    const uint32_t* ops;       // op list storage
    // FP64 vectors of the drivers (refinement / PCG); fine level, ld = ldv
    double* u;           // user solution
    const double* f;     // user right-hand side (unscaled)
    int32_t ldu, ldf;
    double* r;           // PCG residual
    double* z;           // PCG preconditioned residual
    double* p;           // PCG search direction
    double* q;           // PCG A p
    int32_t ldv;         // leading dimension of r, z, p, q
    int32_t n0;          // fine size
    double h2;           // fine h^2
    double h2inv;        // fine 1/h^2
    const double* x;     // generic FP64 input of apply / gradient (x or lam)
    double* y;           // generic FP64 output of apply, second input (u) of gradient
    int32_t ldx, ldy;
    double ds_th[9];     // d stencil / d theta (fine, unscaled coefficients)
    double ds_ep[9];     // d stencil / d eps
};

// per-instance solver state, written by the finalize kernel of reductions
struct InstState {
    double ssf;        // ||F||^2 (scaled units)
    double relres;     // last relative residual
    double relres0;    // first relative residual
    double scale;      // power-of-two scale for the next FP32 right-hand side
    double scale_used; // scale applied to the current FP32 right-hand side
    double rz;         // PCG r.z
    double pq;         // PCG p.q
    double alpha, beta;
    double tol;
    double dth, deps;  // gradient results
    int32_t iters;     // completed cycles / iterations
    int32_t status;    // kc_status of this instance once done
    int32_t done;      // nonzero: every kernel skips this instance
    int32_t maxit;
    int32_t check;     // PCG: the recurrence residual passed tol; the true residual decides next
};

// reduction kinds, applied per instance by the finalize kernel after a reduction
enum Finalize : int32_t {
    FIN_NONE = 0,
    FIN_SSF = 1,        // ssf = sum; relres0 bookkeeping reset
    FIN_STOP = 2,       // stand-alone stop test on sum = ||F - S v||^2
    FIN_STOP_IR = 3,    // same, plus the FP32 scale for the next cycle
    FIN_PQ = 4,         // pq = sum; alpha = rz / pq (breakdown check)
    FIN_PCG_R = 5,      // PCG residual test on sum = ||r||^2, plus FP32 scale
    FIN_RZ = 6,         // rz_new = sum; beta = rz_new / rz
    FIN_GRAD = 7,       // dth, deps = sums
    FIN_PCG_INIT = 8,   // ssf = ||r_0||^2, first residual test, FP32 scale
    FIN_PCG_TRUE = 9,   // PCG true-residual test on sum = ||F - S u||^2 (instances with check set)
};

// persistent coarse kernel operations
enum SubOp : uint32_t {
    SOP_WCALL = 0,    // a whole call (counter k) on a level that wave 0 runs in registers
    SOP_PRE = 1,      // nu1 sweeps (zero guess flag) + residual + full weighting to depth+1
    SOP_POST = 2,     // prolong-add from depth+1 + nu2 sweeps
    SOP_SOLVE = 3,    // coarsest direct solve
};
// op word: kind (bits 0-1) | depth (2-5) | zero-guess flag (6) | lg = log2(n + 1)
// of the level (7-9) | counter k of a register call (10-14) | LDS element
// offset of the level's three arrays (15-31)
constexpr uint32_t SOP_KMAX = 31, SOP_OFFMAX = (1u << 17) - 1;
__host__ __device__ inline uint32_t sop_make(uint32_t op, uint32_t depth, uint32_t zg, uint32_t lg, uint32_t off,
                                             uint32_t k = 0)
{
    return op | (depth << 2) | (zg << 6) | (lg << 7) | (k << 10) | (off << 15);
}
__host__ __device__ inline int sop_kind(uint32_t w) { return (int)(w & 3u); }
__host__ __device__ inline int sop_depth(uint32_t w) { return (int)((w >> 2) & 15u); }
__host__ __device__ inline bool sop_zg(uint32_t w) { return ((w >> 6) & 1u) != 0; }
__host__ __device__ inline int sop_lg(uint32_t w) { return (int)((w >> 7) & 7u); }
__host__ __device__ inline int sop_k(uint32_t w) { return (int)((w >> 10) & 31u); }
__host__ __device__ inline int sop_off(uint32_t w) { return (int)(w >> 15); }

// arguments of a grid-wide stage launch
struct StageArgs {
    const InstDev* inst;
    InstState* st;
    const int32_t* tile_off;  // prefix sums over instances of tiles at this depth (count + 1)
    double* partial;          // per block: two Dot2 sums (value, error term each)
    double* hist;             // relres history, HIST_CAP per instance
    int32_t count;
    int32_t depth;
    int32_t zg;               // current estimate is zero on entry
    int32_t fin;              // Finalize kind of this launch's reduction
    int32_t nu;               // sweeps for fused pre/post kernels
    int32_t src, dst;         // buffer selectors for unfused kernels (0 = A, 1 = B)
    int32_t flags;            // fused kernels' shape: bit 0 = 16 x 16 tiles; bit 4 = 32 x 32 tiles; bit 5 = 8 x 8
                              // tiles; bit 1 = streaming strips, rows 16 << bits 2-3; none = 64 x 32 tiles
    int32_t semi;             // one-kernel-per-operation launch on semi-coarsened (rectangular) levels:
                              // transfers along y only
};

// arguments of a persistent coarse-kernel launch
struct SubArgs {
    const InstDev* inst;
    InstState* st;
    const int32_t* list;      // instance ids handled (one workgroup each)
    int32_t count;
    int32_t first;            // list[0] (a launch for one instance reads no list)
    int32_t depth;            // depth of the calls
    int32_t kappa;            // counter of the first call
    int32_t pair;             // 1: call(kappa) then call(kappa-1) from zero; 0: one call from A
    int32_t nu1, nu2;
    int32_t zg;               // single call: estimate is zero on entry
    int32_t fin;              // single call: FIN_STOP computes the stop test first
    int32_t wave_n;           // levels with n <= wave_n are run by one wave
    int32_t smoother;         // 0 damped Jacobi, 1 alternating zebra line relaxation
    double* hist;
    // single-instance launch on an internal level (the library's own arrays): what the
    // kernel would otherwise read from the instance table before it can issue its loads
    // (op lists of the two calls, the top level's arrays, the coarsest factor); ops1 is
    // null when the kernel reads them from the table
    const uint32_t* ops1;
    const uint32_t* ops2;
    int32_t n1, n2;           // op counts of the first and the second call (0: none)
    int32_t n0;               // size of the top level
    int32_t sub_lds;          // LDS elements of the instance's levels
    const void* F0;           // top level's right-hand side and current estimate
    void* A0;
    int32_t ldf0, lda0;
    double fs0;               // fscale of F0
    const void* chol0;        // coarsest factor in the hierarchy's precision
};

// kernel launchers (kc_kernels.hip)
enum GridKernel : int32_t {
    GK_SWEEP = 1,      // unfused: dst = src + w (F - S src)
    GK_RESID = 2,      // unfused: dst = F - S src
    GK_RESTRICT = 3,   // unfused: F[d+1] = P^T src
    GK_ZERO = 4,       // unfused: A[d] = 0
    GK_PROLONG = 5,    // unfused: dst = P A[d+1]
    GK_ADD = 6,        // unfused: src += dst
    GK_COPY = 7,       // unfused: dst = src
    GK_NORM = 8,       // ||F - S A||^2 with finalize
    GK_PRE = 9,        // fused pre-smoothing + residual + restriction (optional input norm)
    GK_POST = 10,      // fused prolong-add + post-smoothing
    GK_SSF = 11,       // ||F||^2 at level 0
    GK_IR_RESID = 12,  // r = F - S u (FP64), norm, F32 = scale * r
    GK_IR_UPDATE = 13, // u += A32 / scale
    GK_PCG_INIT = 14,  // u = 0, r = F, ||r||^2
    GK_PCG_PRECIN = 15,// level-0 cycle input from r (FP32 scaled copy or FP64 alias)
    GK_PCG_RZ = 16,    // z from the cycle (FP32 -> FP64 unscale), r.z, beta
    GK_PCG_P = 21,     // p = z + beta p
    GK_PCG_AP = 17,    // q = S p, p.q, alpha
    GK_PCG_UPD = 18,   // u += alpha p, r -= alpha q, ||r||^2
    GK_APPLY = 19,     // y = S x / h^2
    GK_GRAD = 20,      // -lam^T dS u / h^2 for theta and eps
    GK_ZERO_SELF = 22, // unfused: A[d] = 0 on the launch's own level
    GK_POSTPRE = 23,   // fused junction of sibling calls: post (nu2 = src) of the first + pre (nu) of the second
    GK_ZEBRA = 24,     // zebra line relaxation in place on buffer src, lines of colour dst, direction nu (0 x, 1 y)
    GK_PCG_TRUE = 25,  // instances with check set: r = F - S u (FP64, replaces the recurrence residual), ||r||^2
};

// launches kernel k (and, when a.fin is set and with_finalize, the finalize kernel after it)
hipError_t launch_grid(GridKernel k, bool f32, const StageArgs& a, int32_t nblocks, hipStream_t s, bool with_finalize = true);
hipError_t launch_finalize(const StageArgs& a, hipStream_t s);
hipError_t launch_subtree(bool f32, const SubArgs& a, int32_t threads, int32_t lds_bytes, hipStream_t s);
hipError_t launch_coarsest(bool f32, const SubArgs& a, hipStream_t s);
hipError_t prepare_subtree(bool f32, int32_t lds_bytes);
int32_t max_lds_bytes();

}  // namespace kc
