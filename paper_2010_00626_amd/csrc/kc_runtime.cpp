// kc_runtime.cpp -- host runtime of libkcycle.so: hierarchy setup, workspace
// layout, the flattened kappa-cycle schedule, hipGraph capture and replay, the
// stand-alone / refinement / PCG drivers and the C-ABI (include/kcycle.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/kcycle.h"
#include "kc_internal.h"

using namespace kc;

namespace {

thread_local std::string g_err;

kc_status fail(kc_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) return fail(KC_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t ALIGN = 256;
constexpr int OPS_CAP = 4096;          // op words reserved per instance
constexpr int KMAX = MAXL + 1;         // counters above this all give the W-cycle

size_t align_up(size_t x, size_t a = ALIGN) { return (x + a - 1) / a * a; }
int ld_of(int n) { return (n + 63) / 64 * 64; }
bool is_pow2(long x) { return x > 0 && (x & (x - 1)) == 0; }

// ---------------------------------------------------------------------------
// discrete problem on the host (Section 4): fine stencil, its derivatives,
// Galerkin coarse stencils and the coarsest inverse
// ---------------------------------------------------------------------------
void fine_stencil(double theta, double eps, double s[9])
{
    const double C = std::cos(theta), S = std::sin(theta);
    const double cross = 0.5 * (1.0 - eps) * C * S;
    const double we = -(C * C + eps * S * S);
    const double sn = -(eps * C * C + S * S);
    const double t[9] = {-cross, sn, cross, we, 2.0 * (1.0 + eps), we, cross, sn, -cross};
    std::memcpy(s, t, sizeof t);
}

// convection-diffusion -div(D grad u) + b . grad u on an n x n grid: the
// diffusion stencil plus first-order upwind convection (backward along a
// positive velocity component, forward along a negative one), h^2-scaled: the
// centre gains h |bx| + h |by|, the upwind neighbours lose h max(+-b, 0).  Coarse
// levels take the same operator at their own mesh width (rediscretisation):
// Galerkin stencils of the upwind operator lose the M-matrix property on
// coarse levels and the cycle diverges.
void convection_stencil(int n, double theta, double eps, double bx, double by, double s[9])
{
    fine_stencil(theta, eps, s);
    const double h = 1.0 / (double)(n + 1);
    const double cx = h * bx, cy = h * by;
    s[4] = s[4] + (std::fabs(cx) + std::fabs(cy));
    s[3] = s[3] - std::fmax(cx, 0.0);
    s[5] = s[5] - std::fmax(-cx, 0.0);
    s[1] = s[1] - std::fmax(cy, 0.0);
    s[7] = s[7] - std::fmax(-cy, 0.0);
}

void fine_stencil_derivs(double theta, double eps, double dth[9], double deps[9])
{
    const double C = std::cos(theta), S = std::sin(theta);
    const double xc = 0.5 * (1.0 - eps) * (C * C - S * S), xw = 2.0 * (1.0 - eps) * C * S;
    const double a[9] = {-xc, -xw, xc, xw, 0.0, xw, xc, -xw, -xc};
    std::memcpy(dth, a, sizeof a);
    const double ec = -0.5 * C * S, ew = -S * S, en = -C * C;
    const double b[9] = {-ec, en, ec, ew, 2.0, ew, ec, en, -ec};
    std::memcpy(deps, b, sizeof b);
}

double w1(int a) { return a == 0 ? 1.0 : 0.5; }

// Galerkin coarse stencil, A_c = R A P with R = P^T / 4 (bilinear P): with
// h_c = 2h the h^2-scaled stencil is S_c = 4 R S P.  It is read off by applying
// P, then S, then R to a coarse unit vector on a 5 x 5 coarse grid (11 x 11
// fine), far enough from the boundary that nothing is cut off.  Every sum runs
// south to north, west to east, so each entry is rounded exactly as the
// level operators of the definition round it.
void galerkin(const double sf[9], double sc[9])
{
    constexpr int NC = 5, NF = 11;
    double e[NF * NF], ae[NF * NF];
    auto ec = [](int J, int I) { return (J == 2 && I == 2) ? 1.0 : 0.0; };
    for (int j = 0; j < NF; ++j)          // e = P e_c (gather)
        for (int i = 0; i < NF; ++i) {
            double acc = 0.0;
            for (int J = (j - 1) / 2 - 1; J <= j / 2; ++J) {
                const int dy = j - (2 * J + 1);
                if (dy < -1 || dy > 1) continue;
                for (int I = (i - 1) / 2 - 1; I <= i / 2; ++I) {
                    const int dx = i - (2 * I + 1);
                    if (dx < -1 || dx > 1) continue;
                    const double v = (J < 0 || J >= NC || I < 0 || I >= NC) ? 0.0 : ec(J, I);
                    acc += (w1(dx) * w1(dy)) * v;
                }
            }
            e[j * NF + i] = acc;
        }
    for (int j = 0; j < NF; ++j)          // ae = S e
        for (int i = 0; i < NF; ++i) {
            double acc = 0.0;
            for (int b = -1; b <= 1; ++b)
                for (int a = -1; a <= 1; ++a) {
                    const int jj = j + b, ii = i + a;
                    const double x = (jj < 0 || jj >= NF || ii < 0 || ii >= NF) ? 0.0 : e[jj * NF + ii];
                    acc += sf[3 * (b + 1) + (a + 1)] * x;
                }
            ae[j * NF + i] = acc * 1.0;
        }
    for (int b0 = -1; b0 <= 1; ++b0)      // S_c = 4 R ae around coarse (2, 2)
        for (int a0 = -1; a0 <= 1; ++a0) {
            const int J = 2 + b0, I = 2 + a0;
            double acc = 0.0;
            for (int b = -1; b <= 1; ++b)
                for (int a = -1; a <= 1; ++a)
                    acc += (w1(a) * w1(b) / 4.0) * ae[(2 * J + 1 + b) * NF + (2 * I + 1 + a)];
            sc[3 * (b0 + 1) + (a0 + 1)] = 4.0 * acc;
        }
}

// Galerkin stencil of the next semi-coarsened level (Section 4, fifth and sixth
// solvers), s_c = R s P with P linear interpolation along y and R = P^T / 2,
// every stencil in units of the fine level's h^2 (x is never coarsened).  It is
// read off by applying P, then s, then R to a coarse unit vector on a grid of 5
// columns and 5 coarse (11 fine) lines, with the same loop orders as the
// definition, so each entry is rounded as the definition rounds it.
void semi_galerkin(const double sf[9], double sc[9])
{
    constexpr int NX = 5, NYC = 5, NYF = 11;
    double e[NX * NYF], ae[NX * NYF];
    for (int j = 0; j < NYF; ++j)          // e = P e_c (gather along y)
        for (int i = 0; i < NX; ++i) {
            double acc = 0.0;
            for (int J = (j - 1) / 2 - 1; J <= j / 2; ++J) {
                const int dy = j - (2 * J + 1);
                if (dy < -1 || dy > 1) continue;
                const double v = (J < 0 || J >= NYC) ? 0.0 : ((J == 2 && i == 2) ? 1.0 : 0.0);
                acc += w1(dy) * v;
            }
            e[j * NX + i] = acc;
        }
    for (int j = 0; j < NYF; ++j)          // ae = s e
        for (int i = 0; i < NX; ++i) {
            double acc = 0.0;
            for (int b = -1; b <= 1; ++b)
                for (int a = -1; a <= 1; ++a) {
                    const int jj = j + b, ii = i + a;
                    const double x = (jj < 0 || jj >= NYF || ii < 0 || ii >= NX) ? 0.0 : e[jj * NX + ii];
                    acc += sf[3 * (b + 1) + (a + 1)] * x;
                }
            ae[j * NX + i] = acc * 1.0;
        }
    for (int b0 = -1; b0 <= 1; ++b0)      // s_c = R ae around coarse line 2, column 2
        for (int a0 = -1; a0 <= 1; ++a0) {
            const int J = 2 + b0, i = 2 + a0;
            double acc = 0.0;
            for (int b = -1; b <= 1; ++b) acc += (w1(b) / 2.0) * ae[(2 * J + 1 + b) * NX + i];
            sc[3 * (b0 + 1) + (a0 + 1)] = acc;
        }
}

// lower Cholesky factor (row-major) of the coarsest matrix of stencil s on an
// nc x nc grid, in the arithmetic type R; the h^2 scaling of the system is a
// power of four, so this factor is the unscaled one times a power of two
template <typename R>
bool coarse_cholesky(int nc, const double s64[9], std::vector<R>& Lc)
{
    const int m = nc * nc;
    Lc.assign((size_t)m * m, R(0));
    std::vector<R>& A = Lc;
    for (int j = 0; j < nc; ++j)
        for (int i = 0; i < nc; ++i)
            for (int b = -1; b <= 1; ++b)
                for (int a = -1; a <= 1; ++a) {
                    const int jj = j + b, ii = i + a;
                    if (jj < 0 || jj >= nc || ii < 0 || ii >= nc) continue;
                    A[(size_t)(j * nc + i) * m + (jj * nc + ii)] = (R)s64[3 * (b + 1) + (a + 1)];
                }
    for (int p = 0; p < m; ++p) {
        for (int q = 0; q <= p; ++q) {
            R acc = A[(size_t)p * m + q];
            for (int k = 0; k < q; ++k) acc -= A[(size_t)p * m + k] * A[(size_t)q * m + k];
            if (p == q) {
                if (!(acc > R(0))) return false;
                A[(size_t)p * m + p] = (R)std::sqrt((double)acc);
            } else {
                A[(size_t)p * m + q] = acc / A[(size_t)q * m + q];
            }
        }
        for (int q = p + 1; q < m; ++q) A[(size_t)p * m + q] = R(0);
    }
    return true;
}

kc_status check_problem(const kc_problem& p, int& L)
{
    if (p.n < 1 || p.n_coarsest < 1 || p.n_coarsest > p.n || !is_pow2((long)p.n + 1) ||
        !is_pow2((long)p.n_coarsest + 1) || p.n_coarsest > 7)
        return fail(KC_ERR_ARG, "n and n_coarsest must be 2^k - 1 with n_coarsest in {1, 3, 7} and <= n");
    if (!(p.eps > 0.0) || !std::isfinite(p.eps) || !std::isfinite(p.theta))
        return fail(KC_ERR_ARG, "eps must be positive and theta finite");
    L = 1;
    while (((p.n + 1) >> (L - 1)) > p.n_coarsest + 1) ++L;
    if (L > MAXL) return fail(KC_ERR_ARG, "too many levels");
    return KC_OK;
}

// ---------------------------------------------------------------------------
// workspace layout (independent of execution options)
// ---------------------------------------------------------------------------
struct InstLayout {
    int L = 0;
    int n[MAXL] = {}, ld[MAXL] = {};
    int nx[MAXL] = {};           // points per line: n, or the fine n on semi-coarsened levels
    bool semi = false;           // levels coarsened along y only
    size_t A[MAXL] = {}, B[MAXL] = {}, F[MAXL] = {};   // cycle arrays by level (A, F of level 0 unused in F64)
    size_t chol64 = 0, chol32 = 0, ops = 0;
    size_t r = 0, z = 0, p = 0, q = 0;
    size_t zt64 = 0, zt32 = 0;   // zebra line-solve tables, per level [1/pivots x | multipliers x | 1/pivots y | multipliers y]
    size_t zoff[MAXL] = {};      // element offset of level d's tables
};

struct Layout {
    size_t inst = 0, state = 0, tiles = 0, lists = 0, partial = 0, hist = 0;
    size_t total = 0;
    int ntables = 0;       // NTABLES tile tables of (count + 1)
    int total_tiles0 = 0;
    std::vector<InstLayout> il;
};

int tiles_of(int n) { return ((n + TX - 1) / TX) * ((n + TY - 1) / TY); }
int tiles_small(int n) { return ((n + TS - 1) / TS) * ((n + TS - 1) / TS); }
int tiles_mid(int n) { return ((n + TM - 1) / TM) * ((n + TM - 1) / TM); }
int tiles_tiny(int n) { return ((n + TT - 1) / TT) * ((n + TT - 1) / TT); }
// zebra launches: the lines of one colour, ZEBRA_QUAD_LPW or two per wave on levels whose lines
// have nx >= quad_n > 0 or nx >= wave_n > 0 points, else one per thread (64 per workgroup);
// k_zebra takes the same decision per instance from the thresholds packed by zebra_flags
int zebra_blocks_lines(int lines, int nx, int wave_n, int quad_n)
{
    const int per_colour = (lines + 1) / 2;
    if (!(wave_n > 0 && nx >= wave_n)) return (per_colour + 63) / 64;
    const int per_block = (GRID_THREADS / 64) * ((quad_n > 0 && nx >= quad_n) ? ZEBRA_QUAD_LPW : 2);
    return (per_colour + per_block - 1) / per_block;
}
int zebra_blocks(int n, int wave_n, int quad_n) { return zebra_blocks_lines(n, n, wave_n, quad_n); }
int zebra_flags(const kc_exec& e) { return e.zebra_wave_n | (e.zebra_quad_n << 15); }
int tiles_rect(int nx, int ny) { return ((nx + TX - 1) / TX) * ((ny + TY - 1) / TY); }
// streaming blocks: STRIP_BLOCK_W columns x R rows, R = 16 << code; 32 rows from 2047^2 up for both
// parts (measured faster than 16 or 64 at 8191^2 and 16383^2); the post-smoothing keeps a shape of its
// own per depth (shape_post) so that the two parts can take different heights
int strip_rows_code(int n) { return n >= 2047 ? 1 : 0; }
int tiles_stream(int n, int code) { return ((n + STRIP_BLOCK_W - 1) / STRIP_BLOCK_W) * ((n + (16 << code) - 1) / (16 << code)); }

// semi: levels coarsened along y only down to one line (every instance the same n)
kc_status make_layout(const kc_problem* probs, int count, kc_precision prec, Layout& lay, bool semi = false)
{
    if (!probs || count < 1) return fail(KC_ERR_ARG, "need at least one problem");
    if (semi)
        for (int i = 0; i < count; ++i) {
            if (probs[i].n != probs[0].n) return fail(KC_ERR_ARG, "semi-coarsened instances must share n");
            if (probs[i].n_coarsest != 1) return fail(KC_ERR_ARG, "semi-coarsening: n_coarsest must be 1 (unused)");
            if (probs[i].n > 16383) return fail(KC_ERR_ARG, "semi-coarsening (x-line zebra) takes n <= 16383");
        }
    if (prec != KC_F64 && prec != KC_F32_CYCLE) return fail(KC_ERR_ARG, "unknown precision");
    const size_t T = (prec == KC_F64) ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return o;
    };
    lay.il.assign(count, InstLayout());
    lay.inst = take(sizeof(InstDev) * count);
    lay.state = take(sizeof(InstState) * count);
    lay.ntables = NTABLES;
    lay.tiles = take(sizeof(int32_t) * (size_t)lay.ntables * (count + 1));
    lay.lists = take(sizeof(int32_t) * (size_t)2 * MAXL * count);
    int tiles0 = 0;
    for (int i = 0; i < count; ++i) {
        int L;
        kc_status st = check_problem(probs[i], L);
        if (st != KC_OK) return st;
        tiles0 += std::max(std::max(std::max(tiles_of(probs[i].n), tiles_small(probs[i].n)), tiles_stream(probs[i].n, 0)),
                           tiles_tiny(probs[i].n));   // any shape at depth 0
    }
    lay.total_tiles0 = tiles0;
    lay.partial = take(sizeof(double) * 4 * (size_t)tiles0);
    lay.hist = take(sizeof(double) * (size_t)HIST_CAP * count);
    for (int i = 0; i < count; ++i) {
        InstLayout& il = lay.il[i];
        check_problem(probs[i], il.L);
        il.semi = semi;
        if (semi) {   // down to a single line
            il.L = 1;
            while (((probs[i].n + 1) >> (il.L - 1)) > 2) ++il.L;
        }
        for (int d = 0; d < il.L; ++d) {
            il.n[d] = ((probs[i].n + 1) >> d) - 1;
            il.nx[d] = semi ? probs[i].n : il.n[d];
            il.ld[d] = ld_of(il.nx[d]);
            const size_t bytes = (size_t)il.n[d] * il.ld[d] * T;
            il.B[d] = take(bytes);
            if (d > 0 || prec == KC_F32_CYCLE) {
                il.A[d] = take(bytes);
                il.F[d] = take(bytes);
            }
        }
        const int m = probs[i].n_coarsest * probs[i].n_coarsest;
        il.chol64 = take(sizeof(double) * m * m);
        il.chol32 = take(sizeof(float) * m * m);
        il.ops = take(sizeof(uint32_t) * OPS_CAP);
        size_t zt = 0;
        for (int d = 0; d < il.L; ++d) {
            il.zoff[d] = zt;
            zt += 4 * (size_t)il.nx[d];
        }
        il.zt64 = take(sizeof(double) * zt);
        il.zt32 = take(sizeof(float) * zt);
        const size_t v64 = (size_t)il.n[0] * il.ld[0] * 8;
        il.r = take(v64);
        il.z = take(v64);
        il.p = take(v64);
        il.q = take(v64);
    }
    lay.total = off;
    return KC_OK;
}

// ---------------------------------------------------------------------------
// schedule
// ---------------------------------------------------------------------------
enum LaunchType { L_GRID, L_SUB, L_COARSEST };

struct Launch {
    LaunchType type;
    GridKernel gk;
    bool f32;
    StageArgs sa;
    int nblocks;
    SubArgs ba;
    int threads;
    int lds;
};

struct HostInst {
    kc_problem p;
    bool conv = false;            // convection-diffusion operator (kc_set_convection)
    double bx = 0.0, by = 0.0;
    InstLayout il;
    int cut = 0;
    double s[MAXL][9];
    std::vector<uint32_t> ops;
    int ops_beg[KMAX] = {}, ops_len[KMAX] = {};
    int zops_beg[KMAX] = {}, zops_len[KMAX] = {};   // zebra relaxation: lists without register calls
    int lds_off[MAXL] = {}, lds_elems = 0;
};

int lg_of(int n)
{
    int lg = 0;
    while ((1 << lg) - 1 < n) ++lg;
    return lg;
}

// op list lengths / starts for a smoother (0 damped Jacobi, 1 zebra)
const int* olen(const HostInst& hi, int smoother) { return smoother == 1 ? hi.zops_len : hi.ops_len; }
const int* obeg(const HostInst& hi, int smoother) { return smoother == 1 ? hi.zops_beg : hi.ops_beg; }

// op list of one call at depth d with counter k (Algorithm 3), levels in LDS;
// a call on a level of at most reg_n points per side becomes one register call
void gen_sub_call(const HostInst& h, int d, int k, bool zg, int reg_n, std::vector<uint32_t>& out)
{
    const uint32_t lg = (uint32_t)lg_of(h.il.n[d]), off = (uint32_t)h.lds_off[d];
    if (h.il.n[d] <= reg_n) {
        out.push_back(sop_make(SOP_WCALL, d, zg ? 1 : 0, lg, off, (uint32_t)std::min<int>(k, SOP_KMAX)));
        return;
    }
    if (d == h.il.L - 1) {
        out.push_back(sop_make(SOP_SOLVE, d, 0, lg, off));
        return;
    }
    out.push_back(sop_make(SOP_PRE, d, zg ? 1 : 0, lg, off));
    gen_sub_call(h, d + 1, k, true, reg_n, out);
    if (k > 1) gen_sub_call(h, d + 1, k - 1, false, reg_n, out);
    out.push_back(sop_make(SOP_POST, d, 0, lg, off));
}

}  // namespace

struct kc_hier {
    int count = 0;
    kc_precision prec = KC_F64;
    bool semi = false;   // levels coarsened along y only (x-line zebra, one kernel per operation)
    kc_exec ex{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t user_stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr, t0 = nullptr, t1 = nullptr;
    hipEvent_t ev_upload = nullptr;   // last copy out of the pinned mirrors
    bool upload_pending = false;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    Layout lay;
    std::vector<HostInst> hi;
    InstDev* h_inst = nullptr;   // pinned mirrors
    InstState* h_st = nullptr;
    InstDev* d_inst = nullptr;
    InstState* d_st = nullptr;
    int32_t* d_tiles = nullptr;
    int32_t* d_lists = nullptr;
    double* d_partial = nullptr;
    double* d_hist = nullptr;
    std::vector<std::vector<int32_t>> tiles;   // host copies of the tile tables
    std::vector<std::vector<int32_t>> lists;   // host copies of the instance lists
    int max_cut = 0, max_L = 0;
    int shape[MAXL] = {};                      // StageArgs::flags of the fused grid kernels at depth d
    int shape_post[MAXL] = {};                 // the same for the post-smoothing kernel
    bool compacted = false;                    // the tables cover only the instances still iterating
    int last_compactions = 0;                  // table compactions during the last driver call
    int sub_lds = 0;
    int sub_lds_z = 0;                         // with the zebra line-solve tables after the levels
    // (driver, kappa, nu1, nu2, smoother, iterations captured)
    std::map<std::tuple<int, int, int, int, double, int>, hipGraphExec_t> graphs;
    double omega_set = -1.0;
    // stats
    int64_t last_grid = 0, last_sub = 0, last_sub_stages = 0, last_cycles = 0, last_launched = 0;
    double last_ms = 0.0;
    std::string last_driver;
    std::vector<int32_t> last_iters;           // per instance, last kc_solve / kc_pcg
};

static bool any_convection(const kc_hier* h)
{
    for (const HostInst& hi : h->hi)
        if (hi.conv) return true;
    return false;
}

namespace {

// tile table indices
int tt_all0() { return 0; }
int tt_cut(int d) { return 1 + d; }          // instances with cut > d
int tt_lvl(int d) { return 1 + MAXL + d; }   // instances with L - 1 > d and cut > d (one kernel per operation)
int tt_zeb(int d) { return 1 + 2 * MAXL + d; }   // zebra line groups of those instances
int tt_cut_post(int d) { return 1 + 3 * MAXL + d; }   // fused post-smoothing strips where they differ from tt_cut
int lt_sub(int d) { return d; }              // instances with cut == d
int lt_coarse(int d) { return MAXL + d; }    // instances with L - 1 == d

const int32_t* dev_tiles(kc_hier* h, int t) { return h->d_tiles + (size_t)t * (h->count + 1); }
const int32_t* dev_list(kc_hier* h, int t) { return h->d_lists + (size_t)t * h->count; }
int ntiles(kc_hier* h, int t) { return h->tiles[t][h->count]; }
int nlist(kc_hier* h, int t) { return (int)h->lists[t].size(); }

StageArgs base_args(kc_hier* h, int table)
{
    StageArgs a{};
    a.inst = h->d_inst;
    a.st = h->d_st;
    a.tile_off = dev_tiles(h, table);
    a.partial = h->d_partial;
    a.hist = h->d_hist;
    a.count = h->count;
    a.semi = h->semi ? 1 : 0;
    return a;
}

Launch grid(kc_hier* h, GridKernel gk, bool f32, int table, int depth)
{
    Launch L{};
    L.type = L_GRID;
    L.gk = gk;
    L.f32 = f32;
    L.sa = base_args(h, table);
    L.sa.depth = depth;
    L.nblocks = ntiles(h, table);
    return L;
}

// fused PRE/POST launch at depth d, in the tile shape chosen for that depth
Launch fused_grid(kc_hier* h, GridKernel gk, bool f32, int d)
{
    const bool own = gk == GK_POST && h->shape_post[d] != h->shape[d];   // post strips of their own height
    Launch L = grid(h, gk, f32, own ? tt_cut_post(d) : tt_cut(d), d);
    L.sa.flags = gk == GK_POST ? h->shape_post[d] : h->shape[d];
    return L;
}

Launch sub(kc_hier* h, bool f32, int depth, int kappa, bool pair, int nu1, int nu2, bool zg, int fin, int smoother = 0)
{
    Launch L{};
    L.type = L_SUB;
    L.f32 = f32;
    L.ba.inst = h->d_inst;
    L.ba.st = h->d_st;
    L.ba.list = dev_list(h, lt_sub(depth));
    L.ba.count = nlist(h, lt_sub(depth));
    L.ba.first = L.ba.count > 0 ? h->lists[lt_sub(depth)][0] : 0;
    L.ba.depth = depth;
    L.ba.kappa = kappa;
    L.ba.pair = pair ? 1 : 0;
    L.ba.nu1 = nu1;
    L.ba.nu2 = nu2;
    L.ba.zg = zg ? 1 : 0;
    L.ba.fin = fin;
    L.ba.wave_n = h->ex.coarse_wave_n;
    L.ba.smoother = smoother;
    L.ba.hist = h->d_hist;
    L.threads = h->ex.coarse_threads;
    L.lds = smoother == 1 ? h->sub_lds_z : h->sub_lds;
    if (L.ba.count == 1 && depth > 0 && h->h_inst && h->ws) {
        // one instance on an internal level: its tables are fixed for the plan, so the
        // launch carries them and the kernel issues every load in one round
        const int i = L.ba.first;
        const HostInst& hi = h->hi[i];
        const InstDev& I = h->h_inst[i];
        const int k1 = std::min(kappa, KMAX), k2 = std::min(std::max(kappa - 1, 1), KMAX);
        const int* ob = obeg(hi, smoother);
        const int* ol = olen(hi, smoother);
        const uint32_t* ops = (const uint32_t*)(h->ws + hi.il.ops);
        L.ba.ops1 = ops + ob[k1 - 1];
        L.ba.n1 = ol[k1 - 1];
        L.ba.ops2 = ops + ob[k2 - 1];
        L.ba.n2 = (pair && kappa > 1) ? ol[k2 - 1] : 0;
        const LevelDev& Lv = I.lev[depth];
        L.ba.n0 = Lv.n;
        L.ba.sub_lds = I.sub_lds;
        L.ba.F0 = Lv.F;
        L.ba.A0 = Lv.A;
        L.ba.ldf0 = Lv.ldf;
        L.ba.lda0 = Lv.lda;
        L.ba.fs0 = Lv.fscale;
        L.ba.chol0 = f32 ? (const void*)I.chol32 : (const void*)I.chol64;
    }
    return L;
}

// fused schedule of one cycle: grid-wide PRE/POST above each instance's cut,
// one persistent launch per parent node for the pair of calls at the cut
void gen_fused(kc_hier* h, int d, int k, bool zg, int fin, const kc_cycle_params& c, bool f32,
               std::vector<Launch>& out)
{
    Launch pre = fused_grid(h, GK_PRE, f32, d);
    pre.sa.zg = zg ? 1 : 0;
    pre.sa.fin = fin;
    pre.sa.nu = c.nu1;
    out.push_back(pre);
    if (nlist(h, lt_sub(d + 1)) > 0) out.push_back(sub(h, f32, d + 1, k, true, c.nu1, c.nu2, false, FIN_NONE));
    if (d + 1 < h->max_cut) {
        gen_fused(h, d + 1, k, true, FIN_NONE, c, f32, out);
        if (k > 1) gen_fused(h, d + 1, k - 1, false, FIN_NONE, c, f32, out);
    }
    Launch post = fused_grid(h, GK_POST, f32, d);
    post.sa.nu = c.nu2;
    out.push_back(post);
}

// a post-smoothing launch followed by the pre-smoothing of the next sibling call on the same
// level (16 x 16 tiles) becomes one fused junction launch
void fuse_junctions(std::vector<Launch>& ls, size_t from)
{
    std::vector<Launch> out(ls.begin(), ls.begin() + from);
    for (size_t k = from; k < ls.size(); ++k) {
        const Launch& L = ls[k];
        if (k + 1 < ls.size()) {
            const Launch& M = ls[k + 1];
            if (L.type == L_GRID && M.type == L_GRID && L.gk == GK_POST && M.gk == GK_PRE && L.f32 == M.f32 &&
                L.sa.depth == M.sa.depth && L.sa.tile_off == M.sa.tile_off && (L.sa.flags == 1 || L.sa.flags == 32) &&
                M.sa.flags == L.sa.flags &&
                M.sa.zg == 0 && M.sa.fin == FIN_NONE && L.sa.fin == FIN_NONE) {
                Launch F = M;
                F.gk = GK_POSTPRE;
                F.sa.src = L.sa.nu;   // nu2 of the first call
                out.push_back(F);
                ++k;
                continue;
            }
        }
        out.push_back(L);
    }
    ls.swap(out);
}

void cycle_fused(kc_hier* h, const kc_cycle_params& c, int kappa, bool zg, int fin, bool f32, std::vector<Launch>& out)
{
    const size_t from = out.size();
    if (nlist(h, lt_sub(0)) > 0) out.push_back(sub(h, f32, 0, kappa, false, c.nu1, c.nu2, zg, fin));
    if (h->max_cut > 0) gen_fused(h, 0, kappa, zg, fin, c, f32, out);
    if (h->ex.fuse_junctions) fuse_junctions(out, from);
}

// Algorithm 4: one launch per operation; cur[d] tracks which buffer holds v_d.
// With zebra relaxation in the fused execution mode the same schedule runs the
// levels above each instance's cut, and one persistent launch per parent call
// runs the pair of child calls at the cut (every coarser level, the coarsest
// solve included, stays inside it)
void gen_paper(kc_hier* h, int d, int k, const kc_cycle_params& c, bool f32, int cur[], std::vector<Launch>& out)
{
    const bool hybrid = h->ex.mode == 0;
    if (h->semi && d == h->max_L - 1) {
        // semi-coarsening: the coarsest level is one x-line without neighbours, solved exactly
        // by one zebra relaxation of its only line (colour 0; the input does not enter)
        Launch L = grid(h, GK_ZEBRA, f32, tt_zeb(d), d);
        L.sa.src = cur[d];
        L.sa.dst = 0;
        L.sa.nu = 0;
        L.sa.flags = zebra_flags(h->ex);
        out.push_back(L);
        return;
    }
    if (!hybrid && nlist(h, lt_coarse(d)) > 0) {
        Launch L{};
        L.type = L_COARSEST;
        L.f32 = f32;
        L.ba.inst = h->d_inst;
        L.ba.st = h->d_st;
        L.ba.list = dev_list(h, lt_coarse(d));
        L.ba.count = nlist(h, lt_coarse(d));
        L.ba.first = L.ba.count > 0 ? h->lists[lt_coarse(d)][0] : 0;
        L.ba.depth = d;
        out.push_back(L);
        cur[d] = 0;
    }
    if (ntiles(h, tt_lvl(d)) == 0) return;
    auto op = [&](GridKernel gk, int src, int dst) {
        Launch L = grid(h, gk, f32, tt_lvl(d), d);
        L.sa.src = src;
        L.sa.dst = dst;
        out.push_back(L);
    };
    // relaxation r: a damped-Jacobi sweep into the other buffer, or a zebra
    // relaxation in place (x-lines for even r, y-lines for odd r; two launches,
    // lines of even index first): src = buffer, dst = colour, nu = direction
    auto relax = [&](int r) {
        if (c.smoother == 1) {
            for (int color = 0; color < 2; ++color) {
                Launch L = grid(h, GK_ZEBRA, f32, tt_zeb(d), d);
                L.sa.src = cur[d];
                L.sa.dst = color;
                L.sa.nu = h->semi ? 0 : (r & 1);   // semi-coarsening relaxes x-lines only
                L.sa.flags = zebra_flags(h->ex);   // per instance: lines per wave from the line length
                out.push_back(L);
            }
        } else {
            op(GK_SWEEP, cur[d], cur[d] ^ 1);
            cur[d] ^= 1;
        }
    };
    for (int s = 0; s < c.nu1; ++s) relax(s);
    op(GK_RESID, cur[d], cur[d] ^ 1);
    op(GK_RESTRICT, cur[d] ^ 1, 0);
    op(GK_ZERO, 0, 0);
    cur[d + 1] = 0;
    if (hybrid && nlist(h, lt_sub(d + 1)) > 0)   // result in the level's first buffer
        out.push_back(sub(h, f32, d + 1, k, true, c.nu1, c.nu2, false, FIN_NONE, c.smoother));
    gen_paper(h, d + 1, k, c, f32, cur, out);
    if (k > 1) gen_paper(h, d + 1, k - 1, c, f32, cur, out);
    {
        Launch L = grid(h, GK_PROLONG, f32, tt_lvl(d), d);
        L.sa.src = cur[d + 1];
        L.sa.dst = cur[d] ^ 1;
        out.push_back(L);
    }
    op(GK_ADD, cur[d], cur[d] ^ 1);
    for (int s = 0; s < c.nu2; ++s) relax(s);
}

void cycle_paper(kc_hier* h, const kc_cycle_params& c, int kappa, bool zg, bool f32, std::vector<Launch>& out)
{
    int cur[MAXL + 1] = {};
    if (zg) out.push_back(grid(h, GK_ZERO_SELF, f32, tt_all0(), 0));   // v_1 <- 0 for a zero-guess call
    if (h->ex.mode == 0 && nlist(h, lt_sub(0)) > 0)   // instances below the cutover altogether
        out.push_back(sub(h, f32, 0, kappa, false, c.nu1, c.nu2, false, FIN_NONE, c.smoother));
    gen_paper(h, 0, kappa, c, f32, cur, out);
    if (cur[0] != 0) {
        Launch L = grid(h, GK_COPY, f32, tt_lvl(0), 0);
        L.sa.src = cur[0];
        L.sa.dst = 0;
        out.push_back(L);
    }
}

int clamp_kappa(kc_hier* h, int kappa) { return std::min(kappa, h->max_L + 1); }

hipError_t run(kc_hier* h, const std::vector<Launch>& ls)
{
    for (const Launch& L : ls) {
        hipError_t e = hipSuccess;
        if (L.type == L_GRID) e = launch_grid(L.gk, L.f32, L.sa, L.nblocks, h->stream);
        else if (L.type == L_SUB) e = launch_subtree(L.f32, L.ba, L.threads, L.lds, h->stream);
        else e = launch_coarsest(L.f32, L.ba, h->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void count_launches(const std::vector<Launch>& ls, int64_t& grid_n, int64_t& sub_n)
{
    grid_n = sub_n = 0;
    for (const Launch& L : ls) {
        if (L.type == L_SUB) { if (L.ba.count > 0) ++sub_n; }
        else if (L.type == L_COARSEST) { if (L.ba.count > 0) ++grid_n; }
        else if (L.nblocks > 0) ++grid_n;
    }
}

// tile prefix tables and instance lists of every stage, over the instances
// marked in `active` (all when null): a finished instance can be left out of
// the launches altogether, its blocks would only check its stop flag and exit
kc_status build_tables(kc_hier* h, const std::vector<char>* active)
{
    const int cnt = h->count;
    h->tiles.assign(NTABLES, std::vector<int32_t>(cnt + 1, 0));
    h->lists.assign(2 * MAXL, std::vector<int32_t>());
    for (int i = 0; i < cnt; ++i) {
        if (active && !(*active)[i]) continue;
        const HostInst& hi = h->hi[i];
        const int L = hi.il.L;
        h->tiles[tt_all0()][i + 1] = tiles_of(hi.il.n[0]);
        for (int d = 0; d < MAXL; ++d) {
            const int sh = h->shape[d];
            const int tc = (sh & 2)    ? tiles_stream(hi.il.n[d], (sh >> 2) & 3)
                           : (sh & 32) ? tiles_tiny(hi.il.n[d])
                           : (sh & 1)  ? tiles_small(hi.il.n[d])
                           : (sh & 16) ? tiles_mid(hi.il.n[d])
                                       : tiles_of(hi.il.n[d]);
            h->tiles[tt_cut(d)][i + 1] = (d < L && hi.cut > d) ? tc : 0;
            const int shp = h->shape_post[d];
            h->tiles[tt_cut_post(d)][i + 1] = (d < L && hi.cut > d && shp != sh) ? tiles_stream(hi.il.n[d], (shp >> 2) & 3) : 0;
            // one-kernel-per-operation stages: levels above the instance's cut (all of them in
            // the paper-structured mode, where the cut is L)
            const bool lvl = d < L - 1 && hi.cut > d;
            if (h->semi) {   // rectangular levels; the coarsest line is solved by the zebra kernel
                h->tiles[tt_lvl(d)][i + 1] = lvl ? tiles_rect(hi.il.nx[d], hi.il.n[d]) : 0;
                h->tiles[tt_zeb(d)][i + 1] = d < L ? zebra_blocks_lines(hi.il.n[d], hi.il.nx[d], h->ex.zebra_wave_n, h->ex.zebra_quad_n) : 0;
                continue;
            }
            h->tiles[tt_lvl(d)][i + 1] = lvl ? tiles_of(hi.il.n[d]) : 0;
            h->tiles[tt_zeb(d)][i + 1] = lvl ? zebra_blocks(hi.il.n[d], h->ex.zebra_wave_n, h->ex.zebra_quad_n) : 0;
            if (hi.cut == d && d < L) h->lists[lt_sub(d)].push_back(i);
            if (L - 1 == d) h->lists[lt_coarse(d)].push_back(i);
        }
    }
    for (auto& t : h->tiles)
        for (int i = 0; i < cnt; ++i) t[i + 1] += t[i];
    std::vector<int32_t> flat((size_t)NTABLES * (cnt + 1));
    for (size_t t = 0; t < h->tiles.size(); ++t) std::copy(h->tiles[t].begin(), h->tiles[t].end(), flat.begin() + t * (cnt + 1));
    std::vector<int32_t> lflat((size_t)2 * MAXL * cnt, 0);
    for (size_t t = 0; t < h->lists.size(); ++t) std::copy(h->lists[t].begin(), h->lists[t].end(), lflat.begin() + t * cnt);
    h->compacted = active != nullptr;
    if (h->d_tiles) {
        HIPCHK(hipMemcpyAsync(h->d_tiles, flat.data(), flat.size() * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->d_lists, lflat.data(), lflat.size() * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    return KC_OK;
}

// ---------------------------------------------------------------------------
// execution plan (depends on the exec options): cut depths, op lists, LDS
// ---------------------------------------------------------------------------
kc_status plan_exec(kc_hier* h)
{
    const size_t T = (h->prec == KC_F64) ? 8 : 4;
    const int cutover = h->ex.coarse_cutover;
    h->max_cut = 0;
    h->max_L = 0;
    h->sub_lds = 0;
    h->sub_lds_z = 0;
    for (int i = 0; i < h->count; ++i) {
        HostInst& hi = h->hi[i];
        const int L = hi.il.L;
        int cut = L - 1;
        for (int d = 0; d < L; ++d)
            if (hi.il.n[d] <= cutover) { cut = d; break; }
        if (h->ex.mode == 1) cut = L;   // paper-structured mode never uses the persistent kernel
        hi.cut = cut;
        h->max_cut = std::max(h->max_cut, std::min(cut, L));
        h->max_L = std::max(h->max_L, L);
        int off = 0;
        for (int d = 0; d < MAXL; ++d) hi.lds_off[d] = 0;
        if (cut < L) {
            for (int d = cut; d < L; ++d) {   // two sweep buffers and F, each (n+2)^2 with a zero ring
                hi.lds_off[d] = off;
                off += 3 * (hi.il.n[d] + 2) * (hi.il.n[d] + 2);
            }
        }
        if (off > (int)SOP_OFFMAX) return fail(KC_ERR_ARG, "coarse levels too large for the op encoding");
        // levels wave 0 runs alone go to registers (the register engine's coarsest solve is 1 x 1)
        const int reg_n = (h->ex.wave_regs && hi.p.n_coarsest == 1) ? std::min(h->ex.coarse_wave_n, 15) : 0;
        hi.ops.clear();
        for (int k = 1; k <= KMAX; ++k) {
            hi.ops_beg[k - 1] = (int)hi.ops.size();
            if (cut < L) {
                const int below = L - cut;
                if (k <= below + 1 || k == 1) gen_sub_call(hi, cut, k, false, reg_n, hi.ops);
                else {   // same as the W-cycle list
                    hi.ops_beg[k - 1] = hi.ops_beg[below];
                    hi.ops_len[k - 1] = hi.ops_len[below];
                    continue;
                }
            }
            hi.ops_len[k - 1] = (int)hi.ops.size() - hi.ops_beg[k - 1];
        }
        // zebra relaxation has no register engine: its lists run every level phase by phase
        for (int k = 1; k <= KMAX; ++k) {
            hi.zops_beg[k - 1] = hi.ops_beg[k - 1];
            hi.zops_len[k - 1] = hi.ops_len[k - 1];
        }
        if (reg_n > 0 && cut < L) {
            const int below = L - cut;
            for (int k = 1; k <= KMAX; ++k) {
                if (k <= below + 1 || k == 1) {
                    hi.zops_beg[k - 1] = (int)hi.ops.size();
                    gen_sub_call(hi, cut, k, false, 0, hi.ops);
                    hi.zops_len[k - 1] = (int)hi.ops.size() - hi.zops_beg[k - 1];
                } else {
                    hi.zops_beg[k - 1] = hi.zops_beg[below];
                    hi.zops_len[k - 1] = hi.zops_len[below];
                }
            }
        }
        if ((int)hi.ops.size() > OPS_CAP) return fail(KC_ERR_ARG, "coarse cutover too large for the op buffer");
        hi.lds_elems = off;
        h->sub_lds = std::max(h->sub_lds, (int)(off * T));
        if (cut < L) h->sub_lds_z = std::max(h->sub_lds_z, (int)((off + ZLDS_TABLE) * T));
    }
    if (h->sub_lds > 0 && h->d_tiles) {
        const int maxl = max_lds_bytes() - 8192;   // the kernel's static parameter block stays below 8 KB
        if (h->sub_lds > maxl)
            return fail(KC_ERR_ARG, "coarse cutover needs " + std::to_string(h->sub_lds) + " B of LDS, device allows " +
                                        std::to_string(maxl));
    }
    const int cnt = h->count;
    for (int d = 0; d < MAXL; ++d) {
        int maxn = 0;
        for (int i = 0; i < cnt; ++i)
            if (d < h->hi[i].il.L && h->hi[i].cut > d) maxn = std::max(maxn, h->hi[i].il.n[d]);
        int f = 0;
        if (maxn > 0 && h->ex.stream_n > 0 && maxn >= h->ex.stream_n) f = 2 | (strip_rows_code(maxn) << 2);
        else if (maxn > 0 && maxn <= h->ex.tiny_tile_n) f = 32;
        else if (maxn > 0 && maxn <= h->ex.small_tile_n) f = 1;
        else if (maxn > 0 && maxn <= h->ex.mid_tile_n) f = 16;
        h->shape[d] = f;
        h->shape_post[d] = f;
    }
    kc_status st = build_tables(h, nullptr);
    if (st != KC_OK) return st;
    if (h->d_tiles) {
        for (int i = 0; i < cnt; ++i) {
            const HostInst& hi = h->hi[i];
            HIPCHK(hipMemcpyAsync(h->ws + hi.il.ops, hi.ops.data(), hi.ops.size() * 4, hipMemcpyHostToDevice, h->stream));
        }
        HIPCHK(hipStreamSynchronize(h->stream));
        if (std::max(h->sub_lds, h->sub_lds_z) > 65536) {
            HIPCHK(prepare_subtree(h->prec == KC_F32_CYCLE, std::max(h->sub_lds, h->sub_lds_z)));
        }
    }
    return KC_OK;
}

// Zebra line relaxation (Section 4, third and fourth solvers): along a line
// the matrix is tridiagonal with constant entries lo (previous point), the
// diagonal and up (next point), in h^2-scaled units; elimination uses the
// pivots p_q (p_0 = diag, p_q = diag - lo u_{q-1}) through their reciprocals
// r_q = 1 / p_q, and the upper multipliers u_q = up / p_q.  Appends [r, u] for
// x-lines (west / centre / east entries) and then for y-lines (south /
// centre / north) of one level, computed in T from the stencil rounded to T.
template <typename T>
void line_tables(int n, const double s64[9], std::vector<T>& out)
{
    T s[9];
    for (int q = 0; q < 9; ++q) s[q] = (T)s64[q];
    for (int dir = 0; dir < 2; ++dir) {
        const T lo = dir == 0 ? s[3] : s[1], dg = s[4], up = dir == 0 ? s[5] : s[7];
        std::vector<T> r((size_t)n), u((size_t)n);
        T piv = dg;
        u[0] = up / piv;
        r[0] = T(1) / piv;
        for (int q = 1; q < n; ++q) {
            piv = dg - lo * u[q - 1];
            u[q] = up / piv;
            r[q] = T(1) / piv;
        }
        out.insert(out.end(), r.begin(), r.end());
        out.insert(out.end(), u.begin(), u.end());
    }
}

void fill_inst_static(kc_hier* h)
{
    const bool f64 = h->prec == KC_F64;
    for (int i = 0; i < h->count; ++i) {
        const HostInst& hi = h->hi[i];
        InstDev& I = h->h_inst[i];
        I.L = hi.il.L;
        I.cut = hi.cut;
        I.nc2 = hi.p.n_coarsest * hi.p.n_coarsest;
        I.sub_lds = hi.lds_elems;
        for (int d = 0; d < hi.il.L; ++d) {
            for (int q = 0; q < 9; ++q) {
                I.s64[d][q] = hi.s[d][q];
                I.s32[d][q] = (float)hi.s[d][q];
            }
            LevelDev& Lv = I.lev[d];
            Lv.n = hi.il.n[d];
            Lv.nx = hi.il.nx[d];
            Lv.lda = Lv.ldb = Lv.ldf = hi.il.ld[d];
            const bool own = d > 0 || !f64;   // FP64 level 0 binds the caller's arrays per call
            Lv.A = own ? (void*)(h->ws + hi.il.A[d]) : nullptr;
            Lv.B = h->ws + hi.il.B[d];
            Lv.F = own ? (void*)(h->ws + hi.il.F[d]) : nullptr;
            Lv.fscale = 1.0;
            I.lds_off[d] = hi.lds_off[d];
        }
        for (int k = 0; k < KMAX; ++k) {
            I.ops_beg[k] = hi.ops_beg[k];
            I.ops_len[k] = hi.ops_len[k];
            I.zops_beg[k] = hi.zops_beg[k];
            I.zops_len[k] = hi.zops_len[k];
        }
        I.ops = (const uint32_t*)(h->ws + hi.il.ops);
        I.chol64 = (const double*)(h->ws + hi.il.chol64);
        I.chol32 = (const float*)(h->ws + hi.il.chol32);
        for (int d = 0; d < hi.il.L; ++d) {
            I.zt64[d] = (const double*)(h->ws + hi.il.zt64) + hi.il.zoff[d];
            I.zt32[d] = (const float*)(h->ws + hi.il.zt32) + hi.il.zoff[d];
        }
        I.r = (double*)(h->ws + hi.il.r);
        I.z = (double*)(h->ws + hi.il.z);
        I.p = (double*)(h->ws + hi.il.p);
        I.q = (double*)(h->ws + hi.il.q);
        I.ldv = hi.il.ld[0];
        I.n0 = hi.il.n[0];
        const double hh = 1.0 / (double)(hi.il.n[0] + 1);
        I.h2 = hh * hh;
        I.h2inv = (double)(hi.il.n[0] + 1) * (double)(hi.il.n[0] + 1);
        fine_stencil_derivs(hi.p.theta, hi.p.eps, I.ds_th, I.ds_ep);
    }
}

void set_omega(kc_hier* h, double omega)
{
    for (int i = 0; i < h->count; ++i) {
        InstDev& I = h->h_inst[i];
        for (int d = 0; d < I.L; ++d) {
            I.w64[d] = omega / I.s64[d][4];
            I.w32[d] = (float)I.w64[d];
        }
    }
}

kc_status upload_inst(kc_hier* h)
{
    HIPCHK(hipMemcpyAsync(h->d_inst, h->h_inst, sizeof(InstDev) * h->count, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipEventRecord(h->ev_upload, h->stream));
    h->upload_pending = true;
    return KC_OK;
}

kc_status upload_state(kc_hier* h, double tol, int maxit)
{
    for (int i = 0; i < h->count; ++i) {
        InstState& s = h->h_st[i];
        std::memset(&s, 0, sizeof s);
        s.tol = tol;
        s.maxit = maxit;
        s.scale = 1.0;
        s.scale_used = 1.0;
    }
    HIPCHK(hipMemcpyAsync(h->d_st, h->h_st, sizeof(InstState) * h->count, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipEventRecord(h->ev_upload, h->stream));
    h->upload_pending = true;
    return KC_OK;
}

kc_status check_cycle(const kc_cycle_params* c)
{
    if (!c) return fail(KC_ERR_ARG, "null cycle parameters");
    if (c->kappa < 1) return fail(KC_ERR_ARG, "kappa must be >= 1");
    if (c->nu1 < 0 || c->nu2 < 0 || c->nu1 > 3 || c->nu2 > 3) return fail(KC_ERR_ARG, "nu1, nu2 must be in 0..3");
    if (!(c->omega > 0.0) || !std::isfinite(c->omega)) return fail(KC_ERR_ARG, "omega must be positive");
    if (c->smoother != 0 && c->smoother != 1) return fail(KC_ERR_ARG, "smoother must be 0 (damped Jacobi) or 1 (zebra)");
    return KC_OK;
}

enum Driver { DRV_CYCLE = 0, DRV_SOLVE64 = 1, DRV_IR = 2, DRV_PCG = 3 };

// launches of one iteration of a driver
void iteration(kc_hier* h, int drv, const kc_cycle_params& c, std::vector<Launch>& out)
{
    const bool f32 = h->prec == KC_F32_CYCLE;
    const int kappa = clamp_kappa(h, c.kappa);
    // zebra relaxation always takes the one-kernel-per-operation schedule above the
    // persistent kernel (the fused grid kernels are damped Jacobi)
    const bool paper = h->ex.mode == 1 || c.smoother == 1;
    switch (drv) {
    case DRV_CYCLE:
        if (paper) cycle_paper(h, c, kappa, false, false, out);
        else cycle_fused(h, c, kappa, false, FIN_NONE, false, out);
        break;
    case DRV_SOLVE64:
        if (paper) {
            Launch n = grid(h, GK_NORM, false, tt_all0(), 0);
            n.sa.fin = FIN_STOP;
            out.push_back(n);
            cycle_paper(h, c, kappa, false, false, out);
        } else {
            cycle_fused(h, c, kappa, false, FIN_STOP, false, out);
        }
        break;
    case DRV_IR: {
        Launch r = grid(h, GK_IR_RESID, true, tt_all0(), 0);
        r.sa.fin = FIN_STOP_IR;
        out.push_back(r);
        if (paper) cycle_paper(h, c, kappa, true, true, out);
        else cycle_fused(h, c, kappa, true, FIN_NONE, true, out);
        out.push_back(grid(h, GK_IR_UPDATE, true, tt_all0(), 0));
        break;
    }
    case DRV_PCG: {
        if (f32) out.push_back(grid(h, GK_PCG_PRECIN, true, tt_all0(), 0));
        if (paper) cycle_paper(h, c, kappa, true, f32, out);
        else cycle_fused(h, c, kappa, true, FIN_NONE, f32, out);
        Launch rz = grid(h, GK_PCG_RZ, f32, tt_all0(), 0);
        rz.sa.fin = FIN_RZ;
        out.push_back(rz);
        out.push_back(grid(h, GK_PCG_P, f32, tt_all0(), 0));
        Launch ap = grid(h, GK_PCG_AP, f32, tt_all0(), 0);
        ap.sa.fin = FIN_PQ;
        out.push_back(ap);
        Launch up = grid(h, GK_PCG_UPD, f32, tt_all0(), 0);
        up.sa.fin = FIN_PCG_R;
        out.push_back(up);
        Launch tr = grid(h, GK_PCG_TRUE, false, tt_all0(), 0);
        tr.sa.fin = FIN_PCG_TRUE;
        out.push_back(tr);
        break;
    }
    }
}

// iterations captured in one graph: each graph launch costs a fixed gap on the stream (about
// 6 us on MI355X), so runs of GRAPH_ITERS iterations go as one launch and the remainder as
// single-iteration launches (exactly `times` iterations either way; an iteration's launches
// take the same arguments every time, so four captured copies equal four replays of one)
constexpr int GRAPH_ITERS = 4;

// the graph of `reps` consecutive iterations (captured on first use, kept until the plan changes)
kc_status iteration_graph(kc_hier* h, int drv, const kc_cycle_params& c, const std::vector<Launch>& ls, int reps,
                          hipGraphExec_t* out)
{
    auto key = std::make_tuple(drv, clamp_kappa(h, c.kappa), c.nu1, c.nu2, (double)c.smoother, reps);
    auto it = h->graphs.find(key);
    if (it == h->graphs.end()) {
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = run(h, ls);
        hipError_t e2 = hipStreamEndCapture(h->stream, &g);
        if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); return fail(KC_ERR_HIP, std::string("capture: ") + hipGetErrorString(e)); }
        HIPCHK(e2);
        hipGraphExec_t x = nullptr;
        HIPCHK(hipGraphInstantiate(&x, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
        it = h->graphs.emplace(key, x).first;
    }
    *out = it->second;
    return KC_OK;
}

// capture (without launching) every graph that launch_iteration(times) will use
kc_status warm_graphs(kc_hier* h, int drv, const kc_cycle_params& c, int times)
{
    if (!h->ex.use_graph) return KC_OK;
    std::vector<Launch> ls;
    iteration(h, drv, c, ls);
    hipGraphExec_t ge = nullptr;
    if (times >= GRAPH_ITERS) {
        kc_status s = iteration_graph(h, drv, c, ls, GRAPH_ITERS, &ge);
        if (s != KC_OK) return s;
    }
    if (times % GRAPH_ITERS) return iteration_graph(h, drv, c, ls, 1, &ge);
    return KC_OK;
}

kc_status launch_iteration(kc_hier* h, int drv, const kc_cycle_params& c, int times)
{
    std::vector<Launch> ls;
    iteration(h, drv, c, ls);
    if (!h->ex.use_graph) {
        for (int t = 0; t < times; ++t) HIPCHK(run(h, ls));
        return KC_OK;
    }
    hipGraphExec_t ge = nullptr;
    int t = times;
    if (t >= GRAPH_ITERS) {
        kc_status s = iteration_graph(h, drv, c, ls, GRAPH_ITERS, &ge);
        if (s != KC_OK) return s;
        for (; t >= GRAPH_ITERS; t -= GRAPH_ITERS) HIPCHK(hipGraphLaunch(ge, h->stream));
    }
    if (t > 0) {
        kc_status s = iteration_graph(h, drv, c, ls, 1, &ge);
        if (s != KC_OK) return s;
        for (; t > 0; --t) HIPCHK(hipGraphLaunch(ge, h->stream));
    }
    return KC_OK;
}

void drop_graphs(kc_hier* h)
{
    for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
}

kc_status enter(kc_hier* h)
{
    // the pinned mirrors are rewritten by this call: the previous upload must be done
    if (h->upload_pending) {
        HIPCHK(hipEventSynchronize(h->ev_upload));
        h->upload_pending = false;
    }
    if (h->own_stream) {
        HIPCHK(hipEventRecord(h->ev_in, h->user_stream));
        HIPCHK(hipStreamWaitEvent(h->stream, h->ev_in, 0));
    }
    return KC_OK;
}

kc_status leave(kc_hier* h)
{
    if (h->own_stream) {
        HIPCHK(hipEventRecord(h->ev_out, h->stream));
        HIPCHK(hipStreamWaitEvent(h->user_stream, h->ev_out, 0));
    }
    return KC_OK;
}

// poll-driven loop: launch iterations until every instance reports done
kc_status drive(kc_hier* h, int drv, const kc_cycle_params& c, int maxit, int32_t* iters, double* relres,
                int32_t* status)
{
    HIPCHK(hipEventRecord(h->t0, h->stream));
    int launched = 0;
    h->last_compactions = 0;
    int batch = h->ex.poll_every > 0 ? h->ex.poll_every : 2;
    std::vector<double> prev_rel(h->count, -1.0);
    std::vector<int> prev_it(h->count, 0);
    const int limit = maxit + 2;
    for (;;) {
        const int n = std::min(batch, limit - launched);
        if (n <= 0) break;
        kc_status s = launch_iteration(h, drv, c, n);
        if (s != KC_OK) return s;
        launched += n;
        HIPCHK(hipMemcpyAsync(h->h_st, h->d_st, sizeof(InstState) * h->count, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        bool all = true;
        double need = 1.0;
        for (int i = 0; i < h->count; ++i) {
            const InstState& s2 = h->h_st[i];
            if (s2.done) continue;
            all = false;
            // remaining cycles predicted from the observed reduction rate
            if (!(s2.tol > 0.0)) {
                need = std::max(need, (double)(s2.maxit - s2.iters + 1));
            } else if (prev_rel[i] > 0.0 && s2.relres > 0.0 && s2.iters > prev_it[i]) {
                const double rate = std::pow(s2.relres / prev_rel[i], 1.0 / (s2.iters - prev_it[i]));
                if (rate > 0.0 && rate < 1.0) {
                    const double rem = std::log(s2.tol / s2.relres) / std::log(rate);
                    need = std::max(need, rem);
                } else {
                    need = std::max(need, 4.0);
                }
            } else {
                need = std::max(need, 2.0);
            }
            prev_rel[i] = s2.relres;
            prev_it[i] = s2.iters;
        }
        if (all) break;
        if (h->ex.poll_every <= 0) batch = std::max(1, std::min(256, (int)std::ceil(need * 0.9)));
        if (h->count > 1) {   // drop finished instances from the launches once they are half of them
            std::vector<char> act(h->count, 0);
            int64_t live = 0;
            for (int i = 0; i < h->count; ++i)
                if (!h->h_st[i].done) { act[i] = 1; live += tiles_of(h->hi[i].il.n[0]); }
            if (2 * live <= (int64_t)ntiles(h, tt_all0())) {
                kc_status s3 = build_tables(h, &act);
                if (s3 != KC_OK) return s3;
                drop_graphs(h);
                ++h->last_compactions;
            }
        }
    }
    if (h->compacted) {   // later calls start from every instance again
        kc_status s3 = build_tables(h, nullptr);
        if (s3 != KC_OK) return s3;
        drop_graphs(h);
    }
    HIPCHK(hipEventRecord(h->t1, h->stream));
    HIPCHK(hipEventSynchronize(h->t1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, h->t0, h->t1));
    h->last_ms = ms;
    h->last_launched = launched;
    kc_status worst = KC_OK;
    int64_t maxits = 0;
    for (int i = 0; i < h->count; ++i) {
        const InstState& s2 = h->h_st[i];
        kc_status si = s2.done ? (kc_status)s2.status : KC_NOT_CONVERGED;
        if (iters) iters[i] = s2.iters;
        if (relres) relres[i] = s2.relres;
        if (status) status[i] = si;
        maxits = std::max<int64_t>(maxits, s2.iters);
        if (si < 0) worst = (worst < 0) ? std::min(worst, si) : si;
        else if (worst >= 0 && si > worst) worst = si;
    }
    h->last_cycles = maxits;
    return worst;
}

kc_status prepare_call(kc_hier* h, const kc_cycle_params* c)
{
    kc_status s = check_cycle(c);
    if (s != KC_OK) return s;
    if (h->semi && c->smoother != 1)
        return fail(KC_ERR_ARG, "a semi-coarsened hierarchy relaxes by x-line zebra: smoother must be 1");
    if (c->smoother == 1) {
        if (any_convection(h)) return fail(KC_ERR_ARG, "convection-diffusion runs with damped Jacobi only");
        for (int i = 0; i < h->count; ++i)
            if (h->hi[i].il.n[0] > 16383) return fail(KC_ERR_ARG, "the zebra smoother takes n <= 16383");
        if (h->ex.mode == 0 && h->sub_lds_z > max_lds_bytes() - 8192)
            return fail(KC_ERR_ARG, "coarse cutover with zebra tables needs " + std::to_string(h->sub_lds_z) +
                                        " B of LDS, device allows " + std::to_string(max_lds_bytes() - 8192));
    }
    if (c->omega != h->omega_set) {
        set_omega(h, c->omega);
        h->omega_set = c->omega;
    }
    return KC_OK;
}

template <typename PtrT>
kc_status check_ptrs(kc_hier* h, PtrT const* p, const int64_t* ld, const char* what)
{
    if (!p || !ld) return fail(KC_ERR_ARG, std::string("null ") + what);
    for (int i = 0; i < h->count; ++i) {
        if (!p[i]) return fail(KC_ERR_ARG, std::string("null device pointer in ") + what);
        if (ld[i] < h->hi[i].il.n[0] || ld[i] > INT32_MAX) return fail(KC_ERR_ARG, std::string("bad leading dimension of ") + what);
    }
    return KC_OK;
}

// the zebra line kernels index a level with 32-bit offsets (line * ld + point):
// a caller's array bound as the fine level must keep (n - 1) * ld + n - 1 in range
template <typename PtrT>
kc_status check_zebra_ld(kc_hier* h, const kc_cycle_params* c, PtrT const* p, const int64_t* ld, const char* what)
{
    if (c->smoother != 1) return KC_OK;
    for (int i = 0; i < h->count; ++i) {
        const int64_t n = h->hi[i].il.n[0];
        if ((n - 1) * ld[i] + (n - 1) > (int64_t)INT32_MAX)
            return fail(KC_ERR_ARG, std::string("leading dimension of ") + what +
                                        " too large for the zebra smoother ((n - 1) * ld + n - 1 must be < 2^31)");
    }
    (void)p;
    return KC_OK;
}

void record_counts(kc_hier* h, int drv, const kc_cycle_params& c)
{
    std::vector<Launch> ls;
    iteration(h, drv, c, ls);
    count_launches(ls, h->last_grid, h->last_sub);
    int64_t st = 0;
    for (const Launch& L : ls)
        if (L.type == L_SUB)
            for (int idx : h->lists[lt_sub(L.ba.depth)]) {
                const HostInst& hi = h->hi[idx];
                const int kk = std::min(L.ba.kappa, KMAX);
                const int* ln = olen(hi, L.ba.smoother);
                st += ln[kk - 1];
                if (L.ba.pair && L.ba.kappa > 1) st += ln[std::min(L.ba.kappa - 1, KMAX) - 1];
                break;
            }
    h->last_sub_stages = st;
}


// ---------------------------------------------------------------------------
// per-launch profile of one driver iteration: kernel names as the compiler
// emits them (so they match a profiler's), algorithmic bytes and flops
// ---------------------------------------------------------------------------
constexpr double FL_SWEEP = 20.0;     // nine-term sum (9 mul + 8 add, as fused multiply-adds) + sub + multiply-add per point
constexpr double FL_RESID = 18.0;     // nine-term sum + sub
constexpr double FL_FW = 17.0;        // 9 mul + 8 add per coarse point
constexpr double FL_ZEBRA_RHS = 13.0;   // six off-line products and sums + scaled f - sum
constexpr double FL_ZEBRA_SOLVE = 5.0;  // forward multiply-add and product, backward multiply-add
constexpr double FL_PROLONG = 3.0;    // average over injected, edge and centre points

std::string launch_name(const kc_hier* h, const Launch& L)
{
    const char* T = L.f32 ? "float" : "double";
    if (L.type == L_SUB)
        return std::string("k_subtree<") + T + ", " + std::to_string(L.threads) + (L.ba.smoother == 1 ? ", true>" : ", false>");
    if (L.type == L_COARSEST) return std::string("k_coarsest<") + T + ">";
    if (L.gk == GK_POSTPRE)
        return std::string("k_postpre<") + T + ", " + std::to_string(L.sa.src) + ", " + std::to_string(L.sa.nu) +
               (L.sa.flags == 32 ? ", 8, 8>" : ", 16, 16>");
    if (L.gk == GK_PRE || L.gk == GK_POST) {
        const std::string k = L.gk == GK_PRE ? "k_pre" : "k_post";
        const std::string nu = std::to_string(L.sa.nu);
        if (L.sa.flags & 2) return k + "_s<" + T + ", " + nu + ", " + std::to_string(16 << ((L.sa.flags >> 2) & 3)) + ">";
        if (L.sa.flags & 1) return k + "<" + T + ", " + nu + ", 16, 16>";
        if (L.sa.flags & 16) return k + "<" + T + ", " + nu + ", 32, 32>";
        if (L.sa.flags & 32) return k + "<" + T + ", " + nu + ", 8, 8>";
        return k + "<" + T + ", " + nu + ", 64, 32>";
    }
    if (L.gk == GK_ZEBRA) return std::string("k_zebra<") + T + ", " + std::to_string(L.sa.nu) + ">";
    if (L.gk <= GK_NORM || L.gk == GK_ZERO_SELF) return std::string("k_unfused<") + T + ", " + std::to_string(L.gk) + ">";
    return std::string("k_driver<") + (L.f32 ? "true" : "false") + ", " + std::to_string(L.gk) + ">";
    (void)h;
}

// algorithmic bytes and flops of one launch (every input read once, every output written once)
void launch_work(const kc_hier* h, const Launch& L, double& bytes, double& flops)
{
    bytes = flops = 0.0;
    const double T = L.f32 ? 4.0 : 8.0;
    if (L.type == L_SUB) {
        for (int idx : h->lists[lt_sub(L.ba.depth)]) {
            const HostInst& hi = h->hi[idx];
            const double nt = hi.il.n[L.ba.depth];
            bytes += 2.0 * nt * nt * T;
            auto add_list = [&](int k) {
                const int kk = std::min(k, KMAX);
                for (int o = 0; o < olen(hi, L.ba.smoother)[kk - 1]; ++o) {
                    const uint32_t op = hi.ops[obeg(hi, L.ba.smoother)[kk - 1] + o];
                    const double n = hi.il.n[sop_depth(op)], n2 = n * n;
                    if (sop_kind(op) == SOP_PRE) {
                        const double nc = (n - 1) / 2;
                        const double sw = L.ba.nu1 > 0 ? (sop_zg(op) ? 1.0 + FL_SWEEP * (L.ba.nu1 - 1) : FL_SWEEP * L.ba.nu1) : 0.0;
                        flops += n2 * (sw + FL_RESID) + nc * nc * FL_FW;
                    } else if (sop_kind(op) == SOP_POST) {
                        flops += n2 * (FL_PROLONG + FL_SWEEP * L.ba.nu2);
                    } else {
                        flops += 2.0 * n2 * n2;   // triangular solves with the dense factor
                    }
                }
            };
            add_list(L.ba.kappa);
            if (L.ba.pair && L.ba.kappa > 1) add_list(L.ba.kappa - 1);
        }
        return;
    }
    if (L.type == L_COARSEST) return;
    const int d = L.sa.depth;
    for (int i = 0; i < h->count; ++i) {
        const HostInst& hi = h->hi[i];
        if (L.gk == GK_POSTPRE) {
            if (hi.cut <= d) continue;
            const double nf = hi.il.n[d], nc = hi.il.n[d + 1];
            bytes += (3.0 * nf * nf + 2.0 * nc * nc) * T;   // read v, f, v_c; write v, f_c
            flops += nf * nf * (FL_PROLONG + FL_SWEEP * (L.sa.src + L.sa.nu) + FL_RESID) + nc * nc * FL_FW;
            continue;
        }
        if (L.gk == GK_ZEBRA) {
            // one colour: f of its lines and the other colour's lines read, its lines written
            if (hi.cut <= d || d >= hi.il.L) continue;
            const double nl = hi.il.n[d], np = hi.il.nx[d];
            const double own = std::floor((nl + 1 - L.sa.dst) / 2);
            bytes += (2.0 * own + (nl - own)) * np * T;
            flops += own * np * (FL_ZEBRA_RHS + FL_ZEBRA_SOLVE);
            continue;
        }
        if (L.gk == GK_PRE || L.gk == GK_POST) {
            if (hi.cut <= d) continue;
            const double nf = hi.il.n[d], nc = hi.il.n[d + 1];
            bytes += (3.0 * nf * nf + nc * nc) * T;
            flops += (L.gk == GK_PRE) ? nf * nf * (FL_SWEEP * L.sa.nu + FL_RESID) + nc * nc * FL_FW
                                      : nf * nf * (FL_PROLONG + FL_SWEEP * L.sa.nu);
            continue;
        }
        const double n0 = hi.il.n[0], N = n0 * n0;
        switch (L.gk) {
        case GK_IR_RESID: bytes += N * 20.0; break;          // read u, f; write the FP32 right-hand side
        case GK_IR_UPDATE: bytes += N * 20.0; break;         // read e (FP32) and u; write u
        case GK_SSF: bytes += N * 8.0; break;
        case GK_PCG_INIT: bytes += N * 24.0; break;          // read f; write u, r
        case GK_PCG_PRECIN: bytes += N * (L.f32 ? 12.0 : 0.0); break;
        case GK_PCG_RZ: bytes += N * (L.f32 ? 20.0 : 24.0); break;
        case GK_PCG_P: bytes += N * 24.0; break;
        case GK_PCG_AP: bytes += N * 16.0; break;
        case GK_PCG_UPD: bytes += N * 48.0; break;
        default: break;
        }
    }
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

void kc_exec_default(kc_exec* e)
{
    if (!e) return;
    std::memset(e, 0, sizeof *e);
    e->mode = 0;
    e->use_graph = 1;
    e->coarse_cutover = 31;
    e->coarse_threads = 512;
    e->poll_every = 0;
    e->coarse_wave_n = 15;
    e->small_tile_n = 511;
    e->stream_n = 2047;
    e->mid_tile_n = 2047;
    e->tiny_tile_n = 255;
    e->zebra_wave_n = 63;
    e->zebra_quad_n = 8191;
    e->wave_regs = 1;
    e->fuse_junctions = 1;
}

const char* kc_status_string(kc_status s)
{
    switch (s) {
    case KC_OK: return "KC_OK";
    case KC_NOT_CONVERGED: return "KC_NOT_CONVERGED";
    case KC_DIVERGED: return "KC_DIVERGED";
    case KC_BREAKDOWN: return "KC_BREAKDOWN";
    case KC_ERR_ARG: return "KC_ERR_ARG";
    case KC_ERR_HIP: return "KC_ERR_HIP";
    case KC_ERR_WORKSPACE: return "KC_ERR_WORKSPACE";
    case KC_ERR_NONFINITE: return "KC_ERR_NONFINITE";
    case KC_ERR_STATE: return "KC_ERR_STATE";
    }
    return "KC_UNKNOWN";
}

const char* kc_last_error(void) { return g_err.c_str(); }

kc_status kc_workspace_bytes(const kc_problem* probs, int32_t count, kc_precision prec, size_t* bytes)
{
    if (!bytes) return fail(KC_ERR_ARG, "null bytes");
    Layout lay;
    kc_status s = make_layout(probs, count, prec, lay);
    if (s != KC_OK) return s;
    *bytes = lay.total;
    return KC_OK;
}

kc_status kc_workspace_bytes_semi(const kc_problem* probs, int32_t count, kc_precision prec, size_t* bytes)
{
    if (!bytes) return fail(KC_ERR_ARG, "null bytes");
    Layout lay;
    kc_status s = make_layout(probs, count, prec, lay, true);
    if (s != KC_OK) return s;
    *bytes = lay.total;
    return KC_OK;
}

kc_status kc_semi_stencils(const kc_problem* p, int32_t max_levels, int32_t* nlevels, double* stencils)
{
    if (!p || !nlevels) return fail(KC_ERR_ARG, "null argument");
    Layout lay;
    kc_status s = make_layout(p, 1, KC_F64, lay, true);
    if (s != KC_OK) return s;
    const int L = lay.il[0].L;
    *nlevels = L;
    double cur[9];
    fine_stencil(p->theta, p->eps, cur);
    for (int d = 0; d < L && d < max_levels; ++d) {
        if (stencils) std::memcpy(stencils + 9 * d, cur, sizeof cur);
        double nxt[9];
        semi_galerkin(cur, nxt);
        std::memcpy(cur, nxt, sizeof cur);
    }
    return KC_OK;
}

kc_status kc_level_stencils(const kc_problem* p, int32_t max_levels, int32_t* nlevels, double* stencils)
{
    if (!p || !nlevels) return fail(KC_ERR_ARG, "null argument");
    int L;
    kc_status s = check_problem(*p, L);
    if (s != KC_OK) return s;
    *nlevels = L;
    double cur[9];
    fine_stencil(p->theta, p->eps, cur);
    for (int d = 0; d < L && d < max_levels; ++d) {
        if (stencils) std::memcpy(stencils + 9 * d, cur, sizeof cur);
        double nxt[9];
        galerkin(cur, nxt);
        std::memcpy(cur, nxt, sizeof cur);
    }
    return KC_OK;
}

kc_status kc_convection_stencils(const kc_problem* p, double bx, double by, int32_t max_levels, int32_t* nlevels,
                                 double* stencils)
{
    if (!p || !nlevels) return fail(KC_ERR_ARG, "null argument");
    if (!std::isfinite(bx) || !std::isfinite(by)) return fail(KC_ERR_ARG, "bx, by must be finite");
    int L;
    kc_status s = check_problem(*p, L);
    if (s != KC_OK) return s;
    *nlevels = L;
    for (int d = 0; d < L && d < max_levels; ++d)
        if (stencils) convection_stencil(((p->n + 1) >> d) - 1, p->theta, p->eps, bx, by, stencils + 9 * d);
    return KC_OK;
}

// prec: the hierarchy's precision, or -1 for host-only planning
static kc_status validate_exec(const kc_exec* e, int prec)
{
    if (e->mode != 0 && e->mode != 1) return fail(KC_ERR_ARG, "exec.mode must be 0 or 1");
    if (e->coarse_cutover < 7 || e->coarse_cutover > 63) return fail(KC_ERR_ARG, "coarse_cutover must be in 7..63");
    if (e->coarse_threads != 256 && e->coarse_threads != 512 && e->coarse_threads != 1024)
        return fail(KC_ERR_ARG, "coarse_threads must be 256, 512 or 1024");
    if (e->coarse_threads == 1024 && prec == (int)KC_F64)
        return fail(KC_ERR_ARG, "coarse_threads 1024 needs FP32 cycles (the FP64 persistent kernel needs more registers)");
    if (e->poll_every < 0) return fail(KC_ERR_ARG, "poll_every must be >= 0");
    if (e->coarse_wave_n < 0 || e->coarse_wave_n > 15) return fail(KC_ERR_ARG, "coarse_wave_n must be in 0..15");
    if (e->small_tile_n < 0 || e->small_tile_n > 4095) return fail(KC_ERR_ARG, "small_tile_n must be in 0..4095");
    if (e->stream_n < 0) return fail(KC_ERR_ARG, "stream_n must be >= 0");
    if (e->mid_tile_n < 0 || e->mid_tile_n > 4095) return fail(KC_ERR_ARG, "mid_tile_n must be in 0..4095");
    if (e->tiny_tile_n < 0 || e->tiny_tile_n > 4095) return fail(KC_ERR_ARG, "tiny_tile_n must be in 0..4095");
    if (e->zebra_wave_n < 0 || e->zebra_wave_n > 16383) return fail(KC_ERR_ARG, "zebra_wave_n must be in 0..16383");
    if (e->zebra_quad_n < 0 || e->zebra_quad_n > 16383) return fail(KC_ERR_ARG, "zebra_quad_n must be in 0..16383");
    if (e->wave_regs != 0 && e->wave_regs != 1) return fail(KC_ERR_ARG, "wave_regs must be 0 or 1");
    if (e->fuse_junctions != 0 && e->fuse_junctions != 1) return fail(KC_ERR_ARG, "fuse_junctions must be 0 or 1");
    if (e->coarse_threads * 8 < 64 * e->coarse_cutover) return fail(KC_ERR_ARG, "coarse_threads too small for the cutover");
    return KC_OK;
}

// level stencils of one instance: Galerkin coarse operators of the diffusion
// problem, or the rediscretised convection-diffusion operator
static void level_stencils_of(HostInst& hi)
{
    if (hi.conv) {
        for (int d = 0; d < hi.il.L; ++d) convection_stencil(hi.il.n[d], hi.p.theta, hi.p.eps, hi.bx, hi.by, hi.s[d]);
        return;
    }
    fine_stencil(hi.p.theta, hi.p.eps, hi.s[0]);
    for (int d = 1; d < hi.il.L; ++d) {
        if (hi.il.semi) semi_galerkin(hi.s[d - 1], hi.s[d]);
        else galerkin(hi.s[d - 1], hi.s[d]);
    }
}

static void build_host(kc_hier* h, const kc_problem* probs)
{
    h->hi.assign(h->count, HostInst());
    for (int i = 0; i < h->count; ++i) {
        HostInst& hi = h->hi[i];
        hi.p = probs[i];
        hi.il = h->lay.il[i];
        level_stencils_of(hi);
    }
}

// coarsest factors and line-solve tables of instance i, copied into the workspace
static kc_status upload_factors(kc_hier* h, int i)
{
    HostInst& hi = h->hi[i];
    std::vector<double> c64;
    std::vector<float> c32;
    if (!coarse_cholesky<double>(hi.p.n_coarsest, hi.s[hi.il.L - 1], c64) ||
        !coarse_cholesky<float>(hi.p.n_coarsest, hi.s[hi.il.L - 1], c32))
        return fail(KC_ERR_ARG, "coarsest matrix is not positive definite");
    std::vector<double> z64;
    std::vector<float> z32;
    for (int d = 0; d < hi.il.L; ++d) {
        line_tables<double>(hi.il.nx[d], hi.s[d], z64);
        line_tables<float>(hi.il.nx[d], hi.s[d], z32);
    }
    if (hipMemcpyAsync(h->ws + hi.il.chol64, c64.data(), c64.size() * 8, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(h->ws + hi.il.chol32, c32.data(), c32.size() * 4, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(h->ws + hi.il.zt64, z64.data(), z64.size() * 8, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(h->ws + hi.il.zt32, z32.data(), z32.size() * 4, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return fail(KC_ERR_HIP, "upload of the coarsest factor or the line-solve tables failed");
    return KC_OK;
}


kc_status kc_schedule_counts(const kc_problem* probs, int32_t count, const kc_exec* exec, const kc_cycle_params* c,
                             int64_t* grid_launches, int64_t* subtree_launches, int64_t* subtree_stages)
{
    kc_status s = check_cycle(c);
    if (s != KC_OK) return s;
    kc_hier h;
    h.count = count;
    kc_exec_default(&h.ex);
    if (exec) h.ex = *exec;
    if ((s = validate_exec(&h.ex, -1)) != KC_OK) return s;
    if ((s = make_layout(probs, count, KC_F64, h.lay)) != KC_OK) return s;
    build_host(&h, probs);
    // host-only planning: no device tables are written and the LDS limit is not checked
    h.d_tiles = nullptr;
    s = plan_exec(&h);
    if (s != KC_OK) return s;
    std::vector<int32_t> zeros((size_t)NTABLES * (count + 1) + 2 * MAXL * count, 0);
    h.d_tiles = zeros.data();
    h.d_lists = zeros.data() + (size_t)NTABLES * (count + 1);
    std::vector<Launch> ls;
    iteration(&h, DRV_CYCLE, *c, ls);
    int64_t g = 0, sb = 0;
    count_launches(ls, g, sb);
    int64_t st = 0;
    for (const Launch& L : ls)
        if (L.type == L_SUB)
            for (int idx : h.lists[lt_sub(L.ba.depth)]) {
                const HostInst& hi = h.hi[idx];
                st += olen(hi, L.ba.smoother)[std::min(L.ba.kappa, KMAX) - 1];
                if (L.ba.pair && L.ba.kappa > 1) st += olen(hi, L.ba.smoother)[std::min(L.ba.kappa - 1, KMAX) - 1];
                break;
            }
    if (grid_launches) *grid_launches = g;
    if (subtree_launches) *subtree_launches = sb;
    if (subtree_stages) *subtree_stages = st;
    h.d_tiles = nullptr;
    h.d_lists = nullptr;
    return KC_OK;
}

static kc_status create_impl(const kc_problem* probs, int32_t count, kc_precision prec, const kc_exec* exec,
                             void* d_workspace, size_t bytes, void* hip_stream, kc_hier** out, bool semi)
{
    if (!out) return fail(KC_ERR_ARG, "null out");
    *out = nullptr;
    kc_hier* h = new kc_hier();
    h->count = count;
    h->prec = prec;
    h->semi = semi;
    kc_exec_default(&h->ex);
    if (exec) h->ex = *exec;
    if (semi) h->ex.mode = 1;   // one kernel per operation on the rectangular levels
    kc_status s = validate_exec(&h->ex, (int)prec);
    if (s != KC_OK) { delete h; return s; }
    s = make_layout(probs, count, prec, h->lay, semi);
    if (s != KC_OK) { delete h; return s; }
    if (!d_workspace || bytes < h->lay.total) { delete h; return fail(KC_ERR_WORKSPACE, "workspace missing or smaller than kc_workspace_bytes"); }
    if (((uintptr_t)d_workspace) % ALIGN != 0) { delete h; return fail(KC_ERR_WORKSPACE, "workspace must be 256-byte aligned"); }
    h->ws = (char*)d_workspace;
    h->ws_bytes = bytes;
    h->user_stream = (hipStream_t)hip_stream;
    auto cleanup = [&](kc_status st) { kc_destroy(h); return st; };
    if (h->user_stream == nullptr) {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess)
            return cleanup(fail(KC_ERR_HIP, "hipStreamCreateWithFlags failed"));
        h->own_stream = true;
    } else {
        h->stream = h->user_stream;
    }
    if (hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming) != hipSuccess || hipEventCreate(&h->t0) != hipSuccess ||
        hipEventCreate(&h->t1) != hipSuccess || hipEventCreateWithFlags(&h->ev_upload, hipEventDisableTiming) != hipSuccess)
        return cleanup(fail(KC_ERR_HIP, "hipEventCreate failed"));
    if (hipHostMalloc((void**)&h->h_inst, sizeof(InstDev) * count, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h->h_st, sizeof(InstState) * count, hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(KC_ERR_HIP, "hipHostMalloc failed"));
    std::memset(h->h_inst, 0, sizeof(InstDev) * count);
    std::memset(h->h_st, 0, sizeof(InstState) * count);
    h->d_inst = (InstDev*)(h->ws + h->lay.inst);
    h->d_st = (InstState*)(h->ws + h->lay.state);
    h->d_tiles = (int32_t*)(h->ws + h->lay.tiles);
    h->d_lists = (int32_t*)(h->ws + h->lay.lists);
    h->d_partial = (double*)(h->ws + h->lay.partial);
    h->d_hist = (double*)(h->ws + h->lay.hist);
    if ((s = enter(h)) != KC_OK) return cleanup(s);
    build_host(h, probs);
    // coarsest Cholesky factors and line-solve tables
    for (int i = 0; i < count; ++i)
        if ((s = upload_factors(h, i)) != KC_OK) return cleanup(s);
    if ((s = plan_exec(h)) != KC_OK) return cleanup(s);
    fill_inst_static(h);
    set_omega(h, 0.8);
    h->omega_set = 0.8;
    if ((s = upload_inst(h)) != KC_OK) return cleanup(s);
    if ((s = upload_state(h, 0.0, 0)) != KC_OK) return cleanup(s);
    if (hipStreamSynchronize(h->stream) != hipSuccess) return cleanup(fail(KC_ERR_HIP, "setup synchronisation failed"));
    if ((s = leave(h)) != KC_OK) return cleanup(s);
    *out = h;
    return KC_OK;
}

kc_status kc_create(const kc_problem* probs, int32_t count, kc_precision prec, const kc_exec* exec, void* d_workspace,
                    size_t bytes, void* hip_stream, kc_hier** out)
{
    return create_impl(probs, count, prec, exec, d_workspace, bytes, hip_stream, out, false);
}

kc_status kc_create_semi(const kc_problem* probs, int32_t count, kc_precision prec, const kc_exec* exec,
                         void* d_workspace, size_t bytes, void* hip_stream, kc_hier** out)
{
    return create_impl(probs, count, prec, exec, d_workspace, bytes, hip_stream, out, true);
}

kc_status kc_destroy(kc_hier* h)
{
    if (!h) return KC_OK;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    if (h->h_inst) (void)hipHostFree(h->h_inst);
    if (h->h_st) (void)hipHostFree(h->h_st);
    if (h->ev_in) (void)hipEventDestroy(h->ev_in);
    if (h->ev_out) (void)hipEventDestroy(h->ev_out);
    if (h->t0) (void)hipEventDestroy(h->t0);
    if (h->t1) (void)hipEventDestroy(h->t1);
    if (h->ev_upload) (void)hipEventDestroy(h->ev_upload);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return KC_OK;
}

kc_status kc_set_exec(kc_hier* h, const kc_exec* exec)
{
    if (!h || !exec) return fail(KC_ERR_ARG, "null argument");
    kc_status s = validate_exec(exec, (int)h->prec);
    if (s != KC_OK) return s;
    if (h->semi && exec->mode != 1) return fail(KC_ERR_ARG, "a semi-coarsened hierarchy runs one kernel per operation (mode 1)");
    HIPCHK(hipStreamSynchronize(h->stream));
    drop_graphs(h);
    kc_exec old = h->ex;
    h->ex = *exec;
    if ((s = plan_exec(h)) != KC_OK) {
        h->ex = old;
        (void)plan_exec(h);
        return s;
    }
    fill_inst_static(h);
    set_omega(h, h->omega_set);
    if ((s = upload_inst(h)) != KC_OK) return s;
    HIPCHK(hipStreamSynchronize(h->stream));
    return KC_OK;
}

kc_status kc_set_convection(kc_hier* h, const double* bx, const double* by)
{
    if (!h || !bx || !by) return fail(KC_ERR_ARG, "null argument");
    if (h->semi) return fail(KC_ERR_STATE, "convection-diffusion needs full coarsening");
    for (int i = 0; i < h->count; ++i) {
        if (!std::isfinite(bx[i]) || !std::isfinite(by[i])) return fail(KC_ERR_ARG, "bx, by must be finite");
        if (h->hi[i].p.n_coarsest != 1)
            return fail(KC_ERR_ARG, "convection-diffusion needs a 1 x 1 coarsest level (n_coarsest = 1)");
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    drop_graphs(h);
    kc_status s;
    if ((s = enter(h)) != KC_OK) return s;
    for (int i = 0; i < h->count; ++i) {
        HostInst& hi = h->hi[i];
        hi.conv = true;
        hi.bx = bx[i];
        hi.by = by[i];
        level_stencils_of(hi);
        if ((s = upload_factors(h, i)) != KC_OK) return s;
    }
    fill_inst_static(h);
    set_omega(h, h->omega_set);
    if ((s = upload_inst(h)) != KC_OK) return s;
    HIPCHK(hipStreamSynchronize(h->stream));
    return leave(h);
}

// level-0 binding of the cycle arrays for each driver
static void bind_level0_user(kc_hier* h, double* const* v, const int64_t* ldv, const double* const* f, const int64_t* ldf)
{
    for (int i = 0; i < h->count; ++i) {
        InstDev& I = h->h_inst[i];
        const HostInst& hi = h->hi[i];
        LevelDev& L0 = I.lev[0];
        L0.A = v[i];
        L0.lda = (int32_t)ldv[i];
        L0.B = h->ws + hi.il.B[0];
        L0.ldb = hi.il.ld[0];
        L0.F = (void*)f[i];
        L0.ldf = (int32_t)ldf[i];
        L0.fscale = I.h2;
        I.u = v[i];
        I.ldu = (int32_t)ldv[i];
        I.f = f[i];
        I.ldf = (int32_t)ldf[i];
    }
}

static void bind_level0_internal(kc_hier* h, bool pcg64)
{
    for (int i = 0; i < h->count; ++i) {
        InstDev& I = h->h_inst[i];
        const HostInst& hi = h->hi[i];
        LevelDev& L0 = I.lev[0];
        if (pcg64) {   // FP64 preconditioner: cycle on z with right-hand side r
            L0.A = I.z;
            L0.lda = I.ldv;
            L0.B = h->ws + hi.il.B[0];
            L0.ldb = hi.il.ld[0];
            L0.F = I.r;
            L0.ldf = I.ldv;
        } else {       // FP32 cycle arrays
            L0.A = h->ws + hi.il.A[0];
            L0.B = h->ws + hi.il.B[0];
            L0.F = h->ws + hi.il.F[0];
            L0.lda = L0.ldb = L0.ldf = hi.il.ld[0];
        }
        L0.fscale = 1.0;
    }
}

static void bind_user_vectors(kc_hier* h, double* const* u, const int64_t* ldu, const double* const* f, const int64_t* ldf)
{
    for (int i = 0; i < h->count; ++i) {
        InstDev& I = h->h_inst[i];
        I.u = u[i];
        I.ldu = (int32_t)ldu[i];
        I.f = f[i];
        I.ldf = (int32_t)ldf[i];
    }
}

kc_status kc_cycle(kc_hier* h, double* const* d_v, const int64_t* ldv, const double* const* d_f, const int64_t* ldf,
                   const kc_cycle_params* c)
{
    if (!h) return fail(KC_ERR_ARG, "null hierarchy");
    if (h->prec != KC_F64) return fail(KC_ERR_STATE, "kc_cycle needs an FP64 hierarchy");
    kc_status s;
    if ((s = check_ptrs(h, d_v, ldv, "v")) != KC_OK || (s = check_ptrs(h, d_f, ldf, "f")) != KC_OK) return s;
    if ((s = prepare_call(h, c)) != KC_OK) return s;
    if ((s = check_zebra_ld(h, c, d_v, ldv, "v")) != KC_OK || (s = check_zebra_ld(h, c, d_f, ldf, "f")) != KC_OK)
        return s;
    if ((s = enter(h)) != KC_OK) return s;
    bind_level0_user(h, d_v, ldv, d_f, ldf);
    if ((s = upload_inst(h)) != KC_OK) return s;
    if ((s = upload_state(h, 0.0, 0)) != KC_OK) return s;
    if ((s = launch_iteration(h, DRV_CYCLE, *c, 1)) != KC_OK) return s;
    record_counts(h, DRV_CYCLE, *c);
    return leave(h);
}

kc_status kc_solve(kc_hier* h, double* const* d_u, const int64_t* ldu, const double* const* d_f, const int64_t* ldf,
                   const kc_cycle_params* c, double tol, int32_t maxit, int32_t* iters, double* relres, int32_t* status)
{
    if (!h) return fail(KC_ERR_ARG, "null hierarchy");
    kc_status s;
    if ((s = check_ptrs(h, d_u, ldu, "u")) != KC_OK || (s = check_ptrs(h, d_f, ldf, "f")) != KC_OK) return s;
    if (maxit < 0 || !(tol >= 0.0)) return fail(KC_ERR_ARG, "maxit must be >= 0 and tol >= 0");
    if ((s = prepare_call(h, c)) != KC_OK) return s;
    if ((s = check_zebra_ld(h, c, d_u, ldu, "u")) != KC_OK || (s = check_zebra_ld(h, c, d_f, ldf, "f")) != KC_OK)
        return s;
    if ((s = enter(h)) != KC_OK) return s;
    const bool f32 = h->prec == KC_F32_CYCLE;
    if (f32) {
        bind_user_vectors(h, d_u, ldu, d_f, ldf);
        bind_level0_internal(h, false);
    } else {
        bind_level0_user(h, d_u, ldu, d_f, ldf);
    }
    if ((s = upload_inst(h)) != KC_OK) return s;
    if ((s = upload_state(h, tol, maxit)) != KC_OK) return s;
    {
        Launch L = grid(h, GK_SSF, f32, tt_all0(), 0);
        L.sa.fin = FIN_SSF;
        HIPCHK(launch_grid(L.gk, L.f32, L.sa, L.nblocks, h->stream));
    }
    const int drv = f32 ? DRV_IR : DRV_SOLVE64;
    s = drive(h, drv, *c, maxit, iters, relres, status);
    record_counts(h, drv, *c);
    h->last_driver = f32 ? "solve_ir_f32" : "solve_f64";
    if (s >= 0) h->last_iters.assign(iters, iters + h->count);
    else h->last_iters.clear();
    kc_status s2 = leave(h);
    return s2 != KC_OK ? s2 : s;
}

kc_status kc_pcg(kc_hier* h, double* const* d_u, const int64_t* ldu, const double* const* d_f, const int64_t* ldf,
                 const kc_cycle_params* c, double tol, int32_t maxit, int32_t* iters, double* relres, int32_t* status)
{
    if (!h) return fail(KC_ERR_ARG, "null hierarchy");
    kc_status s;
    if ((s = check_ptrs(h, d_u, ldu, "u")) != KC_OK || (s = check_ptrs(h, d_f, ldf, "f")) != KC_OK) return s;
    if (maxit < 0 || !(tol >= 0.0)) return fail(KC_ERR_ARG, "maxit must be >= 0 and tol >= 0");
    if (any_convection(h)) return fail(KC_ERR_STATE, "CG needs a symmetric operator (convection is set)");
    if ((s = prepare_call(h, c)) != KC_OK) return s;
    if ((s = enter(h)) != KC_OK) return s;
    const bool f32 = h->prec == KC_F32_CYCLE;
    bind_user_vectors(h, d_u, ldu, d_f, ldf);
    bind_level0_internal(h, !f32);
    if ((s = upload_inst(h)) != KC_OK) return s;
    if ((s = upload_state(h, tol, maxit)) != KC_OK) return s;
    {
        Launch L = grid(h, GK_PCG_INIT, f32, tt_all0(), 0);
        L.sa.fin = FIN_PCG_INIT;
        HIPCHK(launch_grid(L.gk, L.f32, L.sa, L.nblocks, h->stream));
    }
    s = drive(h, DRV_PCG, *c, maxit, iters, relres, status);
    record_counts(h, DRV_PCG, *c);
    h->last_driver = f32 ? "pcg_f32_precond" : "pcg_f64";
    if (s >= 0) h->last_iters.assign(iters, iters + h->count);
    else h->last_iters.clear();
    kc_status s2 = leave(h);
    return s2 != KC_OK ? s2 : s;
}

kc_status kc_residual_history(kc_hier* h, int32_t instance, double* out, int32_t cap, int32_t* count)
{
    if (!h || !count) return fail(KC_ERR_ARG, "null argument");
    if (instance < 0 || instance >= h->count) return fail(KC_ERR_ARG, "instance out of range");
    if (cap < 0 || (cap > 0 && !out)) return fail(KC_ERR_ARG, "out must hold cap entries");
    if ((int)h->last_iters.size() != h->count) return fail(KC_ERR_STATE, "no kc_solve or kc_pcg has run on this hierarchy");
    const int n = std::min(h->last_iters[instance] + 1, HIST_CAP);
    *count = n;
    const int m = std::min(cap, n);
    if (m > 0) {
        HIPCHK(hipMemcpyAsync(out, h->d_hist + (size_t)instance * HIST_CAP, sizeof(double) * m, hipMemcpyDeviceToHost,
                              h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    return KC_OK;
}

kc_status kc_apply_A(kc_hier* h, double* const* d_y, const int64_t* ldy, const double* const* d_x, const int64_t* ldx)
{
    if (!h) return fail(KC_ERR_ARG, "null hierarchy");
    kc_status s;
    if ((s = check_ptrs(h, d_y, ldy, "y")) != KC_OK || (s = check_ptrs(h, d_x, ldx, "x")) != KC_OK) return s;
    if ((s = enter(h)) != KC_OK) return s;
    for (int i = 0; i < h->count; ++i) {
        InstDev& I = h->h_inst[i];
        I.x = d_x[i];
        I.ldx = (int32_t)ldx[i];
        I.y = d_y[i];
        I.ldy = (int32_t)ldy[i];
    }
    if ((s = upload_inst(h)) != KC_OK) return s;
    if ((s = upload_state(h, 0.0, 0)) != KC_OK) return s;
    Launch L = grid(h, GK_APPLY, false, tt_all0(), 0);
    HIPCHK(launch_grid(L.gk, L.f32, L.sa, L.nblocks, h->stream));
    return leave(h);
}

kc_status kc_grad_params(kc_hier* h, const double* const* d_lam, const int64_t* ldl, const double* const* d_u,
                         const int64_t* ldu, double* dtheta, double* deps)
{
    if (!h) return fail(KC_ERR_ARG, "null hierarchy");
    if (!dtheta || !deps) return fail(KC_ERR_ARG, "null outputs");
    if (any_convection(h)) return fail(KC_ERR_STATE, "the parameter gradients are those of the diffusion operator");
    kc_status s;
    if ((s = check_ptrs(h, d_lam, ldl, "lam")) != KC_OK || (s = check_ptrs(h, d_u, ldu, "u")) != KC_OK) return s;
    if ((s = enter(h)) != KC_OK) return s;
    for (int i = 0; i < h->count; ++i) {
        InstDev& I = h->h_inst[i];
        I.x = d_lam[i];
        I.ldx = (int32_t)ldl[i];
        I.y = (double*)d_u[i];
        I.ldy = (int32_t)ldu[i];
    }
    if ((s = upload_inst(h)) != KC_OK) return s;
    if ((s = upload_state(h, 0.0, 0)) != KC_OK) return s;
    Launch L = grid(h, GK_GRAD, false, tt_all0(), 0);
    L.sa.fin = FIN_GRAD;
    HIPCHK(launch_grid(L.gk, L.f32, L.sa, L.nblocks, h->stream));
    HIPCHK(hipMemcpyAsync(h->h_st, h->d_st, sizeof(InstState) * h->count, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int i = 0; i < h->count; ++i) {
        dtheta[i] = h->h_st[i].dth;
        deps[i] = h->h_st[i].deps;
    }
    return leave(h);
}

kc_status kc_time_stage(kc_hier* h, int32_t which, const kc_cycle_params* c, int32_t reps, double* avg_ms, double* bytes)
{
    if (!h || !avg_ms || !bytes || reps < 1) return fail(KC_ERR_ARG, "bad argument");
    kc_status s = prepare_call(h, c);
    if (s != KC_OK) return s;
    if ((s = enter(h)) != KC_OK) return s;
    if ((s = upload_inst(h)) != KC_OK) return s;
    if ((s = upload_state(h, 0.0, 0)) != KC_OK) return s;   // every instance active, no reduction decisions
    const bool f32 = h->prec == KC_F32_CYCLE;
    const double T = f32 ? 4.0 : 8.0;
    Launch L{};
    double b = 0.0;
    const bool is_pre = which == 0 || (which >= 100 && which < 100 + MAXL);
    const bool is_post = which == 1 || (which >= 200 && which < 200 + MAXL);
    if (is_pre || is_post) {
        const int d = which <= 1 ? 0 : which % 100;
        if (d >= h->max_cut) return fail(KC_ERR_STATE, "no grid-wide stage at that depth (persistent kernel there)");
        L = fused_grid(h, is_pre ? GK_PRE : GK_POST, f32, d);
        L.sa.nu = is_pre ? c->nu1 : c->nu2;
        for (int i = 0; i < h->count; ++i) {
            if (h->hi[i].cut <= d) continue;
            const double nf = h->hi[i].il.n[d], ncs = h->hi[i].il.n[d + 1];
            // pre: read v and f, write v and f_c; post: read v, f and v_c, write v
            b += (3.0 * nf * nf + ncs * ncs) * T;
        }
    } else if (which == 2 || (which >= 300 && which < 300 + MAXL)) {
        int d = -1;
        if (which >= 300) d = which - 300;
        for (int k = 1; k < MAXL && d < 0; ++k)
            if (nlist(h, lt_sub(k)) > 0) d = k;
        if (d < 0 || nlist(h, lt_sub(d)) == 0) return fail(KC_ERR_STATE, "no persistent launch at that depth");
        L = sub(h, f32, d, clamp_kappa(h, c->kappa), true, c->nu1, c->nu2, false, FIN_NONE);
        for (int idx : h->lists[lt_sub(d)]) {
            const double n = h->hi[idx].il.n[d];
            b += 2.0 * n * n * T;   // reads f, writes v of the top level; coarser levels stay in LDS
        }
    } else if (which == 3) {
        if (!f32) return fail(KC_ERR_STATE, "the refinement residual pass exists on FP32 hierarchies");
        L = grid(h, GK_IR_RESID, true, tt_all0(), 0);
        for (int i = 0; i < h->count; ++i) {
            const double n0 = h->hi[i].il.n[0];
            b += n0 * n0 * (8.0 + 8.0 + 4.0);   // read u, f; write the FP32 right-hand side
        }
    } else {
        return fail(KC_ERR_ARG, "unknown stage");
    }
    std::vector<Launch> one(1, L);
    HIPCHK(run(h, one));   // warm
    HIPCHK(hipEventRecord(h->t0, h->stream));
    for (int r = 0; r < reps; ++r) HIPCHK(run(h, one));
    HIPCHK(hipEventRecord(h->t1, h->stream));
    HIPCHK(hipEventSynchronize(h->t1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, h->t0, h->t1));
    *avg_ms = (double)ms / reps;
    *bytes = b;
    return leave(h);
}

kc_status kc_time_cycles(kc_hier* h, double* const* d_v, const int64_t* ldv, const double* const* d_f,
                         const int64_t* ldf, const kc_cycle_params* c, int32_t reps, double* ms_per_cycle)
{
    if (!h || !ms_per_cycle || reps < 1) return fail(KC_ERR_ARG, "bad argument");
    if (h->prec != KC_F64) return fail(KC_ERR_STATE, "kc_time_cycles needs an FP64 hierarchy");
    kc_status s;
    if ((s = check_ptrs(h, d_v, ldv, "v")) != KC_OK || (s = check_ptrs(h, d_f, ldf, "f")) != KC_OK) return s;
    if ((s = prepare_call(h, c)) != KC_OK) return s;
    if ((s = check_zebra_ld(h, c, d_v, ldv, "v")) != KC_OK || (s = check_zebra_ld(h, c, d_f, ldf, "f")) != KC_OK)
        return s;
    if ((s = enter(h)) != KC_OK) return s;
    bind_level0_user(h, d_v, ldv, d_f, ldf);
    if ((s = upload_inst(h)) != KC_OK) return s;
    if ((s = upload_state(h, 0.0, 0)) != KC_OK) return s;
    if ((s = launch_iteration(h, DRV_CYCLE, *c, 1)) != KC_OK) return s;   // capture + warm
    if ((s = warm_graphs(h, DRV_CYCLE, *c, reps)) != KC_OK) return s;     // nothing captured while timed
    HIPCHK(hipEventRecord(h->t0, h->stream));
    if ((s = launch_iteration(h, DRV_CYCLE, *c, reps)) != KC_OK) return s;
    HIPCHK(hipEventRecord(h->t1, h->stream));
    HIPCHK(hipEventSynchronize(h->t1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, h->t0, h->t1));
    *ms_per_cycle = (double)ms / reps;
    record_counts(h, DRV_CYCLE, *c);
    return leave(h);
}

kc_status kc_profile_iteration(kc_hier* h, int32_t driver, const kc_cycle_params* c, int32_t reps, char* out, size_t cap)
{
    if (!h || !out || cap == 0 || reps < 1) return fail(KC_ERR_ARG, "bad argument");
    if (driver != 0 && driver != 1) return fail(KC_ERR_ARG, "driver must be 0 (stand-alone) or 1 (pcg)");
    const bool want_pcg = driver == 1;
    if (h->last_driver.empty() || (h->last_driver.rfind("pcg", 0) == 0) != want_pcg)
        return fail(KC_ERR_STATE, want_pcg ? "run kc_pcg on this hierarchy first" : "run kc_solve on this hierarchy first");
    kc_status s;
    if ((s = prepare_call(h, c)) != KC_OK) return s;
    if ((s = enter(h)) != KC_OK) return s;
    const bool f32 = h->prec == KC_F32_CYCLE;
    if ((s = upload_inst(h)) != KC_OK) return s;
    if ((s = upload_state(h, 0.0, 1 << 30)) != KC_OK) return s;   // tol 0: every instance stays active
    {
        Launch L0 = want_pcg ? grid(h, GK_PCG_INIT, f32, tt_all0(), 0) : grid(h, GK_SSF, f32, tt_all0(), 0);
        L0.sa.fin = want_pcg ? FIN_PCG_INIT : FIN_SSF;
        HIPCHK(launch_grid(L0.gk, L0.f32, L0.sa, L0.nblocks, h->stream));
    }
    const int drv = want_pcg ? DRV_PCG : (f32 ? DRV_IR : DRV_SOLVE64);
    std::vector<Launch> ls;
    iteration(h, drv, *c, ls);
    // each launch of the iteration repeated `reps` times back to back between
    // two events (then its finalize step likewise), in iteration order
    std::vector<hipEvent_t> ev(3 * ls.size(), nullptr);
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    std::vector<double> t_main(ls.size(), 0.0), t_fin(ls.size(), 0.0);
    hipError_t err = run(h, ls);   // warm-up iteration
    for (size_t k = 0; k < ls.size() && err == hipSuccess; ++k) {
        const Launch& L = ls[k];
        err = hipEventRecord(ev[3 * k], h->stream);
        for (int r = 0; r < reps && err == hipSuccess; ++r) {
            if (L.type == L_GRID) err = launch_grid(L.gk, L.f32, L.sa, L.nblocks, h->stream, false);
            else if (L.type == L_SUB) err = launch_subtree(L.f32, L.ba, L.threads, L.lds, h->stream);
            else err = launch_coarsest(L.f32, L.ba, h->stream);
        }
        if (err == hipSuccess) err = hipEventRecord(ev[3 * k + 1], h->stream);
        for (int r = 0; r < reps && err == hipSuccess; ++r)
            if (L.type == L_GRID && L.nblocks > 0) err = launch_finalize(L.sa, h->stream);
        if (err == hipSuccess) err = hipEventRecord(ev[3 * k + 2], h->stream);
    }
    if (err == hipSuccess) err = hipStreamSynchronize(h->stream);
    for (size_t k = 0; k < ls.size() && err == hipSuccess; ++k) {
        float a = 0.f, b = 0.f;
        err = hipEventElapsedTime(&a, ev[3 * k], ev[3 * k + 1]);
        if (err == hipSuccess) err = hipEventElapsedTime(&b, ev[3 * k + 1], ev[3 * k + 2]);
        t_main[k] = a;   // ms of `reps` repetitions
        t_fin[k] = b;
    }
    struct Agg { int launches = 0; double ms = 0.0, bytes = 0.0, flops = 0.0; };
    std::map<std::string, Agg> agg;
    std::vector<std::string> order;
    std::string seq;
    double total = 0.0;
    for (size_t k = 0; k < ls.size(); ++k) {
        const Launch& L = ls[k];
        const bool empty = (L.type == L_GRID) ? L.nblocks <= 0 : L.ba.count <= 0;
        if (empty) continue;
        const std::string nm = launch_name(h, L);
        double b, f;
        launch_work(h, L, b, f);
        if (!agg.count(nm)) order.push_back(nm);
        Agg& A = agg[nm];
        A.launches += 1;
        A.ms += t_main[k] / reps;
        A.bytes += b;
        A.flops += f;
        total += t_main[k] / reps;
        char buf[192];
        std::snprintf(buf, sizeof buf, "%s[\"%s\", %d, %.5f, %.1f]", seq.empty() ? "" : ", ", nm.c_str(),
                      L.type == L_GRID ? L.sa.depth : L.ba.depth, t_main[k] / reps, b);
        seq += buf;
        if (L.type == L_GRID && L.sa.fin != FIN_NONE) {
            if (!agg.count("k_finalize")) order.push_back("k_finalize");
            Agg& F = agg["k_finalize"];
            F.launches += 1;
            F.ms += t_fin[k] / reps;
            total += t_fin[k] / reps;
        }
    }
    std::string js = "{\"driver\": \"" + std::string(want_pcg ? "pcg" : (f32 ? "solve_ir_f32" : "solve_f64")) + "\"";
    char buf[256];
    std::snprintf(buf, sizeof buf, ", \"reps\": %d, \"iteration_ms\": %.6f, \"kernels\": [", reps, total);
    js += buf;
    bool first = true;
    for (const std::string& nm : order) {
        const Agg& A = agg[nm];
        std::snprintf(buf, sizeof buf,
                      "%s{\"name\": \"%s\", \"launches\": %d, \"ms\": %.6f, \"avg_ms\": %.6f, \"bytes_per_launch\": %.1f, "
                      "\"flops_per_launch\": %.1f}",
                      first ? "" : ", ", nm.c_str(), A.launches, A.ms, A.ms / A.launches, A.bytes / A.launches,
                      A.flops / A.launches);
        js += buf;
        first = false;
    }
    js += "], \"sequence\": [" + seq + "]}";
    if (js.size() + 1 > cap) return fail(KC_ERR_ARG, "profile buffer too small");
    std::memcpy(out, js.c_str(), js.size() + 1);
    return leave(h);
}

kc_status kc_stats(const kc_hier* h, char* out, size_t cap)
{
    if (!h || !out || cap == 0) return fail(KC_ERR_ARG, "null argument");
    std::string js = "{";
    js += "\"count\": " + std::to_string(h->count);
    js += ", \"precision\": \"" + std::string(h->prec == KC_F64 ? "f64" : "f32_cycle") + "\"";
    js += ", \"mode\": \"" + std::string(h->ex.mode == 1 ? "paper" : "fused") + "\"";
    js += ", \"graph\": " + std::to_string(h->ex.use_graph);
    js += ", \"coarse_cutover\": " + std::to_string(h->ex.coarse_cutover);
    js += ", \"coarse_threads\": " + std::to_string(h->ex.coarse_threads);
    js += ", \"coarse_wave_n\": " + std::to_string(h->ex.coarse_wave_n);
    js += ", \"small_tile_n\": " + std::to_string(h->ex.small_tile_n);
    js += ", \"stream_n\": " + std::to_string(h->ex.stream_n);
    js += ", \"mid_tile_n\": " + std::to_string(h->ex.mid_tile_n);
    js += ", \"tiny_tile_n\": " + std::to_string(h->ex.tiny_tile_n);
    js += ", \"zebra_wave_n\": " + std::to_string(h->ex.zebra_wave_n);
    js += ", \"zebra_quad_n\": " + std::to_string(h->ex.zebra_quad_n);
    js += ", \"wave_regs\": " + std::to_string(h->ex.wave_regs);
    js += ", \"fuse_junctions\": " + std::to_string(h->ex.fuse_junctions);
    js += ", \"subtree_lds_bytes\": " + std::to_string(h->sub_lds);
    js += ", \"workspace_bytes\": " + std::to_string(h->lay.total);
    js += ", \"driver\": \"" + h->last_driver + "\"";
    js += ", \"grid_launches_per_iteration\": " + std::to_string(h->last_grid);
    js += ", \"subtree_launches_per_iteration\": " + std::to_string(h->last_sub);
    js += ", \"subtree_stages_per_iteration\": " + std::to_string(h->last_sub_stages);
    js += ", \"iterations_launched\": " + std::to_string(h->last_launched);
    js += ", \"compactions\": " + std::to_string(h->last_compactions);
    js += ", \"max_iterations\": " + std::to_string(h->last_cycles);
    char buf[64];
    std::snprintf(buf, sizeof buf, "%.6f", h->last_ms);
    js += ", \"last_ms\": " + std::string(buf);
    js += ", \"levels\": [";
    for (int i = 0; i < h->count; ++i) {
        if (i) js += ", ";
        js += "{\"L\": " + std::to_string(h->hi[i].il.L) + ", \"cut\": " + std::to_string(h->hi[i].cut) +
              ", \"n\": " + std::to_string(h->hi[i].il.n[0]) + "}";
    }
    js += "]}";
    if (js.size() + 1 > cap) return fail(KC_ERR_ARG, "stats buffer too small");
    std::memcpy(out, js.c_str(), js.size() + 1);
    return KC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// gradient inner products without a hierarchy or workspace: the instance table,
// the per-instance state, the block table and the Dot2 block partials live in a
// static device array of fixed size (one copy per GPU, held until the process
// ends); nothing allocates device memory
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[KC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;                       // host staging below and the per-device addresses
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {}; // device address of `scratch` on each GPU

struct NoallocStaging {
    InstDev inst[KC_NOALLOC_MAX_INSTANCES];
    InstState st[KC_NOALLOC_MAX_INSTANCES];
    int32_t tile_off[KC_NOALLOC_MAX_INSTANCES + 1];
};
NoallocStaging g_noalloc_host;                 // host-side tables of the call in progress (guarded by the mutex)

// the scratch array's address on the current device, looked up once per device
kc_status scratch_address(void** out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(KC_ERR_ARG, "device index out of range");
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(KC_ERR_HIP, "hipGetSymbolAddress returned a null scratch address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return KC_OK;
}

}  // namespace

extern "C" kc_status kc_grad_params_noalloc(const kc_problem* probs, int32_t count, const double* const* d_lam,
                                            const int64_t* ldl, const double* const* d_u, const int64_t* ldu,
                                            void* hip_stream, double* dtheta, double* deps)
{
    if (!probs || !d_lam || !ldl || !d_u || !ldu || !dtheta || !deps) return fail(KC_ERR_ARG, "null argument");
    if (count < 1 || count > KC_NOALLOC_MAX_INSTANCES)
        return fail(KC_ERR_ARG, "count must be in 1.." + std::to_string(KC_NOALLOC_MAX_INSTANCES));
    // scratch layout: instance table | states | block table | partials (4 doubles per 64 x 32 tile)
    const size_t off_st = align_up(sizeof(InstDev) * (size_t)count);
    const size_t off_tiles = off_st + align_up(sizeof(InstState) * (size_t)count);
    const size_t off_part = off_tiles + align_up(sizeof(int32_t) * (size_t)(count + 1));
    int64_t tiles = 0;
    for (int i = 0; i < count; ++i) {
        int L;
        kc_status st = check_problem(probs[i], L);
        if (st != KC_OK) return st;
        tiles += tiles_of(probs[i].n);
    }
    if (off_part + (size_t)tiles * 4 * sizeof(double) > (size_t)KC_NOALLOC_SCRATCH_BYTES)
        return fail(KC_ERR_ARG, "inputs need " + std::to_string(off_part + (size_t)tiles * 32) +
                                    " B of scratch; the static array holds " + std::to_string(KC_NOALLOC_SCRATCH_BYTES));
    for (int i = 0; i < count; ++i) {
        const int64_t n = probs[i].n;
        if (!d_lam[i] || !d_u[i]) return fail(KC_ERR_ARG, "null device pointer in lam or u");
        if (ldl[i] < n || ldl[i] > INT32_MAX || ldu[i] < n || ldu[i] > INT32_MAX)
            return fail(KC_ERR_ARG, "bad leading dimension of lam or u");
    }
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    void* base = nullptr;
    kc_status s = scratch_address(&base);
    if (s != KC_OK) return s;
    unsigned char* sc = (unsigned char*)base;
    NoallocStaging& hs = g_noalloc_host;
    hs.tile_off[0] = 0;
    for (int i = 0; i < count; ++i) {
        const kc_problem& p = probs[i];
        InstDev& I = hs.inst[i];
        std::memset(&I, 0, sizeof I);
        I.L = 1;
        I.n0 = p.n;
        double s9[9];
        fine_stencil(p.theta, p.eps, s9);
        for (int q = 0; q < 9; ++q) I.s64[0][q] = s9[q];
        const double hh = 1.0 / (double)(p.n + 1);
        I.h2 = hh * hh;
        I.h2inv = (double)(p.n + 1) * (double)(p.n + 1);
        fine_stencil_derivs(p.theta, p.eps, I.ds_th, I.ds_ep);
        I.x = d_lam[i];
        I.ldx = (int32_t)ldl[i];
        I.y = (double*)d_u[i];
        I.ldy = (int32_t)ldu[i];
        std::memset(&hs.st[i], 0, sizeof(InstState));
        hs.tile_off[i + 1] = hs.tile_off[i] + tiles_of(p.n);
    }
    hipStream_t stream = (hipStream_t)hip_stream;
    HIPCHK(hipMemcpyAsync(sc, hs.inst, sizeof(InstDev) * count, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(sc + off_st, hs.st, sizeof(InstState) * count, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(sc + off_tiles, hs.tile_off, sizeof(int32_t) * (count + 1), hipMemcpyHostToDevice, stream));
    StageArgs a{};
    a.inst = (const InstDev*)sc;
    a.st = (InstState*)(sc + off_st);
    a.tile_off = (const int32_t*)(sc + off_tiles);
    a.partial = (double*)(sc + off_part);
    a.hist = nullptr;
    a.count = count;
    a.fin = FIN_GRAD;
    HIPCHK(launch_grid(GK_GRAD, false, a, (int32_t)tiles, stream));
    HIPCHK(hipMemcpyAsync(hs.st, sc + off_st, sizeof(InstState) * count, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    for (int i = 0; i < count; ++i) {
        dtheta[i] = hs.st[i].dth;
        deps[i] = hs.st[i].deps;
    }
    return KC_OK;
}
