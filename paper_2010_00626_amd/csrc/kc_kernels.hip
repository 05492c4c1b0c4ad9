// kc_kernels.hip -- HIP kernels (gfx950, wave64) of the kappa-cycle multigrid
// solver for the rotated anisotropic diffusion problem.
//
// Every quantity on the GPU is in h^2-scaled units: level d solves S_d v = F_d
// with S_d the 3x3 stencil of h_d^2 A_d and F_d = h_d^2 f_d.  For a power-of-two
// h this is an exact rescaling of A_d v = f_d (Section 4 stencil, Galerkin
// coarse operators), so every rounded result equals the unscaled one times a
// power of two.
//
// Arithmetic order (shared by every kernel, one rounding per + and *, no
// contraction): a stencil sum visits the south row, then the centre row, then
// the north row, west to east in each; full weighting visits the 3x3
// neighbourhood in the same order with weights w(a) w(b), w(0)=1, w(+-1)=1/2;
// bilinear prolongation gathers the one, two or four coarse neighbours south
// to north, west to east, and scales the sum by 1/2 or 1/4.
//
// Grid-wide kernels work on 64 x 32 tiles of one level of every instance in a
// batch (blockIdx -> instance by a prefix table).  Reductions are
// deterministic: one partial per block, summed in a fixed order by the last
// block of the instance to arrive, which also applies the solver's decision
// (stop test, CG scalars) to the instance's state.
#include <math.h>

#include "../../include/kcycle.h"
#include "kc_internal.h"

namespace kc {

// ---------------------------------------------------------------------------
// precision traits
// ---------------------------------------------------------------------------
template <typename T> struct P;
template <> struct P<double> {
    static __device__ const double* s(const InstDev& I, int d) { return I.s64[d]; }
    static __device__ double w(const InstDev& I, int d) { return I.w64[d]; }
    static __device__ const double* chol(const InstDev& I) { return I.chol64; }
};
template <> struct P<float> {
    static __device__ const float* s(const InstDev& I, int d) { return I.s32[d]; }
    static __device__ float w(const InstDev& I, int d) { return I.w32[d]; }
    static __device__ const float* chol(const InstDev& I) { return I.chol32; }
};

template <typename T> struct Sten {
    T c[9];
    __device__ void load(const T* s)
    {
#pragma unroll
        for (int k = 0; k < 9; ++k) c[k] = s[k];
    }
    // sum over the 3x3 neighbourhood of x at (row pointer p, stride st), fixed order
    __device__ T apply(const T* x, int st) const
    {
        T acc = T(0);
        acc += c[0] * x[-st - 1];
        acc += c[1] * x[-st];
        acc += c[2] * x[-st + 1];
        acc += c[3] * x[-1];
        acc += c[4] * x[0];
        acc += c[5] * x[1];
        acc += c[6] * x[st - 1];
        acc += c[7] * x[st];
        acc += c[8] * x[st + 1];
        return acc;
    }
};

__device__ inline bool inside(int j, int i, int n) { return (unsigned)j < (unsigned)n && (unsigned)i < (unsigned)n; }

template <typename T>
__device__ inline T gload(const T* p, int ld, int n, int j, int i)
{
    return inside(j, i, n) ? p[(size_t)j * ld + i] : T(0);
}

// stencil sum reading global memory with zero outside the grid
template <typename T>
__device__ inline T gapply(const Sten<T>& s, const T* x, int ld, int n, int j, int i)
{
    T acc = T(0);
    acc += s.c[0] * gload(x, ld, n, j - 1, i - 1);
    acc += s.c[1] * gload(x, ld, n, j - 1, i);
    acc += s.c[2] * gload(x, ld, n, j - 1, i + 1);
    acc += s.c[3] * gload(x, ld, n, j, i - 1);
    acc += s.c[4] * gload(x, ld, n, j, i);
    acc += s.c[5] * gload(x, ld, n, j, i + 1);
    acc += s.c[6] * gload(x, ld, n, j + 1, i - 1);
    acc += s.c[7] * gload(x, ld, n, j + 1, i);
    acc += s.c[8] * gload(x, ld, n, j + 1, i + 1);
    return acc;
}

// full weighting sum around the fine point at r (stride st)
template <typename T>
__device__ inline T fw_sum(const T* r, int st)
{
    const T q = T(0.25), h = T(0.5);
    T acc = T(0);
    acc += q * r[-st - 1];
    acc += h * r[-st];
    acc += q * r[-st + 1];
    acc += h * r[-1];
    acc += T(1) * r[0];
    acc += h * r[1];
    acc += q * r[st - 1];
    acc += h * r[st];
    acc += q * r[st + 1];
    return acc;
}

// bilinear prolongation at fine (j, i) from coarse values V(J, I)
template <typename T, typename Get>
__device__ inline T prolong_at(int j, int i, Get V)
{
    const int Js = (j - 1) >> 1, Is = (i - 1) >> 1;
    const bool jo = j & 1, io = i & 1;
    if (jo && io) return V(Js, Is);
    if (jo) return T(0.5) * (V(Js, Is) + V(Js, Is + 1));
    if (io) return T(0.5) * (V(Js, Is) + V(Js + 1, Is));
    return T(0.25) * (((V(Js, Is) + V(Js, Is + 1)) + V(Js + 1, Is)) + V(Js + 1, Is + 1));
}

// ---------------------------------------------------------------------------
// block -> (instance, tile) and deterministic reductions
// ---------------------------------------------------------------------------
struct Tile {
    int inst, blk, nblk, x0, y0;
};

__device__ inline int find_inst(const int32_t* off, int count, int b)
{
    int lo = 0, hi = count;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// returns false when the instance is finished (the whole block leaves together)
__device__ inline bool get_tile(const StageArgs& a, int depth_for_size, bool fine_user, Tile& t)
{
    const int b = blockIdx.x;
    const int i = find_inst(a.tile_off, a.count, b);
    t.inst = i;
    t.blk = b - a.tile_off[i];
    t.nblk = a.tile_off[i + 1] - a.tile_off[i];
    const InstDev& I = a.inst[i];
    const int n = fine_user ? I.n0 : I.lev[depth_for_size].n;
    const int tx = (n + TX - 1) / TX;
    t.x0 = (t.blk % tx) * TX;
    t.y0 = (t.blk / tx) * TY;
    return a.st[i].done == 0;
}

template <int NT>
__device__ inline double block_sum(double v, double* red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NT / 64; ++k) s += red[k];
    }
    return s;   // valid in thread 0
}

__device__ inline double ir_scale(double ss, double npts)
{
    double t = ss / npts;
    if (!(t > 0.0) || !isfinite(t)) return 1.0;
    int e2;
    (void)frexp(t, &e2);      // t = m 2^e2, m in [0.5, 1)
    const int e = e2 - 1;     // t = m' 2^e, m' in [1, 2)
    const int k = (e >= 0) ? (e / 2) : -((-e + 1) / 2);
    return ldexp(1.0, -k);
}

// stand-alone stop test (shared by grid finalisation and the persistent kernel)
__device__ inline void stop_test(InstState& s, double* hist, int inst, double ss)
{
    const double rel = (s.ssf > 0.0) ? sqrt(ss) / sqrt(s.ssf) : 0.0;
    const int k = s.iters;
    if (k < HIST_CAP) hist[(size_t)inst * HIST_CAP + k] = rel;
    s.relres = rel;
    if (k == 0) s.relres0 = rel;
    if (!isfinite(rel)) { s.status = KC_ERR_NONFINITE; s.done = 1; }
    else if (rel < s.tol) { s.status = KC_OK; s.done = 1; }
    else if (rel > 1e3 * s.relres0) { s.status = KC_DIVERGED; s.done = 1; }
    else if (k >= s.maxit) { s.status = KC_NOT_CONVERGED; s.done = 1; }
    else s.iters = k + 1;
}

__device__ void apply_fin(const StageArgs& a, int inst, double S0, double S1)
{
    InstState& s = a.st[inst];
    const InstDev& I = a.inst[inst];
    const double npts = (double)I.n0 * (double)I.n0;
    switch (a.fin) {
    case FIN_SSF:
        s.ssf = S0;
        s.iters = 0;
        s.relres0 = 0.0;
        s.scale = ir_scale(S0, npts);
        s.scale_used = s.scale;
        if (!isfinite(S0)) { s.status = KC_ERR_NONFINITE; s.done = 1; }
        break;
    case FIN_STOP:
        stop_test(s, a.hist, inst, S0);
        break;
    case FIN_STOP_IR:
        s.scale_used = s.scale;
        s.scale = ir_scale(S0, npts);
        stop_test(s, a.hist, inst, S0);
        break;
    case FIN_PCG_INIT: {
        s.ssf = S0;
        s.iters = 0;
        s.scale = ir_scale(S0, npts);
        const double rel = (S0 > 0.0) ? 1.0 : 0.0;
        s.relres = rel;
        s.relres0 = rel;
        a.hist[(size_t)inst * HIST_CAP] = rel;
        if (!isfinite(S0)) { s.status = KC_ERR_NONFINITE; s.done = 1; }
        else if (rel < s.tol) { s.status = KC_OK; s.done = 1; }
        else if (s.maxit <= 0) { s.status = KC_NOT_CONVERGED; s.done = 1; }
        break;
    }
    case FIN_RZ:
        s.beta = (s.iters == 0) ? 0.0 : S0 / s.rz;
        s.rz = S0;
        break;
    case FIN_PQ:
        s.pq = S0;
        if (!(S0 > 0.0) || !isfinite(S0)) {
            s.status = isfinite(S0) ? KC_BREAKDOWN : KC_ERR_NONFINITE;
            s.done = 1;
        } else {
            s.alpha = s.rz / S0;
        }
        break;
    case FIN_PCG_R: {
        const double rel = sqrt(S0) / sqrt(s.ssf);
        s.iters += 1;
        s.relres = rel;
        if (s.iters < HIST_CAP) a.hist[(size_t)inst * HIST_CAP + s.iters] = rel;
        s.scale = ir_scale(S0, npts);
        if (!isfinite(rel)) { s.status = KC_ERR_NONFINITE; s.done = 1; }
        else if (rel < s.tol) { s.status = KC_OK; s.done = 1; }
        else if (s.iters >= s.maxit) { s.status = KC_NOT_CONVERGED; s.done = 1; }
        break;
    }
    case FIN_GRAD:
        s.dth = -S0;
        s.deps = -S1;
        break;
    default:
        break;
    }
}

// every block of a reducing launch calls this once with its thread values
__device__ void reduce_finalize(const StageArgs& a, const Tile& t, double v0, double v1)
{
    __shared__ double red[2][GRID_THREADS / 64];
    __shared__ int am_last;
    const double s0 = block_sum<GRID_THREADS>(v0, red[0]);
    const double s1 = block_sum<GRID_THREADS>(v1, red[1]);
    const int gb = a.tile_off[t.inst] + t.blk;
    if (threadIdx.x == 0) {
        a.partial[2 * gb] = s0;
        a.partial[2 * gb + 1] = s1;
        __threadfence();
        const int prev = atomicAdd(&a.st[t.inst].counter, 1);
        am_last = (prev == t.nblk - 1);
    }
    __syncthreads();
    if (!am_last) return;
    __threadfence();
    const int b0 = a.tile_off[t.inst];
    double t0 = 0.0, t1 = 0.0;
    for (int k = threadIdx.x; k < t.nblk; k += GRID_THREADS) {
        t0 += __builtin_nontemporal_load(&a.partial[2 * (b0 + k)]);
        t1 += __builtin_nontemporal_load(&a.partial[2 * (b0 + k) + 1]);
    }
    const double S0 = block_sum<GRID_THREADS>(t0, red[0]);
    const double S1 = block_sum<GRID_THREADS>(t1, red[1]);
    if (threadIdx.x == 0) {
        a.st[t.inst].counter = 0;
        apply_fin(a, t.inst, S0, S1);
    }
}

template <typename T> __device__ inline T* buf(const LevelDev& L, int sel) { return (T*)(sel ? L.B : L.A); }

// ---------------------------------------------------------------------------
// unfused kernels: one kernel per operation of Algorithm 4
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(GRID_THREADS) k_unfused(StageArgs a, int kind)
{
    Tile t;
    if (!get_tile(a, a.depth, false, t)) return;
    const InstDev& I = a.inst[t.inst];
    const int d = a.depth;
    const LevelDev& Lv = I.lev[d];
    const int n = Lv.n;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    Sten<T> s;
    s.load(P<T>::s(I, d));
    const T w = P<T>::w(I, d);
    const T fs = (T)Lv.fscale;
    const T* F = (const T*)Lv.F;
    double nrm = 0.0;
    const int lds_ = a.src ? Lv.ldb : Lv.lda;   // leading dimension of the source buffer
    const int ldd_ = a.dst ? Lv.ldb : Lv.lda;   // leading dimension of the destination buffer

    if (kind == GK_RESTRICT || kind == GK_ZERO) {
        // coarse points whose fine position lies in this tile
        const LevelDev& Lc = I.lev[d + 1];
        const int nc = Lc.n;
        const T* r = buf<T>(Lv, a.src);
        const int ld = lds_;
        for (int k = threadIdx.x; k < (TX / 2) * (TY / 2); k += GRID_THREADS) {
            const int Ic = (t.x0 >> 1) + (k % (TX / 2)), Jc = (t.y0 >> 1) + (k / (TX / 2));
            if (Ic >= nc || Jc >= nc) continue;
            if (kind == GK_ZERO) {
                ((T*)Lc.A)[(size_t)Jc * Lc.lda + Ic] = T(0);
            } else {
                const int j = 2 * Jc + 1, i = 2 * Ic + 1;
                const T q = T(0.25), h = T(0.5);
                T acc = T(0);
                acc += q * gload(r, ld, n, j - 1, i - 1);
                acc += h * gload(r, ld, n, j - 1, i);
                acc += q * gload(r, ld, n, j - 1, i + 1);
                acc += h * gload(r, ld, n, j, i - 1);
                acc += T(1) * gload(r, ld, n, j, i);
                acc += h * gload(r, ld, n, j, i + 1);
                acc += q * gload(r, ld, n, j + 1, i - 1);
                acc += h * gload(r, ld, n, j + 1, i);
                acc += q * gload(r, ld, n, j + 1, i + 1);
                ((T*)Lc.F)[(size_t)Jc * Lc.ldf + Ic] = acc;
            }
        }
        return;
    }

    for (int k = ty; k < TY; k += GRID_THREADS / 64) {
        const int j = t.y0 + k, i = t.x0 + tx;
        const bool in = (j < n) && (i < n);
        const size_t gs = (size_t)j * lds_ + i, gd = (size_t)j * ldd_ + i, gf = (size_t)j * Lv.ldf + i;
        switch (kind) {
        case GK_SWEEP: {
            if (!in) break;
            const T* x = buf<T>(Lv, a.src);
            const T acc = gapply(s, x, lds_, n, j, i);
            buf<T>(Lv, a.dst)[gd] = x[gs] + w * (fs * F[gf] - acc);
            break;
        }
        case GK_RESID: {
            if (!in) break;
            const T* x = buf<T>(Lv, a.src);
            buf<T>(Lv, a.dst)[gd] = fs * F[gf] - gapply(s, x, lds_, n, j, i);
            break;
        }
        case GK_PROLONG: {
            if (!in) break;
            const LevelDev& Lc = I.lev[d + 1];
            const T* vc = buf<T>(Lc, a.src);
            const int nc = Lc.n, ldc = a.src ? Lc.ldb : Lc.lda;
            buf<T>(Lv, a.dst)[gd] = prolong_at<T>(j, i, [&](int J, int II) { return gload(vc, ldc, nc, J, II); });
            break;
        }
        case GK_ADD: {
            if (!in) break;
            T* v = buf<T>(Lv, a.src);
            v[gs] = v[gs] + buf<T>(Lv, a.dst)[gd];
            break;
        }
        case GK_COPY: {
            if (!in) break;
            buf<T>(Lv, a.dst)[gd] = buf<T>(Lv, a.src)[gs];
            break;
        }
        case GK_ZERO_SELF: {
            if (!in) break;
            ((T*)Lv.A)[(size_t)j * Lv.lda + i] = T(0);
            break;
        }
        case GK_NORM: {
            if (!in) break;
            const T* x = (const T*)Lv.A;
            const double r = (double)(fs * F[gf] - gapply(s, x, Lv.lda, n, j, i));
            nrm += r * r;
            break;
        }
        default:
            break;
        }
    }
    if (kind == GK_NORM) reduce_finalize(a, t, nrm, 0.0);
}

// ---------------------------------------------------------------------------
// fused pre-smoothing: nu sweeps + residual + full weighting in one pass
// (input region = tile + halo nu+1, swept in LDS); optional input norm
// ---------------------------------------------------------------------------
template <typename T, int NU>
__global__ void __launch_bounds__(GRID_THREADS) k_pre(StageArgs a)
{
    constexpr int H = NU + 1;
    constexpr int RW = TX + 2 * H + 1, RH = TY + 2 * H + 1;
    __shared__ T sv[2][RH * RW];
    __shared__ T sf[RH * RW];
    Tile t;
    if (!get_tile(a, a.depth, false, t)) return;
    const InstDev& I = a.inst[t.inst];
    const int d = a.depth;
    const LevelDev& Lv = I.lev[d];
    const int n = Lv.n;
    const T* A = (const T*)Lv.A;
    T* B = (T*)Lv.B;
    const T* F = (const T*)Lv.F;
    const T fs = (T)Lv.fscale;
    const int rx0 = t.x0 - H, ry0 = t.y0 - H;
    Sten<T> s;
    s.load(P<T>::s(I, d));
    const T w = P<T>::w(I, d);
    const bool zg = a.zg != 0;

    for (int p = threadIdx.x; p < RH * RW; p += GRID_THREADS) {
        const int rj = p / RW, ri = p - rj * RW;
        const int j = ry0 + rj, i = rx0 + ri;
        const bool in = inside(j, i, n);
        sf[p] = in ? fs * F[(size_t)j * Lv.ldf + i] : T(0);
        sv[0][p] = (in && !zg) ? A[(size_t)j * Lv.lda + i] : T(0);
    }
    __syncthreads();

    double nrm = 0.0;
    if (a.fin == FIN_STOP) {
        for (int p = threadIdx.x; p < TX * TY; p += GRID_THREADS) {
            const int rj = H + p / TX, ri = H + (p % TX);
            if (!inside(ry0 + rj, rx0 + ri, n)) continue;
            const int q = rj * RW + ri;
            const double r = (double)(sf[q] - s.apply(&sv[0][q], RW));
            nrm += r * r;
        }
    }

    int cur = 0;
#pragma unroll
    for (int k = 1; k <= NU; ++k) {
        const int ww = RW - 2 * k, hh = RH - 2 * k;
        for (int p = threadIdx.x; p < ww * hh; p += GRID_THREADS) {
            const int rj = k + p / ww, ri = k + (p % ww);
            const int q = rj * RW + ri;
            T val = T(0);
            if (inside(ry0 + rj, rx0 + ri, n)) {
                if (k == 1 && zg) val = w * sf[q];
                else val = sv[cur][q] + w * (sf[q] - s.apply(&sv[cur][q], RW));
            }
            sv[cur ^ 1][q] = val;
        }
        __syncthreads();
        cur ^= 1;
    }

    // smoothed estimate on the tile
    for (int p = threadIdx.x; p < TX * TY; p += GRID_THREADS) {
        const int y = p / TX, x = p % TX;
        const int j = t.y0 + y, i = t.x0 + x;
        if (j < n && i < n) B[(size_t)j * Lv.ldb + i] = sv[cur][(H + y) * RW + (H + x)];
    }
    // residual on [x0, x0+TX] x [y0, y0+TY]
    for (int p = threadIdx.x; p < (TX + 1) * (TY + 1); p += GRID_THREADS) {
        const int y = p / (TX + 1), x = p % (TX + 1);
        const int q = (H + y) * RW + (H + x);
        const int j = t.y0 + y, i = t.x0 + x;
        sv[cur ^ 1][q] = inside(j, i, n) ? sf[q] - s.apply(&sv[cur][q], RW) : T(0);
    }
    __syncthreads();
    {
        const LevelDev& Lc = I.lev[d + 1];
        const int nc = Lc.n, ldc = Lc.ldf;
        T* Fc = (T*)Lc.F;
        const T* r = sv[cur ^ 1];
        for (int p = threadIdx.x; p < (TX / 2) * (TY / 2); p += GRID_THREADS) {
            const int Ic = (t.x0 >> 1) + (p % (TX / 2)), Jc = (t.y0 >> 1) + (p / (TX / 2));
            if (Ic >= nc || Jc >= nc) continue;
            const int q = (2 * Jc + 1 - ry0) * RW + (2 * Ic + 1 - rx0);
            Fc[(size_t)Jc * ldc + Ic] = fw_sum(&r[q], RW);
        }
    }
    if (a.fin == FIN_STOP) reduce_finalize(a, t, nrm, 0.0);
}

// ---------------------------------------------------------------------------
// fused post-smoothing: prolong-add + nu sweeps (input region = tile + halo nu)
// ---------------------------------------------------------------------------
template <typename T, int NU>
__global__ void __launch_bounds__(GRID_THREADS) k_post(StageArgs a)
{
    constexpr int H = NU;
    constexpr int RW = TX + 2 * H, RH = TY + 2 * H;
    constexpr int CW = TX / 2 + H + 3, CH = TY / 2 + H + 3;
    __shared__ T sv[2][RH * RW];
    __shared__ T sf[RH * RW];
    __shared__ T sc[CH * CW];
    Tile t;
    if (!get_tile(a, a.depth, false, t)) return;
    const InstDev& I = a.inst[t.inst];
    const int d = a.depth;
    const LevelDev& Lv = I.lev[d];
    const LevelDev& Lc = I.lev[d + 1];
    const int n = Lv.n, nc = Lc.n, ldc = Lc.lda;
    T* A = (T*)Lv.A;
    const T* B = (const T*)Lv.B;
    const T* F = (const T*)Lv.F;
    const T* Vc = (const T*)Lc.A;
    const T fs = (T)Lv.fscale;
    const int rx0 = t.x0 - H, ry0 = t.y0 - H;
    const int cx0 = (rx0 - 1) >> 1, cy0 = (ry0 - 1) >> 1;
    Sten<T> s;
    s.load(P<T>::s(I, d));
    const T w = P<T>::w(I, d);

    for (int p = threadIdx.x; p < RH * RW; p += GRID_THREADS) {
        const int rj = p / RW, ri = p - rj * RW;
        const int j = ry0 + rj, i = rx0 + ri;
        const bool in = inside(j, i, n);
        sf[p] = in ? fs * F[(size_t)j * Lv.ldf + i] : T(0);
        sv[0][p] = in ? B[(size_t)j * Lv.ldb + i] : T(0);
    }
    for (int p = threadIdx.x; p < CH * CW; p += GRID_THREADS) {
        const int cj = p / CW, ci = p - cj * CW;
        sc[p] = gload(Vc, ldc, nc, cy0 + cj, cx0 + ci);
    }
    __syncthreads();
    for (int p = threadIdx.x; p < RH * RW; p += GRID_THREADS) {
        const int rj = p / RW, ri = p - rj * RW;
        const int j = ry0 + rj, i = rx0 + ri;
        if (!inside(j, i, n)) continue;
        const T e = prolong_at<T>(j, i, [&](int J, int II) { return sc[(J - cy0) * CW + (II - cx0)]; });
        sv[0][p] = sv[0][p] + e;
    }
    __syncthreads();
    int cur = 0;
#pragma unroll
    for (int k = 1; k <= NU; ++k) {
        const int ww = RW - 2 * k, hh = RH - 2 * k;
        for (int p = threadIdx.x; p < ww * hh; p += GRID_THREADS) {
            const int rj = k + p / ww, ri = k + (p % ww);
            const int q = rj * RW + ri;
            T val = T(0);
            if (inside(ry0 + rj, rx0 + ri, n)) val = sv[cur][q] + w * (sf[q] - s.apply(&sv[cur][q], RW));
            sv[cur ^ 1][q] = val;
        }
        __syncthreads();
        cur ^= 1;
    }
    for (int p = threadIdx.x; p < TX * TY; p += GRID_THREADS) {
        const int y = p / TX, x = p % TX;
        const int j = t.y0 + y, i = t.x0 + x;
        if (j < n && i < n) A[(size_t)j * Lv.lda + i] = sv[cur][(H + y) * RW + (H + x)];
    }
}

// exact coarsest solve with the lower Cholesky factor Lc (m x m, row-major):
// L y = F, then L^T v = y, both by substitution in index order (one thread);
// F and v are read and written through strides sf / sv
template <typename T>
__device__ inline void chol_solve(int m, const T* Lc, const T* F, int sf, T* v, int sv)
{
    for (int p = 0; p < m; ++p) {
        T acc = F[p * sf];
        for (int q = 0; q < p; ++q) acc -= Lc[p * m + q] * v[q * sv];
        v[p * sv] = acc / Lc[p * m + p];
    }
    for (int p = m - 1; p >= 0; --p) {
        T acc = v[p * sv];
        for (int q = p + 1; q < m; ++q) acc -= Lc[q * m + p] * v[q * sv];
        v[p * sv] = acc / Lc[p * m + p];
    }
}

// ---------------------------------------------------------------------------
// persistent coarse kernel: one workgroup runs whole calls of the cycle on the
// coarse levels of one instance, all levels resident in LDS.  Rows are spread
// over waves (row j on wave j mod waves, column i on lane i), n <= 63.
// ---------------------------------------------------------------------------
template <typename T>
struct Sub {
    T* sm;
    const InstDev* I;
    int nu1, nu2;

    __device__ T* v(int d) const { return sm + I->lds_off[d]; }
    __device__ T* f(int d) const { return sm + I->lds_off[d] + I->lev[d].n * I->lev[d].n; }
    __device__ T* tmp() const { return sm + I->lds_tmp; }

    template <typename Fn>
    __device__ void each(int n, Fn fn) const
    {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
        if (lane < n)
            for (int j = wv; j < n; j += nw) fn(j, lane);
    }

    __device__ T at(const T* x, int n, int j, int i) const { return inside(j, i, n) ? x[j * n + i] : T(0); }

    __device__ T lapply(const Sten<T>& s, const T* x, int n, int j, int i) const
    {
        T acc = T(0);
        acc += s.c[0] * at(x, n, j - 1, i - 1);
        acc += s.c[1] * at(x, n, j - 1, i);
        acc += s.c[2] * at(x, n, j - 1, i + 1);
        acc += s.c[3] * at(x, n, j, i - 1);
        acc += s.c[4] * at(x, n, j, i);
        acc += s.c[5] * at(x, n, j, i + 1);
        acc += s.c[6] * at(x, n, j + 1, i - 1);
        acc += s.c[7] * at(x, n, j + 1, i);
        acc += s.c[8] * at(x, n, j + 1, i + 1);
        return acc;
    }

    // nu sweeps on level d; v(d) holds the result
    __device__ void sweeps(int d, int nu, bool zg) const
    {
        const int n = I->lev[d].n;
        Sten<T> s;
        s.load(P<T>::s(*I, d));
        const T w = P<T>::w(*I, d);
        T* cur = v(d);
        T* oth = tmp();
        const T* F = f(d);
        for (int k = 0; k < nu; ++k) {
            const bool z = zg && k == 0;
            each(n, [&](int j, int i) {
                const int q = j * n + i;
                oth[q] = z ? w * F[q] : cur[q] + w * (F[q] - lapply(s, cur, n, j, i));
            });
            __syncthreads();
            T* tt = cur; cur = oth; oth = tt;
        }
        if (cur != v(d)) {
            T* vd = v(d);
            each(n, [&](int j, int i) { vd[j * n + i] = cur[j * n + i]; });
            __syncthreads();
        }
        if (zg && nu == 0) {
            T* vd = v(d);
            each(n, [&](int j, int i) { vd[j * n + i] = T(0); });
            __syncthreads();
        }
    }

    __device__ void pre(int d, bool zg) const
    {
        sweeps(d, nu1, zg);
        const int n = I->lev[d].n, nc = I->lev[d + 1].n;
        Sten<T> s;
        s.load(P<T>::s(*I, d));
        const T* vd = v(d);
        const T* F = f(d);
        T* r = tmp();
        each(n, [&](int j, int i) { r[j * n + i] = F[j * n + i] - lapply(s, vd, n, j, i); });
        __syncthreads();
        T* Fc = f(d + 1);
        each(nc, [&](int J, int II) {
            const int j = 2 * J + 1, i = 2 * II + 1;
            const T q = T(0.25), h = T(0.5);
            T acc = T(0);
            acc += q * at(r, n, j - 1, i - 1);
            acc += h * at(r, n, j - 1, i);
            acc += q * at(r, n, j - 1, i + 1);
            acc += h * at(r, n, j, i - 1);
            acc += T(1) * at(r, n, j, i);
            acc += h * at(r, n, j, i + 1);
            acc += q * at(r, n, j + 1, i - 1);
            acc += h * at(r, n, j + 1, i);
            acc += q * at(r, n, j + 1, i + 1);
            Fc[J * nc + II] = acc;
        });
        __syncthreads();
    }

    __device__ void post(int d) const
    {
        const int n = I->lev[d].n, nc = I->lev[d + 1].n;
        T* vd = v(d);
        const T* vc = v(d + 1);
        each(n, [&](int j, int i) {
            const T e = prolong_at<T>(j, i, [&](int J, int II) { return at(vc, nc, J, II); });
            vd[j * n + i] = vd[j * n + i] + e;
        });
        __syncthreads();
        sweeps(d, nu2, false);
    }

    __device__ void solve(int d) const
    {
        if (threadIdx.x == 0) chol_solve<T>(I->nc2, P<T>::chol(*I), f(d), 1, v(d), 1);
        __syncthreads();
    }

    __device__ void call(int k) const
    {
        const int kk = min(k, MAXL + 1);
        const uint32_t* ops = I->ops + I->ops_beg[kk - 1];
        const int nops = I->ops_len[kk - 1];
        for (int o = 0; o < nops; ++o) {
            const uint32_t op = ops[o];
            const int kind = op & 15, d = (op >> 4) & 255;
            const bool zg = (op >> 12) & 1;
            if (kind == SOP_PRE) pre(d, zg);
            else if (kind == SOP_POST) post(d);
            else solve(d);
        }
    }
};

template <typename T>
__global__ void __launch_bounds__(1024) k_subtree(SubArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int inst = a.list[blockIdx.x];
    if (a.st[inst].done) return;
    const InstDev& I = a.inst[inst];
    Sub<T> S{reinterpret_cast<T*>(smem_raw), &I, a.nu1, a.nu2};
    const int d0 = a.depth;
    const LevelDev& Lv = I.lev[d0];
    const int n = Lv.n;
    const T fs = (T)Lv.fscale;
    const T* Fg = (const T*)Lv.F;
    T* Ag = (T*)Lv.A;
    T* v0 = S.v(d0);
    T* f0 = S.f(d0);
    const bool zero = a.pair || a.zg;
    S.each(n, [&](int j, int i) {
        f0[j * n + i] = fs * Fg[(size_t)j * Lv.ldf + i];
        v0[j * n + i] = zero ? T(0) : Ag[(size_t)j * Lv.lda + i];
    });
    __syncthreads();

    if (a.fin == FIN_STOP) {
        __shared__ double red[16];
        __shared__ int stop;
        Sten<T> s;
        s.load(P<T>::s(I, d0));
        double nrm = 0.0;
        S.each(n, [&](int j, int i) {
            const double r = (double)(f0[j * n + i] - S.lapply(s, v0, n, j, i));
            nrm += r * r;
        });
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
        __syncthreads();
        if (threadIdx.x == 0) {
            double ss = 0.0;
            for (int k = 0; k < (int)(blockDim.x >> 6); ++k) ss += red[k];
            stop_test(a.st[inst], a.hist, inst, ss);
            stop = a.st[inst].done;
        }
        __syncthreads();
        if (stop) return;
    }

    S.call(a.kappa);
    if (a.pair && a.kappa > 1) S.call(a.kappa - 1);

    S.each(n, [&](int j, int i) { Ag[(size_t)j * Lv.lda + i] = v0[j * n + i]; });
}

// coarsest direct solve on global memory (paper-structured mode); the coarsest
// grid is at most 7 x 7, staged through LDS
template <typename T>
__global__ void __launch_bounds__(64) k_coarsest(SubArgs a)
{
    __shared__ T fb[64], vb[64];
    const int inst = a.list[blockIdx.x];
    if (a.st[inst].done) return;
    const InstDev& I = a.inst[inst];
    const LevelDev& Lv = I.lev[a.depth];
    const int m = I.nc2, n = Lv.n;
    const T* F = (const T*)Lv.F;
    const T fs = (T)Lv.fscale;
    T* A = (T*)Lv.A;
    for (int p = threadIdx.x; p < m; p += 64) fb[p] = fs * F[(size_t)(p / n) * Lv.ldf + (p % n)];
    __syncthreads();
    if (threadIdx.x == 0) chol_solve<T>(m, P<T>::chol(I), fb, 1, vb, 1);
    __syncthreads();
    for (int p = threadIdx.x; p < m; p += 64) A[(size_t)(p / n) * Lv.lda + (p % n)] = vb[p];
}

// ---------------------------------------------------------------------------
// driver kernels on the fine level (FP64 vectors)
// ---------------------------------------------------------------------------
template <bool F32>
__global__ void __launch_bounds__(GRID_THREADS) k_driver(StageArgs a, int kind)
{
    Tile t;
    if (!get_tile(a, 0, true, t)) return;
    const InstDev& I = a.inst[t.inst];
    InstState& st = a.st[t.inst];
    const int n = I.n0;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    Sten<double> s;
    s.load(I.s64[0]);
    const double h2 = I.h2;
    double acc0 = 0.0, acc1 = 0.0;
    const LevelDev& L0 = I.lev[0];
    const double scale = st.scale, scale_used = st.scale_used;
    const double alpha = st.alpha, beta = st.beta;
    const bool first = st.iters == 0;
    for (int k = ty; k < TY; k += GRID_THREADS / 64) {
        const int j = t.y0 + k, i = t.x0 + tx;
        if (j >= n || i >= n) continue;
        const size_t gu = (size_t)j * I.ldu + i, gf = (size_t)j * I.ldf + i, gv = (size_t)j * I.ldv + i;
        const size_t g0 = (size_t)j * L0.lda + i;   // FP32 level-0 arrays share one leading dimension
        switch (kind) {
        case GK_SSF: {
            const double F = h2 * I.f[gf];
            acc0 += F * F;
            break;
        }
        case GK_IR_RESID: {
            const double r = h2 * I.f[gf] - gapply(s, (const double*)I.u, I.ldu, n, j, i);
            acc0 += r * r;
            if (F32) ((float*)L0.F)[g0] = (float)(scale * r);
            break;
        }
        case GK_IR_UPDATE: {
            const double e = F32 ? (double)((const float*)L0.A)[g0] : ((const double*)L0.A)[g0];
            I.u[gu] = I.u[gu] + e / scale_used;
            break;
        }
        case GK_PCG_INIT: {
            const double F = h2 * I.f[gf];
            I.u[gu] = 0.0;
            I.r[gv] = F;
            acc0 += F * F;
            break;
        }
        case GK_PCG_PRECIN: {
            ((float*)L0.F)[g0] = (float)(scale * I.r[gv]);
            break;
        }
        case GK_PCG_RZ: {
            double z;
            if (F32) {
                z = (double)((const float*)L0.A)[g0] / scale;
                I.z[gv] = z;
            } else {
                z = I.z[gv];
            }
            acc0 += I.r[gv] * z;
            break;
        }
        case GK_PCG_P: {
            I.p[gv] = first ? I.z[gv] : I.z[gv] + beta * I.p[gv];
            break;
        }
        case GK_PCG_AP: {
            const double q = gapply(s, (const double*)I.p, I.ldv, n, j, i);
            I.q[gv] = q;
            acc0 += I.p[gv] * q;
            break;
        }
        case GK_PCG_UPD: {
            I.u[gu] = I.u[gu] + alpha * I.p[gv];
            const double r = I.r[gv] - alpha * I.q[gv];
            I.r[gv] = r;
            acc0 += r * r;
            break;
        }
        case GK_APPLY: {
            I.y[(size_t)j * I.ldy + i] = gapply(s, I.x, I.ldx, n, j, i) * I.h2inv;
            break;
        }
        case GK_GRAD: {
            Sten<double> dt, de;
            dt.load(I.ds_th);
            de.load(I.ds_ep);
            const double lam = I.x[(size_t)j * I.ldx + i];
            const double yt = gapply(dt, (const double*)I.y, I.ldy, n, j, i) * I.h2inv;
            const double ye = gapply(de, (const double*)I.y, I.ldy, n, j, i) * I.h2inv;
            acc0 += lam * yt;
            acc1 += lam * ye;
            break;
        }
        default:
            break;
        }
    }
    if (a.fin != FIN_NONE) reduce_finalize(a, t, acc0, acc1);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
static hipError_t launch_pre(const StageArgs& a, int nb, hipStream_t s)
{
    switch (a.nu) {
    case 0: k_pre<T, 0><<<nb, GRID_THREADS, 0, s>>>(a); break;
    case 1: k_pre<T, 1><<<nb, GRID_THREADS, 0, s>>>(a); break;
    case 2: k_pre<T, 2><<<nb, GRID_THREADS, 0, s>>>(a); break;
    case 3: k_pre<T, 3><<<nb, GRID_THREADS, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_post(const StageArgs& a, int nb, hipStream_t s)
{
    switch (a.nu) {
    case 0: k_post<T, 0><<<nb, GRID_THREADS, 0, s>>>(a); break;
    case 1: k_post<T, 1><<<nb, GRID_THREADS, 0, s>>>(a); break;
    case 2: k_post<T, 2><<<nb, GRID_THREADS, 0, s>>>(a); break;
    case 3: k_post<T, 3><<<nb, GRID_THREADS, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_grid(GridKernel k, bool f32, const StageArgs& a, int32_t nb, hipStream_t s)
{
    if (nb <= 0) return hipSuccess;
    switch (k) {
    case GK_PRE: return f32 ? launch_pre<float>(a, nb, s) : launch_pre<double>(a, nb, s);
    case GK_POST: return f32 ? launch_post<float>(a, nb, s) : launch_post<double>(a, nb, s);
    case GK_SWEEP: case GK_RESID: case GK_RESTRICT: case GK_ZERO: case GK_PROLONG: case GK_ADD: case GK_COPY:
    case GK_NORM: case GK_ZERO_SELF:
        if (f32) k_unfused<float><<<nb, GRID_THREADS, 0, s>>>(a, (int)k);
        else k_unfused<double><<<nb, GRID_THREADS, 0, s>>>(a, (int)k);
        return hipGetLastError();
    default:
        if (f32) k_driver<true><<<nb, GRID_THREADS, 0, s>>>(a, (int)k);
        else k_driver<false><<<nb, GRID_THREADS, 0, s>>>(a, (int)k);
        return hipGetLastError();
    }
}

hipError_t launch_subtree(bool f32, const SubArgs& a, int32_t threads, int32_t lds_bytes, hipStream_t s)
{
    if (a.count <= 0) return hipSuccess;
    if (f32) k_subtree<float><<<a.count, threads, lds_bytes, s>>>(a);
    else k_subtree<double><<<a.count, threads, lds_bytes, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_coarsest(bool f32, const SubArgs& a, hipStream_t s)
{
    if (a.count <= 0) return hipSuccess;
    if (f32) k_coarsest<float><<<a.count, 64, 0, s>>>(a);
    else k_coarsest<double><<<a.count, 64, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t prepare_subtree(bool f32, int32_t lds_bytes)
{
    if (f32) return hipFuncSetAttribute((const void*)k_subtree<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    return hipFuncSetAttribute((const void*)k_subtree<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}

int32_t max_lds_bytes()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
    return v;
}

}  // namespace kc
