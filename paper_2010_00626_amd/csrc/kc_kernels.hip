// kc_kernels.hip -- HIP kernels (gfx950, wave64) of the kappa-cycle multigrid
// solver for the rotated anisotropic diffusion problem.
//
// Every quantity on the GPU is in h^2-scaled units: level d solves S_d v = F_d
// with S_d the 3x3 stencil of h_d^2 A_d and F_d = h_d^2 f_d.  For a power-of-two
// h this is an exact rescaling of A_d v = f_d (Section 4 stencil, Galerkin
// coarse operators), so every rounded result equals the unscaled one times a
// power of two.
//
// Arithmetic order (shared by every kernel; the compiler contracts nothing,
// and each product of a stencil sum, the Jacobi update and both steps of the
// line elimination is an explicit fused multiply-add, fmadd): a stencil sum
// visits the south row, then the centre row, then the north row, west to east
// in each, accumulating product by product; full weighting visits the 3x3
// neighbourhood in the same order with weights w(a) w(b), w(0)=1, w(+-1)=1/2;
// bilinear prolongation gathers the one, two or four coarse neighbours south
// to north, west to east, and scales the sum by 1/2 or 1/4.
//
// Grid-wide kernels work on tiles (8 x 8 to 64 x 32) or row strips of one
// level of every instance in a batch (blockIdx -> instance by a prefix table).
// Reductions are deterministic Dot2 sums: one (value, error) partial per block,
// merged in a fixed order by a finalize kernel (one workgroup per instance),
// which also applies the solver's decision (stop test, CG scalars) to the
// instance's state.  Calls
// below a cutover level run in a persistent kernel, one workgroup per instance
// with the levels in LDS.
#include <math.h>

#include <type_traits>

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

// a * b + c with one rounding: every product of a stencil sum, the Jacobi update
// and both steps of the line elimination (the oracle calls fma() at the same places)
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T> struct Sten {
    T c[9];
    __device__ void load(const T* s)
    {
#pragma unroll
        for (int k = 0; k < 9; ++k) c[k] = s[k];
    }
    // sum over the 3x3 neighbourhood of x at (row pointer p, stride st), fixed order
    __device__ __forceinline__ T apply(const T* x, int st) const
    {
        T acc = T(0);
        acc = fmadd(c[0], x[-st - 1], acc);
        acc = fmadd(c[1], x[-st], acc);
        acc = fmadd(c[2], x[-st + 1], acc);
        acc = fmadd(c[3], x[-1], acc);
        acc = fmadd(c[4], x[0], acc);
        acc = fmadd(c[5], x[1], acc);
        acc = fmadd(c[6], x[st - 1], acc);
        acc = fmadd(c[7], x[st], acc);
        acc = fmadd(c[8], x[st + 1], acc);
        return acc;
    }
};

__device__ inline bool inside(int j, int i, int n) { return (unsigned)j < (unsigned)n && (unsigned)i < (unsigned)n; }

// Loads whose result may be masked read a clamped (always valid) address and
// select afterwards: a load inside a branch makes the compiler wait for it at
// the branch's end, which serialises loads that could all be in flight.
__device__ __forceinline__ int clampi(int v, int n) { return min(max(v, 0), n - 1); }


// Arrays reached through the instance table are global memory, but a pointer
// loaded from memory is generic to the compiler, which then emits FLAT
// accesses; those count against the LDS wait counter as well, so every wait
// for a lane shuffle or LDS access would also wait for all loads in flight.
// The kernels therefore convert them to global-address-space pointers.
template <typename T> using gp = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gp<T> glob(void* p) { return (gp<T>)p; }
template <typename T> __device__ __forceinline__ gp<const T> glob(const void* p) { return (gp<const T>)p; }

template <typename T>
__device__ inline T gload(gp<const T> p, int ld, int n, int j, int i)
{
    const T v = p[(size_t)clampi(j, n) * ld + clampi(i, n)];
    return inside(j, i, n) ? v : T(0);
}

template <typename T>
__device__ inline T gload(const T* p, int ld, int n, int j, int i)
{
    const T v = p[(size_t)clampi(j, n) * ld + clampi(i, n)];
    return inside(j, i, n) ? v : T(0);
}

// stencil sum reading global memory with zero outside the grid
template <typename T>
__device__ inline T gapply(const Sten<T>& s, const T* x, int ld, int n, int j, int i)
{
    T acc = T(0);
    acc = fmadd(s.c[0], gload(x, ld, n, j - 1, i - 1), acc);
    acc = fmadd(s.c[1], gload(x, ld, n, j - 1, i), acc);
    acc = fmadd(s.c[2], gload(x, ld, n, j - 1, i + 1), acc);
    acc = fmadd(s.c[3], gload(x, ld, n, j, i - 1), acc);
    acc = fmadd(s.c[4], gload(x, ld, n, j, i), acc);
    acc = fmadd(s.c[5], gload(x, ld, n, j, i + 1), acc);
    acc = fmadd(s.c[6], gload(x, ld, n, j + 1, i - 1), acc);
    acc = fmadd(s.c[7], gload(x, ld, n, j + 1, i), acc);
    acc = fmadd(s.c[8], gload(x, ld, n, j + 1, i + 1), acc);
    return acc;
}

template <typename T>
__device__ inline T gapply(const Sten<T>& s, gp<const T> x, int ld, int n, int j, int i)
{
    T acc = T(0);
    acc = fmadd(s.c[0], gload(x, ld, n, j - 1, i - 1), acc);
    acc = fmadd(s.c[1], gload(x, ld, n, j - 1, i), acc);
    acc = fmadd(s.c[2], gload(x, ld, n, j - 1, i + 1), acc);
    acc = fmadd(s.c[3], gload(x, ld, n, j, i - 1), acc);
    acc = fmadd(s.c[4], gload(x, ld, n, j, i), acc);
    acc = fmadd(s.c[5], gload(x, ld, n, j, i + 1), acc);
    acc = fmadd(s.c[6], gload(x, ld, n, j + 1, i - 1), acc);
    acc = fmadd(s.c[7], gload(x, ld, n, j + 1, i), acc);
    acc = fmadd(s.c[8], gload(x, ld, n, j + 1, i + 1), acc);
    return acc;
}

// full weighting sum around the fine point at r (stride st)
template <typename T>
__device__ __forceinline__ T fw_sum(const T* r, int st)
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
__device__ __forceinline__ T prolong_at(int j, int i, Get V)
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
// orders one wave's LDS accesses around a point (no other wave takes part)
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

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
template <int BX = TX, int BY = TY>
__device__ inline bool get_tile(const StageArgs& a, int depth_for_size, bool fine_user, Tile& t)
{
    const int b = blockIdx.x;
    const int i = find_inst(a.tile_off, a.count, b);
    t.inst = i;
    t.blk = b - a.tile_off[i];
    t.nblk = a.tile_off[i + 1] - a.tile_off[i];
    const InstDev& I = a.inst[i];
    const int n = fine_user ? I.n0 : I.lev[depth_for_size].n;
    const int tx = (n + BX - 1) / BX;
    t.x0 = (t.blk % tx) * BX;
    t.y0 = (t.blk / tx) * BY;
    return a.st[i].done == 0;
}

// Norms and dot products are Dot2 sums (Ogita, Rump and Oishi, "Accurate sum
// and dot product", 2005): each product is split into its rounded value and
// its exact error (explicit fused multiply-add), the running sum into its
// rounded value and the exact error of the addition (TwoSum), and the errors
// are summed apart and added once at the end.  Two partial sums combine by a
// TwoSum of their values plus the sum of their error terms, so a thread, a
// wave, a block and the finalize kernel each merge in their own fixed order
// and the result is still as accurate as a sum in twice the working
// precision, rounded once: it equals a sequential Dot2 of the same terms
// unless the exact value lies within about n u^2 (relative) of a rounding
// boundary.
struct Acc2 {
    double s, c;
    __device__ __forceinline__ Acc2() : s(0.0), c(0.0) {}
    __device__ __forceinline__ void add_prod(double a, double b)
    {
        const double p = a * b;
        const double e = fma(a, b, -p);
        const double x = s + p;
        const double z = x - s;
        const double q = (s - (x - z)) + (p - z);
        s = x;
        c = c + (q + e);
    }
    __device__ __forceinline__ void add_sq(double a) { add_prod(a, a); }
    // TwoSum is exact in either argument order and the error terms add
    // commutatively, so both lanes of a shuffle pair hold the same result
    __device__ __forceinline__ void merge(double s2, double c2)
    {
        const double x = s + s2;
        const double z = x - s;
        const double q = (s - (x - z)) + (s2 - z);
        s = x;
        c = (c + c2) + q;
    }
    __device__ __forceinline__ double value() const { return s + c; }
};

__device__ __forceinline__ void wave_merge(Acc2& v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v.merge(__shfl_xor(v.s, off, 64), __shfl_xor(v.c, off, 64));
}

// block total of a Dot2 accumulator (valid in thread 0); red holds 2 doubles per wave
template <int NT>
__device__ inline Acc2 block_sum(Acc2 v, double* red)
{
    wave_merge(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) {
        red[2 * w] = v.s;
        red[2 * w + 1] = v.c;
    }
    __syncthreads();
    Acc2 t;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NT / 64; ++k) t.merge(red[2 * k], red[2 * k + 1]);
    }
    return t;
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
        // the recurrence residual drifts from F - S u by rounding: once it passes
        // tol, the true residual (next launch) decides and, if still above tol,
        // replaces it
        const double rel = sqrt(S0) / sqrt(s.ssf);
        s.iters += 1;
        s.relres = rel;
        if (s.iters < HIST_CAP) a.hist[(size_t)inst * HIST_CAP + s.iters] = rel;
        s.scale = ir_scale(S0, npts);
        if (!isfinite(rel)) { s.status = KC_ERR_NONFINITE; s.done = 1; }
        else if (rel < s.tol) s.check = 1;
        else if (s.iters >= s.maxit) { s.status = KC_NOT_CONVERGED; s.done = 1; }
        break;
    }
    case FIN_PCG_TRUE: {
        if (!s.check) break;
        s.check = 0;
        const double rel = sqrt(S0) / sqrt(s.ssf);
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

// every block of a reducing launch stores its two block sums (value and error
// term of each); the finalize kernel (one workgroup per instance, launched next
// on the stream) merges them in block order and applies the solver's decision
__device__ void reduce_partial(const StageArgs& a, const Tile& t, const Acc2& v0, const Acc2& v1)
{
    __shared__ double red[2][2 * (GRID_THREADS / 64)];
    const Acc2 s0 = block_sum<GRID_THREADS>(v0, red[0]);
    const Acc2 s1 = block_sum<GRID_THREADS>(v1, red[1]);
    if (threadIdx.x == 0) {
        const int gb = a.tile_off[t.inst] + t.blk;
        a.partial[4 * gb] = s0.s;
        a.partial[4 * gb + 1] = s0.c;
        a.partial[4 * gb + 2] = s1.s;
        a.partial[4 * gb + 3] = s1.c;
    }
}

__global__ void __launch_bounds__(GRID_THREADS) k_finalize(StageArgs a)
{
    __shared__ double red[2][2 * (GRID_THREADS / 64)];
    const int inst = blockIdx.x;
    const int b0 = a.tile_off[inst], nb = a.tile_off[inst + 1] - b0;
    if (nb == 0 || a.st[inst].done) return;
    // thread t merges partials t, t + 256, ... in that order; loads go in groups of
    // four (clamped indices, masked at use) so that they are in flight together
    constexpr int G = 4;
    Acc2 t0, t1;
    const double4* P4 = (const double4*)a.partial;
    for (int k0 = threadIdx.x; k0 < nb; k0 += G * GRID_THREADS) {
        double4 p[G];
#pragma unroll
        for (int g = 0; g < G; ++g) p[g] = P4[b0 + min(k0 + g * GRID_THREADS, nb - 1)];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (k0 + g * GRID_THREADS < nb) {
                t0.merge(p[g].x, p[g].y);
                t1.merge(p[g].z, p[g].w);
            }
        }
    }
    const Acc2 S0 = block_sum<GRID_THREADS>(t0, red[0]);
    const Acc2 S1 = block_sum<GRID_THREADS>(t1, red[1]);
    if (threadIdx.x == 0) apply_fin(a, inst, S0.value(), S1.value());
}

template <typename T> __device__ inline T* buf(const LevelDev& L, int sel) { return (T*)(sel ? L.B : L.A); }

// ---------------------------------------------------------------------------
// unfused kernels: one kernel per operation of Algorithm 4
// ---------------------------------------------------------------------------
template <typename T, int kind>
__global__ void __launch_bounds__(GRID_THREADS) k_unfused(StageArgs a)
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
    Acc2 nrm;
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

#pragma unroll
    for (int k = ty; k < TY; k += GRID_THREADS / 64) {
        const int j = t.y0 + k, i = t.x0 + tx;
        const bool in = (j < n) && (i < n);
        const size_t gs = (size_t)j * lds_ + i, gd = (size_t)j * ldd_ + i, gf = (size_t)j * Lv.ldf + i;
        switch (kind) {
        case GK_SWEEP: {
            if (!in) break;
            const T* x = buf<T>(Lv, a.src);
            const T acc = gapply(s, x, lds_, n, j, i);
            buf<T>(Lv, a.dst)[gd] = fmadd(w, fs * F[gf] - acc, x[gs]);
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
            nrm.add_sq(r);
            break;
        }
        default:
            break;
        }
    }
    if (kind == GK_NORM) reduce_partial(a, t, nrm, Acc2());
}

// ---------------------------------------------------------------------------
// semi-coarsened levels (Section 4, fifth and sixth solvers): level d has n
// lines (rows) of nx points, x is never coarsened, and every stencil is in units
// of the fine level's h^2 (F of every level carries the same h^2 scale).  One
// kernel per operation on 64 x 32 tiles of (nx, n):
//   residual      r = F - S v (the nine products south row first, west to east);
//   restriction   F_c(J, i) = 1/4 r(2J, i) + 1/2 r(2J+1, i) + 1/4 r(2J+2, i), i.e. R = P^T / 2;
//   prolongation  e(2J+1, i) = v_c(J, i), e(2J, i) = 1/2 v_c(J-1, i) + 1/2 v_c(J, i)
//                 (linear interpolation along y, zero beyond the last lines);
//   zero, add, copy as in the square case.  Relaxation is the x-line zebra kernel.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline T sload(const T* p, int ld, int ny, int nx, int j, int i)
{
    const T v = p[(size_t)min(max(j, 0), ny - 1) * ld + min(max(i, 0), nx - 1)];
    return ((unsigned)j < (unsigned)ny && (unsigned)i < (unsigned)nx) ? v : T(0);
}

template <typename T, int kind>
__global__ void __launch_bounds__(GRID_THREADS) k_semi(StageArgs a)
{
    const int b = blockIdx.x;
    const int inst = find_inst(a.tile_off, a.count, b);
    if (a.st[inst].done) return;
    const InstDev& I = a.inst[inst];
    const int d = a.depth;
    const LevelDev& Lv = I.lev[d];
    const int ny = Lv.n, nx = Lv.nx;
    const int blk = b - a.tile_off[inst];
    const int tiles_x = (nx + TX - 1) / TX;
    const int x0 = (blk % tiles_x) * TX, y0 = (blk / tiles_x) * TY;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int i = x0 + tx;
    const int lds_ = a.src ? Lv.ldb : Lv.lda;
    const int ldd_ = a.dst ? Lv.ldb : Lv.lda;

    if constexpr (kind == GK_RESTRICT || kind == GK_ZERO) {
        // coarse lines J whose centre line 2J+1 lies in this tile
        const LevelDev& Lc = I.lev[d + 1];
        const int nyc = Lc.n;
        const T* r = buf<T>(Lv, a.src);
        for (int k = ty; k < TY / 2; k += GRID_THREADS / 64) {
            const int J = (y0 >> 1) + k;
            if (J >= nyc || i >= nx) continue;
            if constexpr (kind == GK_ZERO) {
                ((T*)Lc.A)[(size_t)J * Lc.lda + i] = T(0);
            } else {
                T acc = T(0);
                acc += T(0.25) * r[(size_t)(2 * J) * lds_ + i];
                acc += T(0.5) * r[(size_t)(2 * J + 1) * lds_ + i];
                acc += T(0.25) * r[(size_t)(2 * J + 2) * lds_ + i];
                ((T*)Lc.F)[(size_t)J * Lc.ldf + i] = acc;
            }
        }
        return;
    }
    Sten<T> s;
    s.load(P<T>::s(I, d));
    const T fs = (T)Lv.fscale;
    for (int k = ty; k < TY; k += GRID_THREADS / 64) {
        const int j = y0 + k;
        if (j >= ny || i >= nx) continue;
        const size_t gs = (size_t)j * lds_ + i, gd = (size_t)j * ldd_ + i;
        if constexpr (kind == GK_RESID) {
            const T* x = buf<T>(Lv, a.src);
            T acc = T(0);
            acc = fmadd(s.c[0], sload(x, lds_, ny, nx, j - 1, i - 1), acc);
            acc = fmadd(s.c[1], sload(x, lds_, ny, nx, j - 1, i), acc);
            acc = fmadd(s.c[2], sload(x, lds_, ny, nx, j - 1, i + 1), acc);
            acc = fmadd(s.c[3], sload(x, lds_, ny, nx, j, i - 1), acc);
            acc = fmadd(s.c[4], sload(x, lds_, ny, nx, j, i), acc);
            acc = fmadd(s.c[5], sload(x, lds_, ny, nx, j, i + 1), acc);
            acc = fmadd(s.c[6], sload(x, lds_, ny, nx, j + 1, i - 1), acc);
            acc = fmadd(s.c[7], sload(x, lds_, ny, nx, j + 1, i), acc);
            acc = fmadd(s.c[8], sload(x, lds_, ny, nx, j + 1, i + 1), acc);
            buf<T>(Lv, a.dst)[gd] = fs * ((const T*)Lv.F)[(size_t)j * Lv.ldf + i] - acc;
        } else if constexpr (kind == GK_PROLONG) {
            const LevelDev& Lc = I.lev[d + 1];
            const T* vc = buf<T>(Lc, a.src);
            const int ldc = a.src ? Lc.ldb : Lc.lda, nyc = Lc.n;
            T acc = T(0);
            if (j & 1) {
                acc += T(1) * vc[(size_t)(j >> 1) * ldc + i];
            } else {
                const int Ja = (j >> 1) - 1, Jb = j >> 1;
                const T va = vc[(size_t)max(Ja, 0) * ldc + i], vb = vc[(size_t)min(Jb, nyc - 1) * ldc + i];
                acc += T(0.5) * (Ja >= 0 ? va : T(0));
                acc += T(0.5) * (Jb < nyc ? vb : T(0));
            }
            buf<T>(Lv, a.dst)[gd] = acc;
        } else if constexpr (kind == GK_ADD) {
            T* v = buf<T>(Lv, a.src);
            v[gs] = v[gs] + buf<T>(Lv, a.dst)[gd];
        } else if constexpr (kind == GK_COPY) {
            buf<T>(Lv, a.dst)[gd] = buf<T>(Lv, a.src)[gs];
        } else if constexpr (kind == GK_ZERO_SELF) {
            ((T*)Lv.A)[(size_t)j * Lv.lda + i] = T(0);
        }
    }
}

// ---------------------------------------------------------------------------
// zebra line relaxation on the levels run one kernel per operation: every line of the launch's
// colour (lines 2 m + colour) solves its tridiagonal system exactly with its
// neighbouring lines' current values, in place.  Forward pass:
// d_q = F_q - (six off-line products: line j-1 then j+1, west to east, for
// x-lines; column i-1 then i+1, south to north, for y-lines);
// y_q = (d_q - lo y_{q-1}) r_q, written over the line; backward pass
// x_q = y_q - u_q x_{q+1}.  r, u: the level's reciprocal pivots and upper
// multipliers.  Two mappings with the same arithmetic, chosen per instance:
//
// * lanes (levels below the launch's threshold): one thread per line, 64
//   lines per workgroup (one wave, so a colour's lines spread over as many
//   CUs as waves).  Both passes go along the line in chunks of ZK points:
//   every load of a chunk (the two neighbouring lines one point ahead, F and
//   r; or the line's own y values and u) is issued before the chunk's stores,
//   the neighbouring lines' values at q - 1, q, q + 1 slide through
//   registers, and the chunk's d_q are formed before the recurrence.
// * waves (levels at or above the threshold): two lines per wave (lanes 0-31
//   and 32-63), eight per workgroup.  Lane l holds point q0 + (l mod 32) of a
//   chunk of 32 points of its line: the lanes form the chunk's d_q (and load
//   r) in parallel and put them in the wave's LDS slots; lanes 0 and 32 alone
//   run the two recurrences over the chunk (unrolled, one LDS read per step,
//   so the vector ALU issues only the recurrences' own operations, each
//   advancing both lines, and the LDS returns 2 x 16 bytes per step), write
//   the results back to LDS, and each lane stores its own point; the next
//   chunk's loads are issued before the recurrences, so they are in flight
//   while they run.  A level's n / 2 lines give n / 4 waves, against n / 128
//   for the lane mapping, which is what large levels need to keep memory busy.  The backward pass
//   reads each point's y back in the lane that wrote it.
// ---------------------------------------------------------------------------
template <typename T> struct ZT;
template <> struct ZT<double> { static __device__ const double* t(const InstDev& I, int d) { return I.zt64[d]; } };
template <> struct ZT<float> { static __device__ const float* t(const InstDev& I, int d) { return I.zt32[d]; } };

// per-line constants of one launch (direction DIR: 0 x-lines, 1 y-lines)
template <typename T, int DIR>
struct ZLine {
    gp<T> V;
    gp<const T> F, rpv, mul;
    int n, nl, ldv, ldf, line;   // points per line, lines of the level
    T fs, lo, cm0, cm1, cm2, cp0, cp1, cp2;
    bool hm, hp;
    int Lm, Lp;
    __device__ __forceinline__ int vi(int L, int q) const { return DIR == 0 ? L * ldv + q : q * ldv + L; }
    __device__ __forceinline__ int fi(int q) const { return DIR == 0 ? line * ldf + q : q * ldf + line; }
};

template <typename T, int DIR>
__device__ __forceinline__ void zebra_lanes(const ZLine<T, DIR>& z)
{
    constexpr int ZK = sizeof(T) == 8 ? 8 : 16;
    const int n = z.n;
    T m0 = T(0), p0 = T(0);                                          // previous / next line at q - 1
    T m1 = z.hm ? z.V[z.vi(z.Lm, 0)] : T(0), p1 = z.hp ? z.V[z.vi(z.Lp, 0)] : T(0);   // at q
    T prev = T(0);
    for (int q0 = 0; q0 < n; q0 += ZK) {
        T mn[ZK], pn[ZK], fv[ZK], rv[ZK];
#pragma unroll
        for (int k = 0; k < ZK; ++k) {
            const int qa = q0 + k + 1;                   // position entering the window
            const int qc = min(qa, n - 1), qf = min(q0 + k, n - 1);
            const T xm = z.V[z.vi(z.Lm, qc)], xp = z.V[z.vi(z.Lp, qc)], xf = z.F[z.fi(qf)];
            mn[k] = (z.hm && qa < n) ? xm : T(0);
            pn[k] = (z.hp && qa < n) ? xp : T(0);
            fv[k] = xf;
            rv[k] = z.rpv[qf];
        }
        T dq[ZK];
#pragma unroll
        for (int k = 0; k < ZK; ++k) {
            T acc = T(0);
            acc = fmadd(z.cm0, m0, acc);
            acc = fmadd(z.cm1, m1, acc);
            acc = fmadd(z.cm2, mn[k], acc);
            acc = fmadd(z.cp0, p0, acc);
            acc = fmadd(z.cp1, p1, acc);
            acc = fmadd(z.cp2, pn[k], acc);
            dq[k] = z.fs * fv[k] - acc;
            m0 = m1;
            m1 = mn[k];
            p0 = p1;
            p1 = pn[k];
        }
#pragma unroll
        for (int k = 0; k < ZK; ++k) {
            const int q = q0 + k;
            if (q < n) {
                const T y = (q == 0) ? dq[k] * rv[k] : fmadd(-z.lo, prev, dq[k]) * rv[k];
                z.V[z.vi(z.line, q)] = y;
                prev = y;
            }
        }
    }
    T next = prev;   // x_{n-1} = y_{n-1}
    for (int q1 = n - 2; q1 >= 0; q1 -= ZK) {
        T yv[ZK], mv[ZK];
#pragma unroll
        for (int k = 0; k < ZK; ++k) {
            const int qc = max(q1 - k, 0);
            yv[k] = z.V[z.vi(z.line, qc)];
            mv[k] = z.mul[qc];
        }
#pragma unroll
        for (int k = 0; k < ZK; ++k) {
            const int q = q1 - k;
            if (q >= 0) {
                const T x = fmadd(-mv[k], next, yv[k]);
                z.V[z.vi(z.line, q)] = x;
                next = x;
            }
        }
    }
}

// the loads of one lane for a forward chunk: point q = q0 + lane (clamped
// addresses).  The values are masked where the point or a neighbour is absent
// only when d_q is formed, so that prefetched loads are not waited for early.
template <typename T>
struct ZFwd {
    T m0, m1, m2, p0, p1, p2, f, r;
    bool km0, km1, km2, kp0, kp1, kp2;   // which neighbour values are present
    template <int DIR>
    __device__ __forceinline__ void load(const ZLine<T, DIR>& z, int q)
    {
        const int qc = min(q, z.n - 1), qm = max(qc - 1, 0), qp = min(q + 1, z.n - 1);
        m0 = z.V[z.vi(z.Lm, qm)];
        m1 = z.V[z.vi(z.Lm, qc)];
        m2 = z.V[z.vi(z.Lm, qp)];
        p0 = z.V[z.vi(z.Lp, qm)];
        p1 = z.V[z.vi(z.Lp, qc)];
        p2 = z.V[z.vi(z.Lp, qp)];
        f = z.F[z.fi(qc)];
        r = z.rpv[qc];
        km0 = z.hm && q >= 1;
        km1 = z.hm;
        km2 = z.hm && q + 1 < z.n;
        kp0 = z.hp && q >= 1;
        kp1 = z.hp;
        kp2 = z.hp && q + 1 < z.n;
    }
    template <int DIR>
    __device__ __forceinline__ T dq(const ZLine<T, DIR>& z) const
    {
        T acc = T(0);
        acc = fmadd(z.cm0, (km0 ? m0 : T(0)), acc);
        acc = fmadd(z.cm1, (km1 ? m1 : T(0)), acc);
        acc = fmadd(z.cm2, (km2 ? m2 : T(0)), acc);
        acc = fmadd(z.cp0, (kp0 ? p0 : T(0)), acc);
        acc = fmadd(z.cp1, (kp1 ? p1 : T(0)), acc);
        acc = fmadd(z.cp2, (kp2 ? p2 : T(0)), acc);
        return z.fs * f - acc;
    }
};

// a wave's LDS slots for one chunk of each of its 64 / ZC lines: the lanes' (d_q, r_q)
// or (y_q, u_q) pairs, read back one per step by the lane running that line's
// recurrence, and the chunk's results, written by that lane and read by every
// lane of the line.  ZC (points per chunk and line) is 32 (two lines per wave) or
// 16 (four lines per wave); the slots of a wave take the same bytes either way
template <typename T, int ZC>
struct ZSlots {
    T pair[64 / ZC][ZC][2];
    T res[64 / ZC][ZC];
};

template <typename T, int DIR, int ZC>
__device__ __forceinline__ void zebra_wave(const ZLine<T, DIR>& z, ZSlots<T, ZC>& sl)
{
    static_assert(ZC == 32 || ZC == 16, "a line takes half or a quarter of a wave");
    constexpr int SB = 8;   // steps per block: the block's pairs are read one block ahead
    const int n = z.n, lane = threadIdx.x & 63, h = lane / ZC, p = lane & (ZC - 1);
    const bool runner = p == 0;   // the first lane of each line's group runs its recurrence
    ZFwd<T> cur;
    cur.load(z, p);
    T prev = T(0);
    // one chunk of the forward pass.  Every chunk issues the same memory operations (the next
    // chunk's loads, clamped past the line's end, then one store), and the first chunk runs
    // before the loop: the loop is then entered, like its back edge, with one store behind
    // the loads, so the wait for them need not cover that store
    auto fwd = [&](int q0) {
        sl.pair[h][p][0] = cur.dq(z);
        sl.pair[h][p][1] = cur.r;
        wave_sync();
        cur.load(z, q0 + ZC + p);   // in flight during the recurrence
        const int cnt = min(ZC, n - q0);
        const bool first = q0 == 0;
        // a full chunk keeps every step; in the last one, steps past the line's end
        // (k >= cnt) compute values that are neither kept nor stored
        auto steps = [&](auto partial) {
            T dk[SB], rk[SB];   // the block's pairs, read one block ahead of the recurrence
#pragma unroll
            for (int j = 0; j < SB; ++j) {
                dk[j] = sl.pair[h][j][0];
                rk[j] = sl.pair[h][j][1];
            }
#pragma unroll
            for (int kb = 0; kb < ZC; kb += SB) {
                T dn[SB], rn[SB];
                if (kb + SB < ZC) {
#pragma unroll
                    for (int j = 0; j < SB; ++j) {
                        dn[j] = sl.pair[h][kb + SB + j][0];
                        rn[j] = sl.pair[h][kb + SB + j][1];
                    }
                }
#pragma unroll
                for (int j = 0; j < SB; ++j) {
                    const int k = kb + j;
                    const T t = (k == 0 && first) ? dk[j] : fmadd(-z.lo, prev, dk[j]);   // y_0 = d_0 r_0
                    const T y = t * rk[j];
                    sl.res[h][k] = y;
                    if constexpr (decltype(partial)::value) prev = (k < cnt) ? y : prev;
                    else prev = y;
                }
                if (kb + SB < ZC) {
#pragma unroll
                    for (int j = 0; j < SB; ++j) {
                        dk[j] = dn[j];
                        rk[j] = rn[j];
                    }
                }
            }
        };
        // the runner lanes run the recurrences: each instruction advances every line of the
        // wave, and the LDS returns 16 bytes per line and step
        if (runner) {
            if (cnt == ZC) steps(std::false_type{});
            else steps(std::true_type{});
        }
        wave_sync();
        {   // lanes past the line's end store the last point's value again (same value, same address)
            const int k = min(p, cnt - 1);
            z.V[z.vi(z.line, q0 + k)] = sl.res[h][k];
        }
        wave_sync();   // the slots are rewritten by the next chunk
    };
    fwd(0);
    for (int q0 = ZC; q0 < n; q0 += ZC) fwd(q0);

    // backward, chunks from the last one down; a lane owns the points it wrote above
    const int c_last = (n - 1) / ZC;
    const T ylast = __shfl(prev, lane & (64 - ZC), 64);   // y_{n-1}, kept by the line's runner lane
    T next = prev;   // x_{n-1} = y_{n-1} (runner lanes)
    T yv, uv;
    {
        const int q = min(c_last * ZC + p, n - 1);
        yv = z.V[z.vi(z.line, q)];
        uv = z.mul[q];
    }
    auto bwd = [&](int c) {
        const int q0 = c * ZC;
        sl.pair[h][p][0] = yv;
        sl.pair[h][p][1] = uv;
        wave_sync();
        {   // in flight during the recurrence (every chunk issues it; clamped before the line's start)
            const int q = max(q0 - ZC + p, 0);
            yv = z.V[z.vi(z.line, q)];
            uv = z.mul[q];
        }
        const int top = min(ZC - 1, n - 2 - q0);   // x_{n-1} = y_{n-1} is already in place
        auto steps = [&](auto partial) {
            T yk[SB], uk[SB];   // the block's pairs, read one block ahead of the recurrence
#pragma unroll
            for (int j = 0; j < SB; ++j) {
                yk[j] = sl.pair[h][ZC - SB + j][0];
                uk[j] = sl.pair[h][ZC - SB + j][1];
            }
#pragma unroll
            for (int kb = ZC - SB; kb >= 0; kb -= SB) {
                T yn[SB], un[SB];
                if (kb > 0) {
#pragma unroll
                    for (int j = 0; j < SB; ++j) {
                        yn[j] = sl.pair[h][kb - SB + j][0];
                        un[j] = sl.pair[h][kb - SB + j][1];
                    }
                }
#pragma unroll
                for (int j = SB - 1; j >= 0; --j) {
                    const int k = kb + j;
                    const T x = fmadd(-uk[j], next, yk[j]);
                    sl.res[h][k] = x;
                    if constexpr (decltype(partial)::value) next = (k <= top) ? x : next;
                    else next = x;
                }
                if (kb > 0) {
#pragma unroll
                    for (int j = 0; j < SB; ++j) {
                        yk[j] = yn[j];
                        uk[j] = un[j];
                    }
                }
            }
        };
        if (runner) {
            if (top == ZC - 1) steps(std::false_type{});
            else steps(std::true_type{});
        }
        wave_sync();
        {   // lanes past top store the value at top again; with top = -1 (a chunk holding only
            // the line's last point) every lane stores y_{n-1} back in place
            const int k = min(p, max(top, 0));
            const T xv = top >= 0 ? sl.res[h][k] : ylast;
            z.V[z.vi(z.line, q0 + k)] = xv;
        }
        wave_sync();
    };
    bwd(c_last);
    for (int c = c_last - 1; c >= 0; --c) bwd(c);
}

template <typename T, int DIR>
__global__ void __launch_bounds__(GRID_THREADS) k_zebra(StageArgs a)
{
    __shared__ ZSlots<T, 32> slots[GRID_THREADS / 64];
    const int b = blockIdx.x;
    const int inst = find_inst(a.tile_off, a.count, b);
    if (a.st[inst].done) return;
    const InstDev& I = a.inst[inst];
    const int d = a.depth;
    const LevelDev& Lv = I.lev[d];
    const int n = Lv.n, nx = Lv.nx;   // lines and points per line (equal except on semi-coarsened levels)
    // the launch's thresholds (flags: bits 0-14 two lines per wave from this line length,
    // bits 15-29 four lines per wave) pick the mapping for this instance from the line
    // length; the block table was sized the same way
    const int wave_n = a.flags & 0x7fff, quad_n = (a.flags >> 15) & 0x7fff;
    const bool waves = wave_n > 0 && nx >= wave_n;
    const bool quad = waves && quad_n > 0 && nx >= quad_n;
    int blk = b - a.tile_off[inst];
    int line;
    if (waves) {
        // consecutive line groups on one XCD (workgroups go round-robin over the
        // eight XCDs), so y-lines sharing cache lines share an L2
        const int nb = a.tile_off[inst + 1] - a.tile_off[inst];
        if ((a.tile_off[inst] & 7) == 0 && (nb & 7) == 0) blk = (blk & 7) * (nb >> 3) + (blk >> 3);
        // lpw lines per wave, 64 / lpw lanes each; a line past the level's last one repeats
        // the wave's first (the same values go to the same addresses again)
        const int lpw = quad ? ZEBRA_QUAD_LPW : 2;
        const int first = 2 * (blk * (GRID_THREADS / 64) * lpw + lpw * (int)(threadIdx.x >> 6)) + a.dst;
        if (first >= n) return;   // the whole wave
        line = first + 2 * (int)((threadIdx.x & 63) / (64 / lpw));
        if (line >= n) line = first;
    } else {
        if (threadIdx.x >= 64) return;
        line = 2 * (blk * 64 + (int)threadIdx.x) + a.dst;
    }
    if (line >= n) return;
    ZLine<T, DIR> z;
    z.V = glob<T>(buf<T>(Lv, a.src));
    z.ldv = a.src ? Lv.ldb : Lv.lda;   // element offsets fit 32 bits (n <= 2^14)
    z.ldf = Lv.ldf;
    z.F = glob<T>((const void*)Lv.F);
    z.fs = (T)Lv.fscale;
    z.n = nx;
    z.nl = n;
    z.line = line;
    Sten<T> s;
    s.load(P<T>::s(I, d));
    z.rpv = glob<T>((const void*)(ZT<T>::t(I, d) + (size_t)DIR * 2 * nx));
    z.mul = z.rpv + nx;
    z.lo = DIR == 0 ? s.c[3] : s.c[1];
    // off-line coefficients at q - 1, q, q + 1 of the previous line (m) and the next line (p), in summation order
    z.cm0 = s.c[0];
    z.cm1 = DIR == 0 ? s.c[1] : s.c[3];
    z.cm2 = DIR == 0 ? s.c[2] : s.c[6];
    z.cp0 = DIR == 0 ? s.c[6] : s.c[2];
    z.cp1 = DIR == 0 ? s.c[7] : s.c[5];
    z.cp2 = s.c[8];
    z.hm = line > 0;
    z.hp = line + 1 < n;   // n lines
    z.Lm = z.hm ? line - 1 : line;   // clamped; values masked when absent
    z.Lp = z.hp ? line + 1 : line;
    if (quad) {
        using QS = ZSlots<T, 64 / ZEBRA_QUAD_LPW>;
        static_assert(sizeof(QS) == sizeof(ZSlots<T, 32>), "one slot array serves both mappings");
        zebra_wave<T, DIR, 64 / ZEBRA_QUAD_LPW>(z, *reinterpret_cast<QS*>(&slots[threadIdx.x >> 6]));
    } else if (waves) {
        zebra_wave<T, DIR, 32>(z, slots[threadIdx.x >> 6]);
    } else {
        zebra_lanes<T, DIR>(z);
    }
}

// ---------------------------------------------------------------------------
// band-mapped passes over an LDS region (small tiles): the block's threads
// form bands of BW consecutive lanes, lane l of a band is column C0 + l and
// band b owns the U consecutive rows from R0 + b U.  A thread loads the
// 3 x (U + 2) window around its rows once and computes its U points (U
// independent chains) before storing any.  Same arithmetic as Sten::apply.
// ---------------------------------------------------------------------------
template <int C0, int C1, int R0, int R1>
struct RBand {
    static constexpr int W = C1 - C0;
    static constexpr int BW = W <= 16 ? 16 : (W <= 32 ? 32 : 64);
    static constexpr int NB = GRID_THREADS / BW;
    static constexpr int U = (R1 - R0 + NB - 1) / NB;
};

// dst = src + w (F - S src) on rows [R0, R1) x columns [C0, C1) of a region with row
// stride RW (zero outside the grid); zg: dst = w F; resid: dst = F - S src
template <typename T, int RW, int C0, int C1, int R0, int R1, int MODE>   // MODE 0 sweep, 1 zero-guess sweep, 2 residual
__device__ __forceinline__ void band_pass(const T* src, T* dst, const T* sf, const Sten<T>& s, T w, int ry0, int rx0, int n)
{
    using G = RBand<C0, C1, R0, R1>;
    constexpr int U = G::U;
    const int b = threadIdx.x / G::BW, l = threadIdx.x % G::BW;
    const int c = C0 + l, r0 = R0 + b * U;
    if (c >= C1 || r0 >= R1) return;
    const bool colin = (unsigned)(rx0 + c) < (unsigned)n;
    T val[U];
    if (MODE == 1) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = min(r0 + u, R1 - 1);
            val[u] = (colin && (unsigned)(ry0 + r) < (unsigned)n) ? w * sf[r * RW + c] : T(0);
        }
    } else {
        T win[U + 2][3];
#pragma unroll
        for (int k = 0; k < U + 2; ++k) {
            const int r = min(r0 - 1 + k, R1);
#pragma unroll
            for (int e = 0; e < 3; ++e) win[k][e] = src[r * RW + c - 1 + e];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = min(r0 + u, R1 - 1);
            T acc = T(0);
            acc = fmadd(s.c[0], win[u][0], acc);
            acc = fmadd(s.c[1], win[u][1], acc);
            acc = fmadd(s.c[2], win[u][2], acc);
            acc = fmadd(s.c[3], win[u + 1][0], acc);
            acc = fmadd(s.c[4], win[u + 1][1], acc);
            acc = fmadd(s.c[5], win[u + 1][2], acc);
            acc = fmadd(s.c[6], win[u + 2][0], acc);
            acc = fmadd(s.c[7], win[u + 2][1], acc);
            acc = fmadd(s.c[8], win[u + 2][2], acc);
            const bool in = colin && (unsigned)(ry0 + r) < (unsigned)n;
            const T fr = sf[r * RW + c];
            if (MODE == 2) val[u] = in ? fr - acc : T(0);
            else val[u] = in ? fmadd(w, fr - acc, win[u + 1][1]) : T(0);
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (r0 + u < R1) dst[(r0 + u) * RW + c] = val[u];
}

// NU sweeps of a region of RW x RH (sweep k covers [k, RW - k) x [k, RH - k)), ping-pong in sv
template <typename T, int NU, int RW, int RH, int K = 1>
__device__ __forceinline__ void band_sweeps(T (*sv)[RW * RH], const T* sf, const Sten<T>& s, T w, bool zg, int ry0, int rx0, int n)
{
    if constexpr (K <= NU) {
        const T* src = sv[(K - 1) & 1];
        T* dst = sv[K & 1];
        if (K == 1 && zg) band_pass<T, RW, K, RW - K, K, RH - K, 1>(src, dst, sf, s, w, ry0, rx0, n);
        else band_pass<T, RW, K, RW - K, K, RH - K, 0>(src, dst, sf, s, w, ry0, rx0, n);
        __syncthreads();
        band_sweeps<T, NU, RW, RH, K + 1>(sv, sf, s, w, zg, ry0, rx0, n);
    }
}

// ---------------------------------------------------------------------------
// fused pre-smoothing: nu sweeps + residual + full weighting in one pass
// (input region = tile + halo nu+1, swept in LDS); optional input norm
// ---------------------------------------------------------------------------
template <typename T, int NU, int TX, int TY>
__global__ void __launch_bounds__(GRID_THREADS) k_pre(StageArgs a)
{
    constexpr int H = NU + 1;
    constexpr int RW = TX + 2 * H + 1, RH = TY + 2 * H + 1;
    __shared__ T sv[2][RH * RW];
    __shared__ T sf[RH * RW];
    Tile t;
    if (!get_tile<TX, TY>(a, a.depth, false, t)) return;
    const InstDev& I = a.inst[t.inst];
    const int d = a.depth;
    const LevelDev& Lv = I.lev[d];
    const int n = Lv.n;
    const gp<const T> A = glob<T>((const void*)Lv.A);
    const gp<T> B = glob<T>(Lv.B);
    const gp<const T> F = glob<T>((const void*)Lv.F);
    const T fs = (T)Lv.fscale;
    const int rx0 = t.x0 - H, ry0 = t.y0 - H;
    Sten<T> s;
    s.load(P<T>::s(I, d));
    const T w = P<T>::w(I, d);
    const bool zg = a.zg != 0;
    // a zero guess reads no estimate: F, with its own leading dimension, is a valid stand-in address
    const gp<const T> Av = zg ? F : A;
    const size_t ldav = zg ? (size_t)Lv.ldf : (size_t)Lv.lda;

    {   // every load of the region in flight before the LDS stores
        constexpr int NR = RH * RW, NPT = (NR + GRID_THREADS - 1) / GRID_THREADS;
        T fa[NPT], va[NPT];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int p = threadIdx.x + k * GRID_THREADS;
            const int rj = p / RW, ri = p - rj * RW;
            const int j = ry0 + rj, i = rx0 + ri;
            const bool in = p < NR && inside(j, i, n);
            const size_t jc = (size_t)clampi(j, n), ic = (size_t)clampi(i, n);
            const T lf = F[jc * Lv.ldf + ic];
            const T lv = Av[jc * ldav + ic];
            fa[k] = in ? fs * lf : T(0);
            va[k] = (in && !zg) ? lv : T(0);
        }
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int p = threadIdx.x + k * GRID_THREADS;
            if (p < NR) {
                sf[p] = fa[k];
                sv[0][p] = va[k];
            }
        }
    }
    __syncthreads();

    Acc2 nrm;
    if (a.fin == FIN_STOP) {
        for (int p = threadIdx.x; p < TX * TY; p += GRID_THREADS) {
            const int rj = H + p / TX, ri = H + (p % TX);
            if (!inside(ry0 + rj, rx0 + ri, n)) continue;
            const int q = rj * RW + ri;
            const double r = (double)(sf[q] - s.apply(&sv[0][q], RW));
            nrm.add_sq(r);
        }
    }

    if constexpr (TX == TY && TX <= 32) {
        band_sweeps<T, NU, RW, RH>(sv, sf, s, w, zg, ry0, rx0, n);
    } else {
#pragma unroll
        for (int k = 1; k <= NU; ++k) {
            const int ww = RW - 2 * k, hh = RH - 2 * k;
            T* src = sv[(k - 1) & 1];
            T* dst = sv[k & 1];
            for (int p = threadIdx.x; p < ww * hh; p += GRID_THREADS) {
                const int rj = k + p / ww, ri = k + (p % ww);
                const int q = rj * RW + ri;
                T val = T(0);
                if (inside(ry0 + rj, rx0 + ri, n)) {
                    if (k == 1 && zg) val = w * sf[q];
                    else val = fmadd(w, sf[q] - s.apply(&src[q], RW), src[q]);
                }
                dst[q] = val;
            }
            __syncthreads();
        }
    }
    const T* vs = sv[NU & 1];
    T* rs = sv[(NU + 1) & 1];

    // smoothed estimate on the tile
    for (int p = threadIdx.x; p < TX * TY; p += GRID_THREADS) {
        const int y = p / TX, x = p % TX;
        const int j = t.y0 + y, i = t.x0 + x;
        if (j < n && i < n) B[(size_t)j * Lv.ldb + i] = vs[(H + y) * RW + (H + x)];
    }
    // residual on [x0, x0+TX] x [y0, y0+TY]
    if constexpr (TX == TY && TX <= 32) {
        band_pass<T, RW, H, H + TX + 1, H, H + TY + 1, 2>(vs, rs, sf, s, w, ry0, rx0, n);
    } else {
        for (int p = threadIdx.x; p < (TX + 1) * (TY + 1); p += GRID_THREADS) {
            const int y = p / (TX + 1), x = p % (TX + 1);
            const int q = (H + y) * RW + (H + x);
            rs[q] = inside(t.y0 + y, t.x0 + x, n) ? sf[q] - s.apply(&vs[q], RW) : T(0);
        }
    }
    __syncthreads();
    {
        const LevelDev& Lc = I.lev[d + 1];
        const int nc = Lc.n, ldc = Lc.ldf;
        const gp<T> Fc = glob<T>(Lc.F);
        for (int p = threadIdx.x; p < (TX / 2) * (TY / 2); p += GRID_THREADS) {
            const int Ic = (t.x0 >> 1) + (p % (TX / 2)), Jc = (t.y0 >> 1) + (p / (TX / 2));
            if (Ic >= nc || Jc >= nc) continue;
            const int q = (2 * Jc + 1 - ry0) * RW + (2 * Ic + 1 - rx0);
            Fc[(size_t)Jc * ldc + Ic] = fw_sum(&rs[q], RW);
        }
    }
    if (a.fin == FIN_STOP) reduce_partial(a, t, nrm, Acc2());
}

// ---------------------------------------------------------------------------
// fused post-smoothing: prolong-add + nu sweeps (input region = tile + halo nu)
// ---------------------------------------------------------------------------
template <typename T, int NU, int TX, int TY>
__global__ void __launch_bounds__(GRID_THREADS) k_post(StageArgs a)
{
    constexpr int H = NU;
    constexpr int RW = TX + 2 * H, RH = TY + 2 * H;
    constexpr int CW = TX / 2 + H + 3, CH = TY / 2 + H + 3;
    __shared__ T sv[2][RH * RW];
    __shared__ T sf[RH * RW];
    __shared__ T sc[CH * CW];
    Tile t;
    if (!get_tile<TX, TY>(a, a.depth, false, t)) return;
    const InstDev& I = a.inst[t.inst];
    const int d = a.depth;
    const LevelDev& Lv = I.lev[d];
    const LevelDev& Lc = I.lev[d + 1];
    const int n = Lv.n, nc = Lc.n, ldc = Lc.lda;
    const gp<T> A = glob<T>(Lv.A);
    const gp<const T> B = glob<T>((const void*)Lv.B);
    const gp<const T> F = glob<T>((const void*)Lv.F);
    const gp<const T> Vc = glob<T>((const void*)Lc.A);
    const T fs = (T)Lv.fscale;
    const int rx0 = t.x0 - H, ry0 = t.y0 - H;
    const int cx0 = (rx0 - 1) >> 1, cy0 = (ry0 - 1) >> 1;
    Sten<T> s;
    s.load(P<T>::s(I, d));
    const T w = P<T>::w(I, d);

    {   // every load of the region in flight before the LDS stores
        constexpr int NR = RH * RW, NPT = (NR + GRID_THREADS - 1) / GRID_THREADS;
        constexpr int NC = CH * CW, NPC = (NC + GRID_THREADS - 1) / GRID_THREADS;
        T fa[NPT], va[NPT], ca[NPC];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int p = threadIdx.x + k * GRID_THREADS;
            const int rj = p / RW, ri = p - rj * RW;
            const int j = ry0 + rj, i = rx0 + ri;
            const bool in = p < NR && inside(j, i, n);
            const size_t jc = (size_t)clampi(j, n), ic = (size_t)clampi(i, n);
            const T lf = F[jc * Lv.ldf + ic];
            const T lv = B[jc * Lv.ldb + ic];
            fa[k] = in ? fs * lf : T(0);
            va[k] = in ? lv : T(0);
        }
#pragma unroll
        for (int k = 0; k < NPC; ++k) {
            const int p = threadIdx.x + k * GRID_THREADS;
            const int cj = p / CW, ci = p - cj * CW;
            const T cv = gload(Vc, ldc, nc, cy0 + cj, cx0 + ci);
            ca[k] = (p < NC) ? cv : T(0);
        }
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int p = threadIdx.x + k * GRID_THREADS;
            if (p < NR) {
                sf[p] = fa[k];
                sv[0][p] = va[k];
            }
        }
#pragma unroll
        for (int k = 0; k < NPC; ++k) {
            const int p = threadIdx.x + k * GRID_THREADS;
            if (p < NC) sc[p] = ca[k];
        }
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
    if constexpr (TX == TY && TX <= 32) {
        band_sweeps<T, NU, RW, RH>(sv, sf, s, w, false, ry0, rx0, n);
    } else {
#pragma unroll
        for (int k = 1; k <= NU; ++k) {
            const int ww = RW - 2 * k, hh = RH - 2 * k;
            T* src = sv[(k - 1) & 1];
            T* dst = sv[k & 1];
            for (int p = threadIdx.x; p < ww * hh; p += GRID_THREADS) {
                const int rj = k + p / ww, ri = k + (p % ww);
                const int q = rj * RW + ri;
                T val = T(0);
                if (inside(ry0 + rj, rx0 + ri, n)) val = fmadd(w, sf[q] - s.apply(&src[q], RW), src[q]);
                dst[q] = val;
            }
            __syncthreads();
        }
    }
    const T* vs = sv[NU & 1];
    for (int p = threadIdx.x; p < TX * TY; p += GRID_THREADS) {
        const int y = p / TX, x = p % TX;
        const int j = t.y0 + y, i = t.x0 + x;
        if (j < n && i < n) A[(size_t)j * Lv.lda + i] = vs[(H + y) * RW + (H + x)];
    }
}

// ---------------------------------------------------------------------------
// fused junction of two sibling calls on one level (kappa >= 2): the first
// call's prolong-add + NU2 sweeps and the second call's NU1 sweeps + residual +
// full weighting, in one tile kernel.  The first call's result would be
// written to A only for the second call's pre-smoothing to read it back, so it
// stays in LDS; the input is the first call's pre-smoothed estimate (B), the
// output goes to B and F of the coarse level, as the pre-smoothing writes them.
// Input region = tile + halo NU2 + NU1 + 1 (+1 on the high side for the
// residual ring of the full weighting).
// ---------------------------------------------------------------------------
template <typename T, int NU2, int NU1, int TX, int TY>
__global__ void __launch_bounds__(GRID_THREADS) k_postpre(StageArgs a)
{
    constexpr int NUT = NU2 + NU1, H = NUT + 1;
    constexpr int RW = TX + 2 * H + 1, RH = TY + 2 * H + 1;
    constexpr int CW = TX / 2 + H + 3, CH = TY / 2 + H + 3;
    __shared__ T sv[2][RH * RW];
    __shared__ T sf[RH * RW];
    __shared__ T sc[CH * CW];
    Tile t;
    if (!get_tile<TX, TY>(a, a.depth, false, t)) return;
    const InstDev& I = a.inst[t.inst];
    const int d = a.depth;
    const LevelDev& Lv = I.lev[d];
    const LevelDev& Lc = I.lev[d + 1];
    const int n = Lv.n, nc = Lc.n;
    const gp<T> B = glob<T>(Lv.B);
    const gp<const T> F = glob<T>((const void*)Lv.F);
    const gp<const T> Vc = glob<T>((const void*)Lc.A);
    const gp<T> Fc = glob<T>(Lc.F);
    const T fs = (T)Lv.fscale;
    const int rx0 = t.x0 - H, ry0 = t.y0 - H;
    const int cx0 = (rx0 - 1) >> 1, cy0 = (ry0 - 1) >> 1;
    Sten<T> s;
    s.load(P<T>::s(I, d));
    const T w = P<T>::w(I, d);

    {   // every load of the region in flight before the LDS stores
        constexpr int NR = RH * RW, NPT = (NR + GRID_THREADS - 1) / GRID_THREADS;
        constexpr int NC = CH * CW, NPC = (NC + GRID_THREADS - 1) / GRID_THREADS;
        T fa[NPT], va[NPT], ca[NPC];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int p = threadIdx.x + k * GRID_THREADS;
            const int rj = p / RW, ri = p - rj * RW;
            const int j = ry0 + rj, i = rx0 + ri;
            const bool in = p < NR && inside(j, i, n);
            const size_t jc = (size_t)clampi(j, n), ic = (size_t)clampi(i, n);
            const T lf = F[jc * Lv.ldf + ic];
            const T lv = B[jc * Lv.ldb + ic];
            fa[k] = in ? fs * lf : T(0);
            va[k] = in ? lv : T(0);
        }
#pragma unroll
        for (int k = 0; k < NPC; ++k) {
            const int p = threadIdx.x + k * GRID_THREADS;
            const int cj = p / CW, ci = p - cj * CW;
            const T cv = gload(Vc, Lc.lda, nc, cy0 + cj, cx0 + ci);
            ca[k] = (p < NC) ? cv : T(0);
        }
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int p = threadIdx.x + k * GRID_THREADS;
            if (p < NR) {
                sf[p] = fa[k];
                sv[0][p] = va[k];
            }
        }
#pragma unroll
        for (int k = 0; k < NPC; ++k) {
            const int p = threadIdx.x + k * GRID_THREADS;
            if (p < NC) sc[p] = ca[k];
        }
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
    // NU2 post-sweeps of the first call, then NU1 pre-sweeps of the second: the same Jacobi sweeps
    band_sweeps<T, NUT, RW, RH>(sv, sf, s, w, false, ry0, rx0, n);
    const T* vs = sv[NUT & 1];
    T* rs = sv[(NUT + 1) & 1];
    for (int p = threadIdx.x; p < TX * TY; p += GRID_THREADS) {
        const int y = p / TX, x = p % TX;
        const int j = t.y0 + y, i = t.x0 + x;
        if (j < n && i < n) B[(size_t)j * Lv.ldb + i] = vs[(H + y) * RW + (H + x)];
    }
    band_pass<T, RW, H, H + TX + 1, H, H + TY + 1, 2>(vs, rs, sf, s, w, ry0, rx0, n);
    __syncthreads();
    const int ldc = Lc.ldf;
    for (int p = threadIdx.x; p < (TX / 2) * (TY / 2); p += GRID_THREADS) {
        const int Ic = (t.x0 >> 1) + (p % (TX / 2)), Jc = (t.y0 >> 1) + (p / (TX / 2));
        if (Ic >= nc || Jc >= nc) continue;
        const int q = (2 * Jc + 1 - ry0) * RW + (2 * Ic + 1 - rx0);
        Fc[(size_t)Jc * ldc + Ic] = fw_sum(&rs[q], RW);
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

// the same substitution on an n x n grid stored with a zero ring (stride P)
template <typename T>
__device__ inline void chol_solve_padded(int n, const T* Lc, const T* F, T* v, int P)
{
    const int m = n * n;
    auto at = [&](int p) { return (p / n + 1) * P + (p % n + 1); };
    for (int p = 0; p < m; ++p) {
        T acc = F[at(p)];
        for (int q = 0; q < p; ++q) acc -= Lc[p * m + q] * v[at(q)];
        v[at(p)] = acc / Lc[p * m + p];
    }
    for (int p = m - 1; p >= 0; --p) {
        T acc = v[at(p)];
        for (int q = p + 1; q < m; ++q) acc -= Lc[q * m + p] * v[at(q)];
        v[at(p)] = acc / Lc[p * m + p];
    }
}

// ---------------------------------------------------------------------------
// streaming fused kernels for large levels.  A wave owns a strip of SW output
// columns; its 64 lanes hold the strip plus a halo (lane l is column
// x0 - H + l) and it walks down the strip's R rows plus the halo rows.  Every
// stage produces one row per step, one row behind the stage feeding it, and
// keeps its nine-point sums in rolling form (the open sums of the two rows
// its newest input row still enters), so each input row is read from memory
// once and no stage holds a window of rows; east / west neighbours come from DPP
// whole-wave shifts (the lanes at the wave's edges are halo, whose values are
// never stored: each stage's valid lanes shrink by one per side).  No LDS and
// no barriers: loads, arithmetic and stores of the many resident waves
// overlap.  Arithmetic per point is the tile kernels' (same expressions, same
// order), so results are identical.
// ---------------------------------------------------------------------------
// DPP lane moves (a VALU operand modifier, no LDS round trip); lanes whose source
// lies outside the row or wave read 0.  A double moves as its two 32-bit halves.
template <int CTRL> __device__ __forceinline__ float dpp(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <int CTRL> __device__ __forceinline__ double dpp(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
constexpr int DPP_WAVE_SHR1 = 0x138;   // wave_shr:1 -> value of lane - 1 (0 in lane 0)
constexpr int DPP_WAVE_SHL1 = 0x130;   // wave_shl:1 -> value of lane + 1 (0 in lane 63)

constexpr int SW = 54;        // output columns per wave (pre-smoothing with nu <= 3 fits 64 lanes)
constexpr int SWAVES = 4;     // strips per block, side by side
static_assert(SW * SWAVES == STRIP_BLOCK_W, "strip geometry");

template <typename T> struct Row3 {
    T w, c, e;   // west neighbour, own column, east neighbour
};

template <typename T> __device__ __forceinline__ Row3<T> row3(T v)
{
    return Row3<T>{dpp<DPP_WAVE_SHR1>(v), v, dpp<DPP_WAVE_SHL1>(v)};
}

// fixed-order nine-point sum (south row first, west to east), as Sten::apply
template <typename T>
__device__ __forceinline__ T sten3(const Sten<T>& s, const Row3<T>& S, const Row3<T>& C, const Row3<T>& N)
{
    T acc = T(0);
    acc = fmadd(s.c[0], S.w, acc);
    acc = fmadd(s.c[1], S.c, acc);
    acc = fmadd(s.c[2], S.e, acc);
    acc = fmadd(s.c[3], C.w, acc);
    acc = fmadd(s.c[4], C.c, acc);
    acc = fmadd(s.c[5], C.e, acc);
    acc = fmadd(s.c[6], N.w, acc);
    acc = fmadd(s.c[7], N.c, acc);
    acc = fmadd(s.c[8], N.e, acc);
    return acc;
}

// full weighting centred on window row C, as fw_sum
template <typename T>
__device__ __forceinline__ T fw3(const Row3<T>& S, const Row3<T>& C, const Row3<T>& N)
{
    const T q = T(0.25), h = T(0.5);
    T acc = T(0);
    acc += q * S.w;
    acc += h * S.c;
    acc += q * S.e;
    acc += h * C.w;
    acc += T(1) * C.c;
    acc += h * C.e;
    acc += q * N.w;
    acc += h * N.c;
    acc += q * N.e;
    return acc;
}

struct Strip {
    int inst, blk, x0, y0;
    bool live;   // the strip has columns inside the level
};

template <int R>
__device__ inline bool get_strip(const StageArgs& a, Strip& t)
{
    const int b = blockIdx.x;
    const int i = find_inst(a.tile_off, a.count, b);
    t.inst = i;
    t.blk = b - a.tile_off[i];   // the block's partial-sum slot
    const int n = a.inst[i].lev[a.depth].n;
    const int nbx = (n + STRIP_BLOCK_W - 1) / STRIP_BLOCK_W;
    // workgroups go round-robin over the eight XCDs: give each XCD a contiguous run of
    // strips (whole bands of rows), so that the halo rows and columns neighbouring strips
    // share are read through one L2
    int blk = t.blk;
    {
        const int nb = a.tile_off[i + 1] - a.tile_off[i];
        if ((a.tile_off[i] & 7) == 0 && (nb & 7) == 0) blk = (blk & 7) * (nb >> 3) + (blk >> 3);
    }
    t.x0 = ((blk % nbx) * SWAVES + (int)(threadIdx.x >> 6)) * SW;
    t.y0 = (blk / nbx) * R;
    t.live = t.x0 < n;
    return a.st[i].done == 0;
}

// A stage's nine-point sums in rolling form: when the stage above delivers a
// row X, X is the north row of the oldest open sum (which it completes), the
// centre row of the next and the south row of a new one, so a stage keeps two
// partial sums and one centre value instead of a window of three rows.  Each
// sum takes the products in the stencil order (south row, centre row, north
// row; west to east), as sten3 does, so every completed sum is sten3's.
template <typename T> struct Roll {
    T ac = T(0);   // row r: south and centre parts
    T as = T(0);   // row r + 1: south part
    T cc = T(0);   // row r's own value
};

// feeds row X (= row r + 1 of the stage above); returns row r's completed sum
// and leaves row r's own value in `centre`
template <typename T>
__device__ __forceinline__ T roll(Roll<T>& q, const Sten<T>& s, const Row3<T>& X, T& centre)
{
    T acc = q.ac;
    acc = fmadd(s.c[6], X.w, acc);
    acc = fmadd(s.c[7], X.c, acc);
    acc = fmadd(s.c[8], X.e, acc);
    centre = q.cc;
    T mid = q.as;
    mid = fmadd(s.c[3], X.w, mid);
    mid = fmadd(s.c[4], X.c, mid);
    mid = fmadd(s.c[5], X.e, mid);
    T low = T(0);
    low = fmadd(s.c[0], X.w, low);
    low = fmadd(s.c[1], X.c, low);
    low = fmadd(s.c[2], X.e, low);
    q.ac = mid;
    q.as = low;
    q.cc = X.c;
    return acc;
}

// pre-smoothing: NU sweeps + residual + full weighting (+ input residual norm).
// Step s reads input row i = y0 - H + s; sweep k produces row i - k, the
// residual row i - NU - 1 and full weighting is centred on row i - NU - 2.
// Every stage keeps its sums in rolling form (Roll) and the right-hand sides
// of the last NU + 2 rows sit in a ring.  The loop body is unrolled over G = 6
// steps (the ring rotates and the row parity alternates at compile time);
// input rows are loaded 3 steps ahead.  Steps past the strip compute rows that
// are never stored.
template <typename T, int NU, int R>
__global__ void __launch_bounds__(256) k_pre_s(StageArgs a)
{
    constexpr int H = NU + 1, G = 6;
    constexpr int STEPS = R + 2 * H + 1, NG = (STEPS + G - 1) / G;
    Strip t;
    if (!get_strip<R>(a, t)) return;
    const InstDev& I = a.inst[t.inst];
    const int d = a.depth;
    const LevelDev& Lv = I.lev[d];
    const LevelDev& Lc = I.lev[d + 1];
    const int n = Lv.n, nc = Lc.n;
    const gp<const T> A = glob<T>((const void*)Lv.A);
    const gp<const T> F = glob<T>((const void*)Lv.F);
    const gp<T> B = glob<T>(Lv.B);
    const gp<T> Fc = glob<T>(Lc.F);
    const int lda = Lv.lda, ldf = Lv.ldf, ldb = Lv.ldb, ldc = Lc.ldf;
    const T fs = (T)Lv.fscale;
    Sten<T> s;
    s.load(P<T>::s(I, d));
    const T w = P<T>::w(I, d);
    const bool zg = a.zg != 0, stop = a.fin == FIN_STOP;
    const int lane = threadIdx.x & 63;
    const int x = t.x0 - H + lane;
    const bool col = t.live && (unsigned)x < (unsigned)n;
    const bool own = t.live && lane >= H && lane < H + SW && (unsigned)x < (unsigned)n;
    const bool fwc = own && (x & 1) && ((x - 1) >> 1) < nc;
    const int ylo = t.y0, yhi = min(t.y0 + R, n);   // rows this strip stores
    const int i0 = t.y0 - H;
    Acc2 nrm;

    Roll<T> sw[NU + 1];   // sw[k]: sweep k (k >= 1); sw[0]: the residual
    T fr[NU + 2];         // fr[j]: right-hand side of row i - j
#pragma unroll
    for (int j = 0; j < NU + 2; ++j) fr[j] = T(0);
    T fwp = T(0);         // full weighting of the next odd row: its south part, then its centre part

    // raw rows from clamped (always valid) addresses, masked when they become current;
    // a zero guess reads no estimate (F, with its own leading dimension, stands in)
    const gp<const T> Av = zg ? F : A;
    const size_t ldav = zg ? (size_t)ldf : (size_t)lda;
    const size_t xc = (size_t)clampi(x, n);
    auto load = [&](int i, T& v, T& f) {
        const size_t ic = (size_t)clampi(i, n);
        v = Av[ic * ldav + xc];
        f = F[ic * ldf + xc];
    };
    T pv[3], pf[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) load(i0 + u, pv[u], pf[u]);

    for (int g = 0; g < NG; ++g) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int i = i0 + g * G + u;
            const T rv = pv[u % 3], rf = pf[u % 3];
            load(i + 3, pv[u % 3], pf[u % 3]);
            const bool rin = col && (unsigned)i < (unsigned)n;
            const T vi = (rin && !zg) ? rv : T(0);
#pragma unroll
            for (int j = NU + 1; j > 0; --j) fr[j] = fr[j - 1];
            fr[0] = rin ? fs * rf : T(0);
            Row3<T> X = row3(vi);   // the newest row of the stage feeding the next one
            T top = vi;             // its own value
#pragma unroll
            for (int k = 1; k <= NU; ++k) {   // sweep k: row i - k
                const int r = i - k;
                const bool in = (unsigned)r < (unsigned)n && (unsigned)x < (unsigned)n;
                T centre;
                const T acc = roll(sw[k], s, X, centre);
                T val;
                if (k == 1 && zg) {
                    val = in ? w * fr[1] : T(0);
                } else {
                    const T res = fr[k] - acc;
                    val = in ? fmadd(w, res, centre) : T(0);
                    if (k == 1 && stop && own && r >= ylo && r < yhi) {
                        const double rd = (double)res;
                        nrm.add_sq(rd);
                    }
                }
                X = row3(val);
                top = val;
            }
            {   // smoothed row i - NU (with no sweeps on a zero guess the input rows are zeros)
                const int r = i - NU;
                if (own && r >= ylo && r < yhi) B[(size_t)r * ldb + x] = top;
            }
            Row3<T> Rr;
            {   // residual of row i - NU - 1
                const int r = i - NU - 1;
                const bool in = (unsigned)r < (unsigned)n && (unsigned)x < (unsigned)n;
                T centre;
                const T res = fr[NU + 1] - roll(sw[0], s, X, centre);
                if (NU == 0 && stop && !zg && own && r >= ylo && r < yhi) {
                    const double rd = (double)res;
                    nrm.add_sq(rd);
                }
                Rr = row3(in ? res : T(0));
            }
            {   // full weighting: residual row j = i - NU - 1 (its parity is that of u: y0 and
                // 2 H are even) is the centre row of the odd centre j, or the north row of
                // centre j - 1 (stored) and the south row of centre j + 1
                const T q = T(0.25), h = T(0.5);
                if ((u & 1) != 0) {
                    fwp += h * Rr.w;
                    fwp += T(1) * Rr.c;
                    fwp += h * Rr.e;
                } else {
                    T acc = fwp;
                    acc += q * Rr.w;
                    acc += h * Rr.c;
                    acc += q * Rr.e;
                    const int c = i - NU - 2;
                    if (fwc && c >= ylo && c < yhi) {
                        const int J = (c - 1) >> 1;
                        if (J < nc) Fc[(size_t)J * ldc + ((x - 1) >> 1)] = acc;
                    }
                    fwp = T(0);
                    fwp += q * Rr.w;
                    fwp += h * Rr.c;
                    fwp += q * Rr.e;
                }
            }
        }
    }
    if (stop) {
        Tile tt;
        tt.inst = t.inst;
        tt.blk = t.blk;
        reduce_partial(a, tt, nrm, Acc2());
    }
}

// post-smoothing: prolong-add + NU sweeps.  Step s reads row i = y0 - H + s,
// corrects it with the bilinear interpolant of the coarse solution and sweep
// k produces row i - k (sums in rolling form, right-hand sides in a ring).  A
// lane loads the coarse value at column (x - 1) / 2 of each coarse row once
// (every second step) and takes the value at the next coarse column from its
// east neighbour lane.
template <typename T, int NU, int R>
__global__ void __launch_bounds__(256) k_post_s(StageArgs a)
{
    constexpr int H = NU, G = 6;
    constexpr int STEPS = R + 2 * H, NG = (STEPS + G - 1) / G;
    Strip t;
    if (!get_strip<R>(a, t)) return;
    const InstDev& I = a.inst[t.inst];
    const int d = a.depth;
    const LevelDev& Lv = I.lev[d];
    const LevelDev& Lc = I.lev[d + 1];
    const int n = Lv.n, nc = Lc.n;
    const gp<T> A = glob<T>(Lv.A);
    const gp<const T> B = glob<T>((const void*)Lv.B);
    const gp<const T> F = glob<T>((const void*)Lv.F);
    const gp<const T> Vc = glob<T>((const void*)Lc.A);
    const int lda = Lv.lda, ldf = Lv.ldf, ldb = Lv.ldb, ldc = Lc.lda;
    const T fs = (T)Lv.fscale;
    Sten<T> s;
    s.load(P<T>::s(I, d));
    const T w = P<T>::w(I, d);
    const int lane = threadIdx.x & 63;
    const int x = t.x0 - H + lane;
    const bool col = t.live && (unsigned)x < (unsigned)n;
    const bool own = t.live && lane >= H && lane < H + SW && (unsigned)x < (unsigned)n;
    const int ylo = t.y0, yhi = min(t.y0 + R, n);
    const int i0 = t.y0 - H;
    const int Is = (x - 1) >> 1;                       // coarse column west of (or at) x
    const bool cin = t.live && (unsigned)Is < (unsigned)nc;
    const bool xodd = (x & 1) != 0;

    Roll<T> sw[NU + 1];   // sw[k]: sweep k (k >= 1)
    T fr[NU + 1];         // fr[j]: right-hand side of row i - j
#pragma unroll
    for (int j = 0; j < NU + 1; ++j) fr[j] = T(0);

    // raw rows from clamped (always valid) addresses, masked when they become current
    const size_t xc = (size_t)clampi(x, n), Ic = (size_t)clampi(Is, nc);
    auto load = [&](int i, T& v, T& f) {
        const size_t ic = (size_t)clampi(i, n);
        v = B[ic * ldb + xc];
        f = F[ic * ldf + xc];
    };
    auto craw = [&](int J) -> T { return Vc[(size_t)clampi(J, nc) * ldc + Ic]; };
    auto cmask = [&](int J, T v) -> T { return (cin && (unsigned)J < (unsigned)nc) ? v : T(0); };
    T pv[3], pf[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) load(i0 + u, pv[u], pf[u]);
    // coarse rows Js = (i - 1) >> 1 and Js + 1 of the current row i: ca (this lane's coarse
    // column), cb (the next one, from the east lane); row Js + 2 is prefetched raw
    int Jn = ((i0 - 1) >> 1) + 2;
    T ca0 = cmask(Jn - 2, craw(Jn - 2)), ca1 = cmask(Jn - 1, craw(Jn - 1));
    T cb0 = dpp<DPP_WAVE_SHL1>(ca0), cb1 = dpp<DPP_WAVE_SHL1>(ca1);
    T cr2 = craw(Jn);

    for (int g = 0; g < NG; ++g) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int i = i0 + g * G + u;
            const T rv = pv[u % 3], rf = pf[u % 3];
            load(i + 3, pv[u % 3], pf[u % 3]);
            const bool rin = col && (unsigned)i < (unsigned)n;
            const T vi = rin ? rv : T(0);
#pragma unroll
            for (int j = NU; j > 0; --j) fr[j] = fr[j - 1];
            fr[0] = rin ? fs * rf : T(0);
            // i0 = y0 - H with y0 even, so the parity of i is that of H + u (known at compile time);
            // an odd row starts a new coarse row pair (not at the first step: the pair is loaded)
            if (((H + u) & 1) != 0 && (u > 0 || g > 0)) {
                ca0 = ca1;
                cb0 = cb1;
                ca1 = cmask(Jn, cr2);
                cb1 = dpp<DPP_WAVE_SHL1>(ca1);
                ++Jn;
                cr2 = craw(Jn);
            }
            T e;
            if ((i & 1) != 0) e = xodd ? ca0 : T(0.5) * (ca0 + cb0);
            else e = xodd ? T(0.5) * (ca0 + ca1) : T(0.25) * (((ca0 + cb0) + ca1) + cb1);
            const bool in = col && (unsigned)i < (unsigned)n;
            const T uu = in ? vi + e : T(0);
            Row3<T> X = row3(uu);
            T top = uu;
#pragma unroll
            for (int k = 1; k <= NU; ++k) {
                const int r = i - k;
                const bool rk = (unsigned)r < (unsigned)n && (unsigned)x < (unsigned)n;
                T centre;
                const T acc = roll(sw[k], s, X, centre);
                const T val = rk ? fmadd(w, fr[k] - acc, centre) : T(0);
                X = row3(val);
                top = val;
            }
            const int r = i - NU;
            if (own && r >= ylo && r < yhi) A[(size_t)r * lda + x] = top;
        }
    }
}

// ---------------------------------------------------------------------------
// persistent coarse kernel: one workgroup runs whole calls of the cycle on the
// coarse levels of one instance, every level resident in LDS.  Each level d has
// three (n+2) x (n+2) arrays with a zero ring (two sweep buffers and F), so no
// stencil needs a bounds check.  Bit d of `cur` says which sweep buffer holds
// the current estimate of level d (sweeps ping-pong, nothing is copied).
// Levels with n > wave_n spread rows over all waves and end each phase with a
// workgroup barrier; levels with n <= wave_n are run by wave 0 alone, whose
// phases need only wave-level ordering, while the other waves wait at the next
// workgroup barrier.
// ---------------------------------------------------------------------------
// per-launch copy of everything the persistent kernel reads between phases:
// LDS keeps it out of global memory, whose latency would otherwise be paid
// once per phase (the phase fences forbid caching it in scalar registers)
template <typename T>
struct SubParams {
    static constexpr int OPS = 512, CH = 81;
    T s[MAXL][9];
    T w[MAXL];
    int n[MAXL];
    int off[MAXL];
    uint32_t ops[OPS];
    int nops[2];
    T chol[CH];
};

// LDS pointers: the phase functions are not inlined, so their arguments carry
// the LDS address space explicitly (generic pointers would compile to FLAT
// accesses, which are slower than ds_read / ds_write)
template <typename T> using lds = __attribute__((address_space(3))) T*;
template <typename T> using clds = const __attribute__((address_space(3))) T*;
template <typename T> __device__ __forceinline__ lds<T> to_lds(T* p) { return (lds<T>)(p); }
template <typename T> __device__ __forceinline__ clds<T> to_lds(const T* p) { return (clds<T>)(p); }

// One phase of the persistent kernel touches every interior point of one
// N x N level (N = 2^k - 1, known at compile time) once.  Arrays have a zero
// ring, row stride N + 2.  Point mapping: thread t belongs to band t / (N + 1)
// and column t mod (N + 1); band b owns the U = ceil(N / NB) consecutive rows
// from b U (NB bands in all: 64 / (N + 1) when wave 0 runs the level alone,
// threads / (N + 1) otherwise).  A lane loads the three columns around its
// own for rows b U - 1 .. b U + U once and forms all U stencils from those
// registers, computing every value before it stores any.  Column N (the ring)
// and rows past N are computed on clamped indices and never stored.  Each
// phase is a small out-of-line function: the kernel runs hundreds of phases
// per launch and inlining them all would not fit the instruction cache.
template <int N, int NB>
struct Band {
    static constexpr int B = N + 1, P = N + 2, U = (N + NB - 1) / NB;
};

// rows r0-1 .. r0+U of columns c-1, c, c+1 of x (padded indices clamped to the ring)
template <typename T, int N, int U>
__device__ __forceinline__ void load_rows(clds<T> x, int r0, int c, T (&w)[U + 2][3])
{
    constexpr int P = N + 2;
#pragma unroll
    for (int k = 0; k < U + 2; ++k) {
        const int pr = min(r0 + k, N + 1);
#pragma unroll
        for (int e = 0; e < 3; ++e) w[k][e] = x[pr * P + c + e];
    }
}

// fixed-order nine-point sum centred on window row k + 1 (south row first, west to east)
template <typename T, int U>
__device__ __forceinline__ T sten_win(const T (&s)[9], const T (&w)[U + 2][3], int k)
{
    T acc = T(0);
    acc = fmadd(s[0], w[k][0], acc);
    acc = fmadd(s[1], w[k][1], acc);
    acc = fmadd(s[2], w[k][2], acc);
    acc = fmadd(s[3], w[k + 1][0], acc);
    acc = fmadd(s[4], w[k + 1][1], acc);
    acc = fmadd(s[5], w[k + 1][2], acc);
    acc = fmadd(s[6], w[k + 2][0], acc);
    acc = fmadd(s[7], w[k + 2][1], acc);
    acc = fmadd(s[8], w[k + 2][2], acc);
    return acc;
}

// the U stencil sums of a window at once, coefficient by coefficient: each
// sum takes the same operations in the same order as sten_win, and the U
// independent sums are interleaved so that their latencies overlap
template <typename T, int U>
__device__ __forceinline__ void sten_win_all(const T (&s)[9], const T (&w)[U + 2][3], T (&acc)[U])
{
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = T(0);
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int e = 0; e < 3; ++e)
#pragma unroll
            for (int u = 0; u < U; ++u) acc[u] = fmadd(s[3 * b + e], w[u + b][e], acc[u]);
}

// y = x + w (F - S x) (Jacobi), or y = w F on a zero guess
template <typename T, int N, int NB>
__device__ __noinline__ void ph_sweep(clds<T> __restrict__ x, lds<T> __restrict__ y, clds<T> __restrict__ F,
                                     clds<T> __restrict__ sc, T om, int t, bool zg)
{
    using G = Band<N, NB>;
    constexpr int U = G::U, P = G::P;
    const int b = t / G::B, c = t % G::B;
    const int j0 = b * U;
    if (b >= NB || j0 >= N) return;
    const int cc = min(c, N - 1);
    T val[U];
    if (zg) {
#pragma unroll
        for (int u = 0; u < U; ++u) val[u] = om * F[(min(j0 + u, N - 1) + 1) * P + cc + 1];
    } else {
        T s[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) s[k] = sc[k];
        T w[U + 2][3];
        load_rows<T, N, U>(x, j0, cc, w);
        T acc[U];
        sten_win_all<T, U>(s, w, acc);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const T f = F[(min(j0 + u, N - 1) + 1) * P + cc + 1];
            val[u] = fmadd(om, f - acc[u], w[u + 1][1]);
        }
    }
    if (c < N) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j0 + u < N) y[(j0 + u + 1) * P + c + 1] = val[u];
    }
}

// r = F - S x
template <typename T, int N, int NB>
__device__ __noinline__ void ph_resid(clds<T> __restrict__ x, lds<T> __restrict__ r, clds<T> __restrict__ F,
                                     clds<T> __restrict__ sc, int t)
{
    using G = Band<N, NB>;
    constexpr int U = G::U, P = G::P;
    const int b = t / G::B, c = t % G::B;
    const int j0 = b * U;
    if (b >= NB || j0 >= N) return;
    const int cc = min(c, N - 1);
    T s[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) s[k] = sc[k];
    T w[U + 2][3];
    load_rows<T, N, U>(x, j0, cc, w);
    T val[U], acc[U];
    sten_win_all<T, U>(s, w, acc);
#pragma unroll
    for (int u = 0; u < U; ++u) val[u] = F[(min(j0 + u, N - 1) + 1) * P + cc + 1] - acc[u];
    if (c < N) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j0 + u < N) r[(j0 + u + 1) * P + c + 1] = val[u];
    }
}

// F_c = P^T r: coarse level NC = (N - 1) / 2 in the band mapping of NC (its own
// NB); coarse point (J, I) is centred on fine padded point (2J + 2, 2I + 2)
template <typename T, int NC, int NB>
__device__ __noinline__ void ph_restrict(clds<T> __restrict__ r, lds<T> __restrict__ Fc, int t)
{
    using G = Band<NC, NB>;
    constexpr int U = G::U, Pc = G::P, N = 2 * NC + 1, P = N + 2;
    const int b = t / G::B, c = t % G::B;
    const int J0 = b * U;
    if (b >= NB || J0 >= NC) return;
    const int cc = min(c, NC - 1);
    // fine padded rows 2 J0 + 1 .. 2 (J0 + U - 1) + 3, columns 2 cc + 1 .. 2 cc + 3
    T w[2 * U + 1][3];
#pragma unroll
    for (int k = 0; k < 2 * U + 1; ++k) {
        const int pr = min(2 * J0 + 1 + k, N + 1);
#pragma unroll
        for (int e = 0; e < 3; ++e) w[k][e] = r[pr * P + 2 * cc + 1 + e];
    }
    const T q = T(0.25), h = T(0.5);
    T val[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int k = 2 * u;
        T acc = T(0);
        acc += q * w[k][0];
        acc += h * w[k][1];
        acc += q * w[k][2];
        acc += h * w[k + 1][0];
        acc += T(1) * w[k + 1][1];
        acc += h * w[k + 1][2];
        acc += q * w[k + 2][0];
        acc += h * w[k + 2][1];
        acc += q * w[k + 2][2];
        val[u] = acc;
    }
    if (c < NC) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (J0 + u < NC) Fc[(J0 + u + 1) * Pc + c + 1] = val[u];
    }
}

// x += P vc (each point reads only its own x)
template <typename T, int N, int NB>
__device__ __noinline__ void ph_prolong(lds<T> __restrict__ x, clds<T> __restrict__ vc, int t)
{
    using G = Band<N, NB>;
    constexpr int U = G::U, P = G::P, Pc = (N - 1) / 2 + 2;
    const int b = t / G::B, c = t % G::B;
    const int j0 = b * U;
    if (b >= NB || j0 >= N) return;
    const int cc = min(c, N - 1);
    T val[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = min(j0 + u, N - 1);
        const T e = prolong_at<T>(j, cc, [&](int J, int I) { return vc[(J + 1) * Pc + (I + 1)]; });
        val[u] = x[(j + 1) * P + cc + 1] + e;
    }
    if (c < N) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j0 + u < N) x[(j0 + u + 1) * P + c + 1] = val[u];
    }
}

template <typename T, int N, int NB>
__device__ __noinline__ void ph_zero(lds<T> __restrict__ x, int t)
{
    using G = Band<N, NB>;
    constexpr int U = G::U, P = G::P;
    const int b = t / G::B, c = t % G::B;
    const int j0 = b * U;
    if (b >= NB || j0 >= N || c >= N) return;
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (j0 + u < N) x[(j0 + u + 1) * P + c + 1] = T(0);
}

// run phase PH on a level of size (1 << lg) - 1 in its band mapping: wave 0
// alone (single; levels up to 15 x 15) or the whole block of THREADS
#define KC_LEVEL_CASE(PH, LG, ...)                                                              \
    case LG: {                                                                                   \
        constexpr int NN = (1 << LG) - 1;                                                        \
        constexpr int NBM = THREADS / (NN + 1) > 0 ? THREADS / (NN + 1) : 1;                     \
        if constexpr (LG <= 4) {                                                                 \
            if (single) PH<T, NN, 64 / (NN + 1)>(__VA_ARGS__, threadIdx.x & 63);                \
            else PH<T, NN, NBM>(__VA_ARGS__, threadIdx.x);                                       \
        } else if constexpr (LG == 5 || THREADS >= 512) {                                        \
            PH<T, NN, NBM>(__VA_ARGS__, threadIdx.x);  /* 63 x 63 needs 512 threads */           \
        }                                                                                        \
        break;                                                                                   \
    }
#define KC_LEVEL_SWITCH(LGV, PH, ...)                                                           \
    switch (LGV) {                                                                               \
        KC_LEVEL_CASE(PH, 2, __VA_ARGS__)                                                        \
        KC_LEVEL_CASE(PH, 3, __VA_ARGS__)                                                        \
        KC_LEVEL_CASE(PH, 4, __VA_ARGS__)                                                        \
        KC_LEVEL_CASE(PH, 5, __VA_ARGS__)                                                        \
        KC_LEVEL_CASE(PH, 6, __VA_ARGS__)                                                        \
        default: break;                                                                          \
    }

// sweep with the zero-guess flag last (it follows the thread index in the phase signature)
template <typename T, int N, int NB>
__device__ __forceinline__ void ph_sweep_zg0(clds<T> x, lds<T> y, clds<T> F, clds<T> sc, T om, int t)
{
    ph_sweep<T, N, NB>(x, y, F, sc, om, t, false);
}
template <typename T, int N, int NB>
__device__ __forceinline__ void ph_sweep_zg1(clds<T> x, lds<T> y, clds<T> F, clds<T> sc, T om, int t)
{
    ph_sweep<T, N, NB>(x, y, F, sc, om, t, true);
}

// zebra relaxation of one colour on an N x N level in LDS (zero ring, stride
// N + 2), in place: thread t solves line 2 t + colour with the lane mapping of
// the grid kernel (same arithmetic, same order; the ring supplies the zeros
// that kernel masks in).  tab: the level's reciprocal pivots then upper
// multipliers for the direction, staged in LDS.  Each chunk of ZK points
// loads its neighbour values, right-hand sides and pivots before its stores.
template <typename T, int N, int DIR>
__device__ __forceinline__ void zebra_lds_line(lds<T> x, clds<T> F, clds<T> sc, clds<T> tab, int color, int t)
{
    constexpr int P = N + 2, ZK = 8;
    const int line = 2 * t + color;
    if (line >= N) return;
    auto at = [&](int L, int q) -> int { return DIR == 0 ? (L + 1) * P + (q + 1) : (q + 1) * P + (L + 1); };
    const T cm0 = sc[0], cm1 = DIR == 0 ? sc[1] : sc[3], cm2 = DIR == 0 ? sc[2] : sc[6];
    const T cp0 = DIR == 0 ? sc[6] : sc[2], cp1 = DIR == 0 ? sc[7] : sc[5], cp2 = sc[8];
    const T lo = DIR == 0 ? sc[3] : sc[1];
    T m0 = T(0), p0 = T(0);
    T m1 = x[at(line - 1, 0)], p1 = x[at(line + 1, 0)];
    T prev = T(0);
#pragma unroll
    for (int q0 = 0; q0 < N; q0 += ZK) {
        T mn[ZK], pn[ZK], fv[ZK], rv[ZK];
#pragma unroll
        for (int k = 0; k < ZK; ++k) {
            const int q = q0 + k;
            if (q < N) {
                mn[k] = x[at(line - 1, q + 1)];   // q + 1 = N reads the ring
                pn[k] = x[at(line + 1, q + 1)];
                fv[k] = F[at(line, q)];
                rv[k] = tab[q];
            }
        }
#pragma unroll
        for (int k = 0; k < ZK; ++k) {
            const int q = q0 + k;
            if (q < N) {
                T acc = T(0);
                acc = fmadd(cm0, m0, acc);
                acc = fmadd(cm1, m1, acc);
                acc = fmadd(cm2, mn[k], acc);
                acc = fmadd(cp0, p0, acc);
                acc = fmadd(cp1, p1, acc);
                acc = fmadd(cp2, pn[k], acc);
                const T dq = fv[k] - acc;
                const T y = (q == 0) ? dq * rv[k] : fmadd(-lo, prev, dq) * rv[k];
                x[at(line, q)] = y;
                prev = y;
                m0 = m1;
                m1 = mn[k];
                p0 = p1;
                p1 = pn[k];
            }
        }
    }
    T next = prev;   // x_{N-1} = y_{N-1}
#pragma unroll
    for (int q1 = N - 2; q1 >= 0; q1 -= ZK) {
        T yv[ZK], uv[ZK];
#pragma unroll
        for (int k = 0; k < ZK; ++k) {
            const int q = q1 - k;
            if (q >= 0) {
                yv[k] = x[at(line, q)];
                uv[k] = tab[N + q];
            }
        }
#pragma unroll
        for (int k = 0; k < ZK; ++k) {
            const int q = q1 - k;
            if (q >= 0) {
                const T v = fmadd(-uv[k], next, yv[k]);
                x[at(line, q)] = v;
                next = v;
            }
        }
    }
}
template <typename T, int N, int NB>
__device__ __noinline__ void ph_zebra0(lds<T> x, clds<T> F, clds<T> sc, clds<T> tab, int color, int t)
{
    zebra_lds_line<T, N, 0>(x, F, sc, tab, color, t);
}
template <typename T, int N, int NB>
__device__ __noinline__ void ph_zebra1(lds<T> x, clds<T> F, clds<T> sc, clds<T> tab, int color, int t)
{
    zebra_lds_line<T, N, 1>(x, F, sc, tab, color, t);
}

// LDS element offset of the zebra tables of a level of size 2^lg - 1 (lg >= 1)
// in the persistent kernel's table block: levels in increasing size, 4 n each
__host__ __device__ constexpr int zlds_off(int lg) { return 4 * ((1 << lg) - lg - 1); }
static_assert(zlds_off(7) == ZLDS_TABLE, "zebra table block");

// ---------------------------------------------------------------------------
// register engine: a whole call on a level that wave 0 runs alone (n <= 15),
// with every coarser level of that call, held in registers.  Level N uses
// bands of B = N + 1 lanes: lane b B + c is column c of rows b U .. b U + U - 1
// (U = 4 for N = 15, else 1); column N and rows >= N are the zero ring.
// East / west neighbours come from DPP row shifts (a band never straddles a
// 16-lane DPP row, and the lane across a band edge holds a ring zero), north /
// south ones across bands from lane permutes; restriction and prolongation
// gather between the layouts of two levels with lane permutes.  No LDS access
// and no synchronisation inside the call; arithmetic as in the LDS phases.
// ---------------------------------------------------------------------------
constexpr int DPP_WEST = 0x111;   // row_shr:1 -> value of lane - 1 (0 at a row start)
constexpr int DPP_EAST = 0x101;   // row_shl:1 -> value of lane + 1 (0 at a row end)

template <int N> struct WL {
    static constexpr int B = N + 1, U = (N == 15) ? 4 : 1, LOGB = (N == 15) ? 4 : (N == 7) ? 3 : (N == 3) ? 2 : 1;
};

template <typename T> struct WRow {   // one row around a lane: west, centre, east
    T w, c, e;
};
template <typename T> __device__ __forceinline__ WRow<T> wrow(T v)
{
    return WRow<T>{dpp<DPP_WEST>(v), v, dpp<DPP_EAST>(v)};
}

// rows -1 .. U of this lane's band for a level of size N, from the lane's U values
template <typename T, int N>
__device__ __forceinline__ void wwin(const T (&v)[WL<N>::U], WRow<T> (&r)[WL<N>::U + 2])
{
    constexpr int B = WL<N>::B, U = WL<N>::U;
    const int lane = threadIdx.x & 63;
    const T s = __shfl_up(v[U - 1], B, 64);     // last row of the band below
    const T n = __shfl_down(v[0], B, 64);       // first row of the band above
    r[0] = wrow(lane >= B ? s : T(0));
#pragma unroll
    for (int u = 0; u < U; ++u) r[u + 1] = wrow(v[u]);
    r[U + 1] = wrow(n);
}

template <typename T>
__device__ __forceinline__ T wsten(const T (&s)[9], const WRow<T>& S, const WRow<T>& C, const WRow<T>& N)
{
    T acc = T(0);
    acc = fmadd(s[0], S.w, acc);
    acc = fmadd(s[1], S.c, acc);
    acc = fmadd(s[2], S.e, acc);
    acc = fmadd(s[3], C.w, acc);
    acc = fmadd(s[4], C.c, acc);
    acc = fmadd(s[5], C.e, acc);
    acc = fmadd(s[6], N.w, acc);
    acc = fmadd(s[7], N.c, acc);
    acc = fmadd(s[8], N.e, acc);
    return acc;
}

// the stencil sums of all U rows of a lane at once (each as wsten, the rows interleaved)
template <typename T, int U>
__device__ __forceinline__ void wsten_all(const T (&s)[9], const WRow<T> (&r)[U + 2], T (&acc)[U])
{
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = T(0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = fmadd(s[3 * b], r[u + b].w, acc[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = fmadd(s[3 * b + 1], r[u + b].c, acc[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = fmadd(s[3 * b + 2], r[u + b].e, acc[u]);
    }
}

template <int N> __device__ __forceinline__ bool wvalid(int u)
{
    const int lane = threadIdx.x & 63;
    const int b = lane >> WL<N>::LOGB, c = lane & (WL<N>::B - 1);
    return b * WL<N>::U + u < N && c < N;
}

// stencils and Jacobi weights of the levels below a register call, relative depth 0 = the call's level
template <typename T> struct WPar {
    T s[4][9];
    T w[4];
    T chol;   // coarsest 1 x 1 factor
    int nu1, nu2;
};

template <typename T, int N>
__device__ __forceinline__ void wsweep(T (&v)[WL<N>::U], const T (&f)[WL<N>::U], const T (&s)[9], T om, bool zg)
{
    constexpr int U = WL<N>::U;
    T nv[U];
    if (zg) {
#pragma unroll
        for (int u = 0; u < U; ++u) nv[u] = wvalid<N>(u) ? om * f[u] : T(0);
    } else {
        WRow<T> r[U + 2];
        wwin<T, N>(v, r);
        T acc[U];
        wsten_all<T, U>(s, r, acc);
#pragma unroll
        for (int u = 0; u < U; ++u) nv[u] = wvalid<N>(u) ? fmadd(om, f[u] - acc[u], r[u + 1].c) : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = nv[u];
}

template <typename T, int N, int REL>
__device__ __forceinline__ void wcycle(T (&v)[WL<N>::U], const T (&f)[WL<N>::U], int k, bool zg, const WPar<T>& P)
{
    constexpr int U = WL<N>::U, B = WL<N>::B;
    const int lane = threadIdx.x & 63;
    if constexpr (N == 1) {
        // direct solve of the 1 x 1 level (Cholesky factor L: v = (f / L) / L); ignores the input v
        T x = f[0] / P.chol;
        x = x / P.chol;
        v[0] = (lane == 0) ? x : T(0);
        (void)k;
        (void)zg;
        (void)B;
    } else {
        constexpr int NC = (N - 1) / 2, BC = WL<NC>::B;
        static_assert(WL<NC>::U == 1, "coarse levels of a register call hold one row per band");
        const T(&s)[9] = P.s[REL];
        const T om = P.w[REL];
        // pre-smoothing
        for (int q = 0; q < P.nu1; ++q) wsweep<T, N>(v, f, s, om, zg && q == 0);
        if (zg && P.nu1 == 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = T(0);
        }
        // residual and its full weighting (kept at every fine point; the centres are gathered)
        T r[U];
        {
            WRow<T> w[U + 2];
            wwin<T, N>(v, w);
            T acc[U];
            wsten_all<T, U>(s, w, acc);
#pragma unroll
            for (int u = 0; u < U; ++u) r[u] = wvalid<N>(u) ? f[u] - acc[u] : T(0);
        }
        T fw[U];
        {
            WRow<T> w[U + 2];
            wwin<T, N>(r, w);
            const T fwc[9] = {T(0.25), T(0.5), T(0.25), T(0.5), T(1), T(0.5), T(0.25), T(0.5), T(0.25)};
            wsten_all<T, U>(fwc, w, fw);   // full weighting: the same nine-term order, the rows interleaved
        }
        T fc[1], vc[1];
        {
            const int J = lane >> WL<NC>::LOGB, I = lane & (BC - 1);
            const bool cval = J < NC && I < NC;
            const int jf = 2 * J + 1, cf = 2 * I + 1;
            const int src = cval ? (jf / U) * B + cf : 0;
            T g = __shfl(fw[0], src, 64);
            if constexpr (U == 4) {
                const T g3 = __shfl(fw[3], src, 64);
                const T g1 = __shfl(fw[1], src, 64);
                g = ((jf & 3) == 1) ? g1 : g3;
            }
            fc[0] = cval ? g : T(0);
            vc[0] = T(0);
        }
        wcycle<T, NC, REL + 1>(vc, fc, k, true, P);
        if (k > 1) wcycle<T, NC, REL + 1>(vc, fc, k - 1, false, P);
        // prolongation: coarse value (J, I) lives on lane J BC + I of the coarse layout
        {
            const int b = lane >> WL<N>::LOGB, c = lane & (B - 1);
            const int Is = (c - 1) >> 1;
            const bool io = (c & 1) != 0;
            auto cv = [&](int J, int I) -> T {
                const bool ok = J >= 0 && I >= 0;
                const T x = __shfl(vc[0], ok ? J * BC + I : 0, 64);
                return ok ? x : T(0);
            };
            // coarse rows (j - 1) >> 1 and the one above for the band's rows
            constexpr int NR = (U == 4) ? 3 : 2;
            T a0[NR], a1[NR];
            const int J0 = (U == 4) ? 2 * b - 1 : (b - 1) >> 1;
#pragma unroll
            for (int m = 0; m < NR; ++m) {
                a0[m] = cv(J0 + m, Is);
                a1[m] = cv(J0 + m, Is + 1);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = b * U + u;
                const int m = ((j - 1) >> 1) - J0;   // row index of (j - 1) >> 1 in a0 / a1
                const T A0 = a0[m < 0 ? 0 : (m >= NR ? NR - 1 : m)], A1 = a1[m < 0 ? 0 : (m >= NR ? NR - 1 : m)];
                const int m1 = (m + 1 >= NR) ? NR - 1 : m + 1;
                const T C0 = a0[m1 < 0 ? 0 : m1], C1 = a1[m1 < 0 ? 0 : m1];
                T e;
                if (j & 1) e = io ? A0 : T(0.5) * (A0 + A1);
                else e = io ? T(0.5) * (A0 + C0) : T(0.25) * (((A0 + A1) + C0) + C1);
                v[u] = wvalid<N>(u) ? v[u] + e : T(0);
            }
        }
        for (int q = 0; q < P.nu2; ++q) wsweep<T, N>(v, f, s, om, false);
    }
}

// a register call on level d (size N) of the persistent kernel: f (and v
// unless zg) from the level's LDS arrays, the result back to buffer `cb`
template <typename T, int N>
__device__ __noinline__ void wcall_level(lds<T> vbuf, clds<T> fbuf, clds<T> sd, clds<T> wd, clds<T> chol, int nu1,
                                         int nu2, int k, bool zg)
{
    constexpr int U = WL<N>::U, P = N + 2;
    const int lane = threadIdx.x & 63;
    const int b = lane >> WL<N>::LOGB, c = lane & (WL<N>::B - 1);
    WPar<T> par;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
#pragma unroll
        for (int q = 0; q < 9; ++q) par.s[l][q] = sd[l * 9 + q];
        par.w[l] = wd[l];
    }
    par.chol = chol[0];
    par.nu1 = nu1;
    par.nu2 = nu2;
    T v[U], f[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = b * U + u;
        const bool ok = j < N && c < N;
        const int q = ok ? (j + 1) * P + c + 1 : 0;
        f[u] = ok ? fbuf[q] : T(0);
        v[u] = (ok && !zg) ? vbuf[q] : T(0);
    }
    wcycle<T, N, 0>(v, f, k, zg, par);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = b * U + u;
        if (j < N && c < N) vbuf[(j + 1) * P + c + 1] = v[u];
    }
}

// ZEB: the levels relax by alternating zebra line relaxation (in place, no
// buffer swaps; tables in the LDS block zt) instead of damped Jacobi
template <typename T, int THREADS, bool ZEB>
struct Sub {
    T* sm;
    const SubParams<T>* pp;
    const InstDev* I;
    int nu1, nu2, wave_n;
    uint32_t cur;           // bit d: current estimate of level d is in the second buffer
    T* zt = nullptr;
    bool pending = false;   // wave 0 has written LDS since the last workgroup barrier

    // level d of size n = 2^lg - 1 starts at LDS element off: buffers 0 and 1 (sweeps), 2 (F)
    __device__ __forceinline__ T* bufp(int off, int lg, int which) const
    {
        const int P = (1 << lg) + 1;
        return sm + off + which * P * P;
    }
    __device__ __forceinline__ bool single_lg(int lg) const { return (1 << lg) - 1 <= wave_n; }
    __device__ __forceinline__ void sync_lg(int lg) const
    {
        if (single_lg(lg)) wave_sync();
        else __syncthreads();
    }

    // zebra: a zero-guess call starts from v = 0; relaxation r runs x-lines (r even)
    // or y-lines (r odd), lines of even index first
    __device__ __forceinline__ void zebra_sweeps(int d, int lg, int off, int nu, bool zg)
    {
        const bool single = single_lg(lg);
        const int n = (1 << lg) - 1;
        const lds<T> x = to_lds<T>(bufp(off, lg, (cur >> d) & 1));
        if (zg) {
            KC_LEVEL_SWITCH(lg, ph_zero, x)
            sync_lg(lg);
        }
        const clds<T> F = to_lds<T>((const T*)bufp(off, lg, 2));
        const clds<T> sc = to_lds<T>(&pp->s[d][0]);
        for (int k = 0; k < nu; ++k) {
            const clds<T> tab = to_lds<T>((const T*)(zt + zlds_off(lg) + (k & 1) * 2 * n));
            for (int color = 0; color < 2; ++color) {
                if (k & 1) { KC_LEVEL_SWITCH(lg, ph_zebra1, x, F, sc, tab, color) }
                else { KC_LEVEL_SWITCH(lg, ph_zebra0, x, F, sc, tab, color) }
                sync_lg(lg);
            }
        }
    }

    __device__ __forceinline__ void sweeps(int d, int lg, int off, int nu, bool zg)
    {
        if constexpr (ZEB) {
            zebra_sweeps(d, lg, off, nu, zg);
            return;
        }
        const bool single = single_lg(lg);
        const clds<T> F = to_lds<T>((const T*)bufp(off, lg, 2));
        const clds<T> sc = to_lds<T>(&pp->s[d][0]);
        const T om = pp->w[d];
        for (int k = 0; k < nu; ++k) {
            const int cb = (cur >> d) & 1;
            const clds<T> x = to_lds<T>((const T*)bufp(off, lg, cb));
            const lds<T> y = to_lds<T>(bufp(off, lg, cb ^ 1));
            if (zg && k == 0) { KC_LEVEL_SWITCH(lg, ph_sweep_zg1, x, y, F, sc, om) }
            else { KC_LEVEL_SWITCH(lg, ph_sweep_zg0, x, y, F, sc, om) }
            sync_lg(lg);
            cur ^= 1u << d;
        }
        if (zg && nu == 0) {
            const bool single = single_lg(lg);
            const lds<T> x = to_lds<T>(bufp(off, lg, (cur >> d) & 1));
            KC_LEVEL_SWITCH(lg, ph_zero, x)
            sync_lg(lg);
        }
    }

    __device__ __forceinline__ void pre(int d, int lg, int off, bool zg)
    {
        sweeps(d, lg, off, nu1, zg);
        const int P = (1 << lg) + 1, offc = off + 3 * P * P;
        const int cb = (cur >> d) & 1;
        {
            const bool single = single_lg(lg);
            KC_LEVEL_SWITCH(lg, ph_resid, to_lds<T>((const T*)bufp(off, lg, cb)), to_lds<T>(bufp(off, lg, cb ^ 1)),
                            to_lds<T>((const T*)bufp(off, lg, 2)), to_lds<T>(&pp->s[d][0]))
            sync_lg(lg);
        }
        {
            const int lgc = lg - 1;
            const bool single = single_lg(lgc);
            const clds<T> r = to_lds<T>((const T*)bufp(off, lg, cb ^ 1));
            const lds<T> Fc = to_lds<T>(bufp(offc, lgc, 2));
            if (lgc == 1) {
                if (single) ph_restrict<T, 1, 32>(r, Fc, threadIdx.x & 63);
                else ph_restrict<T, 1, THREADS / 2>(r, Fc, threadIdx.x);
            } else {
                KC_LEVEL_SWITCH(lgc, ph_restrict, r, Fc)
            }
            sync_lg(lgc);
        }
    }

    __device__ __forceinline__ void post(int d, int lg, int off)
    {
        const int P = (1 << lg) + 1, offc = off + 3 * P * P;
        {
            const bool single = single_lg(lg);
            const lds<T> x = to_lds<T>(bufp(off, lg, (cur >> d) & 1));
            const clds<T> vc = to_lds<T>((const T*)bufp(offc, lg - 1, (cur >> (d + 1)) & 1));
            KC_LEVEL_SWITCH(lg, ph_prolong, x, vc)
            sync_lg(lg);
        }
        sweeps(d, lg, off, nu2, false);
    }

    __device__ __forceinline__ void solve(int d, int lg, int off)
    {
        const int n = (1 << lg) - 1;
        const T* Lc = (n * n * n * n <= SubParams<T>::CH) ? pp->chol : P<T>::chol(*I);
        if (threadIdx.x == 0) chol_solve_padded<T>(n, Lc, bufp(off, lg, 2), bufp(off, lg, (cur >> d) & 1), n + 2);
        sync_lg(lg);
    }

    // a whole call on level d in registers (wave 0); the result goes to the level's current buffer
    __device__ __forceinline__ void wcall(int d, int lg, int off, int k, bool zg)
    {
        const lds<T> vb = to_lds<T>(bufp(off, lg, (cur >> d) & 1));
        const clds<T> fb = to_lds<T>((const T*)bufp(off, lg, 2));
        const clds<T> sd = to_lds<T>(&pp->s[d][0]);
        const clds<T> wd = to_lds<T>(&pp->w[d]);
        const clds<T> ch = to_lds<T>(&pp->chol[0]);
        switch (lg) {
        case 4: wcall_level<T, 15>(vb, fb, sd, wd, ch, nu1, nu2, k, zg); break;
        case 3: wcall_level<T, 7>(vb, fb, sd, wd, ch, nu1, nu2, k, zg); break;
        case 2: wcall_level<T, 3>(vb, fb, sd, wd, ch, nu1, nu2, k, zg); break;
        case 1: wcall_level<T, 1>(vb, fb, sd, wd, ch, nu1, nu2, k, zg); break;
        default: break;
        }
        wave_sync();
    }

    // waves that skip a wave-0 operation still follow its buffer swaps
    __device__ __forceinline__ void skip(int kind, int d, bool zg)
    {
        if constexpr (ZEB) return;   // zebra relaxes in place
        int k = 0;
        if (kind == SOP_PRE) k = (zg && nu1 == 0) ? 0 : nu1;
        else if (kind == SOP_POST) k = nu2;
        if (k & 1) cur ^= 1u << d;
    }

    // the operations of one call (list `which` of the staged op lists)
    __device__ void call(int which)
    {
        const int base = which ? pp->nops[0] : 0;
        const int nops = pp->nops[which];
        const bool w0 = (threadIdx.x >> 6) == 0;
        for (int o = 0; o < nops; ++o) {
            const uint32_t op = pp->ops[base + o];
            const int kind = sop_kind(op), d = sop_depth(op), lg = sop_lg(op), off = sop_off(op);
            const bool zg = sop_zg(op);
            const bool sg = single_lg(lg);
            if (sg && !w0) {
                skip(kind, d, zg);
                pending = true;
                continue;
            }
            if (!sg && pending) {
                __syncthreads();
                pending = false;
            }
            if (kind == SOP_WCALL) wcall(d, lg, off, sop_k(op), zg);
            else if (kind == SOP_PRE) pre(d, lg, off, zg);
            else if (kind == SOP_POST) post(d, lg, off);
            else solve(d, lg, off);
            if (sg || (kind == SOP_PRE && single_lg(lg - 1))) pending = true;
        }
    }
};

// top level (N x N) of a persistent launch: F (scaled) and A (unless zero) are
// loaded into registers, the tables staged (stage()), and after a barrier the
// values go to the level's LDS arrays (F in the third, A in the first buffer);
// false when the instance is finished (checked once the loads are in flight)
template <typename T, int THREADS, int N, typename Stage>
__device__ __forceinline__ bool top_level_in(gp<const T> Fg, gp<const T> Ag, int ldf, int lda, T fs, bool zero, bool done,
                                             T* lev, Stage stage)
{
    constexpr int NN = N * N, NP = (NN + THREADS - 1) / THREADS, P = N + 2;
    T fr[NP], ar[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int p = min((int)threadIdx.x + k * THREADS, NN - 1);
        const int j = p / N, i = p - j * N;
        fr[k] = Fg[(size_t)j * ldf + i];
        ar[k] = zero ? T(0) : Ag[(size_t)j * lda + i];
    }
    stage();
    if (done) return false;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int p = (int)threadIdx.x + k * THREADS;
        if (p < NN) {
            const int j = p / N, i = p - j * N;
            lev[2 * P * P + (j + 1) * P + (i + 1)] = fs * fr[k];
            if (!zero) lev[(j + 1) * P + (i + 1)] = ar[k];
        }
    }
    __syncthreads();
    return true;
}

template <typename T, int THREADS, bool ZEB>
__global__ void __launch_bounds__(THREADS) k_subtree(SubArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ SubParams<T> pp;
    // a launch for a single instance names it in its arguments (no list load first)
    const int inst = (a.count == 1) ? a.first : a.list[blockIdx.x];
    const InstDev& I = a.inst[inst];
    const bool done = a.st[inst].done != 0;   // checked once the loads below are in flight
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int d0 = a.depth, L = I.L;

    // the top level's F (and A) are loaded into registers first, so that they are in
    // flight while the tables are staged; the load count is exact for the level size.
    // A single-instance launch on an internal level carries the table entries these
    // loads need (a.ops1 set), so that no load waits for another
    const bool fast = a.ops1 != nullptr;
    const LevelDev& Lv = I.lev[d0];
    const int n = fast ? a.n0 : Lv.n;
    const T fs = (T)(fast ? a.fs0 : Lv.fscale);
    const gp<const T> Fg = glob<T>(fast ? a.F0 : (const void*)Lv.F);
    const gp<T> Ag = glob<T>(fast ? a.A0 : Lv.A);
    const int ldf = fast ? a.ldf0 : Lv.ldf, lda = fast ? a.lda0 : Lv.lda;
    const int sub_lds = fast ? a.sub_lds : I.sub_lds;
    const T* const chol = fast ? (const T*)a.chol0 : P<T>::chol(I);
    const bool zero = a.pair || a.zg;
    const int k1 = min(a.kappa, MAXL + 1), k2 = min(max(a.kappa - 1, 1), MAXL + 1);
    // zebra calls use op lists without register calls
    const int32_t* const obeg = ZEB ? I.zops_beg : I.ops_beg;
    const int32_t* const olen = ZEB ? I.zops_len : I.ops_len;
    const int n1 = fast ? a.n1 : olen[k1 - 1];
    const int n2 = fast ? a.n2 : ((a.pair && a.kappa > 1) ? olen[k2 - 1] : 0);
    auto stage = [&]() {   // parameters, op lists and a small coarsest factor into LDS; LDS levels zeroed
        if (fast) {
            for (int t = threadIdx.x; t < n1 + n2; t += blockDim.x)
                pp.ops[t] = (t < n1) ? a.ops1[t] : a.ops2[t - n1];
        } else {
            for (int t = threadIdx.x; t < n1 + n2; t += blockDim.x)
                pp.ops[t] = (t < n1) ? I.ops[obeg[k1 - 1] + t] : I.ops[obeg[k2 - 1] + (t - n1)];
        }
        for (int t = threadIdx.x; t < MAXL * 9; t += blockDim.x) {
            const int d = t / 9;
            pp.s[d][t % 9] = (d < L) ? P<T>::s(I, d)[t % 9] : T(0);
        }
        if (threadIdx.x < MAXL) {
            const int d = threadIdx.x;
            pp.w[d] = (d < L) ? P<T>::w(I, d) : T(0);
            pp.n[d] = (d < L) ? I.lev[d].n : 0;
            pp.off[d] = I.lds_off[d];
        }
        if (threadIdx.x == 0) {
            pp.nops[0] = n1;
            pp.nops[1] = n2;
        }
        if (I.nc2 * I.nc2 <= SubParams<T>::CH)
            for (int t = threadIdx.x; t < I.nc2 * I.nc2; t += blockDim.x) pp.chol[t] = chol[t];
        for (int p = threadIdx.x; p < sub_lds; p += blockDim.x) sm[p] = T(0);
        if constexpr (ZEB) {   // line-solve tables of the relaxed levels, after the level arrays
            for (int dd = d0; dd < L - 1; ++dd) {
                const int nn = I.lev[dd].n, lgd = 32 - __clz(nn);
                const T* src = ZT<T>::t(I, dd);
                T* dst = sm + I.sub_lds + zlds_off(lgd);
                for (int p = threadIdx.x; p < 4 * nn; p += blockDim.x) dst[p] = src[p];
            }
        }
    };
    // level sizes are 2^k - 1 <= cutover <= 63; the host accepts a 63 x 63 top level only with 512 threads
    T* const lev = sm + I.lds_off[d0];
    bool live = false;
    switch (n) {
    case 1: live = top_level_in<T, THREADS, 1>(Fg, Ag, ldf, lda, fs, zero, done, lev, stage); break;
    case 3: live = top_level_in<T, THREADS, 3>(Fg, Ag, ldf, lda, fs, zero, done, lev, stage); break;
    case 7: live = top_level_in<T, THREADS, 7>(Fg, Ag, ldf, lda, fs, zero, done, lev, stage); break;
    case 15: live = top_level_in<T, THREADS, 15>(Fg, Ag, ldf, lda, fs, zero, done, lev, stage); break;
    case 31: live = top_level_in<T, THREADS, 31>(Fg, Ag, ldf, lda, fs, zero, done, lev, stage); break;
    default:
        if constexpr (THREADS >= 512) live = top_level_in<T, THREADS, 63>(Fg, Ag, ldf, lda, fs, zero, done, lev, stage);
        break;
    }
    if (!live) return;   // the whole workgroup leaves together

    Sub<T, THREADS, ZEB> S{sm, &pp, &I, a.nu1, a.nu2, a.wave_n, 0u};
    if constexpr (ZEB) S.zt = sm + I.sub_lds;
    const int Pst = n + 2, off0 = pp.off[d0];
    const int lg0 = 32 - __clz(n);   // n = 2^lg0 - 1
    T* v0 = S.bufp(off0, lg0, 0);
    T* f0 = S.bufp(off0, lg0, 2);

    if (a.fin == FIN_STOP) {
        __shared__ double red[32];
        __shared__ int stop;
        Sten<T> s;
        s.load(pp.s[d0]);
        Acc2 nrm;
        for (int p = threadIdx.x; p < n * n; p += blockDim.x) {
            const int j = p / n, i = p - j * n;
            const int q = (j + 1) * Pst + (i + 1);
            const double r = (double)(f0[q] - s.apply(&v0[q], Pst));
            nrm.add_sq(r);
        }
        wave_merge(nrm);
        if ((threadIdx.x & 63) == 0) {
            red[2 * (threadIdx.x >> 6)] = nrm.s;
            red[2 * (threadIdx.x >> 6) + 1] = nrm.c;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            Acc2 ss;
            for (int k = 0; k < (int)(blockDim.x >> 6); ++k) ss.merge(red[2 * k], red[2 * k + 1]);
            stop_test(a.st[inst], a.hist, inst, ss.value());
            stop = a.st[inst].done;
        }
        __syncthreads();
        if (stop) return;
    }

    S.call(0);
    if (n2 > 0) S.call(1);
    __syncthreads();
    const T* vr = S.bufp(off0, lg0, (S.cur >> d0) & 1);
    for (int p = threadIdx.x; p < n * n; p += blockDim.x) {
        const int j = p / n, i = p - j * n;
        Ag[(size_t)j * lda + i] = vr[(j + 1) * Pst + (i + 1)];
    }
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
// Each thread owns DR = TY / 4 consecutive rows of one column of a 64 x 32
// tile.  All loads of a thread are issued before its first store (clamped
// addresses, masked at use), so they are in flight together; a store between
// two rows' loads would make the second row wait for the first (the compiler
// cannot tell the arrays apart).  Stencil kinds keep a three-column window of
// DR + 2 rows; every point is summed in the order of gapply.
constexpr int DR = TY / (GRID_THREADS / 64);

template <typename T>
struct DWin {
    double v[DR + 2][3];
    __device__ __forceinline__ void load(gp<const T> x, int ld, int n, int jb, int i)
    {
#pragma unroll
        for (int r = 0; r < DR + 2; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) v[r][c] = (double)gload(x, ld, n, jb - 1 + r, i - 1 + c);
    }
    // stencil sum at the window's row r (grid row jb + r)
    __device__ __forceinline__ double apply(const Sten<double>& s, int r) const
    {
        double acc = 0.0;
        acc = fmadd(s.c[0], v[r][0], acc);
        acc = fmadd(s.c[1], v[r][1], acc);
        acc = fmadd(s.c[2], v[r][2], acc);
        acc = fmadd(s.c[3], v[r + 1][0], acc);
        acc = fmadd(s.c[4], v[r + 1][1], acc);
        acc = fmadd(s.c[5], v[r + 1][2], acc);
        acc = fmadd(s.c[6], v[r + 2][0], acc);
        acc = fmadd(s.c[7], v[r + 2][1], acc);
        acc = fmadd(s.c[8], v[r + 2][2], acc);
        return acc;
    }
};

template <bool F32, int kind>
__global__ void __launch_bounds__(GRID_THREADS) k_driver(StageArgs a)
{
    Tile t;
    if (!get_tile(a, 0, true, t)) return;
    const InstDev& I = a.inst[t.inst];
    InstState& st = a.st[t.inst];
    const int n = I.n0;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int i = t.x0 + tx, jb = t.y0 + ty * DR;
    const int ic = clampi(i, n);
    Sten<double> s;
    s.load(I.s64[0]);
    const double h2 = I.h2;
    Acc2 acc0, acc1;
    const LevelDev& L0 = I.lev[0];
    const double scale = st.scale, scale_used = st.scale_used;
    const double alpha = st.alpha, beta = st.beta;
    const bool first = st.iters == 0;
    const gp<double> U = glob<double>(I.u), R = glob<double>(I.r), Z = glob<double>(I.z), Pv = glob<double>(I.p),
                     Q = glob<double>(I.q), Y = glob<double>(I.y);
    const gp<const double> Fv = glob<double>((const void*)I.f), X = glob<double>((const void*)I.x);
    const gp<const double> Yc = glob<double>((const void*)I.y), Pc = glob<double>((const void*)I.p),
                           Uc = glob<double>((const void*)I.u), Rc = glob<double>((const void*)I.r),
                           Zc = glob<double>((const void*)I.z), Qc = glob<double>((const void*)I.q);
    const gp<float> F32f = glob<float>(L0.F);
    const gp<const float> A32 = glob<float>((const void*)L0.A);
    const gp<const double> A64 = glob<double>((const void*)L0.A);
    // row offsets (clamped rows: every address is inside the arrays)
    auto rowu = [&](int r) { return (size_t)clampi(jb + r, n) * I.ldu + ic; };
    auto rowf = [&](int r) { return (size_t)clampi(jb + r, n) * I.ldf + ic; };
    auto rowv = [&](int r) { return (size_t)clampi(jb + r, n) * I.ldv + ic; };
    auto row0 = [&](int r) { return (size_t)clampi(jb + r, n) * L0.lda + ic; };   // FP32 level-0 arrays share one ld
    auto ok = [&](int r) { return jb + r < n && i < n; };

    if constexpr (kind == GK_SSF) {
        double F[DR];
#pragma unroll
        for (int r = 0; r < DR; ++r) F[r] = Fv[rowf(r)];
#pragma unroll
        for (int r = 0; r < DR; ++r) {
            const double f = h2 * F[r];
            if (ok(r)) acc0.add_sq(f);
        }
    } else if constexpr (kind == GK_IR_RESID) {
        DWin<double> w;
        w.load(Uc, I.ldu, n, jb, i);
        double F[DR];
#pragma unroll
        for (int r = 0; r < DR; ++r) F[r] = Fv[rowf(r)];
#pragma unroll
        for (int r = 0; r < DR; ++r) {
            const double res = h2 * F[r] - w.apply(s, r);
            if (ok(r)) {
                acc0.add_sq(res);
                if (F32) F32f[row0(r)] = (float)(scale * res);
            }
        }
    } else if constexpr (kind == GK_IR_UPDATE) {
        double E[DR], V[DR];
#pragma unroll
        for (int r = 0; r < DR; ++r) {
            E[r] = F32 ? (double)A32[row0(r)] : A64[row0(r)];
            V[r] = Uc[rowu(r)];
        }
#pragma unroll
        for (int r = 0; r < DR; ++r)
            if (ok(r)) U[rowu(r)] = V[r] + E[r] / scale_used;
    } else if constexpr (kind == GK_PCG_INIT) {
        double F[DR];
#pragma unroll
        for (int r = 0; r < DR; ++r) F[r] = Fv[rowf(r)];
#pragma unroll
        for (int r = 0; r < DR; ++r) {
            const double f = h2 * F[r];
            if (ok(r)) {
                U[rowu(r)] = 0.0;
                R[rowv(r)] = f;
                acc0.add_sq(f);
            }
        }
    } else if constexpr (kind == GK_PCG_PRECIN) {
        double V[DR];
#pragma unroll
        for (int r = 0; r < DR; ++r) V[r] = Rc[rowv(r)];
#pragma unroll
        for (int r = 0; r < DR; ++r)
            if (ok(r)) F32f[row0(r)] = (float)(scale * V[r]);
    } else if constexpr (kind == GK_PCG_RZ) {
        double E[DR], V[DR];
#pragma unroll
        for (int r = 0; r < DR; ++r) {
            E[r] = F32 ? (double)A32[row0(r)] : Zc[rowv(r)];
            V[r] = Rc[rowv(r)];
        }
#pragma unroll
        for (int r = 0; r < DR; ++r) {
            const double z = F32 ? E[r] / scale : E[r];
            if (ok(r)) {
                if (F32) Z[rowv(r)] = z;
                acc0.add_prod(V[r], z);
            }
        }
    } else if constexpr (kind == GK_PCG_P) {
        double E[DR], V[DR];
#pragma unroll
        for (int r = 0; r < DR; ++r) {
            E[r] = Zc[rowv(r)];
            V[r] = first ? 0.0 : Pc[rowv(r)];
        }
#pragma unroll
        for (int r = 0; r < DR; ++r)
            if (ok(r)) Pv[rowv(r)] = first ? E[r] : E[r] + beta * V[r];
    } else if constexpr (kind == GK_PCG_AP) {
        DWin<double> w;
        w.load(Pc, I.ldv, n, jb, i);
#pragma unroll
        for (int r = 0; r < DR; ++r) {
            const double q = w.apply(s, r);
            if (ok(r)) {
                Q[rowv(r)] = q;
                acc0.add_prod(w.v[r + 1][1], q);
            }
        }
    } else if constexpr (kind == GK_PCG_UPD) {
        double V[DR], Pp[DR], Rr[DR], Qq[DR];
#pragma unroll
        for (int r = 0; r < DR; ++r) {
            V[r] = Uc[rowu(r)];
            Pp[r] = Pc[rowv(r)];
            Rr[r] = Rc[rowv(r)];
            Qq[r] = Qc[rowv(r)];
        }
#pragma unroll
        for (int r = 0; r < DR; ++r) {
            const double res = Rr[r] - alpha * Qq[r];
            if (ok(r)) {
                U[rowu(r)] = V[r] + alpha * Pp[r];
                R[rowv(r)] = res;
                acc0.add_sq(res);
            }
        }
    } else if constexpr (kind == GK_PCG_TRUE) {
        if (!st.check) return;   // uniform over the block: no barrier is skipped by part of it
        DWin<double> w;
        w.load(Uc, I.ldu, n, jb, i);
        double F[DR];
#pragma unroll
        for (int r = 0; r < DR; ++r) F[r] = Fv[rowf(r)];
#pragma unroll
        for (int r = 0; r < DR; ++r) {
            const double res = h2 * F[r] - w.apply(s, r);
            if (ok(r)) {
                R[rowv(r)] = res;
                acc0.add_sq(res);
            }
        }
    } else if constexpr (kind == GK_APPLY) {
        DWin<double> w;
        w.load(X, I.ldx, n, jb, i);
#pragma unroll
        for (int r = 0; r < DR; ++r) {
            const double y = w.apply(s, r) * I.h2inv;
            if (ok(r)) Y[(size_t)(jb + r) * I.ldy + i] = y;
        }
    } else if constexpr (kind == GK_GRAD) {
        Sten<double> dt, de;
        dt.load(I.ds_th);
        de.load(I.ds_ep);
        DWin<double> w;
        w.load(Yc, I.ldy, n, jb, i);
        double Lm[DR];
#pragma unroll
        for (int r = 0; r < DR; ++r) Lm[r] = X[(size_t)clampi(jb + r, n) * I.ldx + ic];
#pragma unroll
        for (int r = 0; r < DR; ++r) {
            const double yt = w.apply(dt, r) * I.h2inv;
            const double ye = w.apply(de, r) * I.h2inv;
            if (ok(r)) {
                acc0.add_prod(Lm[r], yt);
                acc1.add_prod(Lm[r], ye);
            }
        }
    }
    if (a.fin != FIN_NONE) reduce_partial(a, t, acc0, acc1);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// shape of a fused grid launch (flags): bit 1 = streaming strips with R = 16 << ((flags >> 2) & 3)
// rows, else bit 5 = 8 x 8 tiles, else bit 0 = 16 x 16 tiles, else bit 4 = 32 x 32 tiles, else 64 x 32 tiles
template <typename T, int NU>
static void pre_shape(const StageArgs& a, int nb, hipStream_t s)
{
    if (a.flags & 2) {
        switch ((a.flags >> 2) & 3) {
        case 0: k_pre_s<T, NU, 16><<<nb, 256, 0, s>>>(a); break;
        default: k_pre_s<T, NU, 32><<<nb, 256, 0, s>>>(a); break;
        }
    } else if (a.flags & 32) {
        k_pre<T, NU, 8, 8><<<nb, GRID_THREADS, 0, s>>>(a);
    } else if (a.flags & 1) {
        k_pre<T, NU, 16, 16><<<nb, GRID_THREADS, 0, s>>>(a);
    } else if (a.flags & 16) {
        k_pre<T, NU, 32, 32><<<nb, GRID_THREADS, 0, s>>>(a);
    } else {
        k_pre<T, NU, TX, TY><<<nb, GRID_THREADS, 0, s>>>(a);
    }
}

template <typename T, int NU>
static void post_shape(const StageArgs& a, int nb, hipStream_t s)
{
    if (a.flags & 2) {
        switch ((a.flags >> 2) & 3) {
        case 0: k_post_s<T, NU, 16><<<nb, 256, 0, s>>>(a); break;
        default: k_post_s<T, NU, 32><<<nb, 256, 0, s>>>(a); break;
        }
    } else if (a.flags & 32) {
        k_post<T, NU, 8, 8><<<nb, GRID_THREADS, 0, s>>>(a);
    } else if (a.flags & 1) {
        k_post<T, NU, 16, 16><<<nb, GRID_THREADS, 0, s>>>(a);
    } else if (a.flags & 16) {
        k_post<T, NU, 32, 32><<<nb, GRID_THREADS, 0, s>>>(a);
    } else {
        k_post<T, NU, TX, TY><<<nb, GRID_THREADS, 0, s>>>(a);
    }
}

template <typename T>
static hipError_t launch_pre(const StageArgs& a, int nb, hipStream_t s)
{
    switch (a.nu) {
    case 0: pre_shape<T, 0>(a, nb, s); break;
    case 1: pre_shape<T, 1>(a, nb, s); break;
    case 2: pre_shape<T, 2>(a, nb, s); break;
    case 3: pre_shape<T, 3>(a, nb, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_post(const StageArgs& a, int nb, hipStream_t s)
{
    switch (a.nu) {
    case 0: post_shape<T, 0>(a, nb, s); break;
    case 1: post_shape<T, 1>(a, nb, s); break;
    case 2: post_shape<T, 2>(a, nb, s); break;
    case 3: post_shape<T, 3>(a, nb, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_unfused(GridKernel k, const StageArgs& a, int nb, hipStream_t s)
{
    const dim3 g(nb), b(GRID_THREADS);
    switch (k) {
    case GK_SWEEP: k_unfused<T, GK_SWEEP><<<g, b, 0, s>>>(a); break;
    case GK_RESID: k_unfused<T, GK_RESID><<<g, b, 0, s>>>(a); break;
    case GK_RESTRICT: k_unfused<T, GK_RESTRICT><<<g, b, 0, s>>>(a); break;
    case GK_ZERO: k_unfused<T, GK_ZERO><<<g, b, 0, s>>>(a); break;
    case GK_PROLONG: k_unfused<T, GK_PROLONG><<<g, b, 0, s>>>(a); break;
    case GK_ADD: k_unfused<T, GK_ADD><<<g, b, 0, s>>>(a); break;
    case GK_COPY: k_unfused<T, GK_COPY><<<g, b, 0, s>>>(a); break;
    case GK_NORM: k_unfused<T, GK_NORM><<<g, b, 0, s>>>(a); break;
    case GK_ZERO_SELF: k_unfused<T, GK_ZERO_SELF><<<g, b, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_semi(GridKernel k, const StageArgs& a, int nb, hipStream_t s)
{
    const dim3 g(nb), b(GRID_THREADS);
    switch (k) {
    case GK_RESID: k_semi<T, GK_RESID><<<g, b, 0, s>>>(a); break;
    case GK_RESTRICT: k_semi<T, GK_RESTRICT><<<g, b, 0, s>>>(a); break;
    case GK_ZERO: k_semi<T, GK_ZERO><<<g, b, 0, s>>>(a); break;
    case GK_PROLONG: k_semi<T, GK_PROLONG><<<g, b, 0, s>>>(a); break;
    case GK_ADD: k_semi<T, GK_ADD><<<g, b, 0, s>>>(a); break;
    case GK_COPY: k_semi<T, GK_COPY><<<g, b, 0, s>>>(a); break;
    case GK_ZERO_SELF: k_semi<T, GK_ZERO_SELF><<<g, b, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool F32>
static hipError_t launch_driver(GridKernel k, const StageArgs& a, int nb, hipStream_t s)
{
    const dim3 g(nb), b(GRID_THREADS);
    switch (k) {
    case GK_SSF: k_driver<F32, GK_SSF><<<g, b, 0, s>>>(a); break;
    case GK_IR_RESID: k_driver<F32, GK_IR_RESID><<<g, b, 0, s>>>(a); break;
    case GK_IR_UPDATE: k_driver<F32, GK_IR_UPDATE><<<g, b, 0, s>>>(a); break;
    case GK_PCG_INIT: k_driver<F32, GK_PCG_INIT><<<g, b, 0, s>>>(a); break;
    case GK_PCG_PRECIN: k_driver<F32, GK_PCG_PRECIN><<<g, b, 0, s>>>(a); break;
    case GK_PCG_RZ: k_driver<F32, GK_PCG_RZ><<<g, b, 0, s>>>(a); break;
    case GK_PCG_P: k_driver<F32, GK_PCG_P><<<g, b, 0, s>>>(a); break;
    case GK_PCG_AP: k_driver<F32, GK_PCG_AP><<<g, b, 0, s>>>(a); break;
    case GK_PCG_UPD: k_driver<F32, GK_PCG_UPD><<<g, b, 0, s>>>(a); break;
    case GK_PCG_TRUE: k_driver<F32, GK_PCG_TRUE><<<g, b, 0, s>>>(a); break;
    case GK_APPLY: k_driver<F32, GK_APPLY><<<g, b, 0, s>>>(a); break;
    case GK_GRAD: k_driver<F32, GK_GRAD><<<g, b, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int NU2, int TSZ>
static hipError_t launch_postpre_nu1(const StageArgs& a, int nb, hipStream_t s)
{
    switch (a.nu) {   // a.nu = nu1 of the second call; a.src = nu2 of the first
    case 0: k_postpre<T, NU2, 0, TSZ, TSZ><<<nb, GRID_THREADS, 0, s>>>(a); break;
    case 1: k_postpre<T, NU2, 1, TSZ, TSZ><<<nb, GRID_THREADS, 0, s>>>(a); break;
    case 2: k_postpre<T, NU2, 2, TSZ, TSZ><<<nb, GRID_THREADS, 0, s>>>(a); break;
    case 3: k_postpre<T, NU2, 3, TSZ, TSZ><<<nb, GRID_THREADS, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int TSZ>
static hipError_t launch_postpre_tile(const StageArgs& a, int nb, hipStream_t s)
{
    switch (a.src) {
    case 0: return launch_postpre_nu1<T, 0, TSZ>(a, nb, s);
    case 1: return launch_postpre_nu1<T, 1, TSZ>(a, nb, s);
    case 2: return launch_postpre_nu1<T, 2, TSZ>(a, nb, s);
    case 3: return launch_postpre_nu1<T, 3, TSZ>(a, nb, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t launch_postpre(const StageArgs& a, int nb, hipStream_t s)
{
    if (a.flags == 1) return launch_postpre_tile<T, 16>(a, nb, s);
    if (a.flags == 32) return launch_postpre_tile<T, 8>(a, nb, s);
    return hipErrorInvalidValue;   // 16 x 16 and 8 x 8 tiles only
}

hipError_t launch_finalize(const StageArgs& a, hipStream_t s)
{
    if (a.fin == FIN_NONE) return hipSuccess;
    k_finalize<<<a.count, GRID_THREADS, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_grid(GridKernel k, bool f32, const StageArgs& a, int32_t nb, hipStream_t s, bool with_finalize)
{
    if (nb <= 0) return hipSuccess;
    hipError_t e;
    switch (k) {
    case GK_PRE: e = f32 ? launch_pre<float>(a, nb, s) : launch_pre<double>(a, nb, s); break;
    case GK_POST: e = f32 ? launch_post<float>(a, nb, s) : launch_post<double>(a, nb, s); break;
    case GK_POSTPRE: e = f32 ? launch_postpre<float>(a, nb, s) : launch_postpre<double>(a, nb, s); break;
    case GK_ZEBRA:   // direction a.nu: 0 x-lines, 1 y-lines
        if (f32) {
            if (a.nu) k_zebra<float, 1><<<nb, GRID_THREADS, 0, s>>>(a);
            else k_zebra<float, 0><<<nb, GRID_THREADS, 0, s>>>(a);
        } else {
            if (a.nu) k_zebra<double, 1><<<nb, GRID_THREADS, 0, s>>>(a);
            else k_zebra<double, 0><<<nb, GRID_THREADS, 0, s>>>(a);
        }
        e = hipGetLastError();
        break;
    case GK_SWEEP: case GK_RESID: case GK_RESTRICT: case GK_ZERO: case GK_PROLONG: case GK_ADD: case GK_COPY:
    case GK_NORM: case GK_ZERO_SELF:
        if (a.semi && k != GK_NORM && k != GK_SWEEP)
            e = f32 ? launch_semi<float>(k, a, nb, s) : launch_semi<double>(k, a, nb, s);
        else
            e = f32 ? launch_unfused<float>(k, a, nb, s) : launch_unfused<double>(k, a, nb, s);
        break;
    default:
        e = f32 ? launch_driver<true>(k, a, nb, s) : launch_driver<false>(k, a, nb, s);
        break;
    }
    if (e != hipSuccess || !with_finalize) return e;
    return launch_finalize(a, s);
}

hipError_t launch_subtree(bool f32, const SubArgs& a, int32_t threads, int32_t lds_bytes, hipStream_t s)
{
    if (a.count <= 0) return hipSuccess;
    const bool z = a.smoother == 1;
    if (threads == 256) {
        if (f32) z ? k_subtree<float, 256, true><<<a.count, 256, lds_bytes, s>>>(a)
                   : k_subtree<float, 256, false><<<a.count, 256, lds_bytes, s>>>(a);
        else z ? k_subtree<double, 256, true><<<a.count, 256, lds_bytes, s>>>(a)
               : k_subtree<double, 256, false><<<a.count, 256, lds_bytes, s>>>(a);
    } else if (threads == 512) {
        if (f32) z ? k_subtree<float, 512, true><<<a.count, 512, lds_bytes, s>>>(a)
                   : k_subtree<float, 512, false><<<a.count, 512, lds_bytes, s>>>(a);
        else z ? k_subtree<double, 512, true><<<a.count, 512, lds_bytes, s>>>(a)
               : k_subtree<double, 512, false><<<a.count, 512, lds_bytes, s>>>(a);
    } else if (threads == 1024 && f32) {   // FP32 only: the FP64 kernel does not fit 128 registers
        z ? k_subtree<float, 1024, true><<<a.count, 1024, lds_bytes, s>>>(a)
          : k_subtree<float, 1024, false><<<a.count, 1024, lds_bytes, s>>>(a);
    } else {
        return hipErrorInvalidValue;
    }
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
    const void* ks[] = {(const void*)k_subtree<float, 256, false>,  (const void*)k_subtree<float, 512, false>,
                        (const void*)k_subtree<float, 1024, false>, (const void*)k_subtree<float, 256, true>,
                        (const void*)k_subtree<float, 512, true>,   (const void*)k_subtree<float, 1024, true>,
                        (const void*)k_subtree<double, 256, false>, (const void*)k_subtree<double, 512, false>,
                        (const void*)k_subtree<double, 256, true>,  (const void*)k_subtree<double, 512, true>};
    hipError_t e = hipSuccess;
    for (int k = f32 ? 0 : 6; k < (f32 ? 6 : 10) && e == hipSuccess; ++k)
        e = hipFuncSetAttribute(ks[k], hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    return e;
}

int32_t max_lds_bytes()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
    return v;
}

}  // namespace kc
