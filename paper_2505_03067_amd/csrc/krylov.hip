// Restarted GMRES for the implicit-Euler step (paper Sec. 2.4), batched over every
// (problem, species) system of a context.
//
// Data layout.  All systems share one index space of "global unknowns": problem p,
// species s, compact domain voxel l sits at off_p + s * Npad_p + l.  Each Krylov
// vector V_k, the work vector W, the FP64 iterate x and right-hand side b are flat
// arrays over that space, so one launch streams every system at once.  A launch is
// a table of blocks, each owning a contiguous range of one system; the table is
// permuted so that every XCD works through a contiguous stretch of the vectors
// (its L2 then serves the +-y/+-z stencil neighbours).
//
// Per cycle (Jacobi-scaled operator B = S A S, S = diag(A)^(-1/2)):
//   residual:   r = b - A x in FP64; V_0 = S r (stored unnormalised, scale 1/||S r||)
//   step j:     K1  w = B v_j,  h = V_j^T w            (stencil + multi-dot)
//               K2  w -= V_j h, h2 = V_j^T w           (axpy + multi-dot, CGS2 pass 2)
//               K3  w -= V_j h2, ||w||, V_{j+1} = w     (axpy + norm)
//   finish:     Givens rotation of the last column and back-substitution
//   update:     x += S V_m y  (FP64 accumulation)
//
// Global reductions without atomics.  Each kernel publishes one partial sum per
// block and row; every block of the *next* kernel (which is ordered after it by the
// launch boundary) sums the partials of its system itself, in block order.  All
// blocks therefore hold bit-identical totals, the result is deterministic, and no
// block waits on another inside a launch.  The Givens rotation of column j is
// computed the same way by every block of the next step's first kernel; one
// designated block per system (its first) stores the Hessenberg state.  The Krylov
// type T is float (FP32 basis inside FP64 iterative refinement) or double (plain
// FP64 GMRES); both use the same kernels.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <utility>

#include "context.h"

namespace mpm {

// Arnoldi steps launched beyond the previous step's cycle length before the host
// checks whether the cycle has to continue (1 measured 1% faster than 2 on the 128^3
// three-species workload: cycle lengths change slowly from step to step, and every
// launch past the end of all cycles costs a few microseconds).
constexpr int kPredictMargin = 1;

// partial-sum rows
constexpr int kRowB = 0;                    // ||b||^2
constexpr int kRowR = 1;                    // ||r||^2, ||S r||^2
constexpr int kRowP1 = 3;                   // K1: V_j^T w
constexpr int kRowP2 = kRowP1 + kMaxM + 1;  // K2: V_j^T w
constexpr int kRowP3 = kRowP2 + kMaxM + 1;  // K3: ||w||^2
static_assert(kRowP3 + 1 <= kPartRows, "partial rows");

// ------------------------------------------------------------------ helpers
// Pointers read from a block record are generic to the compiler, and generic (flat)
// loads make it wait for every outstanding load at once; these arrays live in device
// global memory, which the address-space cast states.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
template <typename T>
__device__ inline gptr<T> as_global(const T* p) {
    return (gptr<T>)p;
}

template <typename T>
struct VW {
    static constexpr int n = 16 / sizeof(T);
};

template <typename T>
__device__ inline void ld16(const T* p, T (&o)[VW<T>::n]) {
    if constexpr (sizeof(T) == 4) {
        const float4 t = *reinterpret_cast<const float4*>(p);
        o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
    } else {
        const double2 t = *reinterpret_cast<const double2*>(p);
        o[0] = t.x; o[1] = t.y;
    }
}
template <typename T>
__device__ inline void st16(T* p, const T (&v)[VW<T>::n]) {
    if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
        *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ inline void ldg16(gptr<T> p, T (&o)[VW<T>::n]) {
    if constexpr (sizeof(T) == 4) {
        const f32x4 t = *(const __attribute__((address_space(1))) f32x4*)p;
        o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
    } else {
        const f64x2 t = *(const __attribute__((address_space(1))) f64x2*)p;
        o[0] = t.x; o[1] = t.y;
    }
}

__device__ inline double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Reduce-scatter over the wave: NV values per lane in, one row sum per lane out.  Each
// butterfly stage halves the rows a lane carries (the lane with the stage's bit set
// keeps the upper half, its partner the lower half), so the exchanges number about
// 2 NV instead of 6 NV for separate wave sums; the remaining stages are plain
// exchanges.  Returns the sum of row 'row'; every lane with the same row holds the
// same value (lane representative when its low bits are zero).  The order of the
// additions is fixed, so every wave and block computes identical totals.
template <int NV>
struct RS {
    static constexpr int K = NV <= 1 ? 1 : NV <= 2 ? 2 : NV <= 4 ? 4 : NV <= 8 ? 8 : NV <= 16 ? 16 : NV <= 32 ? 32 : 64;
    static constexpr int L = K == 1 ? 0 : K == 2 ? 1 : K == 4 ? 2 : K == 8 ? 3 : K == 16 ? 4 : K == 32 ? 5 : 6;
    static_assert(NV <= 64, "at most 64 rows");
};

template <int NV>
__device__ inline double wave_reduce_scatter(const double (&v)[NV], int& row, bool& rep) {
    constexpr int K = RS<NV>::K, L = RS<NV>::L;
    const int lane = threadIdx.x & 63;
    double w[K];
#pragma unroll
    for (int i = 0; i < K; ++i) w[i] = i < NV ? v[i] : 0.0;
    row = 0;
#pragma unroll
    for (int st = 0; st < L; ++st) {
        const int o = 32 >> st, half = K >> (st + 1);
        const bool bit = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            const double send = bit ? w[i] : w[i + half];
            const double keep = bit ? w[i + half] : w[i];
            w[i] = keep + __shfl_xor(send, o);
        }
        if (bit) row += half;
    }
    double r = w[0];
#pragma unroll
    for (int st = L; st < 6; ++st) r += __shfl_xor(r, 32 >> st);
    rep = (lane & ((1 << (6 - L)) - 1)) == 0;
    return r;
}

// Block-reduce NV per-thread sums and store them in slot 'slot' of rows 0..NV-1.
template <int NV, typename A>
__device__ inline void block_partials(const A (&acc)[NV], double* part, int nslots, int slot) {
    __shared__ double sh[kWaves][NV];
    const int w = threadIdx.x >> 6;
    double t[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) t[v] = (double)acc[v];
    int row;
    bool rep;
    const double r = wave_reduce_scatter<NV>(t, row, rep);
    if (rep && row < NV) sh[w][row] = r;
    __syncthreads();
    for (int v = threadIdx.x; v < NV; v += kThreads) {
        double t = sh[0][v];
#pragma unroll
        for (int i = 1; i < kWaves; ++i) t += sh[i][v];
        part[(long long)v * nslots + slot] = t;
    }
}

// Loads of one block's share of a system's partial sums (rows w, w + kWaves, ... of
// wave w; lane i takes slots i, i + 64, ... up to four of them per row), issued
// together; sum_partials finishes the reduction into out[] (shared).  Every block
// sums in the same order, so all hold bit-identical totals.
template <int NV>
struct PartLoad {
    static constexpr int R = (NV + kWaves - 1) / kWaves;
    double t[R][4];
};

template <int NV>
__device__ inline void load_partials(const double* part, int nslots, int slot0, int nb, PartLoad<NV>& pl) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < PartLoad<NV>::R; ++r) {
        const int v = w + r * kWaves;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = lane + 64 * q;
            pl.t[r][q] = (v < NV && i < nb) ? part[(long long)v * nslots + slot0 + i] : 0.0;
        }
    }
}

template <int NV>
__device__ inline void sum_partials(const double* part, int nslots, int slot0, int nb, PartLoad<NV>& pl,
                                    double* out) {
    constexpr int R = PartLoad<NV>::R;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double t[R];
#pragma unroll
    for (int r = 0; r < R; ++r) t[r] = ((pl.t[r][0] + pl.t[r][1]) + pl.t[r][2]) + pl.t[r][3];
    if (nb > 256) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int v = w + r * kWaves;
            if (v < NV)
                for (int i = lane + 256; i < nb; i += 64) t[r] += part[(long long)v * nslots + slot0 + i];
        }
    }
    int row;
    bool rep;
    const double sum = wave_reduce_scatter<R>(t, row, rep);
    const int v = w + row * kWaves;
    if (rep && row < R && v < NV) out[v] = sum;
    (void)lane;
}

// Sum rows 0..NV-1 of a system's partial slots into out[] (shared), then synchronise.
template <int NV>
__device__ inline void reduce_partials(const double* part, int nslots, int slot0, int nb, double* out) {
    PartLoad<NV> pl;
    load_partials<NV>(part, nslots, slot0, nb, pl);
    sum_partials<NV>(part, nslots, slot0, nb, pl, out);
    __syncthreads();
}

struct Where {
    int sys, p, s;
    long long base;      // global index of l = 0 of this species
    long long locbase;   // problem-local index of l = 0 of this species
    long long tot;       // S * Npad (plane stride of the coupling arrays)
};

template <typename T>
__device__ inline Where where_of(const KArgs<T>& a, const Block& blk, const ProbDev& pd) {
    Where w;
    w.sys = blk.sys;
    w.p = blk.sys / a.S;
    w.s = blk.sys - w.p * a.S;
    w.locbase = (long long)w.s * pd.Npad;
    w.base = pd.off + w.locbase;
    w.tot = (long long)a.S * pd.Npad;
    return w;
}

template <typename T>
__device__ inline const T* couplings(const ProbDev& pd);
template <>
__device__ inline const float* couplings<float>(const ProbDev& pd) { return pd.c32; }
template <>
__device__ inline const double* couplings<double>(const ProbDev& pd) { return pd.c64; }

// Scaled stencil B = S A S (unit diagonal) on VW consecutive unknowns starting at
// global index u0 (local voxel l0).  Returns the centre values of v in xv.
template <typename T>
__device__ inline void stencil_scaled(const T* __restrict__ v, const T* __restrict__ c, const ProbDev& pd,
                                      const Where& wh, long long u0, int l0, T (&xv)[VW<T>::n],
                                      T (&out)[VW<T>::n]) {
    constexpr int n = VW<T>::n;
    const long long loc0 = wh.locbase + l0;
    T cx[n], cy[n], cz[n];
    ld16(v + u0, xv);
    ld16(c + loc0, cx);
    ld16(c + wh.tot + loc0, cy);
    ld16(c + 2 * wh.tot + loc0, cz);
    const T vm = v[u0 - 1], vp = v[u0 + n];
    const T cxm = c[loc0 - 1];
#pragma unroll
    for (int e = 0; e < n; ++e) {
        const int4 nb = pd.nbr[l0 + e];
        const T left = e == 0 ? vm : xv[e - 1];
        const T leftc = e == 0 ? cxm : cx[e - 1];
        const T right = e == n - 1 ? vp : xv[e + 1];
        T r = xv[e];
        r += cx[e] * right;
        r += leftc * left;
        r += cy[e] * v[wh.base + nb.y];
        r += c[wh.tot + wh.locbase + nb.x] * v[wh.base + nb.x];
        r += cz[e] * v[wh.base + nb.w];
        r += c[2 * wh.tot + wh.locbase + nb.z] * v[wh.base + nb.z];
        out[e] = (l0 + e < pd.N) ? r : T(0);
    }
}

// Unscaled FP64 operator (A x)_l for one domain voxel.
__device__ inline double apply_A(const ProbDev& pd, const Where& wh, const double* __restrict__ X, long long u,
                                 int l) {
    const long long loc = wh.locbase + l;
    const int4 nb = pd.nbr[l];
    const double* ax = pd.a64;
    const double* ay = pd.a64 + wh.tot;
    const double* az = pd.a64 + 2 * wh.tot;
    double r = pd.d64[loc] * X[u];
    r += ax[loc] * X[u + 1];
    r += ax[loc - 1] * X[u - 1];
    r += ay[loc] * X[wh.base + nb.y];
    r += ay[wh.locbase + nb.x] * X[wh.base + nb.x];
    r += az[loc] * X[wh.base + nb.w];
    r += az[wh.locbase + nb.z] * X[wh.base + nb.z];
    return r;
}

// ------------------------------------------------------------------ kernels
// Gather c^n from the lattice into x, form b = c^n + q; partials of ||b||^2.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gather(KArgs<T> a) {
    constexpr int n = 4;
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    const double* f = a.fields[blk.p] + (long long)blk.s * blk.nvox;
    const gptr<int> vox = as_global(blk.vox);
    const gptr<double> q = as_global(blk.q64);
    double acc[1] = {0.0};
    for (long long u0 = blk.start + threadIdx.x * n; u0 < blk.end; u0 += kThreads * n) {
        const int l0 = (int)(u0 - blk.base);
        int vx[n];
        double qq[n];
#pragma unroll
        for (int e = 0; e < n; ++e) {
            vx[e] = vox[l0 + e];
            qq[e] = q[blk.locbase + l0 + e];
        }
        double cn[n], bb[n];
#pragma unroll
        for (int e = 0; e < n; ++e) {
            const bool in = l0 + e < blk.N;
            cn[e] = in ? f[vx[e]] : 0.0;
            bb[e] = in ? cn[e] + qq[e] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < n; ++e) {
            a.x[u0 + e] = cn[e];
            a.b[u0 + e] = bb[e];
            acc[0] += bb[e] * bb[e];
        }
        if (a.pcur) {
#pragma unroll
            for (int e = 0; e < n; ++e) a.pcur[u0 + e] = cn[e];
        }
    }
    block_partials<1>(acc, a.part + (long long)kRowB * a.nslots, a.nslots, blk.slot);
}

// BF16 of the network input: round to nearest, ties to even; NaN -> quiet NaN 0x7fc0
__device__ inline uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)0x7fc0u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Grid index of lattice voxel v of a problem's box.
__device__ inline long long grid_of_voxel(const ProbDev& pd, int v) {
    const int plane = pd.nx * pd.ny;
    const int z = v / plane;
    const int rem = v - z * plane;
    const int y = rem / pd.nx;
    const int x = rem - y * pd.nx;
    return ((long long)(z - pd.lo[2]) * pd.gd[1] + (y - pd.lo[1])) * pd.gd[0] + (x - pd.lo[0]);
}

// Which systems a residual evaluation covers: the first one of a step covers all;
// the one after a cycle the not yet converged; the warm-start one the systems not
// converged at c^n; the revert one the systems whose warm start was rejected.
enum ResMode { kResCycle = 0, kResFirst = 1, kResWarm = 2, kResRevert = 3 };

__device__ inline bool res_skip(const SysK* sk, int mode) {
    switch (mode) {
        case kResFirst: return false;
        case kResRevert: return !sk->fallback;
        case kResWarm: return sk->converged != 0;
        default: return sk->converged != 0 || sk->active != kIdle;   // only systems whose cycle ended
    }
}

// r = b - A x (FP64); V_0 = S r; partials of ||r||^2 and ||S r||^2.  Two unknowns per
// thread; the neighbour indices are requested first, the direct operands next, and the
// neighbour values once the indices are in.  PAIR (first residual of a step whose start
// is the network's correction of the extrapolation): the same pass also forms the base
// start x_b = 2 x - c^{n-1} (a.pold) at the seven stencil points and stores V_0 =
// S (b - A x_b) for the network's input instead of S r; the partials stay those of r.
// WSIN (first residual of a step with a network start): the pass also writes the
// network input's per-step channels of its domain voxels, each times its scale, BF16:
// c^n (channel s; x holds c^n) and d = S V_0 (channel 4 S + 1 + s), as k_ws_resid does.
template <typename T, bool PAIR = false, bool WSIN = false>
__global__ __launch_bounds__(kThreads) void k_residual(KArgs<T> a, int mode, const float* scales = nullptr) {
    constexpr int n = 2;
    const int lane = threadIdx.x & 63;
    const int cv = lane < a.nsys ? a.sk[lane].converged : 0;
    const int fb = lane < a.nsys ? a.sk[lane].fallback : 0;
    const int ac = lane < a.nsys ? a.sk[lane].active : 0;
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    const bool skip = mode == kResFirst    ? false
                      : mode == kResRevert ? !__builtin_amdgcn_readlane(fb, blk.sys)
                      : mode == kResWarm   ? __builtin_amdgcn_readlane(cv, blk.sys) != 0
                                           : (__builtin_amdgcn_readlane(cv, blk.sys) != 0 ||
                                            __builtin_amdgcn_readlane(ac, blk.sys) != kIdle);
    if (skip) return;
    const __attribute__((address_space(1))) i32x4* nbr = (const __attribute__((address_space(1))) i32x4*)blk.nbr;
    const gptr<double> A = as_global(blk.a64);
    const gptr<double> d = as_global(blk.d64);
    const gptr<double> sc = as_global(blk.sc64);
    const long long tot = blk.tot;
    T* V0 = a.V;
    double acc[2] = {0.0, 0.0};
    ProbDev pd{};
    float cscale = 0.f, dscale = 0.f;
    if constexpr (WSIN) {
        pd = a.probs[blk.p];
        cscale = scales[blk.s];
        dscale = scales[4 * a.S + 1 + blk.s];
    }
    for (long long u0 = blk.start + threadIdx.x * n; u0 < blk.end; u0 += kThreads * n) {
        const int l0 = (int)(u0 - blk.base);
        const long long loc0 = blk.locbase + l0;
        int4 nb[n];
        int vx[n];
        if constexpr (WSIN) {
#pragma unroll
            for (int e = 0; e < n; ++e) vx[e] = blk.vox[l0 + e];
        }
#pragma unroll
        for (int e = 0; e < n; ++e) {
            const i32x4 t = nbr[l0 + e];
            nb[e] = make_int4(t.x, t.y, t.z, t.w);
        }
        __builtin_amdgcn_sched_barrier(0);
        double xv[n], bv[n], dv[n], ax[n], ay[n], az[n], sv[n], ov[n];
        ld16(a.x + u0, xv);
        ld16(a.b + u0, bv);
        ldg16(d + loc0, dv);
        ldg16(A + loc0, ax);
        ldg16(A + tot + loc0, ay);
        ldg16(A + 2 * tot + loc0, az);
        ldg16(sc + loc0, sv);
        if constexpr (PAIR) ld16(a.pold + u0, ov);
        const double xm = a.x[u0 - 1], xp = a.x[u0 + n];
        const double om = PAIR ? a.pold[u0 - 1] : 0.0, op = PAIR ? a.pold[u0 + n] : 0.0;
        const double axm = A[loc0 - 1];
        __builtin_amdgcn_sched_barrier(0);
        double gyp[n], gym[n], aym[n], gzp[n], gzm[n], azm[n], hyp[n], hym[n], hzp[n], hzm[n];
#pragma unroll
        for (int e = 0; e < n; ++e) {
            gyp[e] = a.x[blk.base + nb[e].y];
            gym[e] = a.x[blk.base + nb[e].x];
            aym[e] = A[tot + blk.locbase + nb[e].x];
            gzp[e] = a.x[blk.base + nb[e].w];
            gzm[e] = a.x[blk.base + nb[e].z];
            azm[e] = A[2 * tot + blk.locbase + nb[e].z];
            if constexpr (PAIR) {
                hyp[e] = a.pold[blk.base + nb[e].y];
                hym[e] = a.pold[blk.base + nb[e].x];
                hzp[e] = a.pold[blk.base + nb[e].w];
                hzm[e] = a.pold[blk.base + nb[e].z];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        T v0[n];
#pragma unroll
        for (int e = 0; e < n; ++e) {
            double r = 0.0, sr = 0.0, srb = 0.0;
            if (l0 + e < blk.N) {
                const double left = e == 0 ? xm : xv[e - 1];
                const double right = e == n - 1 ? xp : xv[e + 1];
                const double leftc = e == 0 ? axm : ax[e - 1];
                double Ax = dv[e] * xv[e];
                Ax += ax[e] * right;
                Ax += leftc * left;
                Ax += ay[e] * gyp[e];
                Ax += aym[e] * gym[e];
                Ax += az[e] * gzp[e];
                Ax += azm[e] * gzm[e];
                r = bv[e] - Ax;
                sr = sv[e] * r;
                if constexpr (PAIR) {
                    // x_b at each stencil point as the extrapolation stores it, summed in
                    // the same order as above
                    const double oleft = e == 0 ? om : ov[e - 1];
                    const double oright = e == n - 1 ? op : ov[e + 1];
                    double Axb = dv[e] * (2.0 * xv[e] - ov[e]);
                    Axb += ax[e] * (2.0 * right - oright);
                    Axb += leftc * (2.0 * left - oleft);
                    Axb += ay[e] * (2.0 * gyp[e] - hyp[e]);
                    Axb += aym[e] * (2.0 * gym[e] - hym[e]);
                    Axb += az[e] * (2.0 * gzp[e] - hzp[e]);
                    Axb += azm[e] * (2.0 * gzm[e] - hzm[e]);
                    srb = sv[e] * (bv[e] - Axb);
                }
            }
            v0[e] = (T)(PAIR ? srb : sr);
            acc[0] += r * r;
            acc[1] += sr * sr;
            if constexpr (WSIN) {
                if (l0 + e < blk.N) {
                    const double dd = sv[e] * (double)v0[e];
                    uint16_t* o = pd.wsin + grid_of_voxel(pd, vx[e]) * ws_channels(a.S);
                    o[4 * a.S + 1 + blk.s] = to_bf16((float)dd * dscale);
                    o[blk.s] = to_bf16((float)xv[e] * cscale);
                }
            }
        }
#pragma unroll
        for (int e = 0; e < n; ++e) V0[u0 + e] = v0[e];
    }
    block_partials<2>(acc, a.part + (long long)kRowR * a.nslots, a.nslots, blk.slot);
}

// Norms, convergence test, start of the next cycle for one system; in warm mode the
// acceptance test of the warm start (kept only if its true residual is below that of
// c^n, else the system falls back to c^n).  Thread 0 stores the outcome.
template <typename T>
__device__ inline void res_final_sys(const KArgs<T>& a, int sys, int mode) {
    SysK* sk = a.sk + sys;
    if (res_skip(sk, mode)) return;
    const bool first = mode == kResFirst;
    __shared__ double tot[3];
    reduce_partials<2>(a.part + (long long)kRowR * a.nslots, a.nslots, sk->slot0, sk->nblocks, tot);
    if (first) reduce_partials<1>(a.part + (long long)kRowB * a.nslots, a.nslots, sk->slot0, sk->nblocks, tot + 2);
    if (threadIdx.x != 0) return;
    const Params& prm = *a.prm;
    if (first) {
        sk->bnorm = sqrt(tot[2]);
        sk->iters = 0;
        sk->cycles = 0;
        sk->refinements = 0;
        sk->mcount = 0;
        sk->breakdown = 0;
        sk->ws_used = 0;
        sk->fallback = 0;
        sk->rel_warm = 0.0;
    }
    const double rn = sqrt(tot[0]), srn = sqrt(tot[1]);
    const double bn = sk->bnorm;
    const double rel = bn > 0.0 ? rn / bn : (rn > 0.0 ? INFINITY : 0.0);
    if (mode == kResWarm) {
        sk->rel_warm = rel;
        if (!(rel < sk->rel_init)) {           // rejected (also catches NaN)
            sk->fallback = 1;
            sk->active = 0;
            return;
        }
        sk->ws_used = 1;
    }
    if (first) sk->rel_init = rel;
    else if (mode == kResCycle) sk->refinements += 1;
    sk->rel_final = rel;
    sk->rnorm = rn;
    sk->srnorm = srn;
    sk->need_update = 0;
    const bool conv = (rn <= prm.tol * bn) || rn == 0.0;
    const bool bad = !(rn == rn) || !(srn > 0.0) || isinf(rn);
    sk->converged = conv ? 1 : 0;
    if (conv || bad) {
        sk->active = 0;
        if (bad && !conv) sk->breakdown = 1;
    } else {
        double eta = 0.9 * prm.tol * bn / (rn * sk->kappa_s);
        if (eta < prm.inner_rtol) eta = prm.inner_rtol;
        if (eta > 0.5) eta = 0.5;
        sk->eta = eta;
        sk->vs[0] = 1.0 / srn;
        sk->gt[0] = srn;
        sk->active = kPending;
    }
}

// One block per system.  Ends every launch of the step (first residual, warm start,
// each cycle), so it also copies each system's status head, whether this launch changed
// it or not, to the host-visible mirror the host reads between cycles.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_res_final(KArgs<T> a, int sys0, int mode) {
    const int sys = sys0 + blockIdx.x;
    res_final_sys<T>(a, sys, mode);
    __syncthreads();
    static_assert(kSysHead % 4 == 0 && kSysHead / 4 <= kThreads, "status head copied as words");
    if (threadIdx.x < kSysHead / 4) {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(a.sk + sys);
        volatile uint32_t* dst = reinterpret_cast<volatile uint32_t*>(a.hsk + sys);
        dst[threadIdx.x] = src[threadIdx.x];
        __threadfence_system();
    }
}

// Value of v in lane i (i uniform), as a wave-uniform double.
__device__ inline double rdl(double v, int i) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), i);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), i);
    return __hiloint2double(hi, lo);
}

// Wave 0 only, one Hessenberg row per lane.  'v' holds the unrotated column Jc
// (rows 0..Jc + 1, sub = row Jc + 1).  Applies the earlier Givens rotations (the
// running value of row i is carried from rotation to rotation), forms rotation Jc,
// updates the rotated right-hand side g and tests the end of the cycle; at the end,
// solves R y = g by columns (lane i keeps row i of g and receives y_k in turn).
// Every block computes the same values in the same order; only 'lead' stores.
// Registers stay O(1) per row, whatever Jc.  Returns done (uniform over the wave).
// Per-system scalars column_tail reads, loaded by the caller (lane i: entry i).
struct TailIn {
    double csl, snl;   // Givens cosine and sine of column lane (lane < Jc)
    double vsl;        // vs[lane]
    double gJ, g0, eta;
};

__device__ inline TailIn load_tail(const SysK* sk, int Jc) {
    const int lane = threadIdx.x & 63;
    TailIn t;
    t.csl = lane < Jc ? sk->cs[lane] : 0.0;
    t.snl = lane < Jc ? sk->sn[lane] : 0.0;
    t.vsl = lane <= Jc ? sk->vs[lane] : 0.0;
    t.gJ = sk->gt[Jc];
    t.g0 = sk->gt[0];
    t.eta = sk->eta;
    return t;
}

template <int Jc>
__device__ inline bool column_tail(SysK* sk, const TailIn& ti, double v, double sub, int restart, bool lead) {
    constexpr int LD = kMaxM + 1;
    const int lane = threadIdx.x & 63;
    const double csl = ti.csl, snl = ti.snl;
    double r = v;
    double run = rdl(v, 0);
#pragma unroll
    for (int i = 0; i < Jc; ++i) {
        const double b = rdl(v, i + 1), c = rdl(csl, i), sn = rdl(snl, i);
        const double top = c * run + sn * b;
        run = -sn * run + c * b;
        if (lane == i) r = top;
    }
    const double rho = sqrt(run * run + sub * sub);
    double cs = 1.0, sn = 0.0;
    if (rho > 0.0) {
        cs = run / rho;
        sn = sub / rho;
    }
    if (lane == Jc) r = rho;
    const double gJ = ti.gJ;
    const double gn = -sn * gJ;
    const bool breakdown = !(sub > 0.0) || !(rho > 0.0);
    const bool done = breakdown || fabs(gn) <= ti.eta * ti.g0 || Jc + 1 >= restart;
    if (lead) {
        if (lane <= Jc) sk->R[Jc * LD + lane] = r;
        if (lane == 0) {
            sk->cs[Jc] = cs;
            sk->sn[Jc] = sn;
            sk->gf[Jc] = cs * gJ;
            sk->gt[Jc + 1] = gn;
        }
    }
    if (done) {
        const int m = Jc + 1;
        double rrow[Jc > 0 ? Jc : 1];
#pragma unroll
        for (int k = 0; k < Jc; ++k) rrow[k] = lane <= k ? sk->R[k * LD + lane] : 0.0;
        double gi = lane < Jc ? sk->gf[lane] : (lane == Jc ? cs * gJ : 0.0);
        double yi = 0.0;
        {
            const double yk = rho != 0.0 ? rdl(gi, Jc) / rho : 0.0;
            if (lane == Jc) yi = yk;
            if (lane < Jc) gi -= r * yk;
        }
#pragma unroll
        for (int k = Jc - 1; k >= 0; --k) {
            const double rkk = rdl(rrow[k], k);
            const double gk = rdl(gi, k);
            const double yk = rkk != 0.0 ? gk / rkk : 0.0;
            if (lane == k) yi = yk;
            if (lane < k) gi -= rrow[k] * yk;
        }
        if (lead) {
            if (lane < m) sk->y[lane] = yi * ti.vsl;
            if (lane == 0) {
                sk->mcount = m;
                sk->active = 0;
                sk->need_update = 1;
                sk->iters += m;
                sk->cycles += 1;
                if (breakdown && !(sub == 0.0)) sk->breakdown = 1;
            }
        }
    }
    return done;
}

// CGS2: column Jc = h1 + h2 with ||w|| = hn below the diagonal; the next basis
// vector's scale 1/hn.  Returns true (to the whole block) if the cycle ended at Jc.
template <int Jc>
__device__ inline bool givens_tail(SysK* sk, double hn, int restart, bool lead) {
    __shared__ int s_done;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const TailIn ti = load_tail(sk, Jc);
        const double v = lane <= Jc ? sk->h1[lane] + sk->h2[lane] : (lane == Jc + 1 ? hn : 0.0);
        const bool done = column_tail<Jc>(sk, ti, v, hn, restart, lead);
        if (lead && lane == 0) sk->vs[Jc + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
        if (lane == 0) s_done = done ? 1 : 0;
    }
    __syncthreads();
    return s_done != 0;
}

// K1: (J > 0: finish step J-1 first) w = B v_J and partials of V_k . w, k <= J.
template <typename T, int J>
__global__ __launch_bounds__(kThreads) void k_spmv_dot(KArgs<T> a) {
    constexpr int n = VW<T>::n;
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    SysK* sk = a.sk + blk.sys;
    T vsJ;
    if constexpr (J == 0) {
        // step 0 takes up pending systems (its first block marks them running)
        if (sk->active == kIdle) return;
        if (blk.slot == sk->slot0 && threadIdx.x == 0) sk->active = kRunning;
        vsJ = (T)sk->vs[0];
    } else {
        if (sk->active != kRunning) return;
        __shared__ double red[1];
        reduce_partials<1>(a.part + (long long)kRowP3 * a.nslots, a.nslots, sk->slot0, sk->nblocks, red);
        const double hn = sqrt(red[0]);
        if (givens_tail<J - 1>(sk, hn, a.prm->restart, blk.slot == sk->slot0)) return;
        vsJ = (T)(hn > 0.0 ? 1.0 / hn : 0.0);
    }
    const ProbDev pd = a.probs[blk.sys / a.S];
    const Where wh = where_of(a, blk, pd);
    const T* c = couplings<T>(pd);
    const T* VJ = a.V + (long long)J * a.ldv;
    double acc[J + 1];
#pragma unroll
    for (int k = 0; k <= J; ++k) acc[k] = 0.0;
    for (long long u0 = blk.start + threadIdx.x * n; u0 < blk.end; u0 += kThreads * n) {
        const int l0 = (int)(u0 - wh.base);
        T xv[n], w[n];
        stencil_scaled<T>(VJ, c, pd, wh, u0, l0, xv, w);
#pragma unroll
        for (int e = 0; e < n; ++e) w[e] *= vsJ;
        st16(a.W + u0, w);
#pragma unroll
        for (int k = 0; k < J; ++k) {
            T vk[n];
            ld16(a.V + (long long)k * a.ldv + u0, vk);
#pragma unroll
            for (int e = 0; e < n; ++e) acc[k] += (double)vk[e] * (double)w[e];
        }
#pragma unroll
        for (int e = 0; e < n; ++e) acc[J] += (double)xv[e] * (double)w[e];
    }
    block_partials<J + 1>(acc, a.part + (long long)kRowP1 * a.nslots, a.nslots, blk.slot);
}

// K2: h = V_J^T w from K1's partials; w -= V_J h; partials of V_J^T w (CGS2 pass 2).
template <typename T, int J>
__global__ __launch_bounds__(kThreads) void k_axpy_dot(KArgs<T> a) {
    constexpr int n = VW<T>::n;
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    SysK* sk = a.sk + blk.sys;
    if (sk->active != kRunning) return;
    __shared__ double red[J + 1];
    reduce_partials<J + 1>(a.part + (long long)kRowP1 * a.nslots, a.nslots, sk->slot0, sk->nblocks, red);
    double cf[J + 1];
#pragma unroll
    for (int k = 0; k <= J; ++k) {
        const double vsk = sk->vs[k];
        const double h = vsk * red[k];
        cf[k] = h * vsk;
        if (blk.slot == sk->slot0 && threadIdx.x == 0) sk->h1[k] = h;
    }
    double acc[J + 1];
#pragma unroll
    for (int k = 0; k <= J; ++k) acc[k] = 0.0;
    for (long long u0 = blk.start + threadIdx.x * n; u0 < blk.end; u0 += kThreads * n) {
        T w[n];
        ld16(a.W + u0, w);
        T vk[J + 1][n];
#pragma unroll
        for (int k = 0; k <= J; ++k) ld16(a.V + (long long)k * a.ldv + u0, vk[k]);
        T wn[n];
#pragma unroll
        for (int e = 0; e < n; ++e) {
            double t = (double)w[e];
#pragma unroll
            for (int k = 0; k <= J; ++k) t -= cf[k] * (double)vk[k][e];
            wn[e] = (T)t;
        }
        st16(a.W + u0, wn);
#pragma unroll
        for (int k = 0; k <= J; ++k)
#pragma unroll
            for (int e = 0; e < n; ++e) acc[k] += (double)vk[k][e] * (double)wn[e];
    }
    block_partials<J + 1>(acc, a.part + (long long)kRowP2 * a.nslots, a.nslots, blk.slot);
}

// K3: h2 from K2's partials; w -= V_J h2; V_{J+1} = w; partials of ||w||^2.
template <typename T, int J>
__global__ __launch_bounds__(kThreads) void k_axpy_norm(KArgs<T> a) {
    constexpr int n = VW<T>::n;
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    SysK* sk = a.sk + blk.sys;
    if (sk->active != kRunning) return;
    __shared__ double red[J + 1];
    reduce_partials<J + 1>(a.part + (long long)kRowP2 * a.nslots, a.nslots, sk->slot0, sk->nblocks, red);
    double cf[J + 1];
#pragma unroll
    for (int k = 0; k <= J; ++k) {
        const double vsk = sk->vs[k];
        const double h = vsk * red[k];
        cf[k] = h * vsk;
        if (blk.slot == sk->slot0 && threadIdx.x == 0) sk->h2[k] = h;
    }
    const bool store = J + 1 < a.prm->restart;
    T* VN = a.V + (long long)(J + 1) * a.ldv;
    double acc[1] = {0.0};
    for (long long u0 = blk.start + threadIdx.x * n; u0 < blk.end; u0 += kThreads * n) {
        T w[n];
        ld16(a.W + u0, w);
        double t[n];
#pragma unroll
        for (int e = 0; e < n; ++e) t[e] = (double)w[e];
#pragma unroll
        for (int k = 0; k <= J; ++k) {
            T vk[n];
            ld16(a.V + (long long)k * a.ldv + u0, vk);
#pragma unroll
            for (int e = 0; e < n; ++e) t[e] -= cf[k] * (double)vk[e];
        }
        T wn[n];
#pragma unroll
        for (int e = 0; e < n; ++e) {
            wn[e] = (T)t[e];
            acc[0] += (double)wn[e] * (double)wn[e];
        }
        if (store) st16(VN + u0, wn);
    }
    block_partials<1>(acc, a.part + (long long)kRowP3 * a.nslots, a.nslots, blk.slot);
}

// After the last Arnoldi step of a cycle: Givens of column J and back-substitution
// (one block per system; systems whose cycle already ended are skipped).
template <typename T, int J>
__global__ __launch_bounds__(kThreads) void k_finish(KArgs<T> a, int sys0) {
    SysK* sk = a.sk + sys0 + blockIdx.x;
    if (sk->active != kRunning) return;
    __shared__ double red[1];
    reduce_partials<1>(a.part + (long long)kRowP3 * a.nslots, a.nslots, sk->slot0, sk->nblocks, red);
    (void)givens_tail<J>(sk, sqrt(red[0]), a.prm->restart, true);
}

// x += S sum_k y_k V_k (FP64 accumulation of the FP32 or FP64 basis).  The basis
// vectors are read eight at a time, all eight requested before any is used.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_update(KArgs<T> a) {
    constexpr int n = VW<T>::n;
    constexpr int G = 8;
    const int lane = threadIdx.x & 63;
    const int nu = lane < a.nsys ? a.sk[lane].need_update : 0;
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    if (!__builtin_amdgcn_readlane(nu, blk.sys)) return;
    const SysK* sk = a.sk + blk.sys;
    const int m = sk->mcount;
    const gptr<double> sc = as_global(blk.sc64);
    for (long long u0 = blk.start + threadIdx.x * n; u0 < blk.end; u0 += kThreads * n) {
        const long long loc0 = blk.locbase + (u0 - blk.base);
        double t[n], xv[n], sv[n];
#pragma unroll
        for (int e = 0; e < n; ++e) {
            t[e] = 0.0;
            xv[e] = a.x[u0 + e];
            sv[e] = sc[loc0 + e];
        }
        for (int k0 = 0; k0 < m; k0 += G) {
            T vk[G][n];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (k0 + g < m) {
                    ld16(a.V + (long long)(k0 + g) * a.ldv + u0, vk[g]);
                } else {
#pragma unroll
                    for (int e = 0; e < n; ++e) vk[g][e] = T(0);
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const double yk = k0 + g < m ? sk->y[k0 + g] : 0.0;
#pragma unroll
                for (int e = 0; e < n; ++e) t[e] += yk * (double)vk[g][e];
            }
        }
#pragma unroll
        for (int e = 0; e < n; ++e) a.x[u0 + e] = xv[e] + sv[e] * t[e];
    }
}

// Write x into the lattice field on the domain voxels.  only_idle: only for the systems
// whose solve has ended (neither running nor waiting for another cycle).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scatter(KArgs<T> a, int only_idle) {
    constexpr int n = 4;
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    if (only_idle && a.sk[blk.sys].active != kIdle) return;
    double* f = a.fields[blk.p] + (long long)blk.s * blk.nvox;
    const gptr<int> vox = as_global(blk.vox);
    for (long long u0 = blk.start + threadIdx.x * n; u0 < blk.end; u0 += kThreads * n) {
        const int l0 = (int)(u0 - blk.base);
        int vx[n];
        double xv[n];
#pragma unroll
        for (int e = 0; e < n; ++e) {
            vx[e] = vox[l0 + e];
            xv[e] = a.x[u0 + e];
        }
#pragma unroll
        for (int e = 0; e < n; ++e)
            if (l0 + e < blk.N) f[vx[e]] = xv[e];
    }
}

// Extremes of A_PP per system (for the scaled/unscaled residual bound).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_diag_extremes(KArgs<T> a) {
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    const ProbDev pd = a.probs[blk.sys / a.S];
    const Where wh = where_of(a, blk, pd);
    double mn = INFINITY, mx = 0.0;
    for (long long u = blk.start + threadIdx.x; u < blk.end; u += kThreads) {
        const int l = (int)(u - wh.base);
        if (l < pd.N) {
            const double d = pd.d64[wh.locbase + l];
            mn = fmin(mn, d);
            mx = fmax(mx, d);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        mn = fmin(mn, __shfl_xor(mn, o));
        mx = fmax(mx, __shfl_xor(mx, o));
    }
    if ((threadIdx.x & 63) == 0 && mx > 0.0) {
        SysK* sk = a.sk + blk.sys;
        atomicMin(&sk->dmin_bits, (unsigned long long)__double_as_longlong(mn));
        atomicMax(&sk->dmax_bits, (unsigned long long)__double_as_longlong(mx));
    }
}

__global__ void k_sys_init(SysK* sk, const int* first, const int* count, int nsys) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys) return;
    sk[s].dmin_bits = 0x7ff0000000000000ull;   // +inf
    sk[s].dmax_bits = 0ull;
    sk[s].nblocks = count[s];
    sk[s].slot0 = first[s];
    sk[s].converged = 0;
    sk[s].active = 0;
    sk[s].need_update = 0;
}

__global__ void k_sys_kappa(SysK* sk, int nsys) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys) return;
    const double mn = __longlong_as_double((long long)sk[s].dmin_bits);
    const double mx = __longlong_as_double((long long)sk[s].dmax_bits);
    sk[s].kappa_s = (mn > 0.0 && mx >= mn) ? sqrt(mx / mn) : 1.0;
}

// Debug: lattice -> global vector (FP64 or the Krylov type), problem-local launch.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dbg_gather(ProbDev pd, int S, const double* lat, double* x64, T* xt) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)S * pd.Npad) return;
    const int s = (int)(i / pd.Npad);
    const int l = (int)(i - (long long)s * pd.Npad);
    const double v = l < pd.N ? lat[(long long)s * pd.nvox + pd.vox[l]] : 0.0;
    x64[pd.off + i] = v;
    xt[pd.off + i] = (T)v;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_dbg_apply(ProbDev pd, int S, const double* x64, const T* xt,
                                                        double* lat, int mode) {
    constexpr int n = VW<T>::n;
    const long long i0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * n;
    if (i0 >= (long long)S * pd.Npad) return;
    const int s = (int)(i0 / pd.Npad);
    const int l0 = (int)(i0 - (long long)s * pd.Npad);
    Where wh;
    wh.sys = s;
    wh.p = 0;
    wh.s = s;
    wh.locbase = (long long)s * pd.Npad;
    wh.base = pd.off + wh.locbase;
    wh.tot = (long long)S * pd.Npad;
    double* out = lat + (long long)s * pd.nvox;
    if (mode == 0) {
        for (int e = 0; e < n; ++e)
            if (l0 + e < pd.N) out[pd.vox[l0 + e]] = apply_A(pd, wh, x64, wh.base + l0 + e, l0 + e);
    } else {
        T xv[n], w[n];
        stencil_scaled<T>(xt, couplings<T>(pd), pd, wh, wh.base + l0, l0, xv, w);
        for (int e = 0; e < n; ++e)
            if (l0 + e < pd.N) out[pd.vox[l0 + e]] = (double)w[e];
    }
}

// ------------------------------------------------------------------ delayed CGS2
// Classical Gram-Schmidt with delayed reorthogonalisation: step j keeps the vector
// u_j = A q_{j-1} - Q_{j-1} h (orthogonalised once) unnormalised and applies the
// stencil to it directly, z = B u_j.  One multi-dot gives s = Q^T u_j, t = Q^T z,
// alpha = u_j.u_j and gamma = u_j.z; then
//   q_j = (u_j - Q s) / beta_j,      beta_j^2 = alpha - |s|^2          (second pass, lagged)
//   H[:, j-1] = h_{j-1} + s,         H[j, j-1] = beta_j
//   A q_j = (z - Q_j g) / beta_j,    g = H s   (Arnoldi relation A Q = Q H)
//   h_j = Q_j^T A q_j = (Q_j^T z - g) / beta_j,  q_j . z = (gamma - s.t) / beta_j
//   u_{j+1} = A q_j - Q_j h_j = z / beta_j - Q_j (g / beta_j + h_j)
// so each step is one stencil + multi-dot kernel and one axpy kernel, one global
// reduction, two passes over the basis.  The Givens rotation of column j-1 runs in
// the axpy kernel of step j.  q_0 = vs[0] V_0; every later q_k is stored normalised.
//
// Partial rows of step j (base kRowD): J = 0: [0] V_0.z; J >= 1: [k] V_k.u,
// [J + k] V_k.z (k < J), [2J] u.u, [2J + 1] u.z.
constexpr int kRowD = 3;
static_assert(kRowD + 2 * kMaxM + 2 <= kPartRows, "partial rows");

// Scaled stencil B = S A S on VW consecutive unknowns of the block's system, addressed
// from the block record alone, in three phases so that the memory system sees as few
// dependent round trips as possible: (1) the neighbour indices are requested first;
// (2) the caller's own loads (basis vectors) and the stencil's direct operands
// follow; (3) once the indices are in, the neighbour values are gathered while the
// rest is still in flight.
template <typename T>
struct StencilIn {
    static constexpr int n = VW<T>::n;
    int4 nb[n];
    T xv[n], cx[n], cy[n], cz[n];
    T vm, vp, cxm;
};

template <typename T>
__device__ inline void stencil_idx(const Block& blk, int l0, StencilIn<T>& si) {
    const __attribute__((address_space(1))) i32x4* nbr = (const __attribute__((address_space(1))) i32x4*)blk.nbr;
#pragma unroll
    for (int e = 0; e < StencilIn<T>::n; ++e) {
        const i32x4 t = nbr[l0 + e];
        si.nb[e] = make_int4(t.x, t.y, t.z, t.w);
    }
}

template <typename T>
__device__ inline void stencil_direct(const T* __restrict__ v, const Block& blk, long long u0, int l0,
                                      StencilIn<T>& si) {
    constexpr int n = VW<T>::n;
    const gptr<T> c = as_global((const T*)blk.c);
    const long long loc0 = blk.locbase + l0;
    ld16(v + u0, si.xv);
    ldg16(c + loc0, si.cx);
    ldg16(c + blk.tot + loc0, si.cy);
    ldg16(c + 2 * blk.tot + loc0, si.cz);
    si.vm = v[u0 - 1];
    si.vp = v[u0 + n];
    si.cxm = c[loc0 - 1];
}

// 16-byte loads at element alignment (a run of neighbours starts anywhere)
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));
typedef double f64x2u __attribute__((ext_vector_type(2), aligned(8)));
template <typename T>
__device__ inline void ldg16u(gptr<T> p, T (&o)[VW<T>::n]) {
    if constexpr (sizeof(T) == 4) {
        const f32x4u t = *(const __attribute__((address_space(1))) f32x4u*)p;
        o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
    } else {
        const f64x2u t = *(const __attribute__((address_space(1))) f64x2u*)p;
        o[0] = t.x; o[1] = t.y;
    }
}

template <typename T>
__device__ inline void stencil_finish(const T* __restrict__ v, const Block& blk, int l0, const StencilIn<T>& si,
                                      T (&out)[VW<T>::n]) {
    constexpr int n = VW<T>::n;
    const gptr<T> c = as_global((const T*)blk.c);
    const gptr<T> vg = as_global(v);
    T gyp[n], gym[n], cym[n], gzp[n], gzm[n], czm[n];
    // When the neighbours of the lane's n consecutive unknowns are n consecutive unknowns
    // in every direction (rows inside the domain), each neighbour operand is one 16-byte
    // load instead of n single-element gathers.  The choice is per lane: both paths read
    // the same elements, and on masked boxes many waves hold a few lanes at the domain's
    // edge (measured against a per-wave choice: config 2 11.7 -> 11.3 us per launch)
    bool run = true;
#pragma unroll
    for (int e = 1; e < n; ++e)
        run = run && si.nb[e].x == si.nb[0].x + e && si.nb[e].y == si.nb[0].y + e && si.nb[e].z == si.nb[0].z + e &&
              si.nb[e].w == si.nb[0].w + e;
    if (run) {
        ldg16u<T>(vg + blk.base + si.nb[0].y, gyp);
        ldg16u<T>(vg + blk.base + si.nb[0].x, gym);
        ldg16u<T>(c + blk.tot + blk.locbase + si.nb[0].x, cym);
        ldg16u<T>(vg + blk.base + si.nb[0].w, gzp);
        ldg16u<T>(vg + blk.base + si.nb[0].z, gzm);
        ldg16u<T>(c + 2 * blk.tot + blk.locbase + si.nb[0].z, czm);
    } else {
#pragma unroll
        for (int e = 0; e < n; ++e) {
            gyp[e] = v[blk.base + si.nb[e].y];
            gym[e] = v[blk.base + si.nb[e].x];
            cym[e] = c[blk.tot + blk.locbase + si.nb[e].x];
            gzp[e] = v[blk.base + si.nb[e].w];
            gzm[e] = v[blk.base + si.nb[e].z];
            czm[e] = c[2 * blk.tot + blk.locbase + si.nb[e].z];
        }
    }
    // keep the gathers ahead of any arithmetic on the direct operands
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int e = 0; e < n; ++e) {
        const T left = e == 0 ? si.vm : si.xv[e - 1];
        const T leftc = e == 0 ? si.cxm : si.cx[e - 1];
        const T right = e == n - 1 ? si.vp : si.xv[e + 1];
        T r = si.xv[e];
        r += si.cx[e] * right;
        r += leftc * left;
        r += si.cy[e] * gyp[e];
        r += cym[e] * gym[e];
        r += si.cz[e] * gzp[e];
        r += czm[e] * gzm[e];
        out[e] = (l0 + e < blk.N) ? r : T(0);
    }
}

// Step J, kernel A: z = B u_J (J = 0: z = B q_0) into W, and the partial sums of the
// step's dot products.  The activity flags of all systems are read with the block
// record, and the basis vectors of the range are requested with the stencil's own
// operands, so a block waits for memory three times: block record, operands,
// neighbour values.
template <typename T, int J>
__global__ __launch_bounds__(kThreads) void k_dc_spmv_dot(KArgs<T> a) {
    constexpr int n = VW<T>::n;
    constexpr int NR = J == 0 ? 1 : 2 * J + 2;
    const int lane = threadIdx.x & 63;
    const int actv = lane < a.nsys ? a.sk[lane].active : 0;
    double vs0v = 0.0;
    if constexpr (J == 0) vs0v = lane < a.nsys ? a.sk[lane].vs[0] : 0.0;
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    const int act = __builtin_amdgcn_readlane(actv, blk.sys);
    T sc = T(1);
    if constexpr (J == 0) {
        // step 0 takes up pending systems (its first block marks them running)
        if (act == kIdle) return;
        if (blk.slot == blk.slot0 && threadIdx.x == 0) a.sk[blk.sys].active = kRunning;
        sc = (T)rdl(vs0v, blk.sys);
    } else {
        if (act != kRunning) return;
    }
    const T* U = a.V + (long long)J * a.ldv;
    // per-thread sums in the Krylov type (a few products each), block sums in FP64
    T acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = T(0);
    // the neighbour indices of the next pass are requested one pass ahead, so that from
    // the second pass on the gathers only wait for indices already in flight
    long long u0 = blk.start + threadIdx.x * n;
    StencilIn<T> si;
    if (u0 < blk.end) stencil_idx<T>(blk, (int)(u0 - blk.base), si);
    for (; u0 < blk.end; u0 += kThreads * n) {
        const int l0 = (int)(u0 - blk.base);
        __builtin_amdgcn_sched_barrier(0);
        T vk[J > 0 ? J : 1][n];
#pragma unroll
        for (int k = 0; k < J; ++k) ld16(a.V + (long long)k * a.ldv + u0, vk[k]);
        stencil_direct<T>(U, blk, u0, l0, si);
        StencilIn<T> nx;
        const long long u1 = u0 + kThreads * n;
        if (u1 < blk.end) stencil_idx<T>(blk, (int)(u1 - blk.base), nx);
        __builtin_amdgcn_sched_barrier(0);
        T z[n];
        stencil_finish<T>(U, blk, l0, si, z);
#pragma unroll
        for (int e = 0; e < n; ++e) si.nb[e] = nx.nb[e];
        const T (&uv)[n] = si.xv;
        if constexpr (J == 0) {
#pragma unroll
            for (int e = 0; e < n; ++e) z[e] *= sc;
        }
        st16(a.W + u0, z);
        if constexpr (J == 0) {
#pragma unroll
            for (int e = 0; e < n; ++e) acc[0] += uv[e] * z[e];
        } else {
#pragma unroll
            for (int k = 0; k < J; ++k) {
#pragma unroll
                for (int e = 0; e < n; ++e) {
                    acc[k] += vk[k][e] * uv[e];
                    acc[J + k] += vk[k][e] * z[e];
                }
            }
#pragma unroll
            for (int e = 0; e < n; ++e) {
                acc[2 * J] += uv[e] * uv[e];
                acc[2 * J + 1] += uv[e] * z[e];
            }
        }
    }
    block_partials<NR>(acc, a.part + (long long)kRowD * a.nslots, a.nslots, blk.slot);
}

// After the last step: the rows of k_dc_spmv_dot without a stencil (t, gamma = 0).
template <typename T, int J>
__global__ __launch_bounds__(kThreads) void k_dc_lastdots(KArgs<T> a) {
    constexpr int n = VW<T>::n;
    constexpr int NR = 2 * J + 2;
    const int lane = threadIdx.x & 63;
    const int actv = lane < a.nsys ? a.sk[lane].active : 0;
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    if (__builtin_amdgcn_readlane(actv, blk.sys) != kRunning) return;
    const T* U = a.V + (long long)J * a.ldv;
    T acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = T(0);
    for (long long u0 = blk.start + threadIdx.x * n; u0 < blk.end; u0 += kThreads * n) {
        T uv[n];
        ld16(U + u0, uv);
#pragma unroll
        for (int k = 0; k < J; ++k) {
            T vk[n];
            ld16(a.V + (long long)k * a.ldv + u0, vk);
#pragma unroll
            for (int e = 0; e < n; ++e) acc[k] += vk[e] * uv[e];
        }
#pragma unroll
        for (int e = 0; e < n; ++e) acc[2 * J] += uv[e] * uv[e];
    }
    block_partials<NR>(acc, a.part + (long long)kRowD * a.nslots, a.nslots, blk.slot);
}

// Scalar work of step J >= 1 (wave 0 of every block, one Hessenberg row per lane; only
// the lead block stores; the first-pass coefficients alternate between two buffers so
// that no block reads what the lead block of the same launch writes): finish column
// J-1 (Givens, convergence, back-substitution when the cycle ends) and, if the cycle
// goes on, the coefficients of q_J on V_k (sq) and of u_{J+1} on V_k and q_J (sc),
// and beta_J.  H holds columns 0..J-2 of the Hessenberg matrix.  Returns done.
template <int J>
__device__ inline bool dc_scalars(SysK* sk, const TailIn& ti, double hprev, const double* red, const double* H,
                                  int restart, bool lead, double* sq, double* sc, double* sbeta) {
    constexpr int LD = kMaxM + 1;
    constexpr int Jc = J - 1;
    const int lane = threadIdx.x & 63;
    const double vsl = lane < J ? ti.vsl : 0.0;
    const double s = lane < J ? vsl * red[lane] : 0.0;
    const double t = lane < J ? vsl * red[J + lane] : 0.0;
    const double ss = wsum(s * s), st = wsum(s * t);
    const double alpha = red[2 * J], gam = red[2 * J + 1];
    const double b2 = alpha - ss;
    const double beta = b2 > 0.0 ? sqrt(b2) : 0.0;
    // column J-1 of the Hessenberg matrix: first pass + correction, beta below
    const double v = lane < J ? hprev + s : (lane == J ? beta : 0.0);
    if (lead) {
        if (lane <= J) sk->Hraw[Jc * LD + lane] = v;
        if (lane == 0) sk->vs[J] = 1.0;
    }
    const bool done = column_tail<Jc>(sk, ti, v, beta, restart, lead);
    if (!done) {
        // g = H[0:J+1, 0:J] s (lane k = row k; column i has rows <= i + 1)
        double g = 0.0;
#pragma unroll
        for (int i = 0; i < Jc; ++i) {
            const double si = rdl(s, i);
            if (lane <= i + 1) g += H[i * LD + lane] * si;
        }
        g += v * rdl(s, Jc);
        const double qz = (gam - st) / beta;
        const double tk = lane < J ? t : qz;
        const double h = (tk - g) / beta;
        const double cc = g / beta + h;
        if (lane <= J) {
            if (lead) sk->hc[J & 1][lane] = h;
            sc[lane] = lane < J ? cc * vsl : cc;
        }
        if (lane < J) sq[lane] = s * vsl;
        if (lane == 0) *sbeta = beta;
    }
    return done;
}

// Step J, kernel B: from the reduced dot products, finish q_J = (u_J - Q s) / beta in
// place and form u_{J+1} = z / beta - Q c (J = 0: u_1 = z - h_00 q_0).  Everything a
// block reads (partial sums, the system's scalars, the Hessenberg columns and the
// vectors of its range) is requested in one go once the block record is in.
template <typename T, int J>
__global__ __launch_bounds__(kThreads) void k_dc_axpy(KArgs<T> a) {
    constexpr int n = VW<T>::n;
    constexpr int NR = J == 0 ? 1 : 2 * J + 2;
    constexpr int LD = kMaxM + 1;
    constexpr int NH = J >= 2 ? (J - 1) * LD : 0;
    constexpr int HPT = (NH + kThreads - 1) / kThreads;
    __shared__ double red[NR];
    __shared__ double sH[NH > 0 ? NH : 1];
    __shared__ double sq[J > 0 ? J : 1];
    __shared__ double scf[J + 1];
    __shared__ double sbeta;
    __shared__ int s_done;
    const int lane = threadIdx.x & 63;
    const int actv = lane < a.nsys ? a.sk[lane].active : 0;
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    if (__builtin_amdgcn_readlane(actv, blk.sys) != kRunning) return;
    SysK* sk = a.sk + blk.sys;
    const bool lead = blk.slot == blk.slot0;
    const double* part = a.part + (long long)kRowD * a.nslots;
    // ---- all loads of the block, issued together
    PartLoad<NR> pl;
    load_partials<NR>(part, a.nslots, blk.slot0, blk.nb, pl);
    TailIn ti{};
    double hprev = 0.0;
    if (threadIdx.x < 64) {
        if constexpr (J == 0) {
            ti.vsl = sk->vs[0];
        } else {
            ti = load_tail(sk, J - 1);
            hprev = lane < J ? sk->hc[(J - 1) & 1][lane] : 0.0;
        }
    }
    double hr[HPT > 0 ? HPT : 1];
#pragma unroll
    for (int q = 0; q < HPT; ++q) {
        const int i = threadIdx.x + q * kThreads;
        hr[q] = i < NH ? sk->Hraw[i] : 0.0;
    }
    T* UJ = a.V + (long long)J * a.ldv;
    T* UN = a.V + (long long)(J + 1) * a.ldv;
    long long u0 = blk.start + threadIdx.x * n;
    T z[n], uj[n], vk[J > 0 ? J : 1][n];
    auto load_range = [&](long long u) {
        ld16(a.W + u, z);
        if constexpr (J > 0) {
            ld16(UJ + u, uj);
#pragma unroll
            for (int k = 0; k < J; ++k) ld16(a.V + (long long)k * a.ldv + u, vk[k]);
        } else {
            ld16(a.V + u, vk[0]);
        }
    };
    if (u0 < blk.end) load_range(u0);
    // ---- reductions and the scalar work
    sum_partials<NR>(part, a.nslots, blk.slot0, blk.nb, pl, red);
#pragma unroll
    for (int q = 0; q < HPT; ++q) {
        const int i = threadIdx.x + q * kThreads;
        if (i < NH) sH[i] = hr[q];
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        bool done = false;
        if constexpr (J == 0) {
            const double vs0 = ti.vsl;
            const double h0 = vs0 * red[0];
            if (lane == 0) {
                if (lead) sk->hc[0][0] = h0;
                scf[0] = h0 * vs0;
                sbeta = 1.0;
            }
        } else {
            done = dc_scalars<J>(sk, ti, hprev, red, sH, a.prm->restart, lead, sq, scf, &sbeta);
        }
        if (lane == 0) s_done = done ? 1 : 0;
    }
    __syncthreads();
    if (s_done) return;
    const double ib = 1.0 / sbeta;
    double cq[J > 0 ? J : 1], cu[J + 1];
#pragma unroll
    for (int k = 0; k < J; ++k) cq[k] = sq[k];
#pragma unroll
    for (int k = 0; k <= J; ++k) cu[k] = scf[k];
    while (u0 < blk.end) {
        double un[n];
        if constexpr (J > 0) {
            double q[n];
#pragma unroll
            for (int e = 0; e < n; ++e) {
                q[e] = (double)uj[e];
                un[e] = (double)z[e] * ib;
            }
#pragma unroll
            for (int k = 0; k < J; ++k)
#pragma unroll
                for (int e = 0; e < n; ++e) {
                    q[e] -= cq[k] * (double)vk[k][e];
                    un[e] -= cu[k] * (double)vk[k][e];
                }
            T qs[n];
#pragma unroll
            for (int e = 0; e < n; ++e) {
                q[e] *= ib;
                qs[e] = (T)q[e];
                un[e] -= cu[J] * (double)qs[e];
            }
            st16(UJ + u0, qs);
        } else {
#pragma unroll
            for (int e = 0; e < n; ++e) un[e] = (double)z[e] - cu[0] * (double)vk[0][e];
        }
        T us[n];
#pragma unroll
        for (int e = 0; e < n; ++e) us[e] = (T)un[e];
        st16(UN + u0, us);
        u0 += kThreads * n;
        if (u0 < blk.end) load_range(u0);
    }
}

// End of the cycle: finish the last column (one block per system).
template <typename T, int J>
__global__ __launch_bounds__(kThreads) void k_dc_finish(KArgs<T> a, int sys0) {
    constexpr int NR = 2 * J + 2;
    constexpr int LD = kMaxM + 1;
    SysK* sk = a.sk + sys0 + blockIdx.x;
    if (sk->active != kRunning) return;
    __shared__ double red[NR];
    __shared__ double sq[J], scf[J + 1], sbeta;
    reduce_partials<NR>(a.part + (long long)kRowD * a.nslots, a.nslots, sk->slot0, sk->nblocks, red);
    if (threadIdx.x < 64) {
        const TailIn ti = load_tail(sk, J - 1);
        const double hprev = (threadIdx.x & 63) < J ? sk->hc[(J - 1) & 1][threadIdx.x & 63] : 0.0;
        // the cycle ends here (J = m): the H columns are not needed
        (void)dc_scalars<J>(sk, ti, hprev, red, sk->Hraw, a.prm->restart, true, sq, scf, &sbeta);
        (void)LD;
    }
}

// ------------------------------------------------------------------ warm start
// Network input on the box grid of problem p: channels [c (S), k (S), D (S), s (S), mask,
// d (S)], each multiplied by its scale, BF16.  This kernel writes the static channels
// (k, D, s and the mask, zero beyond the box) and zero c and d channels; c and d of the
// domain voxels are written by the step's first residual pass (k_residual with WSIN) or,
// for training pairs, by k_ws_resid, so that only those run again while the grid,
// domain and scales stay the same.  Threads (64, 4) over (x, y) of one z plane per
// block row.
__global__ __launch_bounds__(256) void k_ws_input(ProbDev pd, int S, const float* stat, const float* scales,
                                                  uint16_t* in) {
    const int gx = pd.gd[0], gy = pd.gd[1];
    const int x = (int)blockIdx.x * 64 + (int)threadIdx.x;
    const int y = (int)blockIdx.y * 4 + (int)threadIdx.y;
    const int z = (int)blockIdx.z;
    if (x >= gx || y >= gy) return;
    const long long i = ((long long)z * gy + y) * gx + x;
    const int C = ws_channels(S);
    uint16_t val[ws_channels(MPM_MAX_SPECIES)];
    for (int s = 0; s < S; ++s) val[s] = 0;
    const long long G = (long long)gx * gy * pd.gd[2];
    float sc[ws_static_channels(MPM_MAX_SPECIES)], sv[ws_static_channels(MPM_MAX_SPECIES)];
    for (int c = 0; c < ws_static_channels(S); ++c) {
        sc[c] = scales[S + c];
        sv[c] = stat[c * G + i];   // channel-major, zero beyond the box
    }
    for (int c = 0; c < ws_static_channels(S); ++c) val[S + c] = to_bf16(sv[c] * sc[c]);
    for (int c = 4 * S + 1; c < C; ++c) val[c] = 0;
    if (C % 8 == 0 && ((uintptr_t)in & 15) == 0) {   // three species: 16 channels, two 16-byte stores
        uint4* o = reinterpret_cast<uint4*>(in + i * C);
        for (int q = 0; q < C / 8; ++q) {
            const uint16_t* w = val + 8 * q;
            o[q] = make_uint4(w[0] | ((uint32_t)w[1] << 16), w[2] | ((uint32_t)w[3] << 16),
                              w[4] | ((uint32_t)w[5] << 16), w[6] | ((uint32_t)w[7] << 16));
        }
    } else {
        for (int c = 0; c < C; ++c) in[i * C + c] = val[c];
    }
}

// Launch k_ws_input over the grid of problem p.
static void launch_ws_input(const ProbHost& ph, const ProbDev& pd, int S, const float* scales, uint16_t* in,
                            hipStream_t st) {
    const dim3 grid((unsigned)((ph.gd[0] + 63) / 64), (unsigned)((ph.gd[1] + 3) / 4), (unsigned)ph.gd[2]);
    k_ws_input<<<grid, dim3(64, 4), 0, st>>>(pd, S, ph.stat, scales, in);
}

// Grid index of compact voxel l of a problem.
__device__ inline long long grid_index(const ProbDev& pd, int l) { return grid_of_voxel(pd, pd.vox[l]); }

// For the systems not already converged at c^n (x holds c^n): x += out * out_scale
// (MPM_WS_NET), x = 2 x - c^{n-1} (MPM_WS_EXTRAP) or x = (2 x - c^{n-1}) + out * out_scale
// (MPM_WS_NET_EXTRAP: the network's correction of the extrapolated start).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_ws_apply(KArgs<T> a, int mode, const float* scales) {
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    const SysK* sk = a.sk + blk.sys;
    if (sk->converged) return;
    const ProbDev pd = a.probs[blk.sys / a.S];
    const Where wh = where_of(a, blk, pd);
    const float os = scales[kScaleOut + wh.s];
    // four unknowns per thread, every load issued before the first use
    constexpr int n = 4;
    for (long long u0 = blk.start + threadIdx.x * n; u0 < blk.end; u0 += kThreads * n) {
        const int l0 = (int)(u0 - wh.base);
        double xv[n], w[n], o[n];
#pragma unroll
        for (int e = 0; e < n; ++e) {
            const bool in = l0 + e < pd.N;
            xv[e] = in ? a.x[u0 + e] : 0.0;
            w[e] = in && mode != MPM_WS_EXTRAP ? (double)(pd.wsout[grid_index(pd, l0 + e) * a.S + wh.s] * os) : 0.0;
            o[e] = in && mode != MPM_WS_NET ? a.pold[u0 + e] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < n; ++e) {
            if (l0 + e >= pd.N) continue;
            const double xb = mode == MPM_WS_NET ? xv[e] : 2.0 * xv[e] - o[e];
            a.x[u0 + e] = mode == MPM_WS_EXTRAP ? xb : xb + w[e];
        }
    }
}

// The per-step channels of the network input on the domain voxels of problem p (for
// the training pairs; a step writes them in its first residual pass), each times its
// scale, BF16: c^n (channel s, from the lattice field) and the Jacobi-scaled
// residual of the base start, d = r / A_PP = S (S r) (channel 4 S + 1 + s).  V holds
// S r of the base start from the step's first residual pass (which, for the correction
// of the extrapolation, forms it for x_b = 2 c^n - c^{n-1}), before any Arnoldi step
// overwrites it.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_ws_resid(KArgs<T> a, int p, const double* field, const float* scales,
                                                       uint16_t* dst) {
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0 || blk.p != p) return;
    const ProbDev pd = a.probs[p];
    const Where wh = where_of(a, blk, pd);
    const int C = ws_channels(a.S);
    const int ch = 4 * a.S + 1 + wh.s;
    const float scale = scales[ch], cscale = scales[wh.s];
    const double* f = field + (long long)wh.s * pd.nvox;
    // four unknowns per thread, every load issued before the first use
    constexpr int n = 4;
    for (long long u0 = blk.start + threadIdx.x * n; u0 < blk.end; u0 += kThreads * n) {
        const int l0 = (int)(u0 - wh.base);
        int vx[n];
        double sv[n], cv[n];
        T vv[n];
#pragma unroll
        for (int e = 0; e < n; ++e) {
            const bool in = l0 + e < pd.N;
            vx[e] = in ? pd.vox[l0 + e] : 0;
            sv[e] = in ? pd.sc64[wh.locbase + l0 + e] : 0.0;
            vv[e] = in ? a.V[u0 + e] : T(0);
        }
#pragma unroll
        for (int e = 0; e < n; ++e) cv[e] = l0 + e < pd.N ? f[vx[e]] : 0.0;
#pragma unroll
        for (int e = 0; e < n; ++e) {
            if (l0 + e >= pd.N) continue;
            const double d = sv[e] * (double)vv[e];
            uint16_t* o = dst + grid_of_voxel(pd, vx[e]) * C;
            o[ch] = to_bf16((float)d * scale);
            o[wh.s] = to_bf16((float)cv[e] * cscale);
        }
    }
}

// Back to x = c^n for the systems whose warm start was rejected.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_ws_revert(KArgs<T> a) {
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    const SysK* sk = a.sk + blk.sys;
    if (!sk->fallback) return;
    const ProbDev pd = a.probs[blk.sys / a.S];
    const Where wh = where_of(a, blk, pd);
    const double* f = a.fields[wh.p] + (long long)wh.s * pd.nvox;
    for (long long u = blk.start + threadIdx.x; u < blk.end; u += kThreads) {
        const int l = (int)(u - wh.base);
        if (l < pd.N) a.x[u] = f[pd.vox[l]];
    }
}

// x = 2 x - c_prev on the domain unknowns of the blocks' systems (x holds c_old gathered
// from the lattice; c_prev: lattice fields of the step before).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_ws_extrap_x(KArgs<T> a, const double* c_prev) {
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    const ProbDev pd = a.probs[blk.sys / a.S];
    const Where wh = where_of(a, blk, pd);
    const double* f = c_prev + (long long)wh.s * pd.nvox;
    for (long long u = blk.start + threadIdx.x; u < blk.end; u += kThreads) {
        const int l = (int)(u - wh.base);
        if (l < pd.N) a.x[u] = 2.0 * a.x[u] - f[pd.vox[l]];
    }
}

// Training target on the grid: (c_new - x_b) / out_scale on domain voxels, else 0, with
// the base start x_b = c_old, or 2 c_old - c_prev when c_prev is given.
__global__ void k_ws_target(ProbDev pd, int S, int bx, int by, int bz, const double* c_prev, const double* c_old,
                            const double* c_new, const float* stat, const float* scales, float* tgt) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long G = (long long)pd.gd[0] * pd.gd[1] * pd.gd[2];
    if (i >= G) return;
    const int gx = pd.gd[0], gy = pd.gd[1];
    const int x = (int)(i % gx);
    const int y = (int)((i / gx) % gy);
    const int z = (int)(i / ((long long)gx * gy));
    const bool dom = x < bx && y < by && z < bz && stat[3 * S * G + i] > 0.f;   // the mask channel
    const long long v = ((long long)(pd.lo[2] + z) * pd.ny + (pd.lo[1] + y)) * pd.nx + (pd.lo[0] + x);
    for (int s = 0; s < S; ++s) {
        float t = 0.f;
        if (dom) {
            const double xb = c_prev ? 2.0 * c_old[s * pd.nvox + v] - c_prev[s * pd.nvox + v] : c_old[s * pd.nvox + v];
            t = (float)((c_new[s * pd.nvox + v] - xb) / (double)scales[kScaleOut + s]);
        }
        tgt[i * S + s] = t;
    }
}

// ------------------------------------------------------------------ residual loss
// Training loss of the warm start measured by the residual its prediction leaves: for a
// predicted change o (network output, in units of out_scale) and the solved change t of
// the same step, the start c^n + o out_scale leaves b - A (c^n + o out_scale) = -A e
// with e = (o - t) out_scale, so the loss is the Jacobi-scaled residual
//   L = sum_{s,l} (w_{s,l} / out_scale_s)^2 / (S N),  w = S A e  (S = diag(A)^(-1/2)),
// and, A being symmetric, dL/do_{s,l} = 2 (A S w)_{s,l} / (S N out_scale_s).  All in
// FP64 on the domain unknowns of one problem; the grid maps to them by grid_index.

// 7-point product (A y)_P over a problem's compact unknowns, y read through 'val', with
// the couplings of the block's system (FP64, unscaled; the -d coupling of P is the +d
// coupling of its -d neighbour).
template <typename F>
__device__ inline double apply_a64(const Block& blk, int l, F val) {
    const long long loc = blk.locbase + l;
    const int4 nb = blk.nbr[l];
    double r = blk.d64[loc] * val(l);
    r += blk.a64[loc] * val(l + 1) + blk.a64[loc - 1] * val(l - 1);
    r += blk.a64[blk.tot + loc] * val(nb.y) + blk.a64[blk.tot + blk.locbase + nb.x] * val(nb.x);
    r += blk.a64[2 * blk.tot + loc] * val(nb.w) + blk.a64[2 * blk.tot + blk.locbase + nb.z] * val(nb.z);
    return r;
}

// e = (out - target) out_scale on the domain unknowns of problem p (0 on padding).
__global__ __launch_bounds__(kThreads) void k_wsl_err(const Block* blocks, const ProbDev* probs, int S, int p,
                                                      const float* out, const float* tgt, const float* scales,
                                                      double* e) {
    const Block blk = blocks[blockIdx.x];
    if (blk.sys < 0 || blk.p != p) return;
    const ProbDev pd = probs[p];
    const double os = scales[kScaleOut + blk.s];
    for (long long u = blk.start + threadIdx.x; u < blk.end; u += kThreads) {
        const int l = (int)(u - blk.base);
        double v = 0.0;
        if (l < pd.N) {
            const long long gi = grid_index(pd, l) * S + blk.s;
            v = ((double)out[gi] - (double)tgt[gi]) * os;
        }
        e[u] = v;
    }
}

// mode 0: w = S (A e) and per-block partial sums of (w / out_scale)^2 in part[block];
// mode 1: g = A (S w).  x is read on the block's system, y written on it.
__global__ __launch_bounds__(kThreads) void k_wsl_apply(const Block* blocks, int p, int mode, const float* scales,
                                                        const double* x, double* y, double* part) {
    const Block blk = blocks[blockIdx.x];
    const bool mine = blk.sys >= 0 && blk.p == p;
    double acc[1] = {0.0};
    if (mine) {
        const double* xs = x + blk.base;
        const double* sc = blk.sc64 + blk.locbase;
        const double os = scales[kScaleOut + blk.s];
        for (long long u = blk.start + threadIdx.x; u < blk.end; u += kThreads) {
            const int l = (int)(u - blk.base);
            double r = 0.0;
            if (l < blk.N) {
                if (mode == 0) {
                    r = sc[l] * apply_a64(blk, l, [&](int q) { return xs[q]; });
                    acc[0] += (r / os) * (r / os);
                } else {
                    r = apply_a64(blk, l, [&](int q) { return sc[q] * xs[q]; });
                }
            }
            y[u] = r;
        }
    }
    if (mode == 0) block_partials<1>(acc, part, 1, blockIdx.x);
}

// grad[grid voxel of l][s] = coef_s g (domain voxels only; the caller zeroes the grid).
__global__ __launch_bounds__(kThreads) void k_wsl_grad(const Block* blocks, const ProbDev* probs, int S, int p,
                                                       const double* g, double coef, const float* scales,
                                                       float* grad) {
    const Block blk = blocks[blockIdx.x];
    if (blk.sys < 0 || blk.p != p) return;
    const ProbDev pd = probs[p];
    const double cs = coef / (double)scales[kScaleOut + blk.s];
    for (long long u = blk.start + threadIdx.x; u < blk.end; u += kThreads) {
        const int l = (int)(u - blk.base);
        if (l < pd.N) grad[grid_index(pd, l) * S + blk.s] = (float)(cs * g[u]);
    }
}

__global__ void k_fill0(float* p, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// ------------------------------------------------------------------ dispatch tables
template <typename T>
using KFn = void (*)(KArgs<T>);
template <typename T>
using KFinFn = void (*)(KArgs<T>, int);

template <typename T, int... Js>
static std::array<KFn<T>, sizeof...(Js)> table_k1(std::integer_sequence<int, Js...>) {
    return {&k_spmv_dot<T, Js>...};
}
template <typename T, int... Js>
static std::array<KFn<T>, sizeof...(Js)> table_k2(std::integer_sequence<int, Js...>) {
    return {&k_axpy_dot<T, Js>...};
}
template <typename T, int... Js>
static std::array<KFn<T>, sizeof...(Js)> table_k3(std::integer_sequence<int, Js...>) {
    return {&k_axpy_norm<T, Js>...};
}
template <typename T, int... Js>
static std::array<KFinFn<T>, sizeof...(Js)> table_k4(std::integer_sequence<int, Js...>) {
    return {&k_finish<T, Js>...};
}

template <typename T, int... Js>
static std::array<KFn<T>, sizeof...(Js)> table_da(std::integer_sequence<int, Js...>) {
    return {&k_dc_spmv_dot<T, Js>...};
}
template <typename T, int... Js>
static std::array<KFn<T>, sizeof...(Js)> table_db(std::integer_sequence<int, Js...>) {
    return {&k_dc_axpy<T, Js>...};
}
template <typename T, int... Js>
static std::array<KFn<T>, sizeof...(Js)> table_dl(std::integer_sequence<int, Js...>) {
    return {&k_dc_lastdots<T, Js + 1>...};
}
template <typename T, int... Js>
static std::array<KFinFn<T>, sizeof...(Js)> table_df(std::integer_sequence<int, Js...>) {
    return {&k_dc_finish<T, Js + 1>...};
}

template <typename T>
struct Kernels {
    std::array<KFn<T>, kMaxM> k1, k2, k3;
    std::array<KFinFn<T>, kMaxM> k4;
    std::array<KFn<T>, kMaxM> da, db, dl;   // dl[m - 1], df[m - 1]: after m steps
    std::array<KFinFn<T>, kMaxM> df;
    Kernels() {
        k1 = table_k1<T>(std::make_integer_sequence<int, kMaxM>{});
        k2 = table_k2<T>(std::make_integer_sequence<int, kMaxM>{});
        k3 = table_k3<T>(std::make_integer_sequence<int, kMaxM>{});
        k4 = table_k4<T>(std::make_integer_sequence<int, kMaxM>{});
        da = table_da<T>(std::make_integer_sequence<int, kMaxM>{});
        db = table_db<T>(std::make_integer_sequence<int, kMaxM>{});
        dl = table_dl<T>(std::make_integer_sequence<int, kMaxM>{});
        df = table_df<T>(std::make_integer_sequence<int, kMaxM>{});
    }
};

template <typename T>
static const Kernels<T>& kernels() {
    static Kernels<T> k;
    return k;
}

// ------------------------------------------------------------------ host side
static void free_work(Ctx* c) {
    if (c->V) (void)hipFree(c->V);
    if (c->W) (void)hipFree(c->W);
    if (c->x) (void)hipFree(c->x);
    if (c->b) (void)hipFree(c->b);
    c->V = c->W = nullptr;
    c->x = c->b = nullptr;
    c->cap_U = 0;
}

static size_t ksize(const Ctx* c) { return c->opt.precision == MPM_FP64 ? 8 : 4; }

// Split each system into blocks of 'per' unknowns (a multiple of kAlign), build the
// XCD-aware batched table and the per-system tables.
static void build_tables(Ctx* c, long long per, int group) {
    const int S = c->S;
    const int nsys = S * c->P;
    per = std::max<long long>(kAlign, (per + kAlign - 1) / kAlign * kAlign);
    c->block_unknowns = (int)per;
    std::vector<Block> logical;            // per system, in slot order
    c->sys_first.assign(nsys, 0);
    c->sys_count.assign(nsys, 0);
    const bool f64 = c->opt.precision == MPM_FP64;
    int slot = 0;
    for (int p = 0; p < c->P; ++p) {
        const ProbHost& ph = c->probs[p];
        const int nbp = (int)((ph.Npad + per - 1) / per);
        for (int s = 0; s < S; ++s) {
            const int sys = p * S + s;
            const long long base = c->off[p] + (long long)s * ph.Npad;
            c->sys_first[sys] = slot;
            for (int i = 0; i < nbp; ++i) {
                const long long a0 = (long long)i * per;
                Block b{};
                b.sys = sys;
                b.start = (int)(base + a0);
                b.end = (int)(base + std::min<long long>(ph.Npad, a0 + per));
                b.slot = slot++;
                b.slot0 = c->sys_first[sys];
                b.nb = nbp;
                b.N = ph.N;
                b.tot = S * ph.Npad;
                b.base = base;
                b.locbase = (long long)s * ph.Npad;
                b.nbr = ph.nbr;
                b.c = f64 ? (const void*)ph.c64 : (const void*)ph.c32;
                b.a64 = ph.a64;
                b.d64 = ph.d64;
                b.sc64 = ph.sc64;
                b.q64 = ph.q64;
                b.vox = ph.vox;
                b.p = p;
                b.s = s;
                b.nvox = ph.nvox;
                logical.push_back(b);
            }
            c->sys_count[sys] = nbp;
        }
    }
    c->nslots = slot;
    auto swizzle = [](const std::vector<Block>& L, std::vector<Block>& out) {
        const size_t nb = L.size();
        const size_t per = (nb + 7) / 8;
        const size_t padded = per * 8;
        Block idle{};
        idle.sys = -1;
        for (size_t b = 0; b < padded; ++b) {
            const size_t xcd = b % 8, pos = b / 8;
            const size_t li = xcd * per + pos;
            out.push_back(li < nb ? L[li] : idle);
        }
    };
    // batched table: the species of one voxel range next to each other, so that an
    // XCD fetches a range's neighbour table once for all species
    std::vector<Block> inter;
    inter.reserve(logical.size());
    for (int p = 0; p < c->P; ++p) {
        const int nbp = c->sys_count[p * S];
        for (int i = 0; i < nbp; ++i)
            for (int s = 0; s < S; ++s) inter.push_back(logical[c->sys_first[p * S + s] + i]);
    }
    c->blocks.clear();
    swizzle(inter, c->blocks);
    // The delayed scheme's axpy kernel may run over 'group' consecutive blocks of a
    // system per block: fewer blocks each read all partial sums of their system (the
    // bulk of that kernel's traffic at small splits), while the stencil kernel keeps
    // one pass per thread.  The records keep the system's partial-sum layout (slot0,
    // nb) of the batched table; only the first block of a system has slot == slot0.
    c->axpy_group = group;
    std::vector<Block> ax;
    for (int p = 0; p < c->P; ++p) {
        const int nbp = c->sys_count[p * S];
        for (int i = 0; i < nbp; i += group)
            for (int s = 0; s < S; ++s) {
                const int f = c->sys_first[p * S + s];
                Block b = logical[f + i];
                b.end = logical[f + std::min(nbp, i + group) - 1].end;
                ax.push_back(b);
            }
    }
    c->blocks_ax.clear();
    swizzle(ax, c->blocks_ax);
    c->blocks_sys.clear();
    c->sys_tab_first.assign(nsys, 0);
    for (int sys = 0; sys < nsys; ++sys) {
        std::vector<Block> L(logical.begin() + c->sys_first[sys],
                             logical.begin() + c->sys_first[sys] + c->sys_count[sys]);
        c->sys_tab_first[sys] = (int)c->blocks_sys.size();
        swizzle(L, c->blocks_sys);
    }
}

// Unknowns per block when nothing is tuned: about 160 blocks per system, since every
// block re-reads all partial sums of its system.
static long long model_tile(const Ctx* c) {
    long long maxpad = 0;
    for (auto& ph : c->probs) maxpad = std::max<long long>(maxpad, ph.Npad);
    return std::max<long long>(2048, maxpad / 160);
}

// Copy the block tables and problem descriptors to the device (growing buffers).
static int upload_tables(Ctx* c) {
    hipStream_t st = c->stream;
    const size_t nb = c->blocks.size(), nbs = c->blocks_sys.size(), nbx = c->blocks_ax.size();
    if (nb > c->cap_blocks || nbs > c->cap_blocks || nbx > c->cap_blocks) {
        if (c->d_blocks) (void)hipFree(c->d_blocks);
        if (c->d_blocks_sys) (void)hipFree(c->d_blocks_sys);
        if (c->d_blocks_ax) (void)hipFree(c->d_blocks_ax);
        c->d_blocks = c->d_blocks_sys = c->d_blocks_ax = nullptr;
        const size_t cap = std::max(std::max(nb, nbs), nbx) * 2;
        if (hipMalloc(&c->d_blocks, cap * sizeof(Block)) != hipSuccess ||
            hipMalloc(&c->d_blocks_sys, cap * sizeof(Block)) != hipSuccess ||
            hipMalloc(&c->d_blocks_ax, cap * sizeof(Block)) != hipSuccess) {
            (void)hipGetLastError();
            c->cap_blocks = 0;
            set_error("device allocation of block tables failed");
            return MPM_ENOMEM;
        }
        c->cap_blocks = cap;
    }
    if ((size_t)c->nslots > c->cap_slots) {
        if (c->d_part) (void)hipFree(c->d_part);
        c->d_part = nullptr;
        const size_t cap = (size_t)c->nslots * 2;
        if (hipMalloc(&c->d_part, cap * kPartRows * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            c->cap_slots = 0;
            set_error("device allocation of partial sums failed");
            return MPM_ENOMEM;
        }
        c->cap_slots = cap;
    }
    MPM_HIP(hipMemcpyAsync(c->d_blocks, c->blocks.data(), nb * sizeof(Block), hipMemcpyHostToDevice, st));
    MPM_HIP(hipMemcpyAsync(c->d_blocks_sys, c->blocks_sys.data(), nbs * sizeof(Block), hipMemcpyHostToDevice, st));
    MPM_HIP(hipMemcpyAsync(c->d_blocks_ax, c->blocks_ax.data(), nbx * sizeof(Block), hipMemcpyHostToDevice, st));
    std::vector<int> fc(2 * (size_t)c->S * c->P);
    const int nsys = c->S * c->P;
    for (int s = 0; s < nsys; ++s) {
        fc[s] = c->sys_first[s];
        fc[nsys + s] = c->sys_count[s];
    }
    MPM_HIP(hipMemcpyAsync(c->d_sysfc, fc.data(), fc.size() * sizeof(int), hipMemcpyHostToDevice, st));
    k_sys_init<<<1, 64, 0, st>>>(c->d_sk, c->d_sysfc, c->d_sysfc + nsys, nsys);
    MPM_HIP(hipGetLastError());
    return MPM_OK;
}

template <typename T>
static KArgs<T> make_args(Ctx* c, const Block* blocks);

// A state in which every Arnoldi kernel runs its full streaming path and no cycle
// ends: zero scales (so the Gram-Schmidt coefficients vanish and beta^2 = u.u > 0 on
// the non-zero fill of the basis), zero tolerance, identity rotations.  The tables
// are re-initialised and the basis re-zeroed after tuning.
__global__ void k_tune_state(SysK* sk, int nsys, int mcount) {
    const int s = blockIdx.x;
    if (s >= nsys) return;
    SysK& k = sk[s];
    for (int i = threadIdx.x; i < kMaxM + 2; i += blockDim.x) {
        k.vs[i] = 0.0;
        k.gt[i] = 1.0;
        k.cs[i] = 1.0;
        k.sn[i] = 0.0;
        k.hc[0][i] = 0.0;
        k.hc[1][i] = 0.0;
    }
    for (int i = threadIdx.x; i < (kMaxM + 1) * (kMaxM + 1); i += blockDim.x) k.Hraw[i] = 0.0;
    for (int i = threadIdx.x; i < kMaxM + 2; i += blockDim.x) k.y[i] = 0.0;
    if (threadIdx.x == 0) {
        k.eta = 0.0;
        k.active = 1;
        k.need_update = 1;   // the update streams mcount vectors with zero coefficients
        k.mcount = mcount;
    }
}

// Timing-based choice of the unknowns per block: run the kernels of Arnoldi steps 0
// and 8 of the selected Gram-Schmidt variant (in the tuning state above) for each
// candidate split, three times, and keep the split with the fastest repetition.  The
// choice is cached per layout.
template <typename T>
static int autotune_t(Ctx* c, long long* best_out, int* group_out) {
    hipStream_t st = c->stream;
    const Kernels<T>& K = kernels<T>();
    const int J = std::min(8, c->opt.restart - 1);
    if (J < 0 || J + 1 > c->opt.restart) {
        set_error("autotune: restart out of range");
        return MPM_EINVAL;
    }
    const int nsys = c->S * c->P;
    const bool dc = c->opt.ortho == MPM_ORTHO_DCGS2;
    long long maxpad = 0;
    for (auto& ph : c->probs) maxpad = std::max<long long>(maxpad, ph.Npad);
    hipEvent_t e0, e1;
    MPM_HIP(hipEventCreate(&e0));
    MPM_HIP(hipEventCreate(&e1));
    const size_t vbytes = (size_t)(c->opt.restart + 1) * c->ldv * ksize(c);
    MPM_HIP(hipMemsetAsync(c->V, 0x3c, vbytes, st));   // finite, non-zero fill
    // Time one work split: the two kernels of Arnoldi steps 0 and J (the axpy kernel over
    // its grouped table) three times plus one residual and one update; best of three.
    auto time_split = [&](long long tile, int group, float* out) -> int {
        build_tables(c, tile, group);
        int rc = upload_tables(c);
        if (rc != MPM_OK) return rc;
        // the update reads V_0..V_{mcount-1}: never more than the restart + 1 stored vectors
        k_tune_state<<<nsys, 64, 0, st>>>(c->d_sk, nsys, J + 1);
        KArgs<T> a = make_args<T>(c, c->d_blocks);
        KArgs<T> ax = make_args<T>(c, c->d_blocks_ax);
        const unsigned nb = (unsigned)c->blocks.size(), nbx = (unsigned)c->blocks_ax.size();
        float ms = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            MPM_HIP(hipEventRecord(e0, st));
            for (int it = 0; it < 3; ++it) {
                if (dc) {
                    K.da[0]<<<nb, kThreads, 0, st>>>(a);
                    K.db[0]<<<nbx, kThreads, 0, st>>>(ax);
                    K.da[J]<<<nb, kThreads, 0, st>>>(a);
                    K.db[J]<<<nbx, kThreads, 0, st>>>(ax);
                    // once per cycle in the solve; here once per two Arnoldi steps
                    if (it == 0) {
                        k_residual<T><<<nb, kThreads, 0, st>>>(a, kResCycle);
                        k_update<T><<<nb, kThreads, 0, st>>>(a);
                    }
                } else {
                    K.k1[0]<<<nb, kThreads, 0, st>>>(a);
                    K.k2[J]<<<nb, kThreads, 0, st>>>(a);
                    K.k3[J]<<<nb, kThreads, 0, st>>>(a);
                }
            }
            MPM_HIP(hipEventRecord(e1, st));
            MPM_HIP(hipEventSynchronize(e1));
            float t = 0.0f;
            MPM_HIP(hipEventElapsedTime(&t, e0, e1));
            ms = std::min(ms, t);
        }
        *out = ms;
        return MPM_OK;
    };
    float best_ms = 1e30f;
    long long best = model_tile(c);
    // at most eight passes per thread (the residual and update kernels do not overlap
    // their passes), at most 1024 partial-sum slots per system
    const long long max_tile = 8LL * kThreads * VW<T>::n;
    for (long long tile = 1024; tile <= max_tile; tile *= 2) {
        const long long nbsys = (maxpad + tile - 1) / tile;
        if (nbsys > 1024) continue;            // too many partial sums per system
        if (tile > 1024 && nbsys < 8) break;   // too few blocks per system
        float ms = 0.0f;
        int rc = time_split(tile, 1, &ms);
        if (rc != MPM_OK) return rc;
        if (ms < best_ms) {
            best_ms = ms;
            best = tile;
        }
    }
    // then the grouping of the axpy kernel's blocks for that split
    int best_group = 1;
    if (dc) {
        const long long nbsys = (maxpad + best - 1) / best;
        for (int group = 2; group <= 4 && nbsys >= 4 * group; group *= 2) {
            float ms = 0.0f;
            int rc = time_split(best, group, &ms);
            if (rc != MPM_OK) return rc;
            if (ms < best_ms) {
                best_ms = ms;
                best_group = group;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    MPM_HIP(hipMemsetAsync(c->V, 0, vbytes, st));
    *best_out = best;
    *group_out = best_group;
    return MPM_OK;
}

static void drop_graphs(Ctx* c);

// Diagonal extremes per system (for the bound between the scaled and the unscaled
// residual), after the layout or the coefficients changed.
static int refresh_diag_extremes(Ctx* c) {
    KArgs<double> ka{};
    ka.blocks = c->d_blocks;
    ka.probs = c->d_probs;
    ka.sk = c->d_sk;
    ka.S = c->S;
    k_diag_extremes<double><<<(unsigned)c->blocks.size(), kThreads, 0, c->stream>>>(ka);
    k_sys_kappa<<<1, 64, 0, c->stream>>>(c->d_sk, c->S * c->P);
    MPM_HIP(hipGetLastError());
    c->coef_dirty = false;
    return MPM_OK;
}

int ensure_layout(Ctx* c) {
    if (!c->layout_dirty) {
        // new coefficients on the standing layout: only the per-system extremes change
        return c->coef_dirty ? refresh_diag_extremes(c) : MPM_OK;
    }
    for (int p = 0; p < c->P; ++p) {
        if (!c->probs[p].ready) {
            set_error("problem " + std::to_string(p) + " has not been set up (mpm_fv_setup)");
            return MPM_ESTATE;
        }
    }
    hipStream_t st = c->stream;
    c->off.assign(c->P, 0);
    long long run = kLead;
    for (int p = 0; p < c->P; ++p) {
        c->off[p] = run;
        run += (long long)c->S * c->probs[p].Npad;
    }
    c->U = run - kLead;
    if (run + kAlign > 0x7fffffffLL) {
        set_error("problem too large for 32-bit unknown indices");
        return MPM_EINVAL;
    }
    const size_t need = (size_t)(run + kAlign);
    const int m = c->opt.restart;
    if (need > c->cap_U) {
        // room for growth: a box that grows step by step keeps its workspace
        free_work(c);
        const size_t ks = ksize(c);
        const size_t cap = (need + need / 8 + kAlign - 1) / kAlign * kAlign;
        if (hipMalloc(&c->V, (size_t)(m + 1) * cap * ks) != hipSuccess ||
            hipMalloc(&c->W, cap * ks) != hipSuccess || hipMalloc(&c->x, cap * 8) != hipSuccess ||
            hipMalloc(&c->b, cap * 8) != hipSuccess) {
            (void)hipGetLastError();
            free_work(c);
            set_error("device allocation of the Krylov workspace failed");
            return MPM_ENOMEM;
        }
        c->cap_U = cap;
        c->ldv = (long long)cap;
        MPM_HIP(hipMemsetAsync(c->V, 0, (size_t)(m + 1) * cap * ks, st));
        MPM_HIP(hipMemsetAsync(c->W, 0, cap * ks, st));
        MPM_HIP(hipMemsetAsync(c->x, 0, cap * 8, st));
        MPM_HIP(hipMemsetAsync(c->b, 0, cap * 8, st));
    }
    std::vector<ProbDev> pd(c->P);
    for (int p = 0; p < c->P; ++p) {
        const ProbHost& ph = c->probs[p];
        pd[p].vox = ph.vox;
        pd[p].nbr = ph.nbr;
        pd[p].d64 = ph.d64;
        pd[p].q64 = ph.q64;
        pd[p].a64 = ph.a64;
        pd[p].sc64 = ph.sc64;
        pd[p].c32 = ph.c32;
        pd[p].c64 = ph.c64;
        pd[p].off = c->off[p];
        pd[p].nvox = ph.nvox;
        pd[p].N = ph.N;
        pd[p].Npad = ph.Npad;
        pd[p].nx = ph.dims[0];
        pd[p].ny = ph.dims[1];
        for (int d = 0; d < 3; ++d) {
            pd[p].lo[d] = ph.lo[d];
            pd[p].gd[d] = ph.gd[d];
        }
        pd[p].wsout = ph.wsout;
        pd[p].wsin = ph.wsin;
    }
    // previous-step values for the extrapolated start live on the global unknowns
    c->have_prev = false;
    if (extrap_warm_start(c)) {
        // two halves of need unknowns: c^{n-1} and this step's c^n (see prev_half)
        if (2 * need > c->cap_prev) {
            (void)hipFree(c->prev);
            c->prev = nullptr;
            c->cap_prev = 0;
            if (hipMalloc(&c->prev, 2 * need * 8) != hipSuccess) {
                (void)hipGetLastError();
                set_error("device allocation of the previous-step buffer failed");
                return MPM_ENOMEM;
            }
            c->cap_prev = 2 * need;
            // entries no block covers (the lead, the gaps) stay zero: the residual pass of the
            // corrected extrapolation reads them as stencil neighbours, as it reads those of x
            MPM_HIP(hipMemsetAsync(c->prev, 0, 2 * need * 8, st));
        }
        c->prev_n = need;
    }
    c->h_probs = pd;
    MPM_HIP(hipMemcpyAsync(c->d_probs, pd.data(), c->P * sizeof(ProbDev), hipMemcpyHostToDevice, st));
    c->h_prm->restart = m;
    c->h_prm->S = c->S;
    MPM_HIP(hipMemcpyAsync(c->d_prm, c->h_prm, sizeof(Params), hipMemcpyHostToDevice, st));
    c->up_valid = false;
    // work split: fixed override, cached tuning result, or a fresh autotune.  With a
    // fixed split the axpy kernel of the delayed scheme takes two blocks' ranges per
    // block (measured faster at 1024 and at 4096 unknowns per block).
    long long tile = c->opt.tile_override;
    int group = 2;
    if (tile <= 0) {
        // The tuning result is kept per species count, precision, orthogonalisation and
        // problem count, and per size class of the largest problem and of all unknowns
        // (eight classes per doubling); a layout whose classes are both within one class of
        // a tuned one reuses that result, so boxes that grow step by step are tuned again
        // only after they have grown by about a fifth.
        long long maxpad = 0, total = 0;
        for (auto& ph : c->probs) {
            maxpad = std::max<long long>(maxpad, ph.Npad);
            total += (long long)c->S * ph.Npad;
        }
        const TuneKey key{c->S, (int)ksize(c), c->opt.ortho, c->P, (int)std::floor(8.0 * std::log2((double)maxpad)),
                          (int)std::floor(8.0 * std::log2((double)total))};
        auto near = c->tile_cache.end();
        for (auto it = c->tile_cache.begin(); it != c->tile_cache.end(); ++it) {
            const TuneKey& k = it->first;
            if (k.S == key.S && k.ks == key.ks && k.ortho == key.ortho && k.P == key.P &&
                std::abs(k.cmax - key.cmax) <= 1 && std::abs(k.ctot - key.ctot) <= 1) {
                near = it;
                if (k.cmax == key.cmax && k.ctot == key.ctot) break;   // exact match first
            }
        }
        if (near != c->tile_cache.end()) {
            tile = near->second.first;
            group = near->second.second;
        } else if (c->opt.batched) {
            int rc = ksize(c) == 8 ? autotune_t<double>(c, &tile, &group) : autotune_t<float>(c, &tile, &group);
            if (rc != MPM_OK) return rc;
            c->tile_cache[key] = {tile, group};
        } else {
            tile = model_tile(c);
        }
    }
    build_tables(c, tile, group);
    int rc = upload_tables(c);
    if (rc != MPM_OK) return rc;
    rc = refresh_diag_extremes(c);
    if (rc != MPM_OK) return rc;
    MPM_HIP(hipStreamSynchronize(st));
    drop_graphs(c);
    c->layout_dirty = false;
    return MPM_OK;
}

template <typename T>
static KArgs<T> make_args(Ctx* c, const Block* blocks) {
    KArgs<T> a{};
    a.blocks = blocks;
    a.probs = c->d_probs;
    a.sk = c->d_sk;
    a.part = c->d_part;
    a.prm = c->d_prm;
    a.V = (T*)c->V;
    a.W = (T*)c->W;
    a.x = c->x;
    a.b = c->b;
    a.fields = c->d_fields;
    a.hsk = c->hsk_dev;
    a.pcur = nullptr;
    a.pold = c->prev ? c->prev + (size_t)c->prev_half * c->prev_n : nullptr;
    a.ldv = c->ldv;
    a.nslots = c->nslots;
    a.S = c->S;
    a.nsys = c->S * c->P;
    return a;
}

static bool timed(const Ctx* c, int kind, int j) {
    return c->time_kind == kind && (kind > MPM_KERNEL_AXPY_NORM || c->time_j == j);
}
// Event pairs around timed launches; a launch beyond the allocated pairs is not timed.
static bool tev_room(const Ctx* c) { return 2 * (size_t)c->tev_used + 1 < c->tev.size(); }
static void tev_begin(Ctx* c, hipStream_t st) {
    if (tev_room(c)) (void)hipEventRecord(c->tev[2 * c->tev_used], st);
}
static void tev_end(Ctx* c, hipStream_t st) {
    if (!tev_room(c)) return;
    (void)hipEventRecord(c->tev[2 * c->tev_used + 1], st);
    ++c->tev_used;
}

// What follows the Arnoldi steps of a launched segment.
enum Tail {
    kTailNone = 0,     // more steps of this cycle follow
    kTailUpdate = 1,   // every system ended its cycle: update, residual, next cycle's start
    kTailFull = 2,     // the segment reached step m: last column, then as kTailUpdate
};

// Enqueue Arnoldi steps [j0, j1) of a GMRES cycle and the given tail for one block
// table.  'events' records a start/stop event pair around the timed launch.
template <typename T>
static void enqueue_cycle(Ctx* c, const Block* tab, unsigned nb, int sys0, int nsys, hipStream_t st, int j0,
                          int j1, int tail, bool events) {
    const Kernels<T>& K = kernels<T>();
    KArgs<T> a = make_args<T>(c, tab);
    // the batched launch runs the delayed scheme's axpy kernel over its grouped table
    const bool grouped = tab == c->d_blocks;
    KArgs<T> ax = make_args<T>(c, grouped ? c->d_blocks_ax : tab);
    const unsigned nbx = grouped ? (unsigned)c->blocks_ax.size() : nb;
    auto emit = [&](auto launch, bool is_timed) {
        if (is_timed && events) {
            tev_begin(c, st);
            for (int r = 0; r < c->time_repeat; ++r) launch();
            tev_end(c, st);
        } else {
            launch();
        }
    };
    const int m = c->opt.restart;
    const bool dc = c->opt.ortho == MPM_ORTHO_DCGS2;
    for (int j = j0; j < j1; ++j) {
        if (dc) {
            KFn<T> fa = K.da[j], fb = K.db[j];
            emit([&] { fa<<<nb, kThreads, 0, st>>>(a); }, timed(c, MPM_KERNEL_SPMV_DOT, j));
            emit([&] { fb<<<nbx, kThreads, 0, st>>>(ax); }, timed(c, MPM_KERNEL_AXPY_DOT, j));
        } else {
            const KFn<T> fns[3] = {K.k1[j], K.k2[j], K.k3[j]};
            for (int q = 0; q < 3; ++q) {
                KFn<T> fn = fns[q];
                emit([&] { fn<<<nb, kThreads, 0, st>>>(a); }, timed(c, MPM_KERNEL_SPMV_DOT + q, j));
            }
        }
    }
    if (tail == kTailNone) return;
    if (tail == kTailFull) {
        if (dc) {
            KFn<T> fl = K.dl[m - 1];
            KFinFn<T> ff = K.df[m - 1];
            emit([&] { fl<<<nb, kThreads, 0, st>>>(a); }, false);
            emit([&] { ff<<<nsys, kThreads, 0, st>>>(a, sys0); }, false);
        } else {
            KFinFn<T> fin = K.k4[m - 1];
            emit([&] { fin<<<nsys, kThreads, 0, st>>>(a, sys0); }, false);
        }
    }
    emit([&] { k_update<T><<<nb, kThreads, 0, st>>>(a); }, timed(c, MPM_KERNEL_UPDATE, 0));
    emit([&] { k_residual<T><<<nb, kThreads, 0, st>>>(a, kResCycle); }, timed(c, MPM_KERNEL_RESIDUAL, 0));
    emit([&] { k_res_final<T><<<nsys, kThreads, 0, st>>>(a, sys0, kResCycle); }, false);
}

// Add the event times and algorithmic bytes of the cycle that just finished.
template <typename T>
static void account_timing(Ctx* c) {
    const int nsys = c->S * c->P;
    for (int i = 0; i < c->tev_used; ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->tev[2 * i], c->tev[2 * i + 1]) == hipSuccess) c->time_ms += ms;
        c->time_launches += c->time_repeat;
    }
    const double t = (double)sizeof(T);
    const int j = c->time_j;
    for (int s = 0; s < nsys; ++s) {
        const SysK& k = c->h_sk[s];
        if (k.cycles <= c->prev_cycles[s]) continue;       // did not run this cycle
        c->prev_cycles[s] = k.cycles;
        const double N = (double)c->probs[s / c->S].N;
        double per = 0.0;
        switch (c->time_kind) {
            case MPM_KERNEL_SPMV_DOT:
                // the delayed scheme applies the stencil of step j before it learns that
                // the cycle ended with column j - 1
                per = (c->opt.ortho == MPM_ORTHO_DCGS2 ? k.mcount >= j : k.mcount > j) ? t * (j + 5) + 16.0 / c->S
                                                                                         : 0.0;
                break;
            case MPM_KERNEL_AXPY_DOT:
                // delayed Gram-Schmidt: reads Q_j, u_j, z, writes q_j, u_{j+1}
                per = k.mcount > j ? (c->opt.ortho != MPM_ORTHO_DCGS2 ? t * (j + 3) : j == 0 ? 3 * t : t * (j + 4))
                                   : 0.0;
                break;
            case MPM_KERNEL_AXPY_NORM:
                per = k.mcount > j ? t * (j + 2) + (j + 1 < c->opt.restart ? t : 0.0) : 0.0;
                break;
            case MPM_KERNEL_UPDATE: per = t * k.mcount + 24.0; break;
            case MPM_KERNEL_RESIDUAL: per = 56.0 + t + 16.0 / c->S; break;
            default: break;
        }
        c->time_bytes += per * N * c->time_repeat;
    }
}

template <typename T>
static void enqueue_cycle_all(Ctx* c, hipStream_t st, int j0, int j1, int tail, bool events) {
    const int nsys = c->S * c->P;
    if (c->opt.batched) {
        enqueue_cycle<T>(c, c->d_blocks, (unsigned)c->blocks.size(), 0, nsys, st, j0, j1, tail, events);
    } else {
        for (int s = 0; s < nsys; ++s) {
            const int first = c->sys_tab_first[s];
            const int cnt = (s + 1 < nsys ? c->sys_tab_first[s + 1] : (int)c->blocks_sys.size()) - first;
            enqueue_cycle<T>(c, c->d_blocks_sys + first, (unsigned)cnt, s, 1, st, j0, j1, tail, events);
        }
    }
}

static void drop_graphs(Ctx* c) {
    for (auto& kv : c->graphs)
        if (kv.second) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

// Arnoldi steps at the head of a segment that are launched directly when the rest of the
// segment comes from a graph: the GPU runs them while the graph is being submitted.
constexpr int kGraphHead = 2;

// Launch one segment of a cycle: from a cached graph, or directly while a kernel is
// timed (events inside a captured graph cannot be timed).
template <typename T>
static int launch_segment(Ctx* c, hipStream_t st, int j0, int j1, int tail) {
    const bool graph = c->opt.use_graph && c->time_kind == MPM_KERNEL_NONE;
    if (!graph) {
        enqueue_cycle_all<T>(c, st, j0, j1, tail, c->time_kind != MPM_KERNEL_NONE);
        MPM_HIP(hipGetLastError());
        return MPM_OK;
    }
    const int jh = std::min(j1, j0 + kGraphHead);
    if (jh > j0) {
        enqueue_cycle_all<T>(c, st, j0, jh, kTailNone, false);
        MPM_HIP(hipGetLastError());
        j0 = jh;
    }
    if (j0 == j1 && tail == kTailNone) return MPM_OK;
    const int key = (j0 * (kMaxM + 1) + j1) * 3 + tail;
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        hipGraph_t g = nullptr;
        MPM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        enqueue_cycle_all<T>(c, st, j0, j1, tail, false);
        MPM_HIP(hipStreamEndCapture(st, &g));
        hipGraphExec_t ge = nullptr;
        hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        it = c->graphs.emplace(key, ge).first;
    }
    MPM_HIP(hipGraphLaunch(it->second, st));
    return MPM_OK;
}

// Wait until the work enqueued so far has run, when the status heads of every system
// are in the host mirror (the last kernel enqueued is always k_res_final, which writes
// them).  Behind that point, the iterates of the systems whose solve has ended go to the
// lattice fields while the host reads the status: after the last cycle nothing is left
// to launch.  The wait polls the event for up to kSpinMs (a blocking wait adds tens of
// microseconds of wake-up latency to every cycle), then blocks.
constexpr double kSpinMs = 5.0;

template <typename T>
static int fetch_status(Ctx* c, hipStream_t st) {
    MPM_HIP(hipEventRecord(c->ev_status, st));
    k_scatter<T><<<(unsigned)c->blocks.size(), kThreads, 0, st>>>(make_args<T>(c, c->d_blocks), 1);
    MPM_HIP(hipGetLastError());
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t e = hipEventQuery(c->ev_status);
        if (e == hipSuccess) return MPM_OK;
        if (e != hipErrorNotReady) return hip_fail(e, "hipEventQuery");
        if (std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() > kSpinMs) break;
    }
    MPM_HIP(hipEventSynchronize(c->ev_status));
    return MPM_OK;
}

// Before the first residual pass of a step with a network start: the scales are set,
// each problem's network buffers cover its grid, and the input's static channels (k, D,
// s, the mask) are built, once per grid, domain and scales; that pass then writes the
// per-step channels (c^n and d) of the domain voxels.
static int ws_prepare_inputs(Ctx* c, hipStream_t st) {
    if (!c->have_scales) {
        set_error("warm start: no network scales (mpm_attach_net)");
        return MPM_ESTATE;
    }
    for (int p = 0; p < c->P; ++p) {
        ProbHost& ph = c->probs[p];
        const long long G = (long long)ph.gd[0] * ph.gd[1] * ph.gd[2];
        if (G <= 0 || (size_t)G > ph.cap_grid || !ph.wsin || !ph.wsout || !ph.stat) {
            set_error("warm start: the network buffers of a problem do not cover its grid");
            return MPM_ESTATE;
        }
        if (!ph.ws_ready) {
            launch_ws_input(ph, c->h_probs[p], c->S, c->d_scales, ph.wsin, st);
            const hipError_t le = hipGetLastError();
            if (le != hipSuccess) return hip_fail(le, "warm start (network input)");
            ph.ws_ready = true;
        }
    }
    return MPM_OK;
}

// Warm start of every system not converged at c^n: network prediction, linear
// extrapolation, or the network's correction of the extrapolation, accepted per system
// only if its true FP64 residual is smaller than that of c^n (else the system restarts
// from c^n).  The outcome is recorded in the statistics (warm_start_used, fallback,
// rel_res_warm).
template <typename T>
static int warm_start(Ctx* c, hipStream_t st) {
    const int nsys = c->S * c->P;
    KArgs<T> a = make_args<T>(c, c->d_blocks);
    const unsigned nb = (unsigned)c->blocks.size();
    const int mode = c->opt.warm_start;
    // the step's first residual pass has written the network input's per-step channels
    // (c^n and d of the base start x_b; for MPM_WS_NET_EXTRAP it also forms x_b = 2 c^n -
    // c^{n-1}), and k_ws_apply forms the start from c^n, c^{n-1} and the output
    if (net_warm_start(c)) {
        hipStream_t saved = c->net->stream;
        c->net->stream = st;
        for (int p = 0; p < c->P; ++p) {
            ProbHost& ph = c->probs[p];
            // the last level computes only the tiles the domain voxels' outputs read
            const TileLists tl{ph.tl_dev, ph.tl_n[0], ph.tl_dev + std::max(ph.tl_n[0], 0), ph.tl_n[1]};
            int rc = net_forward(c->net, ph.wsin, 1, ph.gd[2], ph.gd[1], ph.gd[0], ph.wsout, true,
                                 ph.tl_n[0] >= 0 ? &tl : nullptr);
            if (rc != MPM_OK) {
                c->net->stream = saved;
                return rc;
            }
        }
        c->net->stream = saved;
    }
    k_ws_apply<T><<<nb, kThreads, 0, st>>>(a, mode, c->d_scales);
    k_residual<T><<<nb, kThreads, 0, st>>>(a, kResWarm);
    k_res_final<T><<<nsys, kThreads, 0, st>>>(a, 0, kResWarm);
    k_ws_revert<T><<<nb, kThreads, 0, st>>>(a);
    k_residual<T><<<nb, kThreads, 0, st>>>(a, kResRevert);
    k_res_final<T><<<nsys, kThreads, 0, st>>>(a, 0, kResRevert);
    MPM_HIP(hipGetLastError());
    return MPM_OK;
}

template <typename T>
static int run_step_t(Ctx* c, double tol) {
    hipStream_t st = c->stream;
    const int nsys = c->S * c->P;
    KArgs<T> a = make_args<T>(c, c->d_blocks);
    const unsigned nb = (unsigned)c->blocks.size();
    // with the extrapolated starts the gather also keeps c^n in the free half of prev
    const bool extrap = extrap_warm_start(c);
    KArgs<T> ag = a;
    if (extrap) ag.pcur = c->prev + (size_t)(1 - c->prev_half) * c->prev_n;
    k_gather<T><<<nb, kThreads, 0, st>>>(ag);
    const int wsm = c->opt.warm_start;
    const bool net_extrap = wsm == MPM_WS_NET_EXTRAP && c->net && c->have_prev;
    const bool net_ws = (wsm == MPM_WS_NET && c->net) || net_extrap;
    if (net_ws) {
        const int prc = ws_prepare_inputs(c, st);
        if (prc != MPM_OK) return prc;
    }
    if (net_extrap)
        k_residual<T, true, true><<<nb, kThreads, 0, st>>>(a, kResFirst, c->d_scales);
    else if (net_ws)
        k_residual<T, false, true><<<nb, kThreads, 0, st>>>(a, kResFirst, c->d_scales);
    else
        k_residual<T><<<nb, kThreads, 0, st>>>(a, kResFirst);
    k_res_final<T><<<nsys, kThreads, 0, st>>>(a, 0, kResFirst);
    if (net_ws || (wsm == MPM_WS_EXTRAP && c->have_prev)) {
        int wrc = warm_start<T>(c, st);
        if (wrc != MPM_OK) return wrc;
    }

    MPM_HIP(hipGetLastError());
    int status = MPM_OK, rc = MPM_OK;
    c->prev_cycles.assign(nsys, 0);
    const int m = c->opt.restart;
    c->cycle_len_next.clear();
    auto any_active = [&] {
        for (int s = 0; s < nsys; ++s)
            if (c->h_sk[s].active) return true;
        return false;
    };
    // The status after the first residual is only needed to skip a cycle nobody runs:
    // when the previous step needed a cycle, the first one is launched at once (blocks
    // of systems converged at c^n exit at their first check).
    const bool speculate = !c->cycle_len.empty() && c->cycle_len[0] > 0;
    auto any_running = [&] {
        for (int s = 0; s < nsys; ++s)
            if (c->h_sk[s].active == kRunning) return true;
        return false;
    };
    bool have_status = false;   // h_sk already holds the end state of the last cycle
    for (int cyc = 0;; ++cyc) {
        const bool spec = cyc == 0 && speculate;   // launched with no status to go by
        if (!spec && !have_status) {
            rc = fetch_status<T>(c, st);
            if (rc != MPM_OK) return rc;
        }
        have_status = false;
        if (cyc > 0) {
            // length of the cycle that just ended (longest over the systems that ran it)
            int len = 0;
            for (int s = 0; s < nsys; ++s)
                if (c->h_sk[s].cycles > c->prev_cycles[s]) len = std::max(len, c->h_sk[s].mcount);
            c->cycle_len_next.push_back(len);
            if (c->time_kind != MPM_KERNEL_NONE) account_timing<T>(c);
            else
                for (int s = 0; s < nsys; ++s) c->prev_cycles[s] = c->h_sk[s].cycles;
        }
        bool bad = false;
        if (!spec)
            for (int s = 0; s < nsys; ++s)
                if (c->h_sk[s].breakdown && !c->h_sk[s].converged) bad = true;
        if (!spec && !any_active()) {
            if (bad) status = MPM_NOT_CONVERGED;
            break;
        }
        if (cyc >= c->opt.max_cycles) {
            status = MPM_NOT_CONVERGED;
            break;
        }
        c->tev_used = 0;
        // Launch the cycle up to the length it took in the previous implicit step (plus
        // a margin) followed by the end-of-cycle work for the systems whose cycle ended
        // there; only if a system is still running at that step is it continued to step
        // m (systems restarted meanwhile are pending and wait for the next step 0).
        // Launches past the end of every system's cycle would only find idle systems.
        int k = m;
        if (cyc < (int)c->cycle_len.size()) k = std::min(m, c->cycle_len[cyc] + kPredictMargin);
        if (k < m) {
            rc = launch_segment<T>(c, st, 0, k, kTailUpdate);
            if (rc != MPM_OK) return rc;
            rc = fetch_status<T>(c, st);
            if (rc != MPM_OK) return rc;
            if (any_running())
                rc = launch_segment<T>(c, st, k, m, kTailFull);
            else
                have_status = true;
        } else {
            rc = launch_segment<T>(c, st, 0, m, kTailFull);
        }
        if (rc != MPM_OK) return rc;
    }
    c->cycle_len = c->cycle_len_next;
    // every system that ended its solve was written behind the last status wait; the
    // others (cycle limit reached) are written here with their best iterate
    if (any_active()) k_scatter<T><<<nb, kThreads, 0, st>>>(a, 0);
    if (extrap) {
        // this step's c^n becomes the previous step of the next extrapolation
        c->prev_half ^= 1;
        c->have_prev = true;
    }
    MPM_HIP(hipGetLastError());
    // the status fetched last in the loop is final (the scatter does not change it); the
    // scatter itself completes on the stream, ordered before the caller's later work
    for (int s = 0; s < nsys; ++s) {
        const SysK& k = c->h_sk[s];
        mpm_stats& o = c->stats[s];
        o.iterations = k.iters;
        o.cycles = k.cycles;
        o.refinements = k.refinements;
        o.converged = k.converged;
        o.warm_start_used = k.ws_used;
        o.fallback = k.fallback;
        o.rel_res_initial = k.rel_init;
        o.rel_res_warm = k.rel_warm;
        o.rel_res_final = k.rel_final;
        if (!k.converged) status = MPM_NOT_CONVERGED;
    }
    return status;
}

int run_step(Ctx* c, double* const* fields, double tol) {
    int rc = ensure_layout(c);
    if (rc != MPM_OK) return rc;
    hipStream_t st = c->stream;
    // field pointers and scalar parameters go to the device only when they change (the
    // previous step waited for its last status copy, which follows these uploads on the
    // stream, so the pinned copies are free)
    bool fields_changed = !c->up_valid;
    for (int p = 0; p < c->P; ++p) {
        if (c->h_fields[p] != fields[p]) fields_changed = true;
        c->h_fields[p] = fields[p];
    }
    if (fields_changed)
        MPM_HIP(hipMemcpyAsync(c->d_fields, c->h_fields, c->P * sizeof(double*), hipMemcpyHostToDevice, st));
    Params np = *c->h_prm;
    np.tol = tol;
    np.inner_rtol = c->opt.precision == MPM_FP64 ? 0.0 : c->opt.inner_rtol;
    np.restart = c->opt.restart;
    np.S = c->S;
    np.first = 1;
    if (!c->up_valid || std::memcmp(&np, c->h_prm, sizeof(Params)) != 0) {
        *c->h_prm = np;
        MPM_HIP(hipMemcpyAsync(c->d_prm, c->h_prm, sizeof(Params), hipMemcpyHostToDevice, st));
    }
    c->up_valid = true;
    return c->opt.precision == MPM_FP64 ? run_step_t<double>(c, tol) : run_step_t<float>(c, tol);
}

template <typename T>
static int debug_apply_t(Ctx* c, int p, const double* x, double* y, int mode) {
    hipStream_t st = c->stream;
    ProbDev pd{};
    const ProbHost& ph = c->probs[p];
    pd.vox = ph.vox;
    pd.nbr = ph.nbr;
    pd.d64 = ph.d64;
    pd.q64 = ph.q64;
    pd.a64 = ph.a64;
    pd.sc64 = ph.sc64;
    pd.c32 = ph.c32;
    pd.c64 = ph.c64;
    pd.off = c->off[p];
    pd.nvox = ph.nvox;
    pd.N = ph.N;
    pd.Npad = ph.Npad;
    const long long tot = (long long)c->S * ph.Npad;
    T* xt = (T*)c->W;
    k_dbg_gather<T><<<(unsigned)((tot + kThreads - 1) / kThreads), kThreads, 0, st>>>(pd, c->S, x, c->x, xt);
    constexpr int n = VW<T>::n;
    const long long thr = (tot + n - 1) / n;
    k_dbg_apply<T><<<(unsigned)((thr + kThreads - 1) / kThreads), kThreads, 0, st>>>(pd, c->S, c->x, xt, y, mode);
    MPM_HIP(hipGetLastError());
    MPM_HIP(hipStreamSynchronize(st));
    return MPM_OK;
}

int select_timing(Ctx* c, int kind, int j, int repeat) {
    // per cycle: one timed launch per system and segment, at most two segments
    const size_t need = 2 * 2 * (size_t)c->S * c->P;
    while (c->tev.size() < need) {
        hipEvent_t e;
        MPM_HIP(hipEventCreate(&e));
        c->tev.push_back(e);
    }
    c->time_kind = kind;
    c->time_j = j;
    c->time_repeat = repeat;
    c->time_ms = 0.0;
    c->time_bytes = 0.0;
    c->time_launches = 0;
    c->tev_used = 0;
    drop_graphs(c);
    return MPM_OK;
}

// Krylov state of one system after the last cycle (test hook): the stored basis columns
// V_0..V_{m-1} (m = mcount) of that system's unknowns widened to FP64, their scales
// vs[0..m-1] (orthonormal v_k = vs[k] V_k) and the unrotated Hessenberg columns
// 0..m-1 (hess[k * (kmax + 1) + i] = H[i][k], rows 0..k+1).  Copies at most kmax columns.
template <typename T>
static int debug_krylov_t(Ctx* c, int p, int sp, int kmax, int* mcount, double* vs, double* basis, double* hess) {
    hipStream_t st = c->stream;
    MPM_HIP(hipStreamSynchronize(st));
    const int sys = p * c->S + sp;
    SysK k{};
    MPM_HIP(hipMemcpy(&k, c->d_sk + sys, sizeof(SysK), hipMemcpyDeviceToHost));
    const ProbHost& ph = c->probs[p];
    const int m = std::min(k.mcount, kmax);
    *mcount = k.mcount;
    std::vector<T> col((size_t)ph.N);
    const long long base = c->off[p] + (long long)sp * ph.Npad;
    constexpr int LD = kMaxM + 1;
    for (int j = 0; j < m; ++j) {
        const T* src = (const T*)c->V + (long long)j * c->ldv + base;
        MPM_HIP(hipMemcpy(col.data(), src, (size_t)ph.N * sizeof(T), hipMemcpyDeviceToHost));
        for (int l = 0; l < ph.N; ++l) basis[(size_t)j * ph.N + l] = (double)col[l];
        vs[j] = k.vs[j];
        for (int i = 0; i <= kmax; ++i) hess[(size_t)j * (kmax + 1) + i] = i <= j + 1 && i < LD ? k.Hraw[j * LD + i] : 0.0;
    }
    return MPM_OK;
}

int debug_krylov(Ctx* c, int p, int sp, int kmax, int* mcount, double* vs, double* basis, double* hess) {
    if (c->opt.ortho != MPM_ORTHO_DCGS2) {
        set_error("mpm_debug_krylov: needs the delayed Gram-Schmidt scheme (the unrotated Hessenberg)");
        return MPM_EINVAL;
    }
    if (c->layout_dirty || !c->V) {
        set_error("mpm_debug_krylov: no step has run on the current layout");
        return MPM_ESTATE;
    }
    return c->opt.precision == MPM_FP64 ? debug_krylov_t<double>(c, p, sp, kmax, mcount, vs, basis, hess)
                                        : debug_krylov_t<float>(c, p, sp, kmax, mcount, vs, basis, hess);
}

int debug_apply(Ctx* c, int p, const double* x, double* y, int mode) {
    int rc = ensure_layout(c);
    if (rc != MPM_OK) return rc;
    if (mode == 1 && c->opt.precision == MPM_FP64) {
        set_error("mpm_debug_apply: mode 1 needs an MPM_FP32_IR context");
        return MPM_EINVAL;
    }
    if (mode == 2 && c->opt.precision != MPM_FP64) {
        set_error("mpm_debug_apply: mode 2 needs an MPM_FP64 context");
        return MPM_EINVAL;
    }
    return c->opt.precision == MPM_FP64 ? debug_apply_t<double>(c, p, x, y, mode)
                                        : debug_apply_t<float>(c, p, x, y, mode);
}

}  // namespace mpm

namespace mpm {

// The residual of a base start for the systems of problem p, with the solver's own
// kernels: c_old gathered as c^n (x, b), x = 2 x - c_prev when c_prev is given, and
// r = b - A x (V holds S r).
template <typename T>
static int ws_first_residual(Ctx* c, int p, const double* c_prev, const double* c_old) {
    hipStream_t st = c->stream;
    const int nsys = c->S * c->P;
    const int first = c->sys_tab_first[p * c->S];
    const int end = (p + 1) * c->S < nsys ? c->sys_tab_first[(p + 1) * c->S] : (int)c->blocks_sys.size();
    // the field pointer of problem p, uploaded alone (the other entries may not be set)
    c->h_fields[p] = const_cast<double*>(c_old);
    MPM_HIP(hipMemcpyAsync(c->d_fields + p, c->h_fields + p, sizeof(double*), hipMemcpyHostToDevice, st));
    KArgs<T> a = make_args<T>(c, c->d_blocks_sys + first);
    k_gather<T><<<(unsigned)(end - first), kThreads, 0, st>>>(a);
    if (c_prev) k_ws_extrap_x<T><<<(unsigned)(end - first), kThreads, 0, st>>>(a, c_prev);
    k_residual<T><<<(unsigned)(end - first), kThreads, 0, st>>>(a, kResFirst);
    MPM_HIP(hipGetLastError());
    return MPM_OK;
}

int ws_loss(Ctx* c, int p, const float* out, const float* target, float* grad, double* loss) {
    int rc = ensure_layout(c);
    if (rc != MPM_OK) return rc;
    hipStream_t st = c->stream;
    const ProbHost& ph = c->probs[p];
    const long long G = (long long)ph.gd[0] * ph.gd[1] * ph.gd[2];
    const unsigned nb = (unsigned)c->blocks.size();
    if (nb > c->cap_lossp) {
        (void)hipFree(c->d_lossp);
        if (c->h_lossp) (void)hipHostFree(c->h_lossp);
        c->d_lossp = nullptr;
        c->h_lossp = nullptr;
        c->cap_lossp = 0;
        MPM_HIP(hipMalloc(&c->d_lossp, nb * sizeof(double)));
        MPM_HIP(hipHostMalloc((void**)&c->h_lossp, nb * sizeof(double), hipHostMallocDefault));
        c->cap_lossp = nb;
    }
    // x and b are scratch between steps (the next step gathers them again)
    k_wsl_err<<<nb, kThreads, 0, st>>>(c->d_blocks, c->d_probs, c->S, p, out, target, c->d_scales, c->x);
    k_wsl_apply<<<nb, kThreads, 0, st>>>(c->d_blocks, p, 0, c->d_scales, c->x, c->b, c->d_lossp);
    k_wsl_apply<<<nb, kThreads, 0, st>>>(c->d_blocks, p, 1, c->d_scales, c->b, c->x, nullptr);
    k_fill0<<<(unsigned)((G * c->S + 255) / 256), 256, 0, st>>>(grad, G * c->S);
    const double count = (double)c->S * ph.N;
    k_wsl_grad<<<nb, kThreads, 0, st>>>(c->d_blocks, c->d_probs, c->S, p, c->x, 2.0 / count, c->d_scales, grad);
    MPM_HIP(hipGetLastError());
    MPM_HIP(hipMemcpyAsync(c->h_lossp, c->d_lossp, nb * sizeof(double), hipMemcpyDeviceToHost, st));
    MPM_HIP(hipStreamSynchronize(st));
    double sum = 0.0;
    for (unsigned i = 0; i < nb; ++i) sum += c->h_lossp[i];
    *loss = sum / count;
    return MPM_OK;
}

int ws_pair(Ctx* c, int p, const double* c_prev, const double* c_old, const double* c_new, uint16_t* in_bf16,
            float* target) {
    int rc = ensure_layout(c);
    if (rc != MPM_OK) return rc;
    hipStream_t st = c->stream;
    const ProbHost& ph = c->probs[p];
    const ProbDev& pd = c->h_probs[p];
    const long long G = (long long)ph.gd[0] * ph.gd[1] * ph.gd[2];
    const int bx = ph.hi[0] - ph.lo[0], by = ph.hi[1] - ph.lo[1], bz = ph.hi[2] - ph.lo[2];
    // x, b, V and the partial sums are scratch until the next step recomputes them; the
    // next step uploads its own field pointers
    double* saved = c->h_fields[p];
    c->up_valid = false;
    rc = ksize(c) == 8 ? ws_first_residual<double>(c, p, c_prev, c_old) : ws_first_residual<float>(c, p, c_prev, c_old);
    if (rc == MPM_OK) {
        launch_ws_input(ph, pd, c->S, c->d_scales, in_bf16, st);
        const unsigned nb = (unsigned)c->blocks.size();
        if (ksize(c) == 8)
            k_ws_resid<double><<<nb, kThreads, 0, st>>>(make_args<double>(c, c->d_blocks), p, c_old, c->d_scales,
                                                        in_bf16);
        else
            k_ws_resid<float><<<nb, kThreads, 0, st>>>(make_args<float>(c, c->d_blocks), p, c_old, c->d_scales,
                                                       in_bf16);
        k_ws_target<<<(unsigned)((G + 255) / 256), 256, 0, st>>>(pd, c->S, bx, by, bz, c_prev, c_old, c_new,
                                                               ph.stat, c->d_scales, target);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    c->h_fields[p] = saved;   // after the copy that read it has run
    if (rc != MPM_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "mpm_ws_pair");
    return MPM_OK;
}

}  // namespace mpm
