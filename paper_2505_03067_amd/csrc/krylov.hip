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
//               K3  w -= V_j h2, ||w||, V_{j+1} = w     (axpy + norm) + Givens on device
//   update:     x += S V_m y  (FP64 accumulation)
// Every global reduction is two-stage and deterministic: per-block partial sums in
// fixed order, then the last block of the system to arrive (an atomic counter)
// sums the partials in block order and runs the scalar work (norms, Givens,
// back-substitution).  The Krylov type T is float (FP32 basis inside FP64
// iterative refinement) or double (plain FP64 GMRES); both use the same kernels.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <utility>

#include "context.h"

namespace mpm {

// ------------------------------------------------------------------ helpers
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

__device__ inline double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Block-reduce NV per-thread sums and store them in slot 'slot' of rows 0..NV-1.
template <int NV>
__device__ inline void block_partials(const double (&acc)[NV], double* part, int nslots, int slot) {
    __shared__ double sh[kWaves][NV];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double t = wsum(acc[v]);
        if (lane == 0) sh[w][v] = t;
    }
    __syncthreads();
    for (int v = threadIdx.x; v < NV; v += kThreads) {
        double t = sh[0][v];
#pragma unroll
        for (int i = 1; i < kWaves; ++i) t += sh[i][v];
        part[(long long)v * nslots + slot] = t;
    }
}

// Release this block's partials; true in exactly one block of the system (the last).
__device__ inline bool arrive_last(int* cnt, int nb) {
    __shared__ int last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const int prev = atomicAdd(cnt, 1);
        last = (prev == nb - 1);
        if (last) atomicExch(cnt, 0);
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// Sum rows 0..NV-1 of the system's partial slots in block order into out[] (shared).
template <int NV>
__device__ inline void final_sums(const double* part, int nslots, int slot0, int nb, double* out) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int v = w; v < NV; v += kWaves) {
        double t = 0.0;
        for (int i = lane; i < nb; i += 64) t += part[(long long)v * nslots + slot0 + i];
        t = wsum(t);
        if (lane == 0) out[v] = t;
    }
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
// Gather c^n from the lattice into x, form b = c^n + q, and ||b||.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gather(KArgs<T> a) {
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    const ProbDev pd = a.probs[blk.sys / a.S];
    const Where wh = where_of(a, blk, pd);
    SysK* sk = a.sk + wh.sys;
    const double* f = a.fields[wh.p] + (long long)wh.s * pd.nvox;
    double acc[1] = {0.0};
    for (long long u = blk.start + threadIdx.x; u < blk.end; u += kThreads) {
        const int l = (int)(u - wh.base);
        double cn = 0.0, bb = 0.0;
        if (l < pd.N) {
            cn = f[pd.vox[l]];
            bb = cn + pd.q64[wh.locbase + l];
        }
        a.x[u] = cn;
        a.b[u] = bb;
        acc[0] += bb * bb;
    }
    block_partials<1>(acc, a.part, a.nslots, blk.slot);
    if (!arrive_last(a.cnt + wh.sys, sk->nblocks)) return;
    __shared__ double tot[1];
    final_sums<1>(a.part, a.nslots, sk->slot0, sk->nblocks, tot);
    if (threadIdx.x == 0) {
        sk->bnorm = sqrt(tot[0]);
        sk->iters = 0;
        sk->cycles = 0;
        sk->refinements = 0;
        sk->converged = 0;
        sk->active = 0;
        sk->need_update = 0;
        sk->mcount = 0;
        sk->breakdown = 0;
        sk->ws_used = 0;
        sk->fallback = 0;
        sk->rel_warm = 0.0;
    }
}

// r = b - A x (FP64); V_0 = S r; norms; convergence test; start of the next cycle.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_residual(KArgs<T> a, int first) {
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    SysK* sk = a.sk + blk.sys;
    if (sk->converged) return;
    const ProbDev pd = a.probs[blk.sys / a.S];
    const Where wh = where_of(a, blk, pd);
    T* V0 = a.V;
    double acc[2] = {0.0, 0.0};
    for (long long u = blk.start + threadIdx.x; u < blk.end; u += kThreads) {
        const int l = (int)(u - wh.base);
        double r = 0.0, sr = 0.0;
        if (l < pd.N) {
            r = a.b[u] - apply_A(pd, wh, a.x, u, l);
            sr = pd.sc64[wh.locbase + l] * r;
        }
        V0[u] = (T)sr;
        acc[0] += r * r;
        acc[1] += sr * sr;
    }
    block_partials<2>(acc, a.part, a.nslots, blk.slot);
    if (!arrive_last(a.cnt + wh.sys, sk->nblocks)) return;
    __shared__ double tot[2];
    final_sums<2>(a.part, a.nslots, sk->slot0, sk->nblocks, tot);
    if (threadIdx.x == 0) {
        const Params& prm = *a.prm;
        const double rn = sqrt(tot[0]), srn = sqrt(tot[1]);
        const double bn = sk->bnorm;
        const double rel = bn > 0.0 ? rn / bn : (rn > 0.0 ? INFINITY : 0.0);
        if (first) sk->rel_init = rel;
        else sk->refinements += 1;
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
            sk->g[0] = srn;
            sk->active = 1;
        }
    }
}

// K1: w = B v_J and h_k = v_k . w for k <= J.
template <typename T, int J>
__global__ __launch_bounds__(kThreads) void k_spmv_dot(KArgs<T> a) {
    constexpr int n = VW<T>::n;
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    SysK* sk = a.sk + blk.sys;
    if (!sk->active) return;
    const ProbDev pd = a.probs[blk.sys / a.S];
    const Where wh = where_of(a, blk, pd);
    const T* c = couplings<T>(pd);
    const T* VJ = a.V + (long long)J * a.ldv;
    const T vsJ = (T)sk->vs[J];
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
    block_partials<J + 1>(acc, a.part, a.nslots, blk.slot);
    if (!arrive_last(a.cnt + wh.sys, sk->nblocks)) return;
    __shared__ double tot[J + 1];
    final_sums<J + 1>(a.part, a.nslots, sk->slot0, sk->nblocks, tot);
    for (int k = threadIdx.x; k <= J; k += kThreads) {
        const double h = sk->vs[k] * tot[k];
        sk->h1[k] = h;
        sk->c1[k] = h * sk->vs[k];
    }
}

// K2: w -= sum_k h_k v_k, then h2_k = v_k . w (classical Gram-Schmidt, second pass).
template <typename T, int J>
__global__ __launch_bounds__(kThreads) void k_axpy_dot(KArgs<T> a) {
    constexpr int n = VW<T>::n;
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    SysK* sk = a.sk + blk.sys;
    if (!sk->active) return;
    double cf[J + 1];
#pragma unroll
    for (int k = 0; k <= J; ++k) cf[k] = sk->c1[k];
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
    block_partials<J + 1>(acc, a.part, a.nslots, blk.slot);
    if (!arrive_last(a.cnt + blk.sys, sk->nblocks)) return;
    __shared__ double tot[J + 1];
    final_sums<J + 1>(a.part, a.nslots, sk->slot0, sk->nblocks, tot);
    for (int k = threadIdx.x; k <= J; k += kThreads) {
        const double h = sk->vs[k] * tot[k];
        sk->h2[k] = h;
        sk->c2[k] = h * sk->vs[k];
    }
}

// Givens rotation of Hessenberg column J, residual estimate, and (when the cycle
// ends) back-substitution R y = g.  Run by all 64 lanes of wave 0 in lock step.
template <int J>
__device__ inline void givens_step(SysK* sk, double hn, int restart) {
    constexpr int LD = kMaxM + 1;
    double col[J + 2];
#pragma unroll
    for (int k = 0; k <= J; ++k) col[k] = sk->h1[k] + sk->h2[k];
    col[J + 1] = hn;
#pragma unroll
    for (int i = 0; i < J; ++i) {            // earlier rotations, in order
        const double cs = sk->cs[i], sn = sk->sn[i];
        const double t = cs * col[i] + sn * col[i + 1];
        col[i + 1] = -sn * col[i] + cs * col[i + 1];
        col[i] = t;
    }
    const double rho = sqrt(col[J] * col[J] + col[J + 1] * col[J + 1]);
    double cs = 1.0, sn = 0.0;
    if (rho > 0.0) {
        cs = col[J] / rho;
        sn = col[J + 1] / rho;
    }
    col[J] = rho;
    const double gJ = sk->g[J];
    const double gn = -sn * gJ;
    const int lane = threadIdx.x & 63;
    const bool breakdown = !(hn > 0.0) || !(rho > 0.0);
    const bool done = breakdown || fabs(gn) <= sk->eta * sk->g[0] || J + 1 >= restart;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k <= J; ++k) sk->R[J * LD + k] = col[k];
        sk->cs[J] = cs;
        sk->sn[J] = sn;
        sk->g[J] = cs * gJ;
        sk->g[J + 1] = gn;
        sk->vs[J + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
    }
    __threadfence_block();   // lane 0's stores are read back by the other lanes below
    if (!done) return;
    // back-substitution by columns: lane i keeps g_i and receives y_k in turn
    const int m = J + 1;
    double gi = lane < m ? sk->g[lane] : 0.0;
    double yi = 0.0;
    for (int k = m - 1; k >= 0; --k) {
        const double rkk = sk->R[k * LD + k];
        const double gk = __shfl(gi, k);
        const double yk = rkk != 0.0 ? gk / rkk : 0.0;
        if (lane == k) yi = yk;
        if (lane < k) gi -= sk->R[k * LD + lane] * yk;
    }
    if (lane < m) sk->y[lane] = yi * sk->vs[lane];
    if (lane == 0) {
        sk->mcount = m;
        sk->active = 0;
        sk->need_update = 1;
        sk->iters += m;
        sk->cycles += 1;
        if (breakdown && !(hn == 0.0)) sk->breakdown = 1;
    }
}

// K3: w -= sum_k h2_k v_k, ||w||, V_{J+1} = w; then the Givens update.
template <typename T, int J>
__global__ __launch_bounds__(kThreads) void k_axpy_norm(KArgs<T> a) {
    constexpr int n = VW<T>::n;
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    SysK* sk = a.sk + blk.sys;
    if (!sk->active) return;
    const int restart = a.prm->restart;
    const bool store = J + 1 < restart;
    double cf[J + 1];
#pragma unroll
    for (int k = 0; k <= J; ++k) cf[k] = sk->c2[k];
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
    block_partials<1>(acc, a.part, a.nslots, blk.slot);
    if (!arrive_last(a.cnt + blk.sys, sk->nblocks)) return;
    __shared__ double tot[1];
    final_sums<1>(a.part, a.nslots, sk->slot0, sk->nblocks, tot);
    if (threadIdx.x < 64) givens_step<J>(sk, sqrt(tot[0]), restart);
}

// x += S sum_k y_k V_k (FP64 accumulation of the FP32 or FP64 basis).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_update(KArgs<T> a) {
    constexpr int n = VW<T>::n;
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    SysK* sk = a.sk + blk.sys;
    if (!sk->need_update) return;
    const ProbDev pd = a.probs[blk.sys / a.S];
    const Where wh = where_of(a, blk, pd);
    const int m = sk->mcount;
    for (long long u0 = blk.start + threadIdx.x * n; u0 < blk.end; u0 += kThreads * n) {
        double t[n];
#pragma unroll
        for (int e = 0; e < n; ++e) t[e] = 0.0;
        for (int k = 0; k < m; ++k) {
            T vk[n];
            ld16(a.V + (long long)k * a.ldv + u0, vk);
            const double yk = sk->y[k];
#pragma unroll
            for (int e = 0; e < n; ++e) t[e] += yk * (double)vk[e];
        }
        const long long loc0 = wh.locbase + (u0 - wh.base);
#pragma unroll
        for (int e = 0; e < n; ++e) a.x[u0 + e] += pd.sc64[loc0 + e] * t[e];
    }
}

// Write x back onto the domain voxels of the lattice fields.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scatter(KArgs<T> a) {
    const Block blk = a.blocks[blockIdx.x];
    if (blk.sys < 0) return;
    const ProbDev pd = a.probs[blk.sys / a.S];
    const Where wh = where_of(a, blk, pd);
    double* f = a.fields[wh.p] + (long long)wh.s * pd.nvox;
    for (long long u = blk.start + threadIdx.x; u < blk.end; u += kThreads) {
        const int l = (int)(u - wh.base);
        if (l < pd.N) f[pd.vox[l]] = a.x[u];
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

// ------------------------------------------------------------------ dispatch tables
template <typename T>
using KFn = void (*)(KArgs<T>);

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

template <typename T>
struct Kernels {
    std::array<KFn<T>, kMaxM> k1, k2, k3;
    Kernels() {
        k1 = table_k1<T>(std::make_integer_sequence<int, kMaxM>{});
        k2 = table_k2<T>(std::make_integer_sequence<int, kMaxM>{});
        k3 = table_k3<T>(std::make_integer_sequence<int, kMaxM>{});
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

// Split each system into blocks, build the XCD-aware batched table and the
// per-system tables.
static void build_tables(Ctx* c) {
    const int S = c->S;
    const int nsys = S * c->P;
    long long maxpad = 0;
    for (auto& ph : c->probs) maxpad = std::max<long long>(maxpad, ph.Npad);
    std::vector<Block> logical;
    c->sys_first.assign(nsys, 0);
    c->sys_count.assign(nsys, 0);
    int slot = 0;
    for (int p = 0; p < c->P; ++p) {
        const ProbHost& ph = c->probs[p];
        // unknowns per block: a fixed override, else enough blocks to fill the GPU
        long long per = c->opt.tile_override > 0 ? c->opt.tile_override : 0;
        if (per <= 0) {
            const long long target = std::max(1, 2048 / std::max(1, nsys));
            per = (ph.Npad + target - 1) / target;
        }
        per = std::max<long long>(kAlign, (per + kAlign - 1) / kAlign * kAlign);
        c->block_unknowns = (int)per;
        for (int s = 0; s < S; ++s) {
            const int sys = p * S + s;
            const long long base = c->off[p] + (long long)s * ph.Npad;
            c->sys_first[sys] = slot;
            int nb = 0;
            for (long long a0 = 0; a0 < ph.Npad; a0 += per) {
                Block b;
                b.sys = sys;
                b.start = (int)(base + a0);
                b.end = (int)(base + std::min<long long>(ph.Npad, a0 + per));
                b.slot = slot++;
                logical.push_back(b);
                ++nb;
            }
            c->sys_count[sys] = nb;
        }
    }
    c->nslots = slot;
    auto swizzle = [](const std::vector<Block>& L, std::vector<Block>& out) {
        const size_t nb = L.size();
        const size_t per = (nb + 7) / 8;
        const size_t padded = per * 8;
        Block idle{-1, 0, 0, 0};
        for (size_t b = 0; b < padded; ++b) {
            const size_t xcd = b % 8, pos = b / 8;
            const size_t li = xcd * per + pos;
            out.push_back(li < nb ? L[li] : idle);
        }
    };
    c->blocks.clear();
    swizzle(logical, c->blocks);
    c->blocks_sys.clear();
    std::vector<int> sfirst(nsys);
    for (int sys = 0; sys < nsys; ++sys) {
        std::vector<Block> L(logical.begin() + c->sys_first[sys],
                             logical.begin() + c->sys_first[sys] + c->sys_count[sys]);
        sfirst[sys] = (int)c->blocks_sys.size();
        swizzle(L, c->blocks_sys);
    }
    // reuse sys_first/sys_count as the slice of blocks_sys per system for launches;
    // the partial-slot ranges go to the device SysK through k_sys_init
    c->sys_tab_first = sfirst;
}

int ensure_layout(Ctx* c) {
    if (!c->layout_dirty) return MPM_OK;
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
        free_work(c);
        const size_t ks = ksize(c);
        if (hipMalloc(&c->V, (size_t)(m + 1) * need * ks) != hipSuccess ||
            hipMalloc(&c->W, need * ks) != hipSuccess || hipMalloc(&c->x, need * 8) != hipSuccess ||
            hipMalloc(&c->b, need * 8) != hipSuccess) {
            (void)hipGetLastError();
            free_work(c);
            set_error("device allocation of the Krylov workspace failed");
            return MPM_ENOMEM;
        }
        c->cap_U = need;
        c->ldv = (long long)need;
        MPM_HIP(hipMemsetAsync(c->V, 0, (size_t)(m + 1) * need * ks, st));
        MPM_HIP(hipMemsetAsync(c->W, 0, need * ks, st));
        MPM_HIP(hipMemsetAsync(c->x, 0, need * 8, st));
        MPM_HIP(hipMemsetAsync(c->b, 0, need * 8, st));
    }
    build_tables(c);
    // device tables
    const size_t nb = c->blocks.size(), nbs = c->blocks_sys.size();
    if (nb > c->cap_blocks || nbs > c->cap_blocks) {
        if (c->d_blocks) (void)hipFree(c->d_blocks);
        if (c->d_blocks_sys) (void)hipFree(c->d_blocks_sys);
        const size_t cap = std::max(nb, nbs) * 2;
        if (hipMalloc(&c->d_blocks, cap * sizeof(Block)) != hipSuccess ||
            hipMalloc(&c->d_blocks_sys, cap * sizeof(Block)) != hipSuccess) {
            (void)hipGetLastError();
            set_error("device allocation of block tables failed");
            return MPM_ENOMEM;
        }
        c->cap_blocks = cap;
    }
    if ((size_t)c->nslots > c->cap_slots) {
        if (c->d_part) (void)hipFree(c->d_part);
        const size_t cap = (size_t)c->nslots * 2;
        if (hipMalloc(&c->d_part, cap * kPartRows * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            set_error("device allocation of partial sums failed");
            return MPM_ENOMEM;
        }
        c->cap_slots = cap;
    }
    // the partial rows are addressed with stride nslots
    MPM_HIP(hipMemcpyAsync(c->d_blocks, c->blocks.data(), nb * sizeof(Block), hipMemcpyHostToDevice, st));
    MPM_HIP(hipMemcpyAsync(c->d_blocks_sys, c->blocks_sys.data(), nbs * sizeof(Block), hipMemcpyHostToDevice, st));
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
    }
    MPM_HIP(hipMemcpyAsync(c->d_probs, pd.data(), c->P * sizeof(ProbDev), hipMemcpyHostToDevice, st));
    // per-system slot ranges and diagonal extremes
    const int nsys = c->S * c->P;
    int* tmp = nullptr;
    MPM_HIP(hipMalloc(&tmp, 2 * nsys * sizeof(int)));
    std::vector<int> fc(2 * nsys);
    for (int s = 0; s < nsys; ++s) {
        fc[s] = c->sys_first[s];
        fc[nsys + s] = c->sys_count[s];
    }
    MPM_HIP(hipMemcpyAsync(tmp, fc.data(), fc.size() * sizeof(int), hipMemcpyHostToDevice, st));
    k_sys_init<<<1, 64, 0, st>>>(c->d_sk, tmp, tmp + nsys, nsys);
    MPM_HIP(hipMemsetAsync(c->d_cnt, 0, kMaxSys * sizeof(int), st));
    KArgs<double> ka{};
    ka.blocks = c->d_blocks;
    ka.probs = c->d_probs;
    ka.sk = c->d_sk;
    ka.S = c->S;
    k_diag_extremes<double><<<(unsigned)nb, kThreads, 0, st>>>(ka);
    k_sys_kappa<<<1, 64, 0, st>>>(c->d_sk, nsys);
    MPM_HIP(hipGetLastError());
    MPM_HIP(hipStreamSynchronize(st));
    (void)hipFree(tmp);
    if (c->graph) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
    }
    c->graph_valid = false;
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
    a.cnt = c->d_cnt;
    a.prm = c->d_prm;
    a.V = (T*)c->V;
    a.W = (T*)c->W;
    a.x = c->x;
    a.b = c->b;
    a.fields = c->d_fields;
    a.ldv = c->ldv;
    a.nslots = c->nslots;
    a.S = c->S;
    return a;
}

// Enqueue one GMRES cycle (m Arnoldi steps, update, residual) for the given table.
template <typename T>
static void enqueue_cycle(Ctx* c, const Block* tab, unsigned nb, hipStream_t st) {
    const Kernels<T>& K = kernels<T>();
    KArgs<T> a = make_args<T>(c, tab);
    for (int j = 0; j < c->opt.restart; ++j) {
        K.k1[j]<<<nb, kThreads, 0, st>>>(a);
        K.k2[j]<<<nb, kThreads, 0, st>>>(a);
        K.k3[j]<<<nb, kThreads, 0, st>>>(a);
    }
    k_update<T><<<nb, kThreads, 0, st>>>(a);
    k_residual<T><<<nb, kThreads, 0, st>>>(a, 0);
}

template <typename T>
static void enqueue_cycle_all(Ctx* c, hipStream_t st) {
    if (c->opt.batched) {
        enqueue_cycle<T>(c, c->d_blocks, (unsigned)c->blocks.size(), st);
    } else {
        const int nsys = c->S * c->P;
        for (int s = 0; s < nsys; ++s) {
            const int first = c->sys_tab_first[s];
            const int cnt = (s + 1 < nsys ? c->sys_tab_first[s + 1] : (int)c->blocks_sys.size()) - first;
            enqueue_cycle<T>(c, c->d_blocks_sys + first, (unsigned)cnt, st);
        }
    }
}

template <typename T>
static int run_step_t(Ctx* c, double tol) {
    hipStream_t st = c->stream;
    const int nsys = c->S * c->P;
    KArgs<T> a = make_args<T>(c, c->d_blocks);
    const unsigned nb = (unsigned)c->blocks.size();
    k_gather<T><<<nb, kThreads, 0, st>>>(a);
    k_residual<T><<<nb, kThreads, 0, st>>>(a, 1);
    MPM_HIP(hipGetLastError());
    int status = MPM_OK;
    for (int cyc = 0;; ++cyc) {
        MPM_HIP(hipMemcpyAsync(c->h_sk, c->d_sk, nsys * sizeof(SysK), hipMemcpyDeviceToHost, st));
        MPM_HIP(hipStreamSynchronize(st));
        bool any = false, bad = false;
        for (int s = 0; s < nsys; ++s) {
            if (c->h_sk[s].breakdown && !c->h_sk[s].converged) bad = true;
            if (c->h_sk[s].active) any = true;
        }
        if (!any) {
            if (bad) status = MPM_NOT_CONVERGED;
            break;
        }
        if (cyc >= c->opt.max_cycles) {
            status = MPM_NOT_CONVERGED;
            break;
        }
        if (c->opt.use_graph) {
            if (!c->graph_valid) {
                hipGraph_t g = nullptr;
                MPM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                enqueue_cycle_all<T>(c, st);
                MPM_HIP(hipStreamEndCapture(st, &g));
                if (c->graph) (void)hipGraphExecDestroy(c->graph);
                c->graph = nullptr;
                hipError_t e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
                c->graph_valid = true;
            }
            MPM_HIP(hipGraphLaunch(c->graph, st));
        } else {
            enqueue_cycle_all<T>(c, st);
            MPM_HIP(hipGetLastError());
        }
    }
    k_scatter<T><<<nb, kThreads, 0, st>>>(a);
    MPM_HIP(hipGetLastError());
    MPM_HIP(hipMemcpyAsync(c->h_sk, c->d_sk, nsys * sizeof(SysK), hipMemcpyDeviceToHost, st));
    MPM_HIP(hipStreamSynchronize(st));
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
    for (int p = 0; p < c->P; ++p) c->h_fields[p] = fields[p];
    MPM_HIP(hipMemcpyAsync(c->d_fields, c->h_fields, c->P * sizeof(double*), hipMemcpyHostToDevice, st));
    c->h_prm->tol = tol;
    c->h_prm->inner_rtol = c->opt.precision == MPM_FP64 ? 0.0 : c->opt.inner_rtol;
    c->h_prm->restart = c->opt.restart;
    c->h_prm->S = c->S;
    c->h_prm->first = 1;
    MPM_HIP(hipMemcpyAsync(c->d_prm, c->h_prm, sizeof(Params), hipMemcpyHostToDevice, st));
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
