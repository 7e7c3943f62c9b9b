// Finite-volume discretisation of one problem on its box (paper Sec. 2.3-2.4).
//
// 1. Count the domain voxels of every box row, scan the counts, and compact the
//    domain voxels in C order (z, y, x) with wave ballots: voxel l of the box
//    gets its lattice index vox[l].
// 2. Neighbour table: the compact index of the -y, +y, -z, +z neighbour of every
//    domain voxel (N = "none", a zero padding slot).  The x neighbours of voxel l
//    are l - 1 and l + 1 whenever they are coupled at all, so they need no table.
// 3. Coefficients per (species, voxel), in FP64:
//      G_f = harmonic-mean D / h^2 toward a domain voxel in the box,
//      G_f = 0 toward a voxel outside the mask,
//      G_f = 2 D_P / h^2 on a box face (Dirichlet value half a voxel away),
//      A_PP = 1 + dt k + dt sum G_f,  A_PQ = -dt G_f (stored for the +x, +y, +z faces;
//      the -d face of P is the +d face of its neighbour),
//      q = dt s + dt sum_{box faces} G_f c_b,
//    and the Jacobi scaling S = diag(A)^(-1/2) with the scaled couplings
//    S_P A_PQ S_Q in FP64 and FP32.
#include <algorithm>
#include <cstring>

#include "context.h"

namespace mpm {

__device__ inline int wsum_int(int v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

struct BoxGeo {
    int nx, ny, nz;      // lattice
    int x0, y0, z0;      // box origin
    int bx, by, bz;      // box size
};

__global__ __launch_bounds__(kThreads) void k_row_count(const uint8_t* __restrict__ mask, BoxGeo g,
                                                   int* __restrict__ rowcnt) {
    const int r = blockIdx.x * kWaves + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    const int rows = g.by * g.bz;
    if (r >= rows) return;
    const int ry = r % g.by, rz = r / g.by;
    const uint8_t* row = mask + ((long long)(g.z0 + rz) * g.ny + (g.y0 + ry)) * g.nx + g.x0;
    int c = 0;
    for (int x = lane; x < g.bx; x += 64) c += row[x] != 0;
    c = wsum_int(c);
    if (lane == 0) rowcnt[r] = c;
}

// Exclusive scan of the n per-row counts in two launches: k_scan_sums totals each chunk
// of kScanChunk rows (one block per chunk), k_scan_apply gives each chunk its offset
// (the sum of the totals before it, summed by the block itself) and scans within the
// chunk.  The grand total goes to *total.  Integer sums: exact in any order.
constexpr int kScanChunk = 4096;                  // rows per block
constexpr int kScanPer = kScanChunk / 256;        // consecutive rows per thread

__device__ inline int block_sum_256(int v, int* sh) {
    v = wsum_int(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const int t = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(256) void k_scan_sums(const int* __restrict__ cnt, int n, int* __restrict__ sums) {
    __shared__ int sh[4];
    const int r0 = blockIdx.x * kScanChunk + threadIdx.x * kScanPer;
    int v = 0;
    for (int i = 0; i < kScanPer; ++i)
        if (r0 + i < n) v += cnt[r0 + i];
    const int t = block_sum_256(v, sh);
    if (threadIdx.x == 0) sums[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_scan_apply(const int* __restrict__ cnt, int n, const int* __restrict__ sums,
                                                    int* __restrict__ start, int* __restrict__ total) {
    __shared__ int sh[4];
    __shared__ int pre[256];
    // offset of this chunk
    int o = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += 256) o += sums[b];
    const int off = block_sum_256(o, sh);
    // per-thread totals of kScanPer consecutive rows, scanned across the block
    const int r0 = blockIdx.x * kScanChunk + threadIdx.x * kScanPer;
    int c[kScanPer];
    int v = 0;
    for (int i = 0; i < kScanPer; ++i) {
        c[i] = r0 + i < n ? cnt[r0 + i] : 0;
        v += c[i];
    }
    pre[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {          // Hillis-Steele inclusive scan
        const int w = threadIdx.x >= d ? pre[threadIdx.x - d] : 0;
        __syncthreads();
        pre[threadIdx.x] += w;
        __syncthreads();
    }
    int run = off + pre[threadIdx.x] - v;
    for (int i = 0; i < kScanPer; ++i) {
        if (r0 + i < n) start[r0 + i] = run;
        run += c[i];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 255) *total = off + pre[255];
}

__global__ __launch_bounds__(kThreads) void k_compact(const uint8_t* __restrict__ mask, BoxGeo g,
                                                 const int* __restrict__ rowstart, int* __restrict__ vox,
                                                 int* __restrict__ boxmap) {
    const int r = blockIdx.x * kWaves + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    const int rows = g.by * g.bz;
    if (r >= rows) return;
    const int ry = r % g.by, rz = r / g.by;
    const long long lrow = ((long long)(g.z0 + rz) * g.ny + (g.y0 + ry)) * g.nx + g.x0;
    const long long brow = (long long)r * g.bx;
    int run = rowstart[r];
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int x0 = 0; x0 < g.bx; x0 += 64) {
        const int x = x0 + lane;
        const bool in = x < g.bx;
        const bool a = in && mask[lrow + x] != 0;
        const unsigned long long bal = __ballot(a);
        if (a) {
            const int l = run + __popcll(bal & below);
            vox[l] = (int)(lrow + x);
            boxmap[brow + x] = l;
        } else if (in) {
            boxmap[brow + x] = -1;
        }
        run += __popcll(bal);
    }
}

__global__ __launch_bounds__(256) void k_neighbors(const int* __restrict__ vox, const int* __restrict__ boxmap,
                                                   BoxGeo g, int N, int Npad, int4* __restrict__ nbr,
                                                   int* __restrict__ voxpad) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= Npad) return;
    if (l >= N) {
        nbr[l] = make_int4(N, N, N, N);
        voxpad[l] = -1;
        return;
    }
    const int v = vox[l];
    const int plane = g.nx * g.ny;
    const int z = v / plane;
    const int rem = v - z * plane;
    const int y = rem / g.nx;
    const int x = rem - y * g.nx;
    const int bxr = x - g.x0, byr = y - g.y0, bzr = z - g.z0;
    const long long bidx = ((long long)bzr * g.by + byr) * g.bx + bxr;
    int4 n;
    int m;
    m = byr > 0 ? boxmap[bidx - g.bx] : -1;
    n.x = m >= 0 ? m : N;
    m = byr + 1 < g.by ? boxmap[bidx + g.bx] : -1;
    n.y = m >= 0 ? m : N;
    m = bzr > 0 ? boxmap[bidx - (long long)g.bx * g.by] : -1;
    n.z = m >= 0 ? m : N;
    m = bzr + 1 < g.bz ? boxmap[bidx + (long long)g.bx * g.by] : -1;
    n.w = m >= 0 ? m : N;
    nbr[l] = n;
}

struct CoefArgs {
    const uint8_t* mask;
    const double* D;
    const double* k;
    const double* src;
    const int* vox;
    double* d64;
    double* q64;
    double* a64;      // [3][S*Npad]
    double* sc64;
    BoxGeo g;
    long long nvox;
    double dt, inv_h2;
    double cb[MPM_MAX_SPECIES];
    int N, Npad, S;
    int* bad;         // set to 1 if a domain voxel has D < 0, k < 0 or a non-finite value
};

__device__ inline double harm(double a, double b) {
    const double s = a + b;
    return s != 0.0 ? 2.0 * a * b / s : 0.0;
}

// One thread per (species, l).  Padding gets A_PP = 1, q = 0, couplings 0, scale 0.
__global__ __launch_bounds__(256) void k_coefs(CoefArgs a) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tot = (long long)a.S * a.Npad;
    if (i >= tot) return;
    const int s = (int)(i / a.Npad);
    const int l = (int)(i - (long long)s * a.Npad);
    const long long stride3 = tot;
    if (l >= a.N) {
        a.d64[i] = 1.0;
        a.q64[i] = 0.0;
        a.a64[i] = 0.0;
        a.a64[i + stride3] = 0.0;
        a.a64[i + 2 * stride3] = 0.0;
        a.sc64[i] = 0.0;
        return;
    }
    const BoxGeo& g = a.g;
    const int v = a.vox[l];
    const int plane = g.nx * g.ny;
    const int z = v / plane;
    const int rem = v - z * plane;
    const int y = rem / g.nx;
    const int x = rem - y * g.nx;
    const int cr[3] = {x - g.x0, y - g.y0, z - g.z0};
    const int bs[3] = {g.bx, g.by, g.bz};
    const long long ls[3] = {1, g.nx, (long long)plane};
    const double* Ds = a.D + (long long)s * a.nvox;
    const double DP = Ds[v];
    {
        const double kv = a.k[(long long)s * a.nvox + v], sv = a.src[(long long)s * a.nvox + v];
        if (!(DP >= 0.0) || !(kv >= 0.0) || isinf(DP) || isinf(kv) || !isfinite(sv)) *a.bad = 1;
    }
    double sumG = 0.0, dir = 0.0;
    double up[3];
    for (int d = 0; d < 3; ++d) {
        for (int side = -1; side <= 1; side += 2) {
            const int c = cr[d] + side;
            double G = 0.0;
            if (c < 0 || c >= bs[d]) {            // box face: Dirichlet at half a voxel
                G = 2.0 * DP * a.inv_h2;
                dir += G;
            } else {
                const long long q = v + side * ls[d];
                if (a.mask[q]) G = harm(DP, Ds[q]) * a.inv_h2;
            }
            sumG += G;
            if (side > 0) up[d] = (c < bs[d]) ? G : 0.0;
        }
    }
    const double ks = a.k[(long long)s * a.nvox + v];
    const double ss = a.src[(long long)s * a.nvox + v];
    const double diag = 1.0 + a.dt * ks + a.dt * sumG;
    a.d64[i] = diag;
    a.q64[i] = a.dt * ss + a.dt * dir * a.cb[s];
    a.a64[i] = -a.dt * up[0];
    a.a64[i + stride3] = -a.dt * up[1];
    a.a64[i + 2 * stride3] = -a.dt * up[2];
    a.sc64[i] = 1.0 / sqrt(diag);
}

// Scaled couplings S_P A_PQ S_Q toward +x, +y, +z.
__global__ __launch_bounds__(256) void k_scaled(const double* __restrict__ a64, const double* __restrict__ sc,
                                                const int4* __restrict__ nbr, int N, int Npad, int S,
                                                double* __restrict__ c64, float* __restrict__ c32) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tot = (long long)S * Npad;
    if (i >= tot) return;
    const int s = (int)(i / Npad);
    const int l = (int)(i - (long long)s * Npad);
    const long long base = (long long)s * Npad;
    double cx = 0.0, cy = 0.0, cz = 0.0;
    if (l < N) {
        const int4 n = nbr[l];
        const double sp = sc[i];
        const double ax = a64[i], ay = a64[i + tot], az = a64[i + 2 * tot];
        if (ax != 0.0) cx = ax * sp * sc[i + 1];
        if (ay != 0.0) cy = ay * sp * sc[base + n.y];
        if (az != 0.0) cz = az * sp * sc[base + n.w];
    }
    c64[i] = cx;
    c64[i + tot] = cy;
    c64[i + 2 * tot] = cz;
    c32[i] = (float)cx;
    c32[i + tot] = (float)cy;
    c32[i + 2 * tot] = (float)cz;
}

// Coefficient arrays carry kAlign zero elements before and after their data so
// that the "left neighbour" read of voxel 0 and the right read of the last
// element stay inside the allocation and see zero couplings.
template <typename T>
static hipError_t alloc_padded(T** p, size_t n) {
    T* raw = nullptr;
    hipError_t e = hipMalloc(&raw, (n + 2 * kAlign) * sizeof(T));
    if (e != hipSuccess) return e;
    e = hipMemset(raw, 0, (n + 2 * kAlign) * sizeof(T));
    *p = raw + kAlign;
    return e;
}
template <typename T>
static void free_padded(T*& p) {
    if (p) (void)hipFree(p - kAlign);
    p = nullptr;
}

// Static input channels of the warm-start network on the box grid (box sizes rounded
// up to multiples of 8), channel-major (stat[c G + i] for grid voxel i of G): k[0..S),
// D[0..S), s[0..S), mask; zero outside the box.
__global__ void k_ws_static(const uint8_t* mask, const double* D, const double* k, const double* src, BoxGeo g,
                            int gx, int gy, int gz, int S, long long nvox, float* stat) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long G = (long long)gx * gy * gz;
    if (i >= G) return;
    const int x = (int)(i % gx);
    const int y = (int)((i / gx) % gy);
    const int z = (int)(i / ((long long)gx * gy));
    const int C = ws_static_channels(S);
    if (x >= g.bx || y >= g.by || z >= g.bz) {
        for (int c = 0; c < C; ++c) stat[c * G + i] = 0.f;
        return;
    }
    const long long v = ((long long)(g.z0 + z) * g.ny + (g.y0 + y)) * g.nx + (g.x0 + x);
    for (int s = 0; s < S; ++s) {
        stat[s * G + i] = (float)k[s * nvox + v];
        stat[(S + s) * G + i] = (float)D[s * nvox + v];
        stat[(2 * S + s) * G + i] = (float)src[s * nvox + v];
    }
    stat[3 * S * G + i] = mask[v] ? 1.f : 0.f;
}

// The network's voxel tiles on the warm-start grid (16 x 4 x 4, as its convolutions
// tile it): per tile, flag[ntiles + t] = 1 when a domain voxel (mask channel of the
// static input) lies in it (the last convolution's tiles); flag[t] = 1 when a domain
// voxel lies in the tile grown by one voxel on every side, i.e. when the tile holds a
// value the last 3x3x3 convolution reads for a domain voxel's output (the tiles of the
// convolution before it).  The last convolution's other outputs, of the voxels off the
// domain, may then read values no launch wrote; nothing reads those outputs.  One wave
// per tile.
constexpr int kWsTX = 16, kWsTY = 4, kWsTZ = 4;
__global__ void k_ws_tile_domain(const float* stat, int S, int gx, int gy, int gz, uint8_t* flag) {
    const int ntx = (gx + kWsTX - 1) / kWsTX, nty = gy / kWsTY, ntz = gz / kWsTZ;
    const int nt = ntx * nty * ntz;
    const int t = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);   // one wave per tile
    if (t >= nt) return;
    const int lane = threadIdx.x & 63;
    const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
    const float* m = stat + (long long)3 * S * gx * gy * gz;   // the mask channel
    bool hit = false;
    for (int v = lane; v < kWsTX * kWsTY * kWsTZ; v += 64) {
        const int x = tx * kWsTX + v % kWsTX, y = ty * kWsTY + (v / kWsTX) % kWsTY;
        const int z = tz * kWsTZ + v / (kWsTX * kWsTY);
        if (x < gx && m[((long long)z * gy + y) * gx + x] > 0.f) hit = true;
    }
    const bool any = __ballot(hit) != 0;
    if (lane == 0) flag[nt + t] = any ? 1 : 0;
}
__global__ void k_ws_tile_near(const float* stat, int S, int gx, int gy, int gz, uint8_t* flag) {
    const int ntx = (gx + kWsTX - 1) / kWsTX, nty = gy / kWsTY, ntz = gz / kWsTZ;
    const int nt = ntx * nty * ntz;
    const int t = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);   // one wave per tile
    if (t >= nt) return;
    const int lane = threadIdx.x & 63;
    const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
    const float* m = stat + (long long)3 * S * gx * gy * gz;   // the mask channel
    constexpr int EX = kWsTX + 2, EY = kWsTY + 2, EZ = kWsTZ + 2;
    bool hit = false;
    for (int v = lane; v < EX * EY * EZ; v += 64) {
        const int x = tx * kWsTX - 1 + v % EX, y = ty * kWsTY - 1 + (v / EX) % EY;
        const int z = tz * kWsTZ - 1 + v / (EX * EY);
        if (x >= 0 && x < gx && y >= 0 && y < gy && z >= 0 && z < gz && m[((long long)z * gy + y) * gx + x] > 0.f)
            hit = true;
    }
    const bool any = __ballot(hit) != 0;
    if (lane == 0) flag[t] = any ? 1 : 0;
}

// Grow a scratch buffer to hold n elements (with room for later growth).
template <typename T>
static hipError_t reserve(T** p, size_t* cap, size_t n) {
    if (n <= *cap) return hipSuccess;
    (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    const size_t want = n + n / 8 + 1024;
    hipError_t e = hipMalloc(p, want * sizeof(T));
    if (e == hipSuccess) *cap = want;
    return e;
}

static void free_scratch(ProbHost& ph) {
    (void)hipFree(ph.s_rowcnt);
    (void)hipFree(ph.s_rowstart);
    (void)hipFree(ph.s_boxmap);
    (void)hipFree(ph.s_vox);
    (void)hipFree(ph.s_total);
    (void)hipFree(ph.s_chunk);
    ph.s_rowcnt = ph.s_rowstart = ph.s_boxmap = ph.s_vox = ph.s_total = ph.s_chunk = nullptr;
    ph.cap_rows = ph.cap_boxvox = ph.cap_svox = 0;
}

// Scratch of one setup call: per-row counts and starts, the box-to-domain map, the
// compacted voxel list (npad elements, 0 = not needed yet) and the total.
static int reserve_scratch(ProbHost& ph, size_t rows, size_t boxvox, size_t npad) {
    hipError_t e = hipSuccess;
    if (rows > ph.cap_rows) {
        (void)hipFree(ph.s_rowcnt);
        (void)hipFree(ph.s_rowstart);
        (void)hipFree(ph.s_chunk);
        ph.s_rowcnt = ph.s_rowstart = ph.s_chunk = nullptr;
        ph.cap_rows = 0;
        const size_t want = rows + rows / 8 + 1024;
        e = hipMalloc(&ph.s_rowcnt, want * sizeof(int));
        if (e == hipSuccess) e = hipMalloc(&ph.s_rowstart, want * sizeof(int));
        if (e == hipSuccess) e = hipMalloc(&ph.s_chunk, (want / kScanChunk + 2) * sizeof(int));
        if (e == hipSuccess) ph.cap_rows = want;
    }
    if (e == hipSuccess) e = reserve(&ph.s_boxmap, &ph.cap_boxvox, boxvox);
    if (e == hipSuccess) e = reserve(&ph.s_vox, &ph.cap_svox, npad);
    if (e == hipSuccess && !ph.s_total) e = hipMalloc(&ph.s_total, sizeof(int));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_scratch(ph);
        set_error("mpm_fv_setup: device allocation failed");
        return MPM_ENOMEM;
    }
    return MPM_OK;
}

void free_problem(ProbHost& ph) {
    free_scratch(ph);
    free_padded(ph.vox);
    free_padded(ph.nbr);
    free_padded(ph.d64);
    free_padded(ph.q64);
    free_padded(ph.a64);
    free_padded(ph.sc64);
    free_padded(ph.c32);
    free_padded(ph.c64);
    ph.cap_pad = 0;
    ph.hw_pad = 0;
    (void)hipFree(ph.stat);
    (void)hipFree(ph.wsin);
    (void)hipFree(ph.wsout);
    ph.stat = nullptr;
    ph.wsin = nullptr;
    ph.wsout = nullptr;
    ph.cap_grid = 0;
    (void)hipFree(ph.tl_dev);
    (void)hipFree(ph.tf_dev);
    if (ph.tl_host) (void)hipHostFree(ph.tl_host);
    if (ph.tf_host) (void)hipHostFree(ph.tf_host);
    ph.tl_dev = nullptr;
    ph.tf_dev = nullptr;
    ph.tl_host = nullptr;
    ph.tf_host = nullptr;
    ph.cap_tiles = 0;
    ph.tl_n[0] = -1;
    ph.tl_n[1] = 0;
}

// Zero elements [from, to) of a padded array (its trailing padding included).
template <typename T>
static hipError_t zero_tail(T* p, size_t from, size_t to, hipStream_t st) {
    return to > from ? hipMemsetAsync(p + from, 0, (to - from) * sizeof(T), st) : hipSuccess;
}

// Coefficient arrays for Npad padded unknowns per species.  They are sized with room
// for growth (a box that grows step by step keeps them).  A layout writes exactly the
// first Npad (per-voxel arrays), S Npad or 3 S Npad elements; when a reused array had
// held a larger layout, the part past the new one is zeroed, so reads past the data see
// zero couplings exactly as in a fresh allocation.
static int alloc_problem(ProbHost& ph, int S, int Npad, hipStream_t st) {
    const size_t n = (size_t)Npad, u = (size_t)S * Npad;
    if (n <= ph.cap_pad) {
        hipError_t e = hipSuccess;
        if (n < ph.hw_pad) {
            const size_t hn = ph.hw_pad, hu = (size_t)S * ph.hw_pad;
            e = zero_tail(ph.vox, n, hn, st);
            if (e == hipSuccess) e = zero_tail(ph.nbr, n, hn, st);
            if (e == hipSuccess) e = zero_tail(ph.d64, u, hu, st);
            if (e == hipSuccess) e = zero_tail(ph.q64, u, hu, st);
            if (e == hipSuccess) e = zero_tail(ph.sc64, u, hu, st);
            if (e == hipSuccess) e = zero_tail(ph.a64, 3 * u, 3 * hu, st);
            if (e == hipSuccess) e = zero_tail(ph.c32, 3 * u, 3 * hu, st);
            if (e == hipSuccess) e = zero_tail(ph.c64, 3 * u, 3 * hu, st);
        }
        ph.hw_pad = n;
        return e == hipSuccess ? MPM_OK : hip_fail(e, "mpm_fv_setup (reuse)");
    }
    // keep the setup scratch, drop the rest
    free_padded(ph.vox);
    free_padded(ph.nbr);
    free_padded(ph.d64);
    free_padded(ph.q64);
    free_padded(ph.a64);
    free_padded(ph.sc64);
    free_padded(ph.c32);
    free_padded(ph.c64);
    ph.cap_pad = 0;
    ph.hw_pad = 0;
    const size_t cn = (n + n / 8 + kAlign - 1) / kAlign * kAlign, cu = (size_t)S * cn;
    if (alloc_padded(&ph.vox, cn) != hipSuccess || alloc_padded(&ph.nbr, cn) != hipSuccess ||
        alloc_padded(&ph.d64, cu) != hipSuccess || alloc_padded(&ph.q64, cu) != hipSuccess ||
        alloc_padded(&ph.a64, 3 * cu) != hipSuccess || alloc_padded(&ph.sc64, cu) != hipSuccess ||
        alloc_padded(&ph.c32, 3 * cu) != hipSuccess || alloc_padded(&ph.c64, 3 * cu) != hipSuccess) {
        free_problem(ph);
        (void)hipGetLastError();
        set_error("mpm_fv_setup: device allocation failed");
        return MPM_ENOMEM;
    }
    ph.cap_pad = cn;
    ph.hw_pad = n;
    return MPM_OK;
}

// Coefficients of problem ph on its compacted layout (N domain voxels, vox their lattice
// indices): face couplings, diagonal, right-hand-side terms, Jacobi scaling, the scaled
// copies and, for the learned warm start, the static network input channels.  flag is a
// device word used as the error flag (negative or non-finite input on a domain voxel);
// synchronises the stream to read it.
static int discretise(Ctx* c, ProbHost& ph, const BoxGeo& g, const uint8_t* mask, const double* D, const double* k,
                      const double* src, const double* cb, double dt, double h, int N, int Npad, const int* vox,
                      int* flag) {
    hipStream_t st = c->stream;
    CoefArgs ca;
    ca.mask = mask; ca.D = D; ca.k = k; ca.src = src; ca.vox = vox;
    ca.d64 = ph.d64; ca.q64 = ph.q64; ca.a64 = ph.a64; ca.sc64 = ph.sc64;
    ca.g = g;
    ca.nvox = (long long)g.nx * g.ny * g.nz;
    ca.dt = dt;
    ca.inv_h2 = 1.0 / (h * h);
    for (int s = 0; s < MPM_MAX_SPECIES; ++s) ca.cb[s] = s < c->S ? cb[s] : 0.0;
    ca.N = N; ca.Npad = Npad; ca.S = c->S;
    ca.bad = flag;
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), st);
    if (e != hipSuccess) return hip_fail(e, "mpm_fv_setup (flag)");
    const long long tot = (long long)c->S * Npad;
    k_coefs<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(ca);
    k_scaled<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(ph.a64, ph.sc64, ph.nbr, N, Npad, c->S, ph.c64,
                                                          ph.c32);
    if (net_warm_start(c)) {
        const int gx = (g.bx + 7) / 8 * 8, gy = (g.by + 7) / 8 * 8, gz = (g.bz + 7) / 8 * 8;
        const size_t G = (size_t)gx * gy * gz;
        if (G > ph.cap_grid) {
            (void)hipFree(ph.stat);
            (void)hipFree(ph.wsin);
            (void)hipFree(ph.wsout);
            ph.stat = nullptr;
            ph.wsin = nullptr;
            ph.wsout = nullptr;
            ph.cap_grid = 0;
            if (hipMalloc(&ph.stat, G * ws_static_channels(c->S) * sizeof(float)) != hipSuccess ||
                hipMalloc(&ph.wsin, G * ws_channels(c->S) * sizeof(uint16_t)) != hipSuccess ||
                hipMalloc(&ph.wsout, G * c->S * sizeof(float)) != hipSuccess) {
                (void)hipGetLastError();
                set_error("mpm_fv_setup: device allocation of the warm-start buffers failed");
                return MPM_ENOMEM;
            }
            ph.cap_grid = G;
        }
        ph.gd[0] = gx;
        ph.gd[1] = gy;
        ph.gd[2] = gz;
        ph.ws_ready = false;
        k_ws_static<<<(unsigned)((G + 255) / 256), 256, 0, st>>>(mask, D, k, src, g, gx, gy, gz, c->S, ca.nvox,
                                                              ph.stat);
        // the tiles of the network's last level that the domain needs (lists built below,
        // once the flags are on the host); entries pack the tile digits in 10, 10 and 11 bits
        const int ntx = (gx + kWsTX - 1) / kWsTX, nty = gy / kWsTY, ntz = gz / kWsTZ;
        const size_t nt = (size_t)ntx * nty * ntz;
        ph.tl_n[0] = -1;
        ph.tl_n[1] = 0;
        if (ntx < 1024 && nty < 1024 && ntz < 2048) {
            if (nt > ph.cap_tiles) {
                (void)hipFree(ph.tl_dev);
                (void)hipFree(ph.tf_dev);
                if (ph.tl_host) (void)hipHostFree(ph.tl_host);
                if (ph.tf_host) (void)hipHostFree(ph.tf_host);
                ph.tl_dev = nullptr;
                ph.tf_dev = nullptr;
                ph.tl_host = nullptr;
                ph.tf_host = nullptr;
                ph.cap_tiles = 0;
                if (hipMalloc(&ph.tl_dev, 2 * nt * sizeof(int)) != hipSuccess ||
                    hipMalloc(&ph.tf_dev, 2 * nt) != hipSuccess ||
                    hipHostMalloc((void**)&ph.tl_host, 2 * nt * sizeof(int), hipHostMallocDefault) != hipSuccess ||
                    hipHostMalloc((void**)&ph.tf_host, 2 * nt, hipHostMallocDefault) != hipSuccess) {
                    (void)hipGetLastError();
                    set_error("mpm_fv_setup: device allocation of the warm-start tile lists failed");
                    return MPM_ENOMEM;
                }
                ph.cap_tiles = nt;
            }
            k_ws_tile_domain<<<(unsigned)((nt + 3) / 4), 256, 0, st>>>(ph.stat, c->S, gx, gy, gz, ph.tf_dev);
            k_ws_tile_near<<<(unsigned)((nt + 3) / 4), 256, 0, st>>>(ph.stat, c->S, gx, gy, gz, ph.tf_dev);
            e = hipGetLastError();
            if (e == hipSuccess) e = hipMemcpyAsync(ph.tf_host, ph.tf_dev, 2 * nt, hipMemcpyDeviceToHost, st);
            if (e != hipSuccess) return hip_fail(e, "mpm_fv_setup (tile flags)");
            ph.tl_n[0] = 0;
        }
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(c->h_small + 1, flag, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "mpm_fv_setup (coefficients)");
    if (c->h_small[1]) {
        set_error("mpm_fv_setup: negative or non-finite D, k or s on a domain voxel");
        return MPM_EINVAL;
    }
    if (net_warm_start(c) && ph.tl_n[0] == 0) {
        const int ntx = (ph.gd[0] + kWsTX - 1) / kWsTX, nty = ph.gd[1] / kWsTY, ntz = ph.gd[2] / kWsTZ;
        const int nt = ntx * nty * ntz;
        int na = 0, nb = 0;
        for (int pass = 0; pass < 2; ++pass)
            for (int t = 0; t < nt; ++t) {
                if (!ph.tf_host[pass * nt + t]) continue;
                const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
                const int entry = tx | ty << 10 | tz << 20;
                if (pass == 0) ph.tl_host[na++] = entry;
                else ph.tl_host[nt + nb++] = entry;   // moved behind the first list below
            }
        std::memmove(ph.tl_host + na, ph.tl_host + nt, (size_t)nb * sizeof(int));
        e = hipMemcpyAsync(ph.tl_dev, ph.tl_host, (size_t)(na + nb) * sizeof(int), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "mpm_fv_setup (tile lists)");
        ph.tl_n[0] = na;
        ph.tl_n[1] = nb;
    }
    return MPM_OK;
}

int setup_problem(Ctx* c, int p, const int* dims, const int* lo, const int* hi, const uint8_t* mask,
                  const double* D, const double* k, const double* src, const double* cb, double dt,
                  double h) {
    ProbHost& ph = c->probs[p];
    hipStream_t st = c->stream;
    BoxGeo g;
    g.nx = dims[0]; g.ny = dims[1]; g.nz = dims[2];
    g.x0 = lo[0]; g.y0 = lo[1]; g.z0 = lo[2];
    g.bx = hi[0] - lo[0]; g.by = hi[1] - lo[1]; g.bz = hi[2] - lo[2];
    const int rows = g.by * g.bz;
    const long long boxvox = (long long)rows * g.bx;

    int rc = reserve_scratch(ph, (size_t)rows, (size_t)boxvox, 0);
    if (rc != MPM_OK) return rc;
    int* total_d = ph.s_total;
    const int gr = (rows + kWaves - 1) / kWaves;
    k_row_count<<<gr, kThreads, 0, st>>>(mask, g, ph.s_rowcnt);
    const int nchunk = (rows + kScanChunk - 1) / kScanChunk;
    k_scan_sums<<<nchunk, 256, 0, st>>>(ph.s_rowcnt, rows, ph.s_chunk);
    k_scan_apply<<<nchunk, 256, 0, st>>>(ph.s_rowcnt, rows, ph.s_chunk, ph.s_rowstart, total_d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(c->h_small, total_d, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "mpm_fv_setup (count)");
    const int total_h = c->h_small[0];
    if (total_h == 0) {
        set_error("mpm_fv_setup: the box holds no domain voxel");
        return MPM_EEMPTY;
    }
    const int N = total_h;
    const int Npad = (int)(((long long)N + 1 + kAlign - 1) / kAlign * kAlign);
    rc = alloc_problem(ph, c->S, Npad, st);
    if (rc != MPM_OK) return rc;
    rc = reserve_scratch(ph, (size_t)rows, (size_t)boxvox, (size_t)Npad);
    if (rc != MPM_OK) return rc;
    int* vox_tmp = ph.s_vox;
    k_compact<<<gr, kThreads, 0, st>>>(mask, g, ph.s_rowstart, vox_tmp, ph.s_boxmap);
    k_neighbors<<<(Npad + 255) / 256, 256, 0, st>>>(vox_tmp, ph.s_boxmap, g, N, Npad, ph.nbr, ph.vox);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "mpm_fv_setup (compaction)");
    // ph.vox receives -1 on padding from k_neighbors; copy the domain part
    e = hipMemcpyAsync(ph.vox, vox_tmp, (size_t)N * sizeof(int), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "mpm_fv_setup (vox)");
    ph.nvox = (long long)dims[0] * dims[1] * dims[2];
    rc = discretise(c, ph, g, mask, D, k, src, cb, dt, h, N, Npad, vox_tmp, total_d);
    if (rc != MPM_OK) {
        ph.ready = false;
        c->layout_dirty = true;
        return rc;
    }

    const bool grew = Npad != ph.Npad;
    ph.N = N;
    ph.Npad = Npad;
    for (int d = 0; d < 3; ++d) {
        ph.dims[d] = dims[d];
        ph.lo[d] = lo[d];
        ph.hi[d] = hi[d];
    }
    ph.dt = dt;
    ph.h = h;
    for (int s = 0; s < c->S; ++s) ph.cb[s] = cb[s];
    ph.ready = true;
    // descriptors (pointers may have moved) and the layout are rebuilt lazily
    c->layout_dirty = true;
    (void)grew;
    return MPM_OK;
}

// New coefficients on the box and domain of the last set-up: the compaction, the
// neighbour table and the launch layout are kept (the caller guarantees that the box and
// the domain voxels are unchanged), only the discretisation is redone.
int update_problem(Ctx* c, int p, const uint8_t* mask, const double* D, const double* k, const double* src,
                   const double* cb, double dt, double h) {
    ProbHost& ph = c->probs[p];
    if (!ph.ready) {
        set_error("mpm_fv_update: the problem has not been set up (mpm_fv_setup)");
        return MPM_ESTATE;
    }
    BoxGeo g;
    g.nx = ph.dims[0]; g.ny = ph.dims[1]; g.nz = ph.dims[2];
    g.x0 = ph.lo[0]; g.y0 = ph.lo[1]; g.z0 = ph.lo[2];
    g.bx = ph.hi[0] - ph.lo[0]; g.by = ph.hi[1] - ph.lo[1]; g.bz = ph.hi[2] - ph.lo[2];
    int rc = discretise(c, ph, g, mask, D, k, src, cb, dt, h, ph.N, ph.Npad, ph.vox, ph.s_total);
    if (rc != MPM_OK) {
        ph.ready = false;
        c->layout_dirty = true;
        return rc;
    }
    ph.dt = dt;
    ph.h = h;
    for (int s = 0; s < c->S; ++s) ph.cb[s] = cb[s];
    // the layout stands; the per-system diagonal extremes are refreshed before the next step
    c->coef_dirty = true;
    return MPM_OK;
}

}  // namespace mpm
