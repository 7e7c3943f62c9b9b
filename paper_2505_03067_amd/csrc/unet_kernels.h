// Device kernels of the warm-start U-Net (BF16 storage, FP32 accumulation).
//
// Activations are NDHWC [n][z][y][x][c] in BF16.  3x3x3 convolutions are implicit
// GEMMs on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16): M = output voxels,
// N = output channels, K = 27 taps x input channels (padded to a multiple of 16), taken
// in 32-wide steps whose 8 consecutive k of one lane always belong to one tap.  The
// input gradient is the same GEMM on the output gradient with the taps mirrored and the
// weights transposed: dX[p] = sum_t dY[p - off(t)] W[t] = sum_t dY[p + off(t)] W[26 - t],
// so the forward kernel runs on packed weights holding W[26 - t] transposed.  The weight
// gradient stages voxel tiles in LDS, transposed so that K runs over voxels, and takes
// all 27 taps from one staged tile.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpm {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// round to nearest, ties to even; overflow rounds to infinity, and every NaN becomes
// the quiet NaN 0x7fc0 (adding the rounding bias to a NaN could carry into the sign)
__device__ inline uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)0x7fc0u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

struct ConvArgs {
    const uint16_t* x;     // GEMM input [P][ldx] (activation, or output gradient for dgrad)
    const uint16_t* gate;  // optional [P][ldx]: use x * (gate > 0) (ReLU backward)
    const uint16_t* w;     // BF16 weights packed in MFMA fragment order (k_pack)
    const float* bias;     // optional [cout]
    uint16_t* y;           // output [P][ldy], channels [yoff, yoff + cout)
    float* yf;             // optional FP32 output [P][cout]
    int ldx, cin_p, nt;    // input stride and padded channels; 16-channel output tiles
    // optional upsample-and-concatenate input: channels [0, c1) are x on the grid of half
    // the resolution (nearest upsampling, stride ldx = c1), channels [c1, cin_p) are x2
    // (stride ldx2); c1 a multiple of 16, never with a gate
    const uint16_t* x2;
    int ldx2, c1;
    int ldy, yoff, cout, relu;
    int n, D, H, W;
    // optional 1x1x1 head fused into the epilogue (one 16-channel output tile): per voxel
    // hout[p][o] = hb[o] + sum_c bf16(y[p][c]) hw[c hcout + o], o < hcout <= 4, in the
    // order of k_head; y itself is stored only when set
    const float* hw;
    const float* hb;
    float* hout;
    int hcout;
    // optional list of the tiles to compute (sample 0 only, n = 1): entry tx | ty << 10 |
    // tz << 20; the other tiles' outputs are left as they are
    const int* tlist;
    int tcount;
    // optional 2x2x2 average pooling of the BF16 output fused into the epilogue: yp
    // [n][D/2][H/2][W/2][cout] (D, H, W even), in the order of k_pool2
    uint16_t* yp;
};

// LDS floats of the fused head's weights (16 x up to 4) and biases
constexpr int kHeadLds = 16 * 4 + 4;
// tile-list entries a block stages (see conv_start)
constexpr int kListMax = 64;

// Keep each BF16 half of x only where the gate half is > 0 (ReLU backward).
__device__ inline uint4 apply_gate(uint4 t, const uint4 g) {
    const uint32_t gw[4] = {g.x, g.y, g.z, g.w};
    uint32_t tw[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t lo = gw[i] & 0xffffu, hi = gw[i] >> 16;
        const bool plo = lo != 0 && !(lo & 0x8000u);
        const bool phi = hi != 0 && !(hi & 0x8000u);
        tw[i] &= (plo ? 0x0000ffffu : 0u) | (phi ? 0xffff0000u : 0u);
    }
    return make_uint4(tw[0], tw[1], tw[2], tw[3]);
}

// 3x3x3 convolution as an implicit GEMM with the input staged in LDS.
// Work items are (voxel tile, output-tile group) pairs: a voxel tile is 16 (x) x 4 (y) x
// 4 (z) voxels of one sample, a group NTB of the GEMM's NT 16-channel output tiles.
// Blocks are persistent: block b takes items b, b + G, b + 2G, ... (G = grid size, a
// multiple of NT / NTB, so a block keeps one output-tile group).  Per item and chunk of
// 16 input channels, the input tile with its one-voxel halo (18 x 6 x 6 voxels) is
// staged in LDS, and all 27 taps read it from there; the global loads of the next
// (item, chunk) are issued before the MFMAs of the current one.  With one chunk (16
// input channels) the block's weights stay in registers for all its items; with more,
// each chunk's weights are staged in LDS beside the tile.  Wave w computes rows (y, z)
// = (0..3, w) of the tile (four 16-voxel M tiles).  K runs over tap x channel in 14 MFMA
// steps of 32 per chunk: the two lane halves h = g / 2 (g = lane / 16; channels
// 8 (g mod 2) .. + 7 of the chunk) take the two taps step_tap(s, h).  Nine of the steps
// pair the taps dx = 0 and 1 of one halo row, so each row read from LDS feeds the MFMAs
// of up to three M tiles (38 A-fragment reads per chunk and wave instead of 56).  The
// taps are unrolled at compile time, so every LDS read is a per-lane base plus an
// immediate.  (Chunks of 32 channels, one tap per step, need 27 steps instead of 28 but
// 78 KB of LDS per block, two blocks per CU instead of three, and measured slower.)
// The MFMAs take the weight fragment as their A operand and the input fragment as B,
// which yields the transposed tile: lane l then holds output channels 4 (l / 16) .. + 3
// of voxel l mod 16, stored straight to global memory as one 8-byte word (16 lanes
// cover 16 consecutive voxels of a row).  The item's tile comes from a mixed-radix
// cursor and every address is a uniform base plus a 32-bit per-lane offset, so the
// per-item integer work is a few instructions (64-bit divisions and per-word address
// arithmetic had cost more issue cycles than the MFMAs).
//
// Packed weights (k_pack): one 16-byte B fragment per (step, output tile, lane), steps
// numbered over the chunks in order; the fragment of lane (n = lane mod 16, g) holds the
// 8 input channels of g at its tap for output channel 16 t + n, so a block's weights for
// one step are NTB contiguous kilobytes.
constexpr int kTX = 16, kTY = 4, kTZ = 4;
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2;
constexpr int kHV = kHX * kHY * kHZ;
#ifndef MPM_CONV_CS
#define MPM_CONV_CS 16
#endif
constexpr int kCS = MPM_CONV_CS;   // LDS channel stride per halo voxel, BF16 values (16: no padding)
static_assert(kCS % 8 == 0 && kCS >= 16, "16-byte aligned halo voxels of 16 channels");
constexpr int kSteps = 14; // MFMA steps per 16-channel chunk

// halo-tile voxel offset of tap t = 9 dz + 3 dy + dx (dz, dy, dx in 0..2)
__host__ __device__ constexpr int tap_vox(int t) { return ((t / 9) * kHY + (t / 3) % 3) * kHX + t % 3; }

// The taps of MFMA step s of a 16-channel chunk in lane half h (lanes 32 h .. 32 h + 31),
// paired so that one A fragment read from LDS serves several M tiles: steps 0-8 pair
// (dz, dy, 0) with (dz, dy, 1) (one halo row; the second tap one voxel further along x),
// so the fragment of M tile mt at dy is that of M tile mt + 1 at dy - 1; steps 9-11 pair
// (dz, 0, 2) with (dz, 1, 2) (the next row), step 12 (0, 2, 2) with (1, 2, 2) (the next
// plane), step 13 (2, 2, 2) with zero weights (tap 27).
__host__ __device__ constexpr int step_tap(int s, int h) {
    return s < 9 ? 9 * (s / 3) + 3 * (s % 3) + h : s < 12 ? 9 * (s - 9) + 2 + 3 * h : s == 12 ? 8 + 9 * h : (h ? 27 : 26);
}
__host__ __device__ constexpr bool step_taps_cover() {
    int seen[28] = {};
    for (int s = 0; s < kSteps; ++s)
        for (int h = 0; h < 2; ++h) ++seen[step_tap(s, h)];
    for (int t = 0; t < 28; ++t)
        if (seen[t] != 1) return false;
    return true;
}
static_assert(step_taps_cover(), "every tap (and the zero tap 27) in exactly one step half");

// LDS of one block: the halo tile (kCS values per voxel: 32 bytes, unpadded; padded
// strides of 48, 64 and 80 bytes measured no faster), then one chunk's weights
__host__ __device__ constexpr int conv_x_bytes() { return kHV * kCS * 2; }
// the block's weights (one chunk's) staged in LDS after the halo tile, except with one
// chunk and one output tile (then they live in registers); then the block's bias values
__host__ __device__ constexpr int conv_w_bytes(int ntb, bool wl) { return wl || ntb > 1 ? kSteps * ntb * 1024 : 0; }
// LDS bytes of the fused pooling's exchange between the waves of a plane pair: per pair
// and lane, two pooled rows of four channels per output tile
__host__ __device__ constexpr int conv_pool_bytes(int ntb) { return 2 * 64 * 8 * ntb * 4; }
__host__ __device__ constexpr int conv_lds_bytes(int ntb, bool wl, bool head = false, bool list = false,
                                                 bool pool = false) {
    // + the block's bias values, the fused head's parameters, the block's tile list and
    // the pooling exchange
    return conv_x_bytes() + conv_w_bytes(ntb, wl) + 64 * ntb + (head ? 4 * kHeadLds : 0) + (list ? 4 * kListMax : 0) +
           (pool ? conv_pool_bytes(ntb) : 0);
}

// Stage the fused head's parameters (a.hout set) in LDS: weights [16][4] at 0 (zero past
// hcout outputs), biases at 64.  Read after the block's first barrier.
__device__ inline void conv_stage_head(const ConvArgs& a, float* head_l) {
    if (!a.hout) return;
    if (threadIdx.x < 64) {
        const int c = threadIdx.x >> 2, o = threadIdx.x & 3;
        head_l[threadIdx.x] = o < a.hcout ? a.hw[c * a.hcout + o] : 0.f;
    }
    if (threadIdx.x < 4) head_l[64 + threadIdx.x] = threadIdx.x < a.hcout ? a.hb[threadIdx.x] : 0.f;
}

// Sum of x over lane l and lane l ^ 16 (v_permlane16_swap trades the odd 16-lane rows of
// its first operand for the even rows of its second), and over l and l ^ 32
// (v_permlane32_swap trades the upper half of the first for the lower half of the
// second).  Both add the two values in the same order in every lane.
__device__ inline float sum_xor16(float x) {
    const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}
__device__ inline float sum_xor32(float x) {
    const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}

// Origin of a voxel tile (tile index: x fastest, then y, z, sample), and whether its
// halo (in) and the tile itself (out) lie inside the grid.
struct ConvTile {
    int x0, y0, z0;
    long long sbase;
    bool in, out;
};
// Tile index as mixed-radix digits (x, y, z tile, sample), advanced by a fixed stride
// (the grid's tiles per round) without divisions.
struct ConvCursor {
    int tx, ty, tz, n;
    int sx, sy, sz, sn;
    int k;   // with a tile list: the block's entry
};
__device__ inline void conv_digits(const ConvArgs& a, unsigned t, int& x, int& y, int& z, int& n) {
    const unsigned ntx = (a.W + kTX - 1) / kTX, nty = (a.H + kTY - 1) / kTY, ntz = (a.D + kTZ - 1) / kTZ;
    x = (int)(t % ntx);
    t /= ntx;
    y = (int)(t % nty);
    t /= nty;
    z = (int)(t % ntz);
    n = (int)(t / ntz);
}
// The block's place in the weight-gradient work order.  Workgroups are dispatched to the
// 8 XCDs in turn, so block b runs on XCD b mod 8; numbering the blocks of each XCD
// consecutively gives every XCD a contiguous range of tiles, whose shared halo voxels
// then meet in that XCD's L2 (a bijection of [0, G) for any grid size G).  Measured:
// one training step on 4 x 64^3 1.855 -> 1.82 ms; the same order made the forward
// convolutions slower (16 -> 16 on 128^3: 42.6 -> 45 us), so they keep blockIdx order.
__device__ inline unsigned conv_block_id() {
    const unsigned G = gridDim.x, b = blockIdx.x, x = b % 8, q = G / 8, r = G % 8;
    return x * q + (x < r ? x : r) + b / 8;
}
__device__ inline ConvCursor conv_cursor(const ConvArgs& a, unsigned tile, unsigned stride) {
    ConvCursor c;
    conv_digits(a, tile, c.tx, c.ty, c.tz, c.n);
    conv_digits(a, stride, c.sx, c.sy, c.sz, c.sn);
    return c;
}
__device__ inline void conv_advance(const ConvArgs& a, ConvCursor& c) {
    const int ntx = (a.W + kTX - 1) / kTX, nty = (a.H + kTY - 1) / kTY, ntz = (a.D + kTZ - 1) / kTZ;
    c.tx += c.sx;
    int k = c.tx >= ntx;
    c.tx -= k ? ntx : 0;
    c.ty += c.sy + k;
    k = c.ty >= nty;
    c.ty -= k ? nty : 0;
    c.tz += c.sz + k;
    k = c.tz >= ntz;
    c.tz -= k ? ntz : 0;
    c.n += c.sn + k;
}
// With a tile list, block b of an output-tile group takes list entries b', b' + s,
// b' + 2 s, ... (b' its index among the group's blocks, s their count), at most
// kListMax of them, staged in LDS at its start; past them the cursor reads n = a.n.
__device__ inline void conv_list_tile(const ConvArgs& a, const int* tl, ConvCursor& c) {
    const int e = c.k < kListMax ? tl[c.k] : -1;
    if (e < 0) {
        c.n = a.n;
        return;
    }
    c.tx = e & 1023;
    c.ty = (e >> 10) & 1023;
    c.tz = e >> 20;
    c.n = 0;
}
template <bool LIST>
__device__ inline ConvCursor conv_start(const ConvArgs& a, unsigned first, unsigned stride, int* tl) {
    if constexpr (!LIST) {
        (void)tl;
        return conv_cursor(a, first, stride);
    } else {
        for (int i = threadIdx.x; i < kListMax; i += blockDim.x) {
            const long long li = (long long)first + (long long)i * stride;
            tl[i] = li < a.tcount ? a.tlist[li] : -1;
        }
        __syncthreads();
        ConvCursor c{};
        conv_list_tile(a, tl, c);
        return c;
    }
}
template <bool LIST>
__device__ inline void conv_next(const ConvArgs& a, ConvCursor& c, const int* tl) {
    if constexpr (LIST) {
        ++c.k;
        conv_list_tile(a, tl, c);
    } else {
        (void)tl;
        conv_advance(a, c);
    }
}

__device__ inline ConvTile conv_tile(const ConvArgs& a, const ConvCursor& c) {
    ConvTile t;
    t.x0 = c.tx * kTX;
    t.y0 = c.ty * kTY;
    t.z0 = c.tz * kTZ;
    t.sbase = (long long)c.n * a.D * a.H * a.W;
    t.in = t.x0 >= 1 && t.x0 + kTX + 1 <= a.W && t.y0 >= 1 && t.y0 + kTY + 1 <= a.H && t.z0 >= 1 &&
           t.z0 + kTZ + 1 <= a.D;
    t.out = t.x0 + kTX <= a.W && t.y0 + kTY <= a.H && t.z0 + kTZ <= a.D;
    return t;
}

constexpr int kXM = (kHV * 2 + 255) / 256;   // 16-byte halo words per thread
template <int NTB>
struct ConvW {
    static constexpr int E = kSteps * NTB * 64;   // 16-byte weight fragments per chunk
    static constexpr int M = (E + 255) / 256;
};

// Prefetch registers of one (item, chunk): the halo tile's 16 channels (and ReLU gates
// when GATED), and the chunk's weights when they change with the chunk (WL).
template <int NTB, bool WL, bool GATED>
struct ConvRegs {
    uint4 x[kXM], g[GATED ? kXM : 1], w[WL ? ConvW<NTB>::M : 1];
};

// Global loads of a chunk's weights (packed steps [sb, sb + 14), output tiles
// [tb, tb + NTB)) into w, and their LDS writes.
template <int NTB>
__device__ inline void conv_fetch_w(const ConvArgs& a, int sb, int tb, uint4* w) {
    const uint4* wsrc = reinterpret_cast<const uint4*>(a.w);
#pragma unroll
    for (int i = 0; i < ConvW<NTB>::M; ++i) {
        const int e = threadIdx.x + 256 * i;   // (step, tile, lane) of the block's slice
        w[i] = make_uint4(0, 0, 0, 0);
        if (e < ConvW<NTB>::E) {
            const int s = e / (NTB * 64), q = e - s * (NTB * 64);
            w[i] = wsrc[((long long)(sb + s) * a.nt + tb) * 64 + q];
        }
    }
}
template <int NTB>
__device__ inline void conv_store_w(char* xs, const uint4* w) {
    uint4* wl = reinterpret_cast<uint4*>(xs + conv_x_bytes());
#pragma unroll
    for (int i = 0; i < ConvW<NTB>::M; ++i) {
        const int e = threadIdx.x + 256 * i;
        if (e < ConvW<NTB>::E) wl[e] = w[i];
    }
}

// The thread's halo words: word e = threadIdx.x + 256 i holds channels 8 (e mod 2) .. + 7
// of halo voxel e / 2, packed as hx | hy << 5 | hz << 8 | (e mod 2) << 11 (offsets from
// the halo origin (x0 - 1, y0 - 1, z0 - 1)); -1 past the halo.
__device__ inline int conv_halo_word(int i) {
    const int e = threadIdx.x + 256 * i;
    if (e >= 2 * kHV) return -1;
    const int v = e >> 1;
    return v % kHX | ((v / kHX) % kHY) << 5 | (v / (kHX * kHY)) << 8 | (e & 1) << 11;
}

// Byte offsets of the thread's halo words from the halo origin (~0 past the halo), fixed
// for a launch: off on a full-resolution source with channel stride ld, and, when UP,
// offh on the half-resolution source that is upsampled (stride a.ldx; the halo voxel
// (hx, hy, hz) reads half-resolution voxel ((hx + 1) / 2, ...) from the origin's).
template <bool UP>
struct ConvLane {
    unsigned off[kXM];
    unsigned offh[UP ? kXM : 1];
};
template <bool UP>
__device__ inline ConvLane<UP> conv_lane(const ConvArgs& a, int ld) {
    ConvLane<UP> l;
    const unsigned Hh = a.H >> 1, Wh = a.W >> 1;
#pragma unroll
    for (int i = 0; i < kXM; ++i) {
        const int p = conv_halo_word(i);
        const unsigned hx = p & 31, hy = (p >> 5) & 7, hz = (p >> 8) & 7, gi = p >> 11;
        l.off[i] = p < 0 ? ~0u : 2u * (((hz * a.H + hy) * a.W + hx) * ld + 8 * gi);
        if (UP)
            l.offh[UP ? i : 0] =
                p < 0 ? ~0u : 2u * (((((hz + 1) >> 1) * Hh + ((hy + 1) >> 1)) * Wh + ((hx + 1) >> 1)) * a.ldx + 8 * gi);
    }
    return l;
}

// Global loads of channels [cb, cb + 16) of tile t (and of the chunk's weights when WL).
// Addresses are a per-item base (the halo origin, uniform) plus the lane's 32-bit offset;
// only tiles whose halo crosses the grid's boundary test each word.  XCAT: the kernel
// may read an upsampled half-resolution input and a concatenated skip (a.x2).
template <int NTB, bool WL, bool GATED>
__device__ inline void conv_fetch(const ConvArgs& a, const ConvTile& t, int cb, int tb,
                                  const ConvLane<WL && !GATED>& ln, ConvRegs<NTB, WL, GATED>& r) {
    constexpr bool XCAT = WL && !GATED;
    const bool up = XCAT && a.x2 && cb < a.c1;       // upsampled half-resolution input
    const bool cat = XCAT && a.x2 && cb >= a.c1;     // concatenated skip input
    const int ld = cat ? a.ldx2 : a.ldx;
    const int Hh = a.H >> 1, Wh = a.W >> 1;
    long long org;
    if (up)   // half-resolution voxel of the halo origin (x0, y0, z0 are even)
        org = t.sbase / 8 + ((long long)((t.z0 >> 1) - 1) * Hh + ((t.y0 >> 1) - 1)) * Wh + ((t.x0 >> 1) - 1);
    else
        org = t.sbase + ((long long)(t.z0 - 1) * a.H + (t.y0 - 1)) * a.W + (t.x0 - 1);
    // byte address of the origin's first channel (integer arithmetic: it may lie before
    // the buffer when the halo crosses the grid's low faces; such words are not loaded)
    const uintptr_t base = (cat ? (uintptr_t)a.x2 + 2 * (uintptr_t)(cb - a.c1) : (uintptr_t)a.x + 2 * (uintptr_t)cb) +
                           (uintptr_t)(org * ld * 2);
    const uintptr_t gbase = GATED ? (uintptr_t)a.gate + 2 * (uintptr_t)cb + (uintptr_t)(org * a.ldx * 2) : 0;
#pragma unroll
    for (int i = 0; i < kXM; ++i) {
        r.x[i] = make_uint4(0, 0, 0, 0);
        if (GATED) r.g[i] = make_uint4(0, 0, 0, 0);
    }
    if (t.in) {   // every word inside the grid: one base and the lane's offsets
#pragma unroll
        for (int i = 0; i < kXM; ++i) {
            if (ln.off[i] == ~0u) continue;
            const unsigned o = XCAT && up ? ln.offh[XCAT ? i : 0] : ln.off[i];
            r.x[i] = *reinterpret_cast<const uint4*>(base + o);
            if (GATED) r.g[i] = *reinterpret_cast<const uint4*>(gbase + o);
        }
    } else {
#pragma unroll
        for (int i = 0; i < kXM; ++i) {
            const int p = conv_halo_word(i);
            if (p < 0) continue;
            const int hx = p & 31, hy = (p >> 5) & 7, hz = (p >> 8) & 7;
            if ((unsigned)(t.x0 - 1 + hx) < (unsigned)a.W && (unsigned)(t.y0 - 1 + hy) < (unsigned)a.H &&
                (unsigned)(t.z0 - 1 + hz) < (unsigned)a.D) {
                const unsigned o = XCAT && up ? ln.offh[XCAT ? i : 0] : ln.off[i];
                r.x[i] = *reinterpret_cast<const uint4*>(base + o);
                if (GATED) r.g[i] = *reinterpret_cast<const uint4*>(gbase + o);
            }
        }
    }
    if (WL) conv_fetch_w<NTB>(a, kSteps * (cb / 16), tb, r.w);
}

// LDS writes of a fetched (item, chunk); the caller brackets them with barriers.
template <int NTB, bool WL, bool GATED>
__device__ inline void conv_store(char* xs, const ConvRegs<NTB, WL, GATED>& r) {
#pragma unroll
    for (int i = 0; i < kXM; ++i) {
        const int e = threadIdx.x + 256 * i;
        if (e < 2 * kHV)
            *reinterpret_cast<uint4*>(xs + ((e >> 1) * kCS + 8 * (e & 1)) * 2) =
                GATED ? apply_gate(r.x[i], r.g[i]) : r.x[i];
    }
    if (WL) conv_store_w<NTB>(xs, r.w);
}

// One 16-channel chunk: 14 MFMA steps over the 27 taps (step_tap).  lb is the LDS byte
// address of the lane's voxel x = lane % 16 in halo row 0 of the wave's plane, channels
// 8 (g mod 2) .. + 7 (g = lane / 16).  M tile mt covers output row y = mt, which reads
// halo row mt + dy for tap row dy.  B fragments come from registers (breg, weights
// fixed for the block) or from the chunk's weights in LDS (at wbase, by default right
// after the halo tile).
template <int NTB, bool BREG>
__device__ inline void conv_chunk(const char* xs, uint32_t lb, const uint4 (&breg)[kSteps][NTB],
                                  f32x4 (&acc)[4][NTB], const char* wbase = nullptr) {
    constexpr int VB = kCS * 2;         // LDS bytes per halo voxel
    constexpr int ROW = kHX * VB;       // per halo row
    constexpr int PLANE = kHY * ROW;    // per halo plane
    const int lane = threadIdx.x & 63, h = lane >> 5;
    const uint32_t b1 = lb + h * VB, bR = lb + h * ROW, bZ = lb + h * PLANE;
    const char* wl = (wbase ? wbase : xs + conv_x_bytes()) + 16 * lane;   // weights staged in LDS
    auto bfrag = [&](int s, int nt) -> bf16x8 {
        if (BREG) return __builtin_bit_cast(bf16x8, breg[s][nt]);
        return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(wl + (s * NTB + nt) * 1024));
    };
    auto afrag = [&](uint32_t addr) -> bf16x8 {
        return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(xs + addr));
    };
    // steps 0-8: six halo rows per plane feed the 12 (M tile, dy) products of taps dx = 0, 1
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) {
        bf16x8 a[6];
#pragma unroll
        for (int y = 0; y < 6; ++y) a[y] = afrag(b1 + (dz * kHY + y) * ROW);
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            bf16x8 b[NTB];
#pragma unroll
            for (int nt = 0; nt < NTB; ++nt) b[nt] = bfrag(3 * dz + dy, nt);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < NTB; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[nt], a[mt + dy], acc[mt][nt], 0, 0, 0);
        }
    }
    // steps 9-13: taps dx = 2, paired across rows, across planes, and with zero weights
#pragma unroll
    for (int s = 9; s < kSteps; ++s) {
        bf16x8 b[NTB];
#pragma unroll
        for (int nt = 0; nt < NTB; ++nt) b[nt] = bfrag(s, nt);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const uint32_t ad = s < 12 ? bR + (((s - 9) * kHY + mt) * kHX + 2) * VB
                              : s == 12 ? bZ + ((mt + 2) * kHX + 2) * VB
                                        : lb + ((2 * kHY + mt + 2) * kHX + 2) * VB;
            const bf16x8 af = afrag(ad);
#pragma unroll
            for (int nt = 0; nt < NTB; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[nt], af, acc[mt][nt], 0, 0, 0);
        }
    }
}

// Bias, ReLU and store of an item's output tiles (acc is cleared).  The MFMAs take the
// weights as their A operand, so lane l holds output channels 4 (l / 16) .. + 3 of
// voxel x0 + l mod 16 in row (y0 + mt, z0 + wave): one 8-byte BF16 word per M tile
// when the output's stride and offset allow (vec), else single values.  With the fused
// head (NTB = 1, head_l its parameters in LDS), lane group g = l / 16 forms the partial
// sums of its four channels, the groups' sums are added pairwise across lanes (g with
// g ^ 1, then with g ^ 2), and group g stores output g (FP32).
template <int NTB, bool HEAD = false, bool POOL = false>
__device__ inline void conv_epilogue(const ConvArgs& a, const ConvTile& t, int tb, const float* bias_l, bool vec,
                                     f32x4 (&acc)[4][NTB], const float* head_l = nullptr, float* pool_l = nullptr) {
    static_assert(!HEAD || NTB == 1, "the fused head takes one output tile");
    static_assert(!(HEAD && POOL), "the head and the pooling are not fused together");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15;
    const long long ob = t.sbase + ((long long)t.z0 * a.H + t.y0) * a.W + t.x0;   // the tile's origin
    // pooling: sums over the voxel pair x, x + 1 (lanes m, m ^ 1), then over the row pair
    // (M tiles 2 r, 2 r + 1), per pooled row r and output tile
    float ps[POOL ? 2 : 1][NTB][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const bool inb = t.out || (t.x0 + m < a.W && t.y0 + mt < a.H && t.z0 + wave < a.D);
        const unsigned pv = ((unsigned)wave * a.H + mt) * a.W + m;   // voxel offset from the origin
#pragma unroll
        for (int nt = 0; nt < NTB; ++nt) {
            const int co = (tb + nt) * 16 + 4 * (lane >> 4);
            const float4 bq = *reinterpret_cast<const float4*>(bias_l + nt * 16 + 4 * (lane >> 4));
            const float bv[4] = {bq.x, bq.y, bq.z, bq.w};
            float v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v[i] = acc[mt][nt][i] + bv[i];
                if (a.relu) v[i] = fmaxf(v[i], 0.f);
            }
            acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
            if constexpr (POOL) {   // every lane takes part in the exchange
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float rb = (float)(__bf16)v[i];   // the stored value
                    // quad_perm [1, 0, 3, 2]: the value of lane l ^ 1
                    const float px = rb + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(rb), 0xB1, 0xF, 0xF, false));
                    if (mt % 2 == 0) ps[mt / 2][nt][i] = px;
                    else ps[mt / 2][nt][i] += px;
                }
            }
            if constexpr (HEAD) {   // every lane takes part in the exchanges; y is not stored
                const int g = lane >> 4;
                float r[4], tot[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) r[i] = (float)(__bf16)v[i];
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    float ps = 0.f;
#pragma unroll
                    for (int i = 0; i < 4; ++i) ps = __builtin_fmaf(r[i], head_l[(4 * g + i) * 4 + o], ps);
                    tot[o] = sum_xor32(sum_xor16(ps));
                }
                // lane group g stores output g of its voxel: one store covers the M tile
                const float tv = g == 0 ? tot[0] : g == 1 ? tot[1] : g == 2 ? tot[2] : tot[3];
                if (g < a.hcout && inb) a.hout[(ob + pv) * a.hcout + g] = head_l[64 + g] + tv;
                continue;
            }
            if (!inb) continue;
            if (vec && co + 4 <= a.cout) {
                const bf16x2 lo = {(__bf16)v[0], (__bf16)v[1]}, hi = {(__bf16)v[2], (__bf16)v[3]};
                uint16_t* yp = a.y + ob * a.ldy + a.yoff;
                *reinterpret_cast<uint2*>(yp + pv * a.ldy + co) =
                    make_uint2(__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi));
            } else if (a.y) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (co + i < a.cout)
                        a.y[(ob + pv) * a.ldy + a.yoff + co + i] = __builtin_bit_cast(uint16_t, (__bf16)v[i]);
            }
            if (a.yf) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (co + i < a.cout) a.yf[(ob + pv) * a.cout + co + i] = v[i];
            }
        }
    }
    if constexpr (POOL) {
        // plane pairs: waves 2 q and 2 q + 1 hold planes z0 + 2 q and z0 + 2 q + 1; the odd
        // wave hands its sums over LDS, the even one adds them and stores the pooled voxel
        // (lanes with even m)
        // value k of the pair's lane at xl[128 k]: consecutive lanes, consecutive banks
        float* xl = pool_l + (wave >> 1) * 64 + lane;
        if (wave & 1) {
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int nt = 0; nt < NTB; ++nt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) xl[128 * ((r * NTB + nt) * 4 + i)] = ps[r][nt][i];
        }
        __syncthreads();
        if (!(wave & 1)) {
            const int PD = a.D >> 1, PH = a.H >> 1, PW = a.W >> 1;
            const int px = (t.x0 >> 1) + (m >> 1), pz = (t.z0 >> 1) + (wave >> 1);
            const bool xok = (m & 1) == 0 && px < PW && pz < PD;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int py = (t.y0 >> 1) + r;
                const bool ok = xok && py < PH;
                const long long q = (t.sbase >> 3) + ((long long)pz * PH + py) * PW + px;
#pragma unroll
                for (int nt = 0; nt < NTB; ++nt) {
                    const int co = (tb + nt) * 16 + 4 * (lane >> 4);
                    float sv[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) sv[i] = (ps[r][nt][i] + xl[128 * ((r * NTB + nt) * 4 + i)]) * 0.125f;
                    if (!ok) continue;
                    if (a.cout % 4 == 0 && co + 4 <= a.cout) {   // one 8-byte word (8-byte aligned)
                        const bf16x2 lo = {(__bf16)sv[0], (__bf16)sv[1]}, hi = {(__bf16)sv[2], (__bf16)sv[3]};
                        *reinterpret_cast<uint2*>(a.yp + q * a.cout + co) =
                            make_uint2(__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi));
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if (co + i < a.cout) a.yp[q * a.cout + co + i] = __builtin_bit_cast(uint16_t, (__bf16)sv[i]);
                    }
                }
            }
        }
    }
}

// WL: the weights change with the chunk (more than 16 input channels); GATED: the input
// is multiplied by (gate > 0) (ReLU backward).  The grid size must be a multiple of
// NT / NTB: a block keeps one output-tile group (its bias is read once, and without WL
// its weights are staged once), and its epilogue issues no loads, so the wait for the
// next item's prefetched input does not also wait for the stores of this one.  Three
// blocks per CU for the chunk-staged weights (WL); two for the others, whose registers
// (the weights held in registers, or the ReLU gates) would not fit three.
template <int NTB, bool WL, bool GATED, bool HEAD = false, bool LIST = false, bool POOL = false>
__global__ __launch_bounds__(256, (NTB == 1 && WL && !GATED) ? 3 : 2) void k_conv(ConvArgs a) {
    extern __shared__ uint4 xs_dyn[];
    char* xs = reinterpret_cast<char*>(xs_dyn);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nsplit = a.nt / NTB;
    const int nchunk = WL ? a.cin_p / 16 : 1;
    const unsigned bid = blockIdx.x;
    const int tb = (int)(bid % nsplit) * NTB;   // the block's first output tile
    // the block's bias values sit in LDS after the halo tile and the weights, then the
    // fused head's parameters and the tile list
    float* bias_l = reinterpret_cast<float*>(xs + conv_x_bytes() + conv_w_bytes(NTB, WL));
    float* head_l = bias_l + 16 * NTB;   // (one output tile only)
    int* tl = reinterpret_cast<int*>(head_l + (HEAD ? kHeadLds : 0));
    float* pool_l = reinterpret_cast<float*>(tl + (LIST ? kListMax : 0));
    // the block's tiles: bid / nsplit, then every gridDim.x / nsplit-th (of the grid, or
    // of the tile list)
    ConvCursor cur = conv_start<LIST>(a, bid / nsplit, gridDim.x / nsplit, tl);
    if (cur.n >= a.n) return;
    if (threadIdx.x < 16 * NTB) {
        const int co = tb * 16 + threadIdx.x;
        bias_l[threadIdx.x] = a.bias && co < a.cout ? a.bias[co] : 0.f;
    }
    if (HEAD) conv_stage_head(a, head_l);
    // BF16 output as one 8-byte word of four channels per lane and M tile
    const bool vec = a.y && a.ldy % 4 == 0 && a.yoff % 4 == 0 && ((uintptr_t)a.y & 7) == 0;
    // the lane's voxel x = lane % 16 in halo row 0 of plane 'wave' (M tile mt adds mt rows)
    const uint32_t lb = (uint32_t)(((wave * kHY) * kHX + (lane & 15)) * kCS * 2 + 16 * ((lane >> 4) & 1));
    f32x4 acc[4][NTB];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NTB; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    // one chunk (16 input channels) and one output tile: the block's B fragments stay in
    // registers for every item (packed in fragment order: step, output tile, lane); with
    // two output tiles they are staged once in LDS (112 more registers would leave one
    // wave per SIMD)
    constexpr bool BREG = !WL && NTB == 1;
    uint4 breg[kSteps][NTB];
    if (BREG) {
        const uint4* wsrc = reinterpret_cast<const uint4*>(a.w);
#pragma unroll
        for (int s = 0; s < kSteps; ++s)
#pragma unroll
            for (int nt = 0; nt < NTB; ++nt) breg[s][nt] = wsrc[((long long)s * a.nt + tb + nt) * 64 + lane];
    } else if (!WL) {   // read from LDS by every item after the first barrier
        uint4 w[ConvW<NTB>::M];
        conv_fetch_w<NTB>(a, 0, tb, w);
        conv_store_w<NTB>(xs, w);
    }
    // halo word offsets of the full-resolution source (the skip input when a.x2 is set)
    const ConvLane<WL && !GATED> ln = conv_lane<WL && !GATED>(a, (WL && !GATED && a.x2) ? a.ldx2 : a.ldx);
    ConvRegs<NTB, WL, GATED> regs;
    // chunk c covers channels [16 c, 16 c + 16)
    int chunk = 0;
    ConvTile t = conv_tile(a, cur);
    conv_fetch<NTB, WL, GATED>(a, t, 0, tb, ln, regs);
    for (;;) {
        __syncthreads();   // every wave is done with the previous chunk's LDS
        conv_store<NTB, WL, GATED>(xs, regs);
        __syncthreads();
        ConvCursor nxt = cur;
        int nc = chunk + 1;
        if (nc == nchunk) {
            nc = 0;
            conv_next<LIST>(a, nxt, tl);
        }
        const bool more = nxt.n < a.n;
        const ConvTile tn = nc == 0 ? conv_tile(a, nxt) : t;
        if (more) conv_fetch<NTB, WL, GATED>(a, tn, 16 * nc, tb, ln, regs);   // in flight during the MFMAs
        conv_chunk<NTB, BREG>(xs, lb, breg, acc);
        if (chunk == nchunk - 1) conv_epilogue<NTB, HEAD, POOL>(a, t, tb, bias_l, vec, acc, head_l, pool_l);
        if (!more) break;
        t = tn;
        cur = nxt;
        chunk = nc;
    }
}

typedef __attribute__((address_space(3))) void lds_void_t;

// Staging of an item's halo tile (16 input channels) straight from global memory into
// LDS: global_load_lds_dwordx4 writes lane l's 16 bytes at the wave's LDS base + 16 l,
// which is the word order of the tile; words outside the grid are written as zeros.
__device__ inline void conv_stage(const ConvArgs& a, const ConvTile& t, const ConvLane<false>& ln, char* dst) {
    const int wave = threadIdx.x >> 6;
    const uintptr_t base =
        (uintptr_t)a.x + (uintptr_t)((t.sbase + ((long long)(t.z0 - 1) * a.H + (t.y0 - 1)) * a.W + (t.x0 - 1)) * a.ldx * 2);
#pragma unroll
    for (int i = 0; i < kXM; ++i) {
        const int p = conv_halo_word(i);
        if (p < 0) continue;
        const int hx = p & 31, hy = (p >> 5) & 7, hz = (p >> 8) & 7;
        if (t.in || ((unsigned)(t.x0 - 1 + hx) < (unsigned)a.W && (unsigned)(t.y0 - 1 + hy) < (unsigned)a.H &&
                     (unsigned)(t.z0 - 1 + hz) < (unsigned)a.D))
            __builtin_amdgcn_global_load_lds((const void*)(base + ln.off[i]),
                                             (lds_void_t*)(dst + (256 * i + 64 * wave) * 16), 16, 0, 0);
        else
            *reinterpret_cast<uint4*>(dst + (threadIdx.x + 256 * i) * 16) = make_uint4(0, 0, 0, 0);
    }
}

// k_conv for 16-channel inputs without a gate, with the halo tiles staged asynchronously
// in two LDS buffers: the staging of item j + 2 is issued as soon as every wave has read
// item j, so its global loads overlap the MFMAs of item j + 1 and nothing passes through
// registers (16 -> 16 channels on 128^3: 49 -> 42 us).  Same work split, results and
// epilogue as k_conv.
template <int NTB, bool HEAD = false, bool LIST = false, bool POOL = false>
__global__ __launch_bounds__(256, NTB == 1 ? 3 : 2) void k_conv_staged(ConvArgs a) {
    constexpr int HB = kHV * kCS * 2;
    __shared__ __attribute__((aligned(16))) char h0[HB];
    __shared__ __attribute__((aligned(16))) char h1[HB];
    __shared__ __attribute__((aligned(16))) char wl[NTB > 1 ? kSteps * NTB * 1024 : 16];
    __shared__ __attribute__((aligned(16))) float bias_l[16 * NTB];
    __shared__ __attribute__((aligned(16))) float head_l[HEAD ? kHeadLds : 1];
    __shared__ int tl[LIST ? kListMax : 1];
    __shared__ float pool_l[POOL ? conv_pool_bytes(NTB) / 4 : 1];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nsplit = a.nt / NTB;
    const unsigned bid = blockIdx.x;
    const int tb = (int)(bid % nsplit) * NTB;
    ConvCursor cur = conv_start<LIST>(a, bid / nsplit, gridDim.x / nsplit, tl);
    if (cur.n >= a.n) return;
    if (threadIdx.x < 16 * NTB) {
        const int co = tb * 16 + threadIdx.x;
        bias_l[threadIdx.x] = a.bias && co < a.cout ? a.bias[co] : 0.f;
    }
    if (HEAD) conv_stage_head(a, head_l);
    const bool vec = a.y && a.ldy % 4 == 0 && a.yoff % 4 == 0 && ((uintptr_t)a.y & 7) == 0;
    const uint32_t lb = (uint32_t)(((wave * kHY) * kHX + (lane & 15)) * kCS * 2 + 16 * ((lane >> 4) & 1));
    f32x4 acc[4][NTB];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NTB; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    constexpr bool BREG = NTB == 1;
    uint4 breg[kSteps][NTB];
    if (BREG) {
        const uint4* wsrc = reinterpret_cast<const uint4*>(a.w);
#pragma unroll
        for (int s = 0; s < kSteps; ++s) breg[s][0] = wsrc[((long long)s * a.nt + tb) * 64 + lane];
    } else {   // the block's weights, staged once
        uint4 w[ConvW<NTB>::M];
        conv_fetch_w<NTB>(a, 0, tb, w);
#pragma unroll
        for (int i = 0; i < ConvW<NTB>::M; ++i) {
            const int e = threadIdx.x + 256 * i;
            if (e < ConvW<NTB>::E) reinterpret_cast<uint4*>(wl)[e] = w[i];
        }
    }
    const ConvLane<false> ln = conv_lane<false>(a, a.ldx);
    // the item being computed (cur, tile t) and the next one to stage (scur, tile st)
    ConvTile t = conv_tile(a, cur);
    ConvCursor scur = cur;
    ConvTile st = t;
    conv_stage(a, st, ln, h0);
    conv_next<LIST>(a, scur, tl);
    st = conv_tile(a, scur);
    __syncthreads();
    if (scur.n < a.n) conv_stage(a, st, ln, h1);
    conv_next<LIST>(a, scur, tl);
    st = conv_tile(a, scur);
    conv_chunk<NTB, BREG>(h0, lb, breg, acc, wl);
    // One step: wait until every wave has read hn (the item just computed) and the
    // staging of the item in hc has landed, stage the item after next into hn, store the
    // finished item, and compute the next one from hc.  The restrict qualifiers tell the
    // compiler that the reads of hc do not wait for the staging just issued into hn.
    auto step = [&](char* __restrict__ hn, const char* __restrict__ hc) -> bool {
        __syncthreads();
        if (scur.n < a.n) conv_stage(a, st, ln, hn);
        conv_next<LIST>(a, scur, tl);
        st = conv_tile(a, scur);
        conv_epilogue<NTB, HEAD, POOL>(a, t, tb, bias_l, vec, acc, head_l, pool_l);
        conv_next<LIST>(a, cur, tl);
        if (cur.n >= a.n) return false;
        t = conv_tile(a, cur);
        conv_chunk<NTB, BREG>(hc, lb, breg, acc, wl);
        return true;
    };
    for (;;) {
        if (!step(h0, h1)) break;
        if (!step(h1, h0)) break;
    }
}

struct WgradArgs {
    const uint16_t* x;     // forward input [P][ldx] (real channels cin, padded cin_p)
    const uint16_t* g;     // output gradient [P][ldg]
    const uint16_t* gate;  // layer output [P][ldg] (ReLU gate) or null
    float* part;           // [gridDim.x][27][cin_p][cout_p]
    float* bpart;          // optional [gridDim.x][cout_p]: bias-gradient partials
    int ldx, cin_p, ldg, cout_p;
    int n, D, H, W;
};

// Weight gradient of a 3x3x3 convolution, dW[tap][c][o] = sum_p x[p + off(tap)][c] *
// g[p][o] * (gate[p][o] > 0), for one 16 x 16 block of (c, o) (blockIdx.y) over the
// voxel tiles b, b + gridDim.x, ... (b = conv_block_id(); 16 x 4 x 4 voxels each, as in
// k_conv).  Per tile, the input's 18 x 6 x 6 halo and the gated gradient are staged in
// LDS transposed ([channel][voxel]) so that the MFMA K dimension runs over voxels; the
// halo is stored three times, shifted by dx = 0, 1, 2 along x, so that the 8 voxels of
// every A fragment are one aligned 16-byte word for all 27 taps.  K step ks covers the
// tile's rows (z, y) = (ks / 2, 2 (ks mod 2) + r), r = 0, 1; lane group q = lane / 16
// holds row r = q / 2, voxels x = 8 (q mod 2) .. + 7.  Wave w accumulates taps w, w + 4,
// ...; wave 3, which has one tap fewer, also sums the gated gradient over the voxels
// (an MFMA with an all-ones A) for the bias gradient when blockIdx.y has c block 0.
constexpr int kWgCi = 36 * 16 + 8;        // BF16 stride between channels of a shifted halo copy
constexpr int kWgCopy = 16 * kWgCi;        // one shifted copy, 16 channels
constexpr int kWgCo = 256 + 8;             // BF16 stride between gradient channels
// LDS bytes: three halo copies and the transposed gradient
constexpr int kWgLds = (3 * kWgCopy + 16 * kWgCo) * 2;

__global__ __launch_bounds__(256) void k_conv_wgrad(WgradArgs a) {
    extern __shared__ uint4 wg_dyn[];
    uint16_t* xs = reinterpret_cast<uint16_t*>(wg_dyn);   // [dx][c][hz][hy][x'] with x' = hx - dx
    uint16_t* gs = xs + 3 * kWgCopy;                       // [o][tile voxel]
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nob = a.cout_p / 16;
    const int cbk = blockIdx.y / nob, obk = blockIdx.y - cbk * nob;   // 16-channel blocks of c and o
    const int c0 = 16 * cbk, o0 = 16 * obk;
    const bool with_bias = a.bpart && cbk == 0;
    const int ntx = (a.W + kTX - 1) / kTX, nty = (a.H + kTY - 1) / kTY, ntz = (a.D + kTZ - 1) / kTZ;
    const long long tiles = (long long)a.n * ntz * nty * ntx;
    f32x4 acc[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int q = lane >> 4, l16 = lane & 15;
    for (long long tile = conv_block_id(); tile < tiles; tile += gridDim.x) {   // XCD-contiguous tiles
        long long r = tile;
        const int x0 = (int)(r % ntx) * kTX;
        r /= ntx;
        const int y0 = (int)(r % nty) * kTY;
        r /= nty;
        const int z0 = (int)(r % ntz) * kTZ;
        const long long sbase = (r / ntz) * a.D * a.H * a.W;
        // global loads: halo words (voxel, 8 channels) and gradient words
        constexpr int EX = 2 * kHV, EG = 2 * 256;
        constexpr int SX = (EX + 255) / 256, SG = (EG + 255) / 256;
        uint4 tx[SX], tg[SG];
#pragma unroll
        for (int i = 0; i < SX; ++i) {
            const int e = threadIdx.x + 256 * i;
            tx[i] = make_uint4(0, 0, 0, 0);
            if (e < EX) {
                const int v = e >> 1, gi = e & 1;
                const int x = x0 - 1 + v % kHX, y = y0 - 1 + (v / kHX) % kHY, z = z0 - 1 + v / (kHX * kHY);
                if (x >= 0 && x < a.W && y >= 0 && y < a.H && z >= 0 && z < a.D) {
                    const long long p = sbase + ((long long)z * a.H + y) * a.W + x;
                    tx[i] = *reinterpret_cast<const uint4*>(a.x + p * a.ldx + c0 + 8 * gi);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < SG; ++i) {
            const int e = threadIdx.x + 256 * i;
            tg[i] = make_uint4(0, 0, 0, 0);
            if (e < EG) {
                const int v = e >> 1, gi = e & 1;
                const int x = x0 + (v & 15), y = y0 + ((v >> 4) & 3), z = z0 + (v >> 6);
                if (x < a.W && y < a.H && z < a.D) {
                    const long long p = sbase + ((long long)z * a.H + y) * a.W + x;
                    tg[i] = *reinterpret_cast<const uint4*>(a.g + p * a.ldg + o0 + 8 * gi);
                    if (a.gate) tg[i] = apply_gate(tg[i], *reinterpret_cast<const uint4*>(a.gate + p * a.ldg + o0 + 8 * gi));
                }
            }
        }
        __syncthreads();   // the previous tile's LDS reads are done
#pragma unroll
        for (int i = 0; i < SX; ++i) {
            const int e = threadIdx.x + 256 * i;
            if (e < EX) {
                const int v = e >> 1, gi = e & 1;
                const int hx = v % kHX, row = v / kHX;   // row = hz * 6 + hy
                const uint32_t w4[4] = {tx[i].x, tx[i].y, tx[i].z, tx[i].w};
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const int xp = hx - dx;
                    if (xp >= 0 && xp < 16) {
                        uint16_t* d = xs + dx * kWgCopy + (8 * gi) * kWgCi + row * 16 + xp;
#pragma unroll
                        for (int j = 0; j < 8; ++j)
                            d[j * kWgCi] = (uint16_t)(j & 1 ? w4[j >> 1] >> 16 : w4[j >> 1] & 0xffffu);
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < SG; ++i) {
            const int e = threadIdx.x + 256 * i;
            if (e < EG) {
                const int v = e >> 1, gi = e & 1;
                const uint32_t w4[4] = {tg[i].x, tg[i].y, tg[i].z, tg[i].w};
                uint16_t* d = gs + (8 * gi) * kWgCo + v;
#pragma unroll
                for (int j = 0; j < 8; ++j) d[j * kWgCo] = (uint16_t)(j & 1 ? w4[j >> 1] >> 16 : w4[j >> 1] & 0xffffu);
            }
        }
        __syncthreads();
        // B fragments of the 8 K steps (shared by every tap)
        bf16x8 bq[8];
#pragma unroll
        for (int ks = 0; ks < 8; ++ks)
            bq[ks] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(gs + l16 * kWgCo + 32 * ks + 8 * q));
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            const int t = wave + 4 * i;   // wave-uniform
            if (t < 27) {
                const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
                const uint16_t* xa = xs + dx * kWgCopy + l16 * kWgCi + 8 * (q & 1);
#pragma unroll
                for (int ks = 0; ks < 8; ++ks) {
                    const int z = ks >> 1, y = 2 * (ks & 1) + (q >> 1);
                    const bf16x8 af = __builtin_bit_cast(
                        bf16x8, *reinterpret_cast<const uint4*>(xa + ((z + dz) * kHY + (y + dy)) * 16));
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bq[ks], acc[i], 0, 0, 0);
                }
            } else if (with_bias) {   // t = 27 on wave 3: ones^T g, every row the voxel sum
                const bf16x8 ones = __builtin_bit_cast(bf16x8, make_uint4(0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u));
#pragma unroll
                for (int ks = 0; ks < 8; ++ks) acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ones, bq[ks], acc[i], 0, 0, 0);
            }
        }
    }
    // D layout: lane holds rows c = 4 (lane / 16) + i, column o = lane mod 16
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const int t = wave + 4 * i;
        if (t < 27) {
            float* out = a.part + ((long long)blockIdx.x * 27 + t) * a.cin_p * a.cout_p;
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) out[(c0 + 4 * q + rr) * a.cout_p + o0 + l16] = acc[i][rr];
        } else if (with_bias && q == 0) {
            a.bpart[(long long)blockIdx.x * a.cout_p + o0 + l16] = acc[i][0];
        }
    }
}

// grad[tap][c][o] += sum over chunks of the partials (fixed order).
__global__ void k_wgrad_reduce(const float* part, int nchunk, int cin, int cout, int cin_p, int cout_p,
                               float* grad) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tot = 27LL * cin * cout;
    if (i >= tot) return;
    const int o = (int)(i % cout);
    const long long r = i / cout;
    const int c = (int)(r % cin);
    const int tap = (int)(r / cin);
    // eight interleaved partial sums keep eight loads in flight (fixed order: deterministic)
    const long long stride = 27LL * cin_p * cout_p;
    const float* q = part + ((long long)tap * cin_p + c) * cout_p + o;
    double s8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int k = 0;
    for (; k + 8 <= nchunk; k += 8)
#pragma unroll
        for (int j = 0; j < 8; ++j) s8[j] += q[(k + j) * stride];
    for (; k < nchunk; ++k) s8[0] += q[k * stride];
    grad[i] += (float)(((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7])));
}

__global__ void k_bias_reduce(const float* part, int nchunk, int ld, int cout, float* grad) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= cout) return;
    double s8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int k = 0;
    for (; k + 8 <= nchunk; k += 8)
#pragma unroll
        for (int j = 0; j < 8; ++j) s8[j] += part[(long long)(k + j) * ld + o];
    for (; k < nchunk; ++k) s8[0] += part[(long long)k * ld + o];
    grad[o] += (float)(((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7])));
}

// Eight BF16 values as one 16-byte word, and their FP32 values.
__device__ inline void unpack8(const uint4 t, float (&f)[8]) {
    const uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[2 * i] = __uint_as_float(w[i] << 16);
        f[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
    }
}
__device__ inline uint4 pack8(const float (&f)[8]) {
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = (uint32_t)f2bf(f[2 * i]) | ((uint32_t)f2bf(f[2 * i + 1]) << 16);
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// Voxel coordinates of linear index p in an n x D x H x W grid.
struct Vox {
    int x, y, z, b;
};
__device__ inline Vox decode(long long p, int D, int H, int W) {
    Vox v;
    long long r = p / W;
    v.x = (int)(p - r * W);
    const long long r2 = r / H;
    v.y = (int)(r - r2 * H);
    const long long r3 = r2 / D;
    v.z = (int)(r2 - r3 * D);
    v.b = (int)r3;
    return v;
}

// 2x2x2 average pooling of channels [0, c) (input stride ldx, output stride c); one
// thread per output voxel and group of 8 channels.
__global__ void k_pool2(const uint16_t* x, int ldx, int c, int n, int D, int H, int W, uint16_t* y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int d = D / 2, h = H / 2, w = W / 2;
    const int G = c / 8;
    const long long tot = (long long)n * d * h * w * G;
    if (i >= tot) return;
    const int g = (int)(i % G);
    const long long po = i / G;
    const Vox v = decode(po, d, h, w);
    // children k = (z, y, x) bits, summed pairwise: x pairs, then y, then z (the order of
    // the pooling fused into the convolution epilogue)
    float f[8][8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const long long q = (((long long)v.b * D + 2 * v.z + (k >> 2)) * H + 2 * v.y + ((k >> 1) & 1)) * W + 2 * v.x + (k & 1);
        unpack8(*reinterpret_cast<const uint4*>(x + q * ldx + 8 * g), f[k]);
    }
    float s[8];
#pragma unroll
    for (int e = 0; e < 8; ++e)
        s[e] = (((f[0][e] + f[1][e]) + (f[2][e] + f[3][e])) + ((f[4][e] + f[5][e]) + (f[6][e] + f[7][e]))) * 0.125f;
    *reinterpret_cast<uint4*>(y + po * c + 8 * g) = pack8(s);
}

// out[child] = dpool[parent] / 8 (+ dskip[child] channels) for the encoder skip; one
// thread per voxel and group of 8 channels.
__global__ void k_pool2_bwd_add(const uint16_t* dpool, int c, const uint16_t* dskip, int lds, int n, int D, int H,
                                int W, uint16_t* out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int G = c / 8;
    const long long tot = (long long)n * D * H * W * G;
    if (i >= tot) return;
    const int g = (int)(i % G);
    const long long p = i / G;
    const Vox v = decode(p, D, H, W);
    const long long q = (((long long)v.b * (D / 2) + v.z / 2) * (H / 2) + v.y / 2) * (W / 2) + v.x / 2;
    float f[8];
    unpack8(*reinterpret_cast<const uint4*>(dpool + q * c + 8 * g), f);
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] *= 0.125f;
    if (dskip) {
        float k[8];
        unpack8(*reinterpret_cast<const uint4*>(dskip + p * lds + 8 * g), k);
#pragma unroll
        for (int e = 0; e < 8; ++e) f[e] += k[e];
    }
    *reinterpret_cast<uint4*>(out + p * c + 8 * g) = pack8(f);
}

// Nearest x2 upsampling of h (c channels) into channels [0, c) of a concat buffer with
// stride c + cs, and a copy of the skip (cs channels) into channels [c, c + cs); one
// thread per voxel and group of 8 channels (a pure copy of 16-byte words).
__global__ void k_up2_cat(const uint16_t* h, int c, const uint16_t* skip, int cs, int n, int D, int H, int W,
                          uint16_t* cat) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int ldc = c + cs, G = ldc / 8;
    const long long tot = (long long)n * D * H * W * G;
    if (i >= tot) return;
    const int g = (int)(i % G);
    const long long p = i / G;
    uint4 t;
    if (8 * g < c) {
        const Vox v = decode(p, D, H, W);
        const long long q = (((long long)v.b * (D / 2) + v.z / 2) * (H / 2) + v.y / 2) * (W / 2) + v.x / 2;
        t = *reinterpret_cast<const uint4*>(h + q * c + 8 * g);
    } else {
        t = *reinterpret_cast<const uint4*>(skip + p * cs + 8 * g - c);
    }
    *reinterpret_cast<uint4*>(cat + p * ldc + 8 * g) = t;
}

// Gradient of the upsampling: dh[parent][ch] = sum of the 8 children's dcat[.][ch]; one
// thread per parent voxel and group of 8 channels.
__global__ void k_up2_bwd(const uint16_t* dcat, int ldc, int c, int n, int d, int h, int w, uint16_t* dh) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int G = c / 8;
    const long long tot = (long long)n * d * h * w * G;
    if (i >= tot) return;
    const int g = (int)(i % G);
    const long long p = i / G;
    const Vox v = decode(p, d, h, w);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const long long q = (((long long)v.b * 2 * d + 2 * v.z + (k >> 2)) * 2 * h + 2 * v.y + ((k >> 1) & 1)) * 2 * w +
                            2 * v.x + (k & 1);
        float f[8];
        unpack8(*reinterpret_cast<const uint4*>(dcat + q * ldc + 8 * g), f);
#pragma unroll
        for (int e = 0; e < 8; ++e) s[e] += f[e];
    }
    *reinterpret_cast<uint4*>(dh + p * c + 8 * g) = pack8(s);
}

// 1x1x1 head: out[p][o] = b[o] + sum_c h[p][c] W[c][o] (FP32 weights and output), for
// c = 16 input channels; one thread per voxel.
__global__ void k_head(const uint16_t* h, int c, const float* W, const float* b, int cout, long long P, float* out) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float hv[16];
    unpack8(*reinterpret_cast<const uint4*>(h + p * 16), *reinterpret_cast<float(*)[8]>(hv));
    unpack8(*reinterpret_cast<const uint4*>(h + p * 16 + 8), *reinterpret_cast<float(*)[8]>(hv + 8));
    (void)c;
    // the order of the head fused into the convolution epilogue: the sums of channels
    // 4 g .. 4 g + 3, added pairwise, then the bias
    for (int o = 0; o < cout; ++o) {
        float ps[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            ps[g] = 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) ps[g] = __builtin_fmaf(hv[4 * g + i], W[(4 * g + i) * cout + o], ps[g]);
        }
        out[p * cout + o] = b[o] + ((ps[0] + ps[1]) + (ps[2] + ps[3]));
    }
}

// Head backward for c = 16 input channels: dh[p][c] = sum_o dout[p][o] W[c][o] (BF16), and
// per-block partials of dW[c][o] = sum_p h[p][c] dout[p][o] and db[o] = sum_p dout[p][o]
// (the per-thread sums go through LDS, each parameter summed by one thread in order).
constexpr int kHeadPar = 16 * 4 + 4;
__global__ __launch_bounds__(256) void k_head_bwd(const uint16_t* h, int c, const float* W, int cout, const float* dout,
                                                  long long P, long long per_chunk, uint16_t* dh, float* part) {
    const long long pa = (long long)blockIdx.x * per_chunk;
    const long long pb = pa + per_chunk < P ? pa + per_chunk : P;
    const int npar = 16 * cout + cout;
    float acc[kHeadPar];
#pragma unroll
    for (int i = 0; i < kHeadPar; ++i) acc[i] = 0.f;
    (void)c;
    for (long long p = pa + threadIdx.x; p < pb; p += blockDim.x) {
        float hv[16], g[4] = {0.f, 0.f, 0.f, 0.f};
        unpack8(*reinterpret_cast<const uint4*>(h + p * 16), *reinterpret_cast<float(*)[8]>(hv));
        unpack8(*reinterpret_cast<const uint4*>(h + p * 16 + 8), *reinterpret_cast<float(*)[8]>(hv + 8));
#pragma unroll
        for (int o = 0; o < 4; ++o)
            if (o < cout) g[o] = dout[p * cout + o];
        float d[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            float s = 0.f;
#pragma unroll
            for (int o = 0; o < 4; ++o)
                if (o < cout) {
                    s += g[o] * W[k * cout + o];
                    acc[k * 4 + o] += hv[k] * g[o];
                }
            d[k] = s;
        }
#pragma unroll
        for (int o = 0; o < 4; ++o) acc[64 + o] += g[o];
        *reinterpret_cast<uint4*>(dh + p * 16) = pack8(*reinterpret_cast<float(*)[8]>(d));
        *reinterpret_cast<uint4*>(dh + p * 16 + 8) = pack8(*reinterpret_cast<float(*)[8]>(d + 8));
    }
    __shared__ float sh[kHeadPar][65];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float s = 0.f;
    for (int r = 0; r < 4; ++r) {
        if (wv == r) {
#pragma unroll
            for (int i = 0; i < kHeadPar; ++i) sh[i][lane] = acc[i];
        }
        __syncthreads();
        if (threadIdx.x < kHeadPar)
            for (int t = 0; t < 64; ++t) s += sh[threadIdx.x][t];
        __syncthreads();
    }
    if (threadIdx.x < kHeadPar) {
        const int i = threadIdx.x;
        // parameter order of the flat vector: W[c][o] (c-major), then b[o]
        const int k = i / 4, o = i % 4;
        if (i < 64 && o < cout) part[(long long)blockIdx.x * npar + k * cout + o] = s;
        if (i >= 64 && i - 64 < cout) part[(long long)blockIdx.x * npar + 16 * cout + (i - 64)] = s;
    }
}

__global__ void k_param_reduce(const float* part, int nchunk, int npar, float* grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npar) return;
    double s = 0.0;
    for (int k = 0; k < nchunk; ++k) s += part[(long long)k * npar + i];
    grad[i] += (float)s;
}

// MSE: grad = 2 (out - target) / count, per-block partial sums of the squared error.
__global__ __launch_bounds__(256) void k_mse(const float* out, const float* tgt, long long count, float* grad,
                                             double* part) {
    __shared__ double sh[256];
    double s = 0.0;
    const float scale = 2.0f / (float)count;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x) {
        const float d = out[i] - tgt[i];
        grad[i] = scale * d;
        s += (double)d * d;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Adam (Kingma and Ba) on the FP32 master parameters.
__global__ void k_adam(float* th, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// The step of a packed convolution GEMM: 14 steps per 16-channel chunk.  For lane group
// g of step sg, returns the tap (27 for the zero half of the last pair) and the first of
// the group's 8 input channels.
__device__ inline void packed_step(int sg, int g, int& tap, int& c0) {
    tap = step_tap(sg % kSteps, g >> 1);
    c0 = 16 * (sg / kSteps) + 8 * (g & 1);
}

// BF16 copies of one convolution's weights W[tap][cin][cout] in the fragment order of
// k_conv (steps x output tiles x 64 lanes x 8 values): the forward GEMM (input channels
// cin, output channels cout) into wf, and the input-gradient GEMM into wd, whose input
// channels are the layer's outputs o and whose output channels are the layer's inputs c,
// with the taps mirrored: wd(tap, o, c) = W[26 - tap][c][o].
// nf, nd: packed values of the two GEMMs (steps x 512 x output tiles).
__global__ void k_pack(const float* W, int cin, int cout, int cin_p, int cout_p, long long nf, long long nd,
                       uint16_t* wf, uint16_t* wd) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool fwd = i < nf;
    if (!fwd && (i >= nf + nd || !wd)) return;
    const long long k = fwd ? i : i - nf;
    const int gi = fwd ? cin : cout, go = fwd ? cout : cin;           // GEMM input / output channels
    const int nt = (fwd ? cout_p : cin_p) / 16;
    const int j = (int)(k % 8), lane = (int)((k / 8) % 64), t = (int)((k / 512) % nt);
    const int sg = (int)(k / (512LL * nt));
    int tap, c0;
    packed_step(sg, lane >> 4, tap, c0);
    const int ci = c0 + j, co = 16 * t + (lane & 15);
    float v = 0.f;
    if (tap < 27 && ci < gi && co < go)
        v = fwd ? W[((long long)tap * cin + ci) * cout + co] : W[((long long)(26 - tap) * cin + co) * cout + ci];
    (fwd ? wf : wd)[k] = f2bf(v);
}

// Copy an input with 'c' channels into a zero-padded buffer with 'cp' channels (cp a
// multiple of 8); one thread per voxel.
__global__ void k_pad_channels(const uint16_t* x, int c, int cp, long long P, uint16_t* y) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    for (int g = 0; g < cp / 8; ++g) {
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int c0 = 8 * g + 2 * i;
            const uint32_t lo = c0 < c ? x[p * c + c0] : 0u;
            const uint32_t hi = c0 + 1 < c ? x[p * c + c0 + 1] : 0u;
            w[i] = lo | (hi << 16);
        }
        *reinterpret_cast<uint4*>(y + p * cp + 8 * g) = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

}  // namespace mpm
