// Device kernels of the warm-start U-Net (BF16 storage, FP32 accumulation).
//
// Activations are NDHWC [n][z][y][x][c] in BF16.  3x3x3 convolutions are implicit
// GEMMs on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16): M = output voxels,
// N = output channels, K = 27 taps x input channels, with the tap/channel index
// k = tap * Cin_p + c (Cin_p a multiple of 8, so the 8 consecutive k of one lane
// always belong to one tap).  The input gradient is the same GEMM on the output
// gradient with the taps mirrored and the weights transposed; the weight gradient
// stages voxel chunks in LDS, transposed so that K runs over voxels.  For the input
// gradient, dX[p] = sum_t dY[p - off(t)] W[t] = sum_t dY[p + off(t)] W[26 - t], so the
// same forward kernel runs on packed weights holding W[26 - t] transposed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpm {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// round to nearest even (finite inputs)
__device__ inline uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

struct ConvArgs {
    const uint16_t* x;     // GEMM input [P][ldx] (activation, or output gradient for dgrad)
    const uint16_t* gate;  // optional [P][ldx]: use x * (gate > 0) (ReLU backward)
    const uint16_t* w;     // [cout_p][kp] BF16, k = tap * cin_p + c
    const float* bias;     // optional [cout]
    uint16_t* y;           // output [P][ldy], channels [yoff, yoff + cout)
    float* yf;             // optional FP32 output [P][cout]
    int ldx, cin_p, kp, taps;
    int ldy, yoff, cout, relu;
    int n, D, H, W;
};

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

// 3x3x3 convolution as an implicit GEMM with the input staged in LDS.  A block owns an
// output tile of 16 (x) x 4 (y) x 4 (z) voxels of one sample; the input tile with its
// one-voxel halo (18 x 6 x 6 voxels) is staged once per chunk of up to 32 input channels
// (voxel stride padded by 8 channels against bank conflicts; every global load of a
// thread is issued before its LDS writes), and all 27 taps read it from LDS.  Wave w
// computes rows (y, z) 4w..4w+3 of the tile (four 16-voxel M tiles) for every
// 16-channel N tile; K runs over tap x channel with k = tap * C + c inside a chunk of C
// channels (C = 16: one 32-wide step covers two taps).
constexpr int kTX = 16, kTY = 4, kTZ = 4;
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2;
constexpr int kHV = kHX * kHY * kHZ;
constexpr int kCS = 40;   // LDS channel stride per voxel (32 + 8 padding), BF16 units

template <int NT>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a) {
    __shared__ uint4 xs[kHV * kCS / 8];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int ntx = (a.W + kTX - 1) / kTX, nty = (a.H + kTY - 1) / kTY, ntz = (a.D + kTZ - 1) / kTZ;
    int bid = blockIdx.x;
    const int tx = bid % ntx;
    bid /= ntx;
    const int ty = bid % nty;
    bid /= nty;
    const int tz = bid % ntz;
    const int sb = bid / ntz;
    const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * kTZ;
    const long long sbase = (long long)sb * a.D * a.H * a.W;
    f32x4 acc[4][NT];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kg = 8 * (lane >> 4);
    for (int cb = 0; cb < a.cin_p; cb += 32) {
        const int C = a.cin_p - cb < 32 ? a.cin_p - cb : 32;
        const int G = C / 8;
        constexpr int SM = (kHV * 4 + 255) / 256;
        uint4 st[SM], sg[SM];
        int sidx[SM];
#pragma unroll
        for (int i = 0; i < SM; ++i) {
            const int e = threadIdx.x + 256 * i;
            st[i] = make_uint4(0, 0, 0, 0);
            sg[i] = make_uint4(0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u);   // BF16 1.0 (gate open)
            sidx[i] = -1;
            if (e < kHV * G) {
                const int v = e / G, g = e - v * G;
                const int hx = v % kHX, hy = (v / kHX) % kHY, hz = v / (kHX * kHY);
                const int x = x0 - 1 + hx, y = y0 - 1 + hy, z = z0 - 1 + hz;
                sidx[i] = v * (kCS / 8) + g;
                if (x >= 0 && x < a.W && y >= 0 && y < a.H && z >= 0 && z < a.D) {
                    const long long q = sbase + ((long long)z * a.H + y) * a.W + x;
                    st[i] = *reinterpret_cast<const uint4*>(a.x + q * a.ldx + cb + 8 * g);
                    if (a.gate) sg[i] = *reinterpret_cast<const uint4*>(a.gate + q * a.ldx + cb + 8 * g);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < SM; ++i)
            if (sidx[i] >= 0) xs[sidx[i]] = a.gate ? apply_gate(st[i], sg[i]) : st[i];
        __syncthreads();
        const int KC = 27 * C;
        for (int kk = 0; kk < KC; kk += 32) {
            const int kl = kk + kg;
            const int tap = kl / C, c0 = kl - tap * C;
            const bool tin = tap < 27;
            bf16x8 bfr[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                uint4 t = make_uint4(0, 0, 0, 0);
                if (tin)
                    t = *reinterpret_cast<const uint4*>(a.w + (long long)(nt * 16 + (lane & 15)) * a.kp +
                                                        tap * a.cin_p + cb + c0);
                bfr[nt] = __builtin_bit_cast(bf16x8, t);
            }
            const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;   // halo offsets 0..2
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const int r = 4 * wave + mt;
                const int yy = r % kTY, zz = r / kTY;
                const int hv = ((zz + dz) * kHY + (yy + dy)) * kHX + (lane & 15) + dx;
                uint4 t = make_uint4(0, 0, 0, 0);
                if (tin) t = xs[hv * (kCS / 8) + c0 / 8];
                const bf16x8 af = __builtin_bit_cast(bf16x8, t);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr[nt], acc[mt][nt], 0, 0, 0);
            }
        }
    }
    // D layout: lane holds rows 4 * (lane / 16) + i (voxels x0 + row), column lane % 16
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const int r = 4 * wave + mt;
        const int y = y0 + r % kTY, z = z0 + r / kTY;
        if (y >= a.H || z >= a.D) continue;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int co = nt * 16 + (lane & 15);
            if (co >= a.cout) continue;
            const float bv = a.bias ? a.bias[co] : 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = x0 + 4 * (lane >> 4) + i;
                if (x >= a.W) continue;
                const long long p = sbase + ((long long)z * a.H + y) * a.W + x;
                float v = acc[mt][nt][i] + bv;
                if (a.relu) v = fmaxf(v, 0.f);
                if (a.y) a.y[p * a.ldy + a.yoff + co] = f2bf(v);
                if (a.yf) a.yf[p * a.cout + co] = v;
            }
        }
    }
}

struct WgradArgs {
    const uint16_t* x;     // forward input [P][ldx] (real channels cin, padded cin_p)
    const uint16_t* g;     // output gradient [P][ldg]
    const uint16_t* gate;  // layer output [P][ldg] (ReLU gate) or null
    float* part;           // [nchunk][27][cin_p][cout_p]
    float* bpart;          // optional [nchunk][cout]: bias-gradient partials (from the centre tap)
    int ldx, cin_p, ldg, cout_p;
    int n, D, H, W;
    long long per_chunk;   // voxels per block (multiple of 64)
};

// Weight gradient of a 3x3x3 convolution for one tap (blockIdx.y) over one voxel
// chunk (blockIdx.x): dW[tap][c][o] = sum_p x[p + off(tap)][c] * g[p][o] * (gate > 0).
// Voxel tiles of 64 are staged in LDS transposed ([channel][voxel]) so that the MFMA
// K dimension runs over voxels.
__global__ __launch_bounds__(256) void k_conv_wgrad(WgradArgs a) {
    constexpr int PT = 64;
    __shared__ uint16_t xs[128 * PT];   // [cin_p][PT]
    __shared__ uint16_t gs[128 * PT];   // [cout_p][PT]
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tap = blockIdx.y;
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const long long P = (long long)a.n * a.D * a.H * a.W;
    const long long pa = (long long)blockIdx.x * a.per_chunk;
    const long long pb = pa + a.per_chunk < P ? pa + a.per_chunk : P;
    const int mtc = a.cin_p / 16, ntc = a.cout_p / 16, ntile = mtc * ntc;
    f32x4 acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int cgx = a.cin_p / 8, cgg = a.cout_p / 8;   // 16-byte groups per voxel
    // the centre tap's block also sums the gated gradient per channel (bias gradient)
    const bool bias = a.bpart && tap == 13;
    float bsum = 0.f;
    for (long long t0 = pa; t0 < pb; t0 += PT) {
        __syncthreads();
        // stage x (shifted by the tap) and the gated gradient, transposed
        for (int e = threadIdx.x; e < PT * (cgx + cgg); e += 256) {
            const bool isx = e < PT * cgx;
            const int ee = isx ? e : e - PT * cgx;
            const int cg = isx ? cgx : cgg;
            const int pv = ee / cg, grp = ee - pv * cg;
            const long long p = t0 + pv;
            uint4 t = make_uint4(0, 0, 0, 0);
            if (p < pb) {
                long long r = p;
                const int xx = (int)(r % a.W); r /= a.W;
                const int yy = (int)(r % a.H); r /= a.H;
                const int zz = (int)(r % a.D);
                const long long nb = r / a.D;
                if (isx) {
                    const int z = zz + dz, y = yy + dy, x = xx + dx;
                    if (z >= 0 && z < a.D && y >= 0 && y < a.H && x >= 0 && x < a.W) {
                        const long long q = ((nb * a.D + z) * a.H + y) * a.W + x;
                        t = *reinterpret_cast<const uint4*>(a.x + q * a.ldx + grp * 8);
                    }
                } else {
                    t = *reinterpret_cast<const uint4*>(a.g + p * a.ldg + grp * 8);
                    if (a.gate) {
                        const uint4 g = *reinterpret_cast<const uint4*>(a.gate + p * a.ldg + grp * 8);
                        const uint32_t gw[4] = {g.x, g.y, g.z, g.w};
                        uint32_t tw[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const uint32_t lo = gw[i] & 0xffffu, hi = gw[i] >> 16;
                            const bool plo = lo != 0 && !(lo & 0x8000u);
                            const bool phi = hi != 0 && !(hi & 0x8000u);
                            tw[i] &= (plo ? 0x0000ffffu : 0u) | (phi ? 0xffff0000u : 0u);
                        }
                        t = make_uint4(tw[0], tw[1], tw[2], tw[3]);
                    }
                }
            }
            const uint32_t w4[4] = {t.x, t.y, t.z, t.w};
            uint16_t* dst = isx ? xs : gs;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                dst[(grp * 8 + 2 * i) * PT + pv] = (uint16_t)(w4[i] & 0xffffu);
                dst[(grp * 8 + 2 * i + 1) * PT + pv] = (uint16_t)(w4[i] >> 16);
            }
        }
        __syncthreads();
        if (bias && (int)threadIdx.x < a.ldg) {
            const uint16_t* row = gs + threadIdx.x * PT;
            for (int pv = 0; pv < PT; ++pv) bsum += bf2f(row[pv]);
        }
#pragma unroll
        for (int kk = 0; kk < PT; kk += 32) {
            const int kq = kk + 8 * (lane >> 4);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int tile = wave + 4 * i;
                if (tile < ntile) {
                    const int mt = tile / ntc, nt = tile - (tile / ntc) * ntc;
                    const uint4 ta = *reinterpret_cast<const uint4*>(xs + (mt * 16 + (lane & 15)) * PT + kq);
                    const uint4 tb = *reinterpret_cast<const uint4*>(gs + (nt * 16 + (lane & 15)) * PT + kq);
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ta),
                                                                     __builtin_bit_cast(bf16x8, tb), acc[i], 0, 0, 0);
                }
            }
        }
    }
    if (bias && (int)threadIdx.x < a.ldg) a.bpart[(long long)blockIdx.x * a.ldg + threadIdx.x] = bsum;
    float* out = a.part + ((long long)blockIdx.x * 27 + tap) * a.cin_p * a.cout_p;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int tile = wave + 4 * i;
        if (tile < ntile) {
            const int mt = tile / ntc, nt = tile - (tile / ntc) * ntc;
            const int co = nt * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ci = mt * 16 + 4 * (lane >> 4) + r;
                out[ci * a.cout_p + co] = acc[i][r];
            }
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
    double s = 0.0;
    for (int k = 0; k < nchunk; ++k) s += part[(((long long)k * 27 + tap) * cin_p + c) * cout_p + o];
    grad[i] += (float)s;
}

__global__ void k_bias_reduce(const float* part, int nchunk, int cout, float* grad) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= cout) return;
    double s = 0.0;
    for (int k = 0; k < nchunk; ++k) s += part[(long long)k * cout + o];
    grad[o] += (float)s;
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
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const long long q = (((long long)v.b * D + 2 * v.z + (k >> 2)) * H + 2 * v.y + ((k >> 1) & 1)) * W + 2 * v.x + (k & 1);
        float f[8];
        unpack8(*reinterpret_cast<const uint4*>(x + q * ldx + 8 * g), f);
#pragma unroll
        for (int e = 0; e < 8; ++e) s[e] += f[e];
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] *= 0.125f;
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
    for (int o = 0; o < cout; ++o) {
        float s = b[o];
#pragma unroll
        for (int k = 0; k < 16; ++k) s += hv[k] * W[k * cout + o];
        out[p * cout + o] = s;
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

// BF16 copies of one convolution's weights: forward [cout_p][kp] with k = tap * cin_p + c,
// and input-gradient [cin_p][kpd] with k = tap * cout_p + o holding W[26 - tap][c][o].
__global__ void k_pack(const float* W, int cin, int cout, int taps, int cin_p, int cout_p, int kp, int kpd,
                       uint16_t* wf, uint16_t* wd) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nf = (long long)cout_p * kp, nd = (long long)cin_p * kpd;
    if (i < nf) {
        const int o = (int)(i / kp), k = (int)(i % kp);
        const int tap = k / cin_p, c = k % cin_p;
        float v = 0.f;
        if (o < cout && tap < taps && c < cin) v = W[((long long)tap * cin + c) * cout + o];
        wf[i] = f2bf(v);
    } else if (i < nf + nd && wd) {
        const long long j = i - nf;
        const int c = (int)(j / kpd), k = (int)(j % kpd);
        const int tap = k / cout_p, o = k % cout_p;
        float v = 0.f;
        if (c < cin && tap < taps && o < cout) v = W[((long long)(taps - 1 - tap) * cin + c) * cout + o];
        wd[j] = f2bf(v);
    }
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
