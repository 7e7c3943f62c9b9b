// Warm-start U-Net: parameters, activations and the forward/backward/Adam driver.
//
// Shape (fixed by the project's specification, not by the paper): L levels of widths
// C_0..C_{L-1}; per level two 3x3x3 convolutions + ReLU; 2x2x2 average pooling between
// encoder levels; decoder levels upsample x2 (nearest), concatenate [upsampled, skip]
// and apply two 3x3x3 convolutions + ReLU; a 1x1x1 head.  FP32 master parameters,
// gradients and Adam moments; BF16 copies of the convolution weights in the layouts
// the MFMA kernels read; BF16 activations; FP32 accumulation.
#include <cmath>
#include <random>
#include <vector>

#include "context.h"
#include "unet.h"
#include "unet_kernels.h"

namespace mpm {

static int roundup(int v, int m) { return (v + m - 1) / m * m; }

int net_build(Net* n, int in_ch, int out_ch, int levels, const int* widths, uint64_t seed) {
    n->in_ch = in_ch;
    n->out_ch = out_ch;
    n->L = levels;
    n->widths.assign(widths, widths + levels);
    auto add = [&](int cin, int cout, int taps) {
        ConvL l;
        l.cin = cin;
        l.cout = cout;
        l.taps = taps;
        l.cin_p = roundup(cin, 16);
        l.cout_p = roundup(cout, 16);
        l.kp = 2 * kSteps * l.cin_p;    // 14 steps of 32 per 16 input channels
        l.kpd = 2 * kSteps * l.cout_p;
        l.woff = n->nparam;
        n->nparam += (size_t)taps * cin * cout;
        l.boff = n->nparam;
        n->nparam += cout;
        n->layers.push_back(l);
    };
    int cin = in_ch;
    for (int l = 0; l < levels; ++l) {
        add(cin, widths[l], 27);
        add(widths[l], widths[l], 27);
        cin = widths[l];
    }
    for (int l = levels - 2; l >= 0; --l) {
        add(widths[l + 1] + widths[l], widths[l], 27);
        add(widths[l], widths[l], 27);
    }
    add(widths[0], out_ch, 1);
    hipStream_t st = n->stream;
    const size_t np = n->nparam;
    MPM_HIP(hipMalloc(&n->theta, np * 4));
    MPM_HIP(hipMalloc(&n->grad, np * 4));
    MPM_HIP(hipMalloc(&n->m, np * 4));
    MPM_HIP(hipMalloc(&n->v, np * 4));
    MPM_HIP(hipMemsetAsync(n->grad, 0, np * 4, st));
    MPM_HIP(hipMemsetAsync(n->m, 0, np * 4, st));
    MPM_HIP(hipMemsetAsync(n->v, 0, np * 4, st));
    for (auto& l : n->layers) {
        if (l.taps != 27) continue;
        MPM_HIP(hipMalloc(&l.wf, (size_t)l.cout_p * l.kp * 2));
        MPM_HIP(hipMalloc(&l.wd, (size_t)l.cin_p * l.kpd * 2));
    }
    // He-normal initialisation (std sqrt(2 / fan_in)), zero biases, small head
    std::vector<float> h(np, 0.0f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (size_t li = 0; li < n->layers.size(); ++li) {
        const ConvL& l = n->layers[li];
        const bool head = li + 1 == n->layers.size();
        const double sd = head ? 1e-2 : std::sqrt(2.0 / (double)(l.taps * l.cin));
        for (size_t i = 0; i < (size_t)l.taps * l.cin * l.cout; ++i) h[l.woff + i] = (float)(sd * nd(rng));
    }
    MPM_HIP(hipMemcpyAsync(n->theta, h.data(), np * 4, hipMemcpyHostToDevice, st));
    MPM_HIP(hipStreamSynchronize(st));
    return net_pack(n);
}

int net_pack(Net* n) {
    hipStream_t st = n->stream;
    for (auto& l : n->layers) {
        if (l.taps != 27) continue;
        const long long nf = (long long)l.cout_p * l.kp, nd = (long long)l.cin_p * l.kpd;
        k_pack<<<(unsigned)((nf + nd + 255) / 256), 256, 0, st>>>(n->theta + l.woff, l.cin, l.cout, l.cin_p, l.cout_p,
                                                                 nf, nd, l.wf, l.wd);
    }
    MPM_HIP(hipGetLastError());
    return MPM_OK;
}

static void free_acts(Net* n) {
    for (auto p : n->bufs) (void)hipFree(p);
    n->bufs.clear();
    n->act.clear();
    n->gin.clear();
    n->pooled.clear();
    n->cat.clear();
    n->dcat.clear();
    (void)hipFree(n->wpart);
    n->wpart = nullptr;
    n->wpart_cap = 0;
    n->dims[0] = n->dims[1] = n->dims[2] = n->dims[3] = 0;
}

void net_free(Net* n) {
    if (!n) return;
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    free_acts(n);
    for (auto& l : n->layers) {
        (void)hipFree(l.wf);
        (void)hipFree(l.wd);
    }
    (void)hipFree(n->theta);
    (void)hipFree(n->grad);
    (void)hipFree(n->m);
    (void)hipFree(n->v);
    (void)hipFree(n->outbuf);
    (void)hipFree(n->dpart);
}

// Activation, gradient and scratch buffers for one input shape.
static int ensure_acts(Net* n, int nb, int D, int H, int W) {
    if (n->dims[0] == nb && n->dims[1] == D && n->dims[2] == H && n->dims[3] == W) return MPM_OK;
    free_acts(n);
    const int L = n->L;
    auto alloc = [&](size_t elems, uint16_t** p) -> int {
        if (hipMalloc(p, elems * 2) != hipSuccess) {
            (void)hipGetLastError();
            set_error("U-Net activation allocation failed");
            return MPM_ENOMEM;
        }
        n->bufs.push_back(*p);
        return MPM_OK;
    };
    auto vox = [&](int lvl) { return (size_t)nb * (D >> lvl) * (H >> lvl) * (W >> lvl); };
    const size_t nl = n->layers.size();
    n->act.assign(nl, nullptr);
    n->gin.assign(nl, nullptr);
    n->pooled.assign(L, nullptr);
    n->cat.assign(L, nullptr);
    n->dcat.assign(L, nullptr);
    int rc = MPM_OK;
    n->xin = nullptr;
    if (n->in_ch != n->layers[0].cin_p && (rc = alloc(vox(0) * n->layers[0].cin_p, &n->xin))) return rc;
    // level of each conv layer
    std::vector<int> lvl_of(nl, 0);
    for (int l = 0; l < L; ++l) lvl_of[2 * l] = lvl_of[2 * l + 1] = l;
    for (int d = 0; d < L - 1; ++d) {
        const int l = L - 2 - d;
        lvl_of[2 * L + 2 * d] = lvl_of[2 * L + 2 * d + 1] = l;
    }
    n->lvl_of = lvl_of;
    for (size_t li = 0; li + 1 < nl; ++li) {
        const ConvL& c = n->layers[li];
        if ((rc = alloc(vox(lvl_of[li]) * c.cout, &n->act[li]))) return rc;
        if ((rc = alloc(vox(lvl_of[li]) * c.cout, &n->gin[li]))) return rc;   // grad wrt this layer's output
    }
    for (int l = 1; l < L; ++l)
        if ((rc = alloc(vox(l) * n->widths[l - 1], &n->pooled[l]))) return rc;
    for (int l = 0; l < L - 1; ++l) {
        const size_t c = (size_t)n->widths[l + 1] + n->widths[l];
        if ((rc = alloc(vox(l) * c, &n->cat[l]))) return rc;
        if ((rc = alloc(vox(l) * c, &n->dcat[l]))) return rc;
    }
    if ((rc = alloc(vox(0) * n->widths[0], &n->ghead))) return rc;
    if ((rc = alloc(vox(1) * n->widths[0] * 8, &n->gscratch))) return rc;   // pooled-input gradient
    n->dims[0] = nb;
    n->dims[1] = D;
    n->dims[2] = H;
    n->dims[3] = W;
    return MPM_OK;
}

// Launch k_conv<NTB, WL, GATED> over all (voxel tile, output-tile group) items: one
// persistent block per LDS slot of the device (capped at the item count, rounded down to
// a multiple of the group count).
// Resident blocks of k_conv<NTB, WL, GATED> on the device (registers and LDS
// permitting), found once; the first call also grants the kernel its LDS.
template <int NTB, bool WL, bool GATED, bool HEAD = false, bool LIST = false, bool POOL = false>
static hipError_t conv_slots(int* out) {
    constexpr int lds = conv_lds_bytes(NTB, WL, HEAD, LIST, POOL);
    static int slots = 0;
    static const hipError_t granted = [] {
        int dev = 0, cap = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess && cap < lds) e = hipErrorInvalidValue;
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_conv<NTB, WL, GATED, HEAD, LIST, POOL>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_conv<NTB, WL, GATED, HEAD, LIST, POOL>, 256,
                                                             lds);
        slots = std::max(1, cus) * std::max(1, per_cu);
        return e;
    }();
    *out = slots;
    return granted;
}

// Blocks of a persistent launch: one per resident slot, capped at the items (voxel tiles,
// or listed tiles, times the output-tile groups) and rounded down to a multiple of the
// group count; with a tile list, enough that no block takes more than kListMax entries.
static long long conv_grid(const ConvArgs& a, int nsplit, int slots) {
    const long long tiles = a.tlist ? (long long)a.tcount
                                    : (long long)a.n * ((a.D + kTZ - 1) / kTZ) * ((a.H + kTY - 1) / kTY) *
                                          ((a.W + kTX - 1) / kTX);
    long long grid = std::min<long long>(tiles * nsplit, slots);
    grid = std::max<long long>(nsplit, grid / nsplit * nsplit);
    if (a.tlist) grid = std::max<long long>(grid, (tiles + kListMax - 1) / kListMax * nsplit);
    return grid;
}

template <int NTB, bool WL, bool GATED, bool HEAD = false, bool LIST = false, bool POOL = false>
static int launch_conv(const ConvArgs& a, hipStream_t st) {
    constexpr int lds = conv_lds_bytes(NTB, WL, HEAD, LIST, POOL);
    int slots = 0;
    const hipError_t granted = conv_slots<NTB, WL, GATED, HEAD, LIST, POOL>(&slots);
    if (granted != hipSuccess) return hip_fail(granted, "U-Net convolution LDS");
    const long long grid = conv_grid(a, a.nt / NTB, slots);
    k_conv<NTB, WL, GATED, HEAD, LIST, POOL><<<(unsigned)grid, 256, lds, st>>>(a);
    return MPM_OK;
}

// k_conv_staged<1> (16 input channels, one output tile, no gate; static LDS): one block
// per resident slot, as launch_conv.
template <bool HEAD = false, bool LIST = false, bool POOL = false>
static hipError_t staged_slots(int* out) {
    static int slots = 0;
    static const hipError_t granted = [] {
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_conv_staged<1, HEAD, LIST, POOL>, 256, 0);
        slots = std::max(1, cus) * std::max(1, per_cu);
        return e;
    }();
    *out = slots;
    return granted;
}

// 16-channel input and one output tile: k_conv_staged once every block has two or more
// tiles (16 -> 16 on 128^3: 50.5 -> 42.6 us; on small grids its longer start costs more
// than it saves), else k_conv.
template <bool HEAD, bool LIST, bool POOL>
static int launch_one_tile(const ConvArgs& a, long long tiles, hipStream_t st) {
    int slots = 0;
    const hipError_t e = staged_slots<HEAD, LIST, POOL>(&slots);
    if (e != hipSuccess) return hip_fail(e, "U-Net convolution occupancy");
    if (tiles * a.nt < 2LL * slots) return launch_conv<1, false, false, HEAD, LIST, POOL>(a, st);
    k_conv_staged<1, HEAD, LIST, POOL><<<(unsigned)conv_grid(a, a.nt, slots), 256, 0, st>>>(a);
    return MPM_OK;
}

// Output tiles per block: two for a 16-channel input with an even tile count (each A
// fragment read from LDS then feeds two MFMAs); for wider inputs two when the grid has
// tiles for at least two rounds of the resident blocks (64^3 layers with 32 outputs:
// 29.3 -> 26.4 us), else one (three blocks per CU instead of two, which the smaller
// grids need to fill the device).  The fused head and tile lists go with one output
// tile, the fused pooling with every variant but the gated ones.
static int conv_dispatch(ConvArgs a, int nt, hipStream_t st) {
    if (nt < 1 || nt > 8 || a.cin_p % 16 || a.cin_p < 16 || (a.x2 && (a.gate || a.c1 % 16))) {
        set_error("unsupported channel count in the U-Net");
        return MPM_EINVAL;
    }
    if (a.hout && (nt != 1 || a.cin_p != 16 || a.gate || a.x2 || a.y || a.hcout < 1 || a.hcout > 4)) {
        set_error("the fused head needs a 16 -> 16 convolution and at most 4 outputs");
        return MPM_EINVAL;
    }
    if (a.tlist && (a.n != 1 || a.gate || nt != 1 || a.tcount < 0 || (a.cin_p == 16 && !a.hout))) {
        set_error("a tile list needs one sample and one output tile (with the fused head for 16 inputs)");
        return MPM_EINVAL;
    }
    if (a.yp && (a.gate || a.hout || a.tlist || a.x2 || !a.y || (a.D | a.H | a.W) & 1)) {
        set_error("the fused pooling needs even grid sizes and a plain convolution");
        return MPM_EINVAL;
    }
    a.nt = nt;
    const bool one = a.cin_p == 16, pool = a.yp != nullptr;
    if (a.tlist && a.tcount == 0) return MPM_OK;   // nothing listed
    if (a.tlist && !one) return launch_conv<1, true, false, false, true>(a, st);
    if (a.gate) {
        if (one) return nt % 2 ? launch_conv<1, false, true>(a, st) : launch_conv<2, false, true>(a, st);
        return launch_conv<1, true, true>(a, st);
    }
    const long long tiles = a.tlist ? (long long)a.tcount
                                    : (long long)a.n * ((a.D + kTZ - 1) / kTZ) * ((a.H + kTY - 1) / kTY) *
                                          ((a.W + kTX - 1) / kTX);
    if (one && nt % 2) {
        if (a.tlist) return launch_one_tile<true, true, false>(a, tiles, st);
        if (a.hout) return launch_one_tile<true, false, false>(a, tiles, st);
        if (pool) return launch_one_tile<false, false, true>(a, tiles, st);
        return launch_one_tile<false, false, false>(a, tiles, st);
    }
    if (one)
        return pool ? launch_conv<2, false, false, false, false, true>(a, st) : launch_conv<2, false, false>(a, st);
    if (nt % 2 == 0) {
        int slots = 0;
        const hipError_t e = pool ? conv_slots<2, true, false, false, false, true>(&slots)
                                  : conv_slots<2, true, false>(&slots);
        if (e != hipSuccess) return hip_fail(e, "U-Net convolution LDS");
        if (tiles * (nt / 2) >= 2LL * slots)
            return pool ? launch_conv<2, true, false, false, false, true>(a, st) : launch_conv<2, true, false>(a, st);
    }
    return pool ? launch_conv<1, true, false, false, false, true>(a, st) : launch_conv<1, true, false>(a, st);
}

static ConvArgs conv_args(const Net* n, int lvl) {
    ConvArgs a{};
    a.n = n->dims[0];
    a.D = n->dims[1] >> lvl;
    a.H = n->dims[2] >> lvl;
    a.W = n->dims[3] >> lvl;
    return a;
}

static unsigned blocks_for(long long count) { return (unsigned)((count + 255) / 256); }

int net_forward(Net* n, const uint16_t* in, int nb, int D, int H, int W, float* out, bool infer,
                const TileLists* tiles) {
    const int L = n->L;
    const int div = 1 << (L - 1);
    if (nb < 1 || D < div || H < div || W < div || D % div || H % div || W % div) {
        set_error("U-Net input sizes must be positive multiples of 2^(levels-1)");
        return MPM_EINVAL;
    }
    int rc = ensure_acts(n, nb, D, H, W);
    if (rc) return rc;
    hipStream_t st = n->stream;
    const long long P0 = (long long)nb * D * H * W;
    const ConvL& l0 = n->layers[0];
    // an input whose channel count is a multiple of 16 is read in place (and must stay
    // unchanged until the backward pass); others are padded with zero channels
    if (n->in_ch == l0.cin_p) {
        n->x0 = in;
    } else {
        k_pad_channels<<<blocks_for(P0), 256, 0, st>>>(in, n->in_ch, l0.cin_p, P0, n->xin);
        n->x0 = n->xin;
    }
    const uint16_t* h = n->x0;
    int hch = l0.cin_p;
    int li = 0;
    for (int lvl = 0; lvl < L; ++lvl) {
        if (lvl > 0) h = n->pooled[lvl];   // pooled by the previous level's second convolution
        for (int r = 0; r < 2; ++r, ++li) {
            const ConvL& c = n->layers[li];
            ConvArgs a = conv_args(n, lvl);
            a.x = h;
            a.ldx = hch;
            a.cin_p = c.cin_p;
            a.w = c.wf;
            a.bias = n->theta + c.boff;
            a.y = n->act[li];
            a.ldy = c.cout;
            a.cout = c.cout;
            a.relu = 1;
            if (r == 1 && lvl + 1 < L) a.yp = n->pooled[lvl + 1];   // the next level's input
            if ((rc = conv_dispatch(a, c.cout_p / 16, st))) return rc;
            h = n->act[li];
            hch = c.cout;
        }
    }
    const ConvL& hd = n->layers.back();
    // inference: the head runs in the last convolution's epilogue, whose output is then
    // not stored (only a 16 -> 16 last layer with its 16-channel head qualifies)
    const int last = (int)n->layers.size() - 2;
    const bool fuse = infer && n->layers[last].cin_p == 16 && n->layers[last].cout == 16 && hd.cin == 16 &&
                      hd.cout <= 4;
    const bool listed = fuse && tiles && nb == 1;
    for (int lvl = L - 2; lvl >= 0; --lvl) {
        const int cu = n->widths[lvl + 1], cs = n->widths[lvl];
        for (int r = 0; r < 2; ++r, ++li) {
            const ConvL& c = n->layers[li];
            ConvArgs a = conv_args(n, lvl);
            a.x = h;
            a.ldx = hch;
            if (r == 0) {   // reads the upsampled input and the skip itself (widths are
                            // multiples of 16: each 16-channel chunk has one source)
                a.x2 = n->act[2 * lvl + 1];
                a.ldx2 = cs;
                a.c1 = cu;
            }
            a.cin_p = c.cin_p;
            a.w = c.wf;
            a.bias = n->theta + c.boff;
            a.y = n->act[li];
            a.ldy = c.cout;
            a.cout = c.cout;
            a.relu = 1;
            if (fuse && li == last) {
                a.y = nullptr;
                a.hw = n->theta + hd.woff;
                a.hb = n->theta + hd.boff;
                a.hout = out;
                a.hcout = hd.cout;
            }
            if (listed && li >= last - 1) {
                a.tlist = li == last ? tiles->domain : tiles->near;
                a.tcount = li == last ? tiles->n_domain : tiles->n_near;
            }
            if ((rc = conv_dispatch(a, c.cout_p / 16, st))) return rc;
            h = n->act[li];
            hch = c.cout;
        }
    }
    if (!fuse)
        k_head<<<blocks_for(P0), 256, 0, st>>>(h, hch, n->theta + hd.woff, n->theta + hd.boff, hd.cout, P0, out);
    MPM_HIP(hipGetLastError());
    n->head_in = fuse ? nullptr : h;
    n->have_fwd = true;
    n->fwd_infer = infer;
    n->fwd_listed = listed;
    return MPM_OK;
}

// Weight and bias gradients of 3x3x3 layer li (input x with ldx channels at level lvl,
// output gradient g gated by the layer's own output).
static int conv_param_grads(Net* n, int li, int lvl, const uint16_t* x, int ldx, const uint16_t* g,
                            const uint16_t* gate, float* gw, float* gb) {
    hipStream_t st = n->stream;
    const ConvL& c = n->layers[li];
    const int D = n->dims[1] >> lvl, H = n->dims[2] >> lvl, W = n->dims[3] >> lvl;
    const long long tiles = (long long)n->dims[0] * ((D + kTZ - 1) / kTZ) * ((H + kTY - 1) / kTY) * ((W + kTX - 1) / kTX);
    // one block per (16 x 16 channel block, voxel-tile stride); about 512 blocks in all,
    // two per CU (63 KB of LDS each)
    const int cblocks = (c.cin_p / 16) * (c.cout_p / 16);
    const long long nchunk = std::max(1LL, std::min(tiles, (long long)std::max(1, 512 / cblocks)));
    const size_t need = (size_t)nchunk * 27 * c.cin_p * c.cout_p;
    if (need > n->wpart_cap) {
        (void)hipFree(n->wpart);
        if (hipMalloc(&n->wpart, need * 4) != hipSuccess) {
            (void)hipGetLastError();
            n->wpart = nullptr;
            n->wpart_cap = 0;
            set_error("U-Net gradient scratch allocation failed");
            return MPM_ENOMEM;
        }
        n->wpart_cap = need;
    }
    WgradArgs w{};
    w.x = x;
    w.g = g;
    w.gate = gate;
    w.part = n->wpart;
    w.ldx = ldx;
    w.cin_p = c.cin_p;
    w.ldg = c.cout;
    w.cout_p = c.cout_p;
    w.n = n->dims[0];
    w.D = D;
    w.H = H;
    w.W = W;
    if ((size_t)nchunk * c.cout_p > n->dpart_cap) {
        (void)hipFree(n->dpart);
        n->dpart_cap = std::max<size_t>((size_t)nchunk * c.cout_p, 64 * 128);
        if (hipMalloc(&n->dpart, n->dpart_cap * 4) != hipSuccess) {
            (void)hipGetLastError();
            n->dpart = nullptr;
            n->dpart_cap = 0;
            set_error("U-Net gradient scratch allocation failed");
            return MPM_ENOMEM;
        }
    }
    w.bpart = gb ? n->dpart : nullptr;
    k_conv_wgrad<<<dim3((unsigned)nchunk, (unsigned)cblocks), 256, kWgLds, st>>>(w);
    const long long tot = 27LL * c.cin * c.cout;
    k_wgrad_reduce<<<blocks_for(tot), 256, 0, st>>>(n->wpart, (int)nchunk, c.cin, c.cout, c.cin_p, c.cout_p, gw);
    if (gb) k_bias_reduce<<<1, 128, 0, st>>>(n->dpart, (int)nchunk, c.cout_p, c.cout, gb);
    MPM_HIP(hipGetLastError());
    return MPM_OK;
}

// Input gradient of 3x3x3 layer li into dx ([P][cin]), from g gated by the layer output.
static int conv_input_grad(Net* n, int li, int lvl, const uint16_t* g, const uint16_t* gate, uint16_t* dx,
                           float* dxf = nullptr) {
    const ConvL& c = n->layers[li];
    ConvArgs a = conv_args(n, lvl);
    a.x = g;
    a.gate = gate;
    a.yf = dxf;
    a.ldx = c.cout;
    a.cin_p = c.cout_p;
    a.w = c.wd;
    a.y = dx;
    a.ldy = c.cin;
    a.cout = c.cin;
    return conv_dispatch(a, c.cin_p / 16, n->stream);
}

int net_backward(Net* n, const float* dout) {
    if (!n->have_fwd || n->fwd_infer) {
        set_error("mpm_net_backward needs a preceding mpm_net_forward (not an inference pass)");
        return MPM_ESTATE;
    }
    hipStream_t st = n->stream;
    const int L = n->L;
    const int nb = n->dims[0], D = n->dims[1], H = n->dims[2], W = n->dims[3];
    const long long P0 = (long long)nb * D * H * W;
    const int nl = (int)n->layers.size();
    int rc;
    // head
    {
        const ConvL& hd = n->layers[nl - 1];
        const long long nchunk = std::max(1LL, std::min(256LL, P0 / 4096));
        const long long per = (P0 + nchunk - 1) / nchunk;
        const int npar = hd.cin * hd.cout + hd.cout;
        if ((size_t)nchunk * npar > n->dpart_cap) {
            (void)hipFree(n->dpart);
            n->dpart_cap = (size_t)nchunk * npar;
            if (hipMalloc(&n->dpart, n->dpart_cap * 4) != hipSuccess) {
                (void)hipGetLastError();
                n->dpart = nullptr;
                n->dpart_cap = 0;
                set_error("U-Net gradient scratch allocation failed");
                return MPM_ENOMEM;
            }
        }
        k_head_bwd<<<(unsigned)nchunk, 256, 0, st>>>(n->head_in, hd.cin, n->theta + hd.woff, hd.cout, dout, P0, per,
                                                     n->ghead, n->dpart);
        k_param_reduce<<<blocks_for(npar), 256, 0, st>>>(n->dpart, (int)nchunk, npar, n->grad + hd.woff);
    }
    // decoder, deepest last in forward order -> first here is level 0
    int li = nl - 2;
    const uint16_t* g = n->ghead;     // gradient wrt the output of layer li
    for (int lvl = 0; lvl <= L - 2; ++lvl) {
        const int cu = n->widths[lvl + 1], cs = n->widths[lvl];
        // second conv of the level: input act[li - 1]
        if ((rc = conv_param_grads(n, li, lvl, n->act[li - 1], n->layers[li].cin, g, n->act[li], n->grad + n->layers[li].woff, n->grad + n->layers[li].boff))) return rc;
        if ((rc = conv_input_grad(n, li, lvl, g, n->act[li], n->gin[li - 1]))) return rc;
        g = n->gin[li - 1];
        --li;
        // first conv of the level: its input, the concatenation of the upsampled deeper
        // output and the skip, which the forward pass read without writing it
        {
            const long long Pl = P0 >> (3 * lvl);
            k_up2_cat<<<blocks_for(Pl * (cu + cs) / 8), 256, 0, st>>>(n->act[li - 1], cu, n->act[2 * lvl + 1], cs, nb,
                                                                   D >> lvl, H >> lvl, W >> lvl, n->cat[lvl]);
        }
        if ((rc = conv_param_grads(n, li, lvl, n->cat[lvl], cu + cs, g, n->act[li], n->grad + n->layers[li].woff, n->grad + n->layers[li].boff))) return rc;
        if ((rc = conv_input_grad(n, li, lvl, g, n->act[li], n->dcat[lvl]))) return rc;
        --li;
        // gradient wrt the upsampled input -> gradient wrt the output of layer li (one level deeper)
        const long long Pd = P0 >> (3 * (lvl + 1));
        k_up2_bwd<<<blocks_for(Pd * cu / 8), 256, 0, st>>>(n->dcat[lvl], cu + cs, cu, nb, D >> (lvl + 1), H >> (lvl + 1),
                                                      W >> (lvl + 1), n->gin[li]);
        g = n->gin[li];
    }
    // encoder, bottom first; li is the second conv of the bottom level
    for (int lvl = L - 1; lvl >= 0; --lvl) {
        const int cinl = lvl == 0 ? n->layers[0].cin_p : n->widths[lvl - 1];
        if ((rc = conv_param_grads(n, li, lvl, n->act[li - 1], n->layers[li].cin, g, n->act[li], n->grad + n->layers[li].woff, n->grad + n->layers[li].boff))) return rc;
        if ((rc = conv_input_grad(n, li, lvl, g, n->act[li], n->gin[li - 1]))) return rc;
        g = n->gin[li - 1];
        --li;
        const uint16_t* xin = lvl == 0 ? n->x0 : n->pooled[lvl];
        if ((rc = conv_param_grads(n, li, lvl, xin, cinl, g, n->act[li], n->grad + n->layers[li].woff, n->grad + n->layers[li].boff))) return rc;
        if (lvl == 0) break;
        // gradient wrt the pooled input, then wrt the previous level's output (+ its skip)
        if ((rc = conv_input_grad(n, li, lvl, g, n->act[li], n->gscratch))) return rc;
        --li;
        const int c = n->widths[lvl - 1];
        const long long Pu = P0 >> (3 * (lvl - 1));
        k_pool2_bwd_add<<<blocks_for(Pu * c / 8), 256, 0, st>>>(n->gscratch, c,
                                                           lvl - 1 <= L - 2 ? n->dcat[lvl - 1] + n->widths[lvl] : nullptr,
                                                           n->widths[lvl] + c, nb, D >> (lvl - 1), H >> (lvl - 1),
                                                           W >> (lvl - 1), n->gin[li]);
        g = n->gin[li];
    }
    MPM_HIP(hipGetLastError());
    return MPM_OK;
}

}  // namespace mpm

// ------------------------------------------------------------------ C ABI
using namespace mpm;

extern "C" int32_t mpm_net_create(mpm_net* out, int32_t in_ch, int32_t out_ch, int32_t levels, const int32_t* widths,
                                  uint64_t seed, void* stream) {
    if (!out || !widths) {
        set_error("mpm_net_create: null pointer");
        return MPM_EINVAL;
    }
    *out = nullptr;
    if (in_ch < 1 || in_ch > 32 || out_ch < 1 || out_ch > 4 || levels < 1 || levels > 6) {
        set_error("mpm_net_create: need 1 <= in_ch <= 32, 1 <= out_ch <= 4, 1 <= levels <= 6");
        return MPM_EINVAL;
    }
    for (int l = 0; l < levels; ++l) {
        if (widths[l] < 16 || widths[l] > 64 || widths[l] % 16 != 0) {
            set_error("mpm_net_create: widths must be 16, 32, 48 or 64");
            return MPM_EINVAL;
        }
        if (l + 1 < levels && widths[l] + widths[l + 1] > 128) {
            set_error("mpm_net_create: a decoder concat may hold at most 128 channels");
            return MPM_EINVAL;
        }
    }
    if (widths[0] > 16) {
        set_error("mpm_net_create: the head reads at most 16 channels (widths[0] = 16)");
        return MPM_EINVAL;
    }
    Net* n = new Net();
    n->stream = (hipStream_t)stream;
    int rc = net_build(n, in_ch, out_ch, levels, widths, seed);
    if (rc == MPM_OK) {
        hipError_t e = hipStreamSynchronize(n->stream);
        if (e != hipSuccess) rc = hip_fail(e, "mpm_net_create");
    }
    if (rc != MPM_OK) {
        net_free(n);
        delete n;
        return rc;
    }
    *out = (mpm_net)n;
    return MPM_OK;
}

extern "C" int32_t mpm_net_params(mpm_net net, float** params, float** grads, int64_t* count) {
    Net* n = (Net*)net;
    if (!n || !params || !grads || !count) {
        set_error("mpm_net_params: null pointer");
        return MPM_EINVAL;
    }
    *params = n->theta;
    *grads = n->grad;
    *count = (int64_t)n->nparam;
    return MPM_OK;
}

extern "C" int32_t mpm_net_sync_weights(mpm_net net) {
    Net* n = (Net*)net;
    if (!n) {
        set_error("mpm_net_sync_weights: null pointer");
        return MPM_EINVAL;
    }
    return net_pack(n);
}

extern "C" int32_t mpm_net_zero_grad(mpm_net net) {
    Net* n = (Net*)net;
    if (!n) {
        set_error("mpm_net_zero_grad: null pointer");
        return MPM_EINVAL;
    }
    MPM_HIP(hipMemsetAsync(n->grad, 0, n->nparam * 4, n->stream));
    return MPM_OK;
}

extern "C" int32_t mpm_net_forward(mpm_net net, const uint16_t* in, int32_t nb, int32_t d, int32_t h, int32_t w,
                                   float* out) {
    Net* n = (Net*)net;
    if (!n || !in || !out) {
        set_error("mpm_net_forward: null pointer");
        return MPM_EINVAL;
    }
    return net_forward(n, in, nb, d, h, w, out, false);
}

extern "C" int32_t mpm_net_infer(mpm_net net, const uint16_t* in, int32_t nb, int32_t d, int32_t h, int32_t w,
                                 float* out) {
    Net* n = (Net*)net;
    if (!n || !in || !out) {
        set_error("mpm_net_infer: null pointer");
        return MPM_EINVAL;
    }
    return net_forward(n, in, nb, d, h, w, out, true);
}

extern "C" int32_t mpm_net_backward(mpm_net net, const float* grad_out) {
    Net* n = (Net*)net;
    if (!n || !grad_out) {
        set_error("mpm_net_backward: null pointer");
        return MPM_EINVAL;
    }
    return net_backward(n, grad_out);
}

extern "C" int32_t mpm_net_mse(mpm_net net, const float* out, const float* target, int64_t count, float* grad_out,
                               double* loss) {
    Net* n = (Net*)net;
    if (!n || !out || !target || !grad_out || !loss || count <= 0) {
        set_error("mpm_net_mse: bad arguments");
        return MPM_EINVAL;
    }
    const int nb = 512;
    if (!n->mse_part) MPM_HIP(hipHostMalloc((void**)&n->mse_part, nb * sizeof(double), hipHostMallocDefault));
    if (!n->mse_dev) MPM_HIP(hipMalloc(&n->mse_dev, nb * sizeof(double)));
    k_mse<<<nb, 256, 0, n->stream>>>(out, target, count, grad_out, n->mse_dev);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(n->mse_part, n->mse_dev, nb * sizeof(double), hipMemcpyDeviceToHost, n->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    if (e != hipSuccess) return hip_fail(e, "mpm_net_mse");
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += n->mse_part[i];
    *loss = s / (double)count;
    return MPM_OK;
}

extern "C" int32_t mpm_net_adam_step(mpm_net net, float lr, float b1, float b2, float eps, int32_t t) {
    Net* n = (Net*)net;
    if (!n || t < 1 || !(lr >= 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps >= 0.f)) {
        set_error("mpm_net_adam_step: bad arguments");
        return MPM_EINVAL;
    }
    const float c1 = 1.0f - std::pow(b1, (float)t), c2 = 1.0f - std::pow(b2, (float)t);
    const long long np = (long long)n->nparam;
    k_adam<<<(unsigned)((np + 255) / 256), 256, 0, n->stream>>>(n->theta, n->grad, n->m, n->v, np, lr, b1, b2, eps, c1,
                                                                 c2);
    MPM_HIP(hipGetLastError());
    return net_pack(n);
}

extern "C" int32_t mpm_net_destroy(mpm_net net) {
    Net* n = (Net*)net;
    if (!n) return MPM_OK;
    if (n->mse_part) (void)hipHostFree(n->mse_part);
    (void)hipFree(n->mse_dev);
    net_free(n);
    delete n;
    return MPM_OK;
}

extern "C" int32_t mpm_net_read(mpm_net net, int32_t what, float* dst) {
    Net* n = (Net*)net;
    if (!n || !dst || (what != 0 && what != 1)) {
        set_error("mpm_net_read: bad arguments");
        return MPM_EINVAL;
    }
    MPM_HIP(hipMemcpyAsync(dst, what == 0 ? n->theta : n->grad, n->nparam * 4, hipMemcpyDeviceToDevice, n->stream));
    MPM_HIP(hipStreamSynchronize(n->stream));
    return MPM_OK;
}

extern "C" int32_t mpm_net_write(mpm_net net, int32_t what, const float* src) {
    Net* n = (Net*)net;
    if (!n || !src || (what != 0 && what != 1)) {
        set_error("mpm_net_write: bad arguments");
        return MPM_EINVAL;
    }
    MPM_HIP(hipMemcpyAsync(what == 0 ? n->theta : n->grad, src, n->nparam * 4, hipMemcpyDeviceToDevice, n->stream));
    if (what == 0) {
        int rc = net_pack(n);
        if (rc != MPM_OK) return rc;
    }
    MPM_HIP(hipStreamSynchronize(n->stream));
    return MPM_OK;
}

extern "C" int32_t mpm_net_debug_layer(mpm_net net, int32_t layer, int32_t mode, int32_t nb, int32_t d, int32_t h,
                                       int32_t w, const uint16_t* x, const uint16_t* g, const uint16_t* gate,
                                       float* out) {
    Net* n = (Net*)net;
    if (!n || !out || layer < 0 || layer + 1 >= (int)n->layers.size() || mode < 0 || mode > 2 || nb < 1 || d < 1 ||
        h < 1 || w < 1 || (mode != 1 && !x) || (mode != 0 && !g)) {
        set_error("mpm_net_debug_layer: bad arguments");
        return MPM_EINVAL;
    }
    const ConvL& c = n->layers[layer];
    hipStream_t st = n->stream;
    int saved[4] = {n->dims[0], n->dims[1], n->dims[2], n->dims[3]};
    n->dims[0] = nb;
    n->dims[1] = d;
    n->dims[2] = h;
    n->dims[3] = w;
    int rc = MPM_OK;
    if (mode == 0) {
        ConvArgs a = conv_args(n, 0);
        a.x = x;
        a.ldx = c.cin_p;
        a.cin_p = c.cin_p;
        a.w = c.wf;
        a.bias = n->theta + c.boff;
        a.yf = out;
        a.cout = c.cout;
        rc = conv_dispatch(a, c.cout_p / 16, st);
    } else if (mode == 1) {
        rc = conv_input_grad(n, layer, 0, g, gate, nullptr, out);
    } else {
        // the reduction accumulates into its target, so start from zero
        hipError_t e = hipMemsetAsync(out, 0, (size_t)27 * c.cin * c.cout * sizeof(float), st);
        rc = e == hipSuccess ? conv_param_grads(n, layer, 0, x, c.cin_p, g, gate, out, nullptr)
                             : hip_fail(e, "mpm_net_debug_layer");
    }
    n->dims[0] = saved[0];
    n->dims[1] = saved[1];
    n->dims[2] = saved[2];
    n->dims[3] = saved[3];
    if (rc == MPM_OK) {
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hip_fail(e, "mpm_net_debug_layer");
    }
    return rc;
}

// Test hooks end with a launch check and a stream synchronisation.
static int net_debug_finish(hipStream_t st) {
    MPM_HIP(hipGetLastError());
    MPM_HIP(hipStreamSynchronize(st));
    return MPM_OK;
}

extern "C" int32_t mpm_net_debug_tensor(mpm_net net, int32_t kind, int32_t index, uint16_t* dst, int64_t* count) {
    Net* n = (Net*)net;
    if (!n || !count || kind < MPM_NT_INPUT || kind > MPM_NT_HEAD_GRAD) {
        set_error("mpm_net_debug_tensor: bad arguments");
        return MPM_EINVAL;
    }
    if (n->dims[0] == 0) {
        set_error("mpm_net_debug_tensor: no forward pass yet");
        return MPM_ESTATE;
    }
    const int L = n->L;
    const int nl = (int)n->layers.size();
    auto vox = [&](int lvl) {
        return (long long)n->dims[0] * (n->dims[1] >> lvl) * (n->dims[2] >> lvl) * (n->dims[3] >> lvl);
    };
    const uint16_t* src = nullptr;
    long long elems = 0;
    switch (kind) {
        case MPM_NT_INPUT:
            src = n->x0;
            elems = vox(0) * n->layers[0].cin_p;
            break;
        case MPM_NT_ACT:
        case MPM_NT_ACT_GRAD:
            if (index < 0 || index >= nl - 1) break;
            if (kind == MPM_NT_ACT && ((index == nl - 2 && n->fwd_infer && !n->head_in) ||
                                       (index == nl - 3 && n->fwd_listed))) {
                set_error("mpm_net_debug_tensor: the last inference pass did not store this output in full");
                return MPM_ESTATE;
            }
            src = kind == MPM_NT_ACT ? n->act[index] : n->gin[index];
            elems = vox(n->lvl_of[index]) * n->layers[index].cout;
            break;
        case MPM_NT_POOLED:
            if (index < 1 || index >= L) break;
            src = n->pooled[index];
            elems = vox(index) * n->widths[index - 1];
            break;
        case MPM_NT_CAT:
        case MPM_NT_CAT_GRAD:
            if (index < 0 || index >= L - 1) break;
            src = kind == MPM_NT_CAT ? n->cat[index] : n->dcat[index];
            elems = vox(index) * (n->widths[index + 1] + n->widths[index]);
            break;
        case MPM_NT_HEAD_GRAD:
            src = n->ghead;
            elems = vox(0) * n->widths[0];
            break;
    }
    if (!src) {
        set_error("mpm_net_debug_tensor: index out of range for this tensor kind");
        return MPM_EINVAL;
    }
    if (!dst) {
        *count = elems;
        return MPM_OK;
    }
    if (*count != elems) {
        set_error("mpm_net_debug_tensor: *count must equal the tensor's element count");
        return MPM_EINVAL;
    }
    MPM_HIP(hipMemcpyAsync(dst, src, (size_t)elems * 2, hipMemcpyDeviceToDevice, n->stream));
    MPM_HIP(hipStreamSynchronize(n->stream));
    return MPM_OK;
}

extern "C" int32_t mpm_net_debug_op(mpm_net net, int32_t op, int32_t nb, int32_t d, int32_t h, int32_t w, int32_t c,
                                    int32_t c2, const void* a, const void* b, void* out, void* out2) {
    Net* n = (Net*)net;
    const bool even = d % 2 == 0 && h % 2 == 0 && w % 2 == 0;
    if (!n || !a || !out || nb < 1 || d < 1 || h < 1 || w < 1 || c < 1 || op < MPM_OP_POOL || op > MPM_OP_PAD ||
        (op != MPM_OP_PAD && c % 8)) {
        set_error("mpm_net_debug_op: bad arguments");
        return MPM_EINVAL;
    }
    hipStream_t st = n->stream;
    const long long P = (long long)nb * d * h * w;
    const uint16_t* A = (const uint16_t*)a;
    const uint16_t* B = (const uint16_t*)b;
    uint16_t* O = (uint16_t*)out;
    switch (op) {
        case MPM_OP_POOL:
            if (!even) break;
            k_pool2<<<blocks_for(P / 8 * c / 8), 256, 0, st>>>(A, c, c, nb, d, h, w, O);
            return net_debug_finish(st);
        case MPM_OP_POOL_BWD_ADD:
            if (!even || (B && (c2 < c || c2 % 8))) break;
            k_pool2_bwd_add<<<blocks_for(P * c / 8), 256, 0, st>>>(A, c, B ? B + (c2 - c) : nullptr, c2, nb, d, h, w, O);
            return net_debug_finish(st);
        case MPM_OP_UP2_CAT:
            if (!even || !B || c2 < 8 || c2 % 8) break;
            k_up2_cat<<<blocks_for(P * (c + c2) / 8), 256, 0, st>>>(A, c, B, c2, nb, d, h, w, O);
            return net_debug_finish(st);
        case MPM_OP_UP2_BWD:
            if (!even || c2 < 0 || c2 % 8) break;
            k_up2_bwd<<<blocks_for(P / 8 * c / 8), 256, 0, st>>>(A, c + c2, c, nb, d / 2, h / 2, w / 2, O);
            return net_debug_finish(st);
        case MPM_OP_HEAD:
        case MPM_OP_HEAD_BWD: {
            const ConvL& hd = n->layers.back();
            if (c != 16 || hd.cin != 16) break;
            if (op == MPM_OP_HEAD) {
                k_head<<<blocks_for(P), 256, 0, st>>>(A, 16, n->theta + hd.woff, n->theta + hd.boff, hd.cout, P,
                                                    (float*)out);
                return net_debug_finish(st);
            }
            if (!B || !out2) break;
            // per-chunk partials as in the backward pass, reduced into out2 (zeroed here)
            const long long nchunk = std::max(1LL, std::min(256LL, P / 4096));
            const long long per = (P + nchunk - 1) / nchunk;
            const int npar = hd.cin * hd.cout + hd.cout;
            float* part = nullptr;
            MPM_HIP(hipMalloc(&part, (size_t)nchunk * npar * 4));
            hipError_t e = hipMemsetAsync(out2, 0, (size_t)npar * 4, st);
            if (e == hipSuccess) {
                k_head_bwd<<<(unsigned)nchunk, 256, 0, st>>>(A, 16, n->theta + hd.woff, hd.cout, (const float*)B, P, per,
                                                             O, part);
                k_param_reduce<<<blocks_for(npar), 256, 0, st>>>(part, (int)nchunk, npar, (float*)out2);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            (void)hipFree(part);
            if (e != hipSuccess) return hip_fail(e, "mpm_net_debug_op");
            return MPM_OK;
        }
        case MPM_OP_PAD:
            if (c2 < c || c2 % 8) break;
            k_pad_channels<<<blocks_for(P), 256, 0, st>>>(A, c, c2, P, O);
            return net_debug_finish(st);
    }
    set_error("mpm_net_debug_op: unsupported shape or channel counts for this operation");
    return MPM_EINVAL;
}
