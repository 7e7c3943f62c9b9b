// Host-side U-Net state (not visible through the C ABI).
#pragma once

#include <vector>

#include "common.h"

namespace mpm {

struct ConvL {
    int cin = 0, cout = 0, taps = 0;
    int cin_p = 0, cout_p = 0, kp = 0, kpd = 0;
    size_t woff = 0, boff = 0;         // offsets in the flat parameter vector
    uint16_t* wf = nullptr;            // BF16 forward weights, cout_p x kp values in fragment order
    uint16_t* wd = nullptr;            // BF16 input-gradient weights (W[26 - tap] transposed), cin_p x kpd
};

struct Net {
    int in_ch = 0, out_ch = 0, L = 0;
    std::vector<int> widths;
    std::vector<ConvL> layers;         // forward order; the last one is the 1x1x1 head
    size_t nparam = 0;
    float* theta = nullptr;            // FP32 master parameters
    float* grad = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    hipStream_t stream = nullptr;
    // buffers for the current input shape
    int dims[4] = {0, 0, 0, 0};        // n, D, H, W
    std::vector<void*> bufs;
    uint16_t* xin = nullptr;           // the input padded to cin_p channels (when in_ch < cin_p)
    const uint16_t* x0 = nullptr;      // what the first layer read in the last forward pass
    std::vector<uint16_t*> act, gin, pooled, cat, dcat;
    std::vector<int> lvl_of;
    uint16_t* ghead = nullptr;
    uint16_t* gscratch = nullptr;
    const uint16_t* head_in = nullptr;
    float* wpart = nullptr;
    size_t wpart_cap = 0;
    float* dpart = nullptr;
    size_t dpart_cap = 0;
    float* outbuf = nullptr;
    bool have_fwd = false;
    bool fwd_infer = false;            // the last forward pass was an inference pass
    bool fwd_listed = false;           // ... that computed listed tiles of the last level only
    // warm-start use
    double* mse_part = nullptr;        // pinned host copy of the MSE partial sums
    double* mse_dev = nullptr;         // device partial sums of the MSE
};

int net_build(Net* n, int in_ch, int out_ch, int levels, const int* widths, uint64_t seed);
int net_pack(Net* n);
void net_free(Net* n);
// Tiles of the last level an inference pass computes (device lists of tile entries, see
// ConvArgs::tlist): those of its first convolution (near) and of its second one and
// the head (domain).
struct TileLists {
    const int* near;
    int n_near;
    const int* domain;
    int n_domain;
};
// infer: an inference pass (the head fused into the last convolution where the widths
// allow; no backward pass may follow); with tiles (one sample, fused head), the last
// level computes only the listed tiles, so the output is valid on the domain tiles only.
int net_forward(Net* n, const uint16_t* in, int nb, int D, int H, int W, float* out, bool infer,
                const TileLists* tiles = nullptr);
int net_backward(Net* n, const float* dout);

}  // namespace mpm
