// Host-side solver context (not visible through the C ABI).
#pragma once

#include <map>
#include <string>
#include <vector>

#include "common.h"
#include "unet.h"

namespace mpm {

// One lattice problem: its box discretisation lives in buffers owned here and is
// addressed with problem-local indices (species * Npad + l).
struct ProbHost {
    bool ready = false;
    int dims[3] = {0, 0, 0};
    int lo[3] = {0, 0, 0};
    int hi[3] = {0, 0, 0};
    int N = 0;
    int Npad = 0;
    long long nvox = 0;
    double dt = 0.0, h = 0.0;
    double cb[MPM_MAX_SPECIES] = {0, 0, 0, 0};
    int* vox = nullptr;
    int4* nbr = nullptr;
    double* d64 = nullptr;
    double* q64 = nullptr;
    double* a64 = nullptr;
    double* sc64 = nullptr;
    float* c32 = nullptr;
    double* c64 = nullptr;
    size_t cap_pad = 0;        // padded unknowns per species the buffers hold (>= Npad)
    size_t hw_pad = 0;         // largest Npad written since the parts past it were zero
    // scratch of mpm_fv_setup, kept between calls (a box that changes every step
    // reuses it): per-row counts and starts, box-to-domain map, compacted voxels, total
    int* s_rowcnt = nullptr;
    int* s_rowstart = nullptr;
    int* s_boxmap = nullptr;
    int* s_vox = nullptr;
    int* s_total = nullptr;
    int* s_chunk = nullptr;            // per-chunk row totals of the scan
    size_t cap_rows = 0, cap_boxvox = 0, cap_svox = 0;
    // warm start: static network input channels on the box grid (k, D, s, mask)
    int gd[3] = {0, 0, 0};
    float* stat = nullptr;     // [3 S + 1][G] FP32, channel-major
    uint16_t* wsin = nullptr;  // BF16 network input [G][ws_channels(S)]
    float* wsout = nullptr;    // network output [G][S]
    size_t cap_grid = 0;       // grid voxels the three buffers above hold
    // tiles of the network's last level the warm start computes (16 x 4 x 4 voxels of the
    // grid, entries tx | ty << 10 | tz << 20): [0, tl_n[0]) those within one voxel of a
    // tile holding domain voxels (its first convolution), then the tl_n[1] tiles holding
    // domain voxels (its second convolution and the head); tl_n[0] < 0: no lists
    int* tl_dev = nullptr;
    int* tl_host = nullptr;    // pinned
    uint8_t* tf_dev = nullptr; // per-tile flags [2][tiles]
    uint8_t* tf_host = nullptr;  // pinned
    size_t cap_tiles = 0;
    int tl_n[2] = {-1, 0};
    bool ws_ready = false;     // wsin holds the static channels (and zero c and d off the
                               // domain) of the current grid, domain and scales (cleared
                               // by a set-up and by new scales)
};

// What a tuning result is kept for: species, basis word size, orthogonalisation,
// problems, and the size classes of the largest problem and of all unknowns.
struct TuneKey {
    int S, ks, ortho, P, cmax, ctot;
    bool operator<(const TuneKey& o) const {
        const int a[6] = {S, ks, ortho, P, cmax, ctot}, b[6] = {o.S, o.ks, o.ortho, o.P, o.cmax, o.ctot};
        for (int i = 0; i < 6; ++i)
            if (a[i] != b[i]) return a[i] < b[i];
        return false;
    }
};

struct Ctx {
    int S = 0, P = 0;
    mpm_options opt{};
    hipStream_t user_stream = nullptr;
    hipStream_t stream = nullptr;      // where the work goes: the caller's stream, or a private
                                       // one when cycles are captured into graphs
    bool own_stream = false;           // stream is private
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipEvent_t ev_status = nullptr;    // the status head has reached the host
    std::vector<ProbHost> probs;

    // global layout of the work vectors: problem p occupies
    // [off_p, off_p + S * Npad_p) starting at kLead.
    bool layout_dirty = true;
    bool coef_dirty = false;           // coefficients changed on a standing layout (mpm_fv_update)
    long long U = 0;                   // unknowns over all problems (padded)
    std::vector<long long> off;
    std::vector<Block> blocks;         // batched launch table (XCD-swizzled)
    std::vector<int> sys_first, sys_count;   // per-system slice of blocks_sys
    std::vector<Block> blocks_sys;     // per-system tables, concatenated
    std::vector<ProbDev> h_probs;      // host copy of the device descriptors
    std::vector<int> sys_tab_first;    // start of each system's table in blocks_sys
    int nslots = 0;
    int block_unknowns = 0;            // unknowns per block (autotuned or fixed)
    int axpy_group = 1;                // blocks of the batched table per block of the axpy table
    std::map<TuneKey, std::pair<long long, int>> tile_cache;   // autotuned split and axpy group

    // device buffers
    ProbDev* d_probs = nullptr;
    SysK* d_sk = nullptr;
    double* d_part = nullptr;
    Params* d_prm = nullptr;
    Block* d_blocks = nullptr;
    Block* d_blocks_sys = nullptr;
    std::vector<Block> blocks_ax;      // batched table of the delayed scheme's axpy kernel
    Block* d_blocks_ax = nullptr;
    int* d_sysfc = nullptr;            // [2][kMaxSys] first slot and block count per system
    double** d_fields = nullptr;
    size_t cap_blocks = 0, cap_slots = 0;
    void* V = nullptr;                 // (restart + 1) vectors of the Krylov type
    void* W = nullptr;
    double* x = nullptr;
    double* b = nullptr;
    long long ldv = 0;
    size_t cap_U = 0;

    // pinned host mirrors (up_valid: the device holds what they hold)
    double** h_fields = nullptr;
    Params* h_prm = nullptr;
    int* h_small = nullptr;            // pinned words read back by mpm_fv_setup
    bool up_valid = false;
    SysK* h_sk = nullptr;
    SysK* hsk_dev = nullptr;           // device address of h_sk (k_res_final writes the heads)

    // graphs of GMRES cycle segments, keyed by (first step, end step, tail kind)
    std::map<int, hipGraphExec_t> graphs;
    // Arnoldi steps taken by each cycle of the previous implicit step (the cycle is
    // first launched up to that length + kPredictMargin, then continued if needed)
    std::vector<int> cycle_len, cycle_len_next;

    std::vector<mpm_stats> stats;
    bool stepped = false;

    // warm start
    Net* net = nullptr;
    float* d_scales = nullptr;         // [kScaleCount]: input channel scales, then output scales
    float h_scales[kScaleCount] = {0};
    bool have_scales = false;
    double* d_lossp = nullptr;         // per-block partial sums of the warm-start loss
    double* h_lossp = nullptr;         // their pinned host copy
    size_t cap_lossp = 0;
    double* prev = nullptr;            // two halves on the global unknowns: c^{n-1} and
                                       // this step's c^n, which trade places every step
    size_t cap_prev = 0;
    size_t prev_n = 0;                 // elements in each half of prev
    int prev_half = 0;                 // the half that holds c^{n-1}
    bool have_prev = false;

    // kernel timing hook
    int time_kind = 0, time_j = 0, time_repeat = 1;
    std::vector<hipEvent_t> tev;       // start/stop pairs, one pair per timed launch
    int tev_used = 0;                  // pairs recorded in the current cycle
    double time_ms = 0.0, time_bytes = 0.0;
    long long time_launches = 0;
    std::vector<int> prev_cycles;
};

// setup.hip
int setup_problem(Ctx* c, int p, const int* dims, const int* lo, const int* hi,
                  const uint8_t* mask, const double* D, const double* k, const double* src,
                  const double* cb, double dt, double h);
void free_problem(ProbHost& ph);
int launch_diag_extremes(Ctx* c, int p);
int update_problem(Ctx* c, int p, const uint8_t* mask, const double* D, const double* k, const double* src,
                   const double* cb, double dt, double h);

// krylov.hip
int run_step(Ctx* c, double* const* fields, double tol);
int debug_apply(Ctx* c, int p, const double* x, double* y, int mode);
int debug_krylov(Ctx* c, int p, int sp, int kmax, int* mcount, double* vs, double* basis, double* hess);
int ensure_layout(Ctx* c);
int select_timing(Ctx* c, int kind, int j, int repeat);
int ws_pair(Ctx* c, int p, const double* c_prev, const double* c_old, const double* c_new, uint16_t* in_bf16,
            float* target);
// the network warm starts (network buffers on the box grid, mpm_attach_net)
inline bool net_warm_start(const Ctx* c) {
    return c->opt.warm_start == MPM_WS_NET || c->opt.warm_start == MPM_WS_NET_EXTRAP;
}
// the starts that keep c^{n-1}
inline bool extrap_warm_start(const Ctx* c) {
    return c->opt.warm_start == MPM_WS_EXTRAP || c->opt.warm_start == MPM_WS_NET_EXTRAP;
}
int ws_loss(Ctx* c, int p, const float* out, const float* target, float* grad, double* loss);

}  // namespace mpm
