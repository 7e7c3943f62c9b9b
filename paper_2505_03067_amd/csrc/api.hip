// C ABI of libmpm: argument checks, context lifetime and stream ordering.
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>

#include "context.h"

namespace mpm {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return MPM_EHIP;
}

static void destroy_ctx(Ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& ph : c->probs) free_problem(ph);
    for (auto& kv : c->graphs)
        if (kv.second) (void)hipGraphExecDestroy(kv.second);
    (void)hipFree(c->d_probs);
    (void)hipFree(c->d_sk);
    (void)hipFree(c->d_part);
    (void)hipFree(c->d_prm);
    (void)hipFree(c->d_blocks);
    (void)hipFree(c->d_blocks_sys);
    (void)hipFree(c->d_blocks_ax);
    (void)hipFree(c->d_sysfc);
    (void)hipFree(c->d_fields);
    (void)hipFree(c->V);
    (void)hipFree(c->W);
    (void)hipFree(c->x);
    (void)hipFree(c->b);
    if (c->h_fields) (void)hipHostFree(c->h_fields);
    if (c->h_prm) (void)hipHostFree(c->h_prm);
    if (c->h_small) (void)hipHostFree(c->h_small);
    if (c->h_sk) (void)hipHostFree(c->h_sk);
    if (c->h_lossp) (void)hipHostFree(c->h_lossp);
    (void)hipFree(c->d_lossp);
    (void)hipFree(c->d_scales);
    (void)hipFree(c->prev);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    if (c->ev_status) (void)hipEventDestroy(c->ev_status);
    for (auto e : c->tev) (void)hipEventDestroy(e);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// With a private stream (graph capture cannot run on the caller's stream, which may be
// the null stream), order it after the caller's stream (entry) and the caller's stream
// after it (exit).  Without one, the work is on the caller's stream already.
static int enter(Ctx* c) {
    if (!c->own_stream) return MPM_OK;
    MPM_HIP(hipEventRecord(c->ev_in, c->user_stream));
    MPM_HIP(hipStreamWaitEvent(c->stream, c->ev_in, 0));
    return MPM_OK;
}
static int leave(Ctx* c) {
    if (!c->own_stream) return MPM_OK;
    MPM_HIP(hipEventRecord(c->ev_out, c->stream));
    MPM_HIP(hipStreamWaitEvent(c->user_stream, c->ev_out, 0));
    return MPM_OK;
}

}  // namespace mpm

using namespace mpm;

extern "C" const char* mpm_last_error(void) { return g_err.c_str(); }

extern "C" int32_t mpm_default_options(mpm_options* opt) {
    if (!opt) {
        set_error("mpm_default_options: null pointer");
        return MPM_EINVAL;
    }
    std::memset(opt, 0, sizeof(*opt));
    opt->restart = 30;
    opt->max_cycles = 50;
    opt->precision = MPM_FP32_IR;
    opt->batched = 1;
    opt->use_graph = 0;
    opt->warm_start = MPM_WS_NONE;
    opt->tile_override = 0;
    opt->inner_rtol = 1e-6;
    opt->ortho = MPM_ORTHO_DCGS2;
    return MPM_OK;
}

extern "C" int32_t mpm_create(mpm_ctx* out, int32_t nspecies, int32_t nproblems, const mpm_options* opt,
                              void* stream) {
    if (!out) {
        set_error("mpm_create: null ctx pointer");
        return MPM_EINVAL;
    }
    *out = nullptr;
    if (nspecies < 1 || nspecies > MPM_MAX_SPECIES || nproblems < 1 || nspecies * nproblems > kMaxSys) {
        set_error("mpm_create: need 1 <= nspecies <= 4, nproblems >= 1 and nspecies * nproblems <= 64");
        return MPM_EINVAL;
    }
    mpm_options o;
    if (opt) o = *opt;
    else mpm_default_options(&o);
    if (o.restart < 1 || o.restart > MPM_MAX_RESTART || o.max_cycles < 1 ||
        (o.precision != MPM_FP64 && o.precision != MPM_FP32_IR) || !(o.inner_rtol >= 0.0 && o.inner_rtol < 1.0) ||
        o.warm_start < MPM_WS_NONE || o.warm_start > MPM_WS_NET_EXTRAP || o.tile_override < 0 ||
        (o.ortho != MPM_ORTHO_CGS2 && o.ortho != MPM_ORTHO_DCGS2) ||
        (o.tile_override % kAlign) != 0) {
        set_error("mpm_create: invalid options");
        return MPM_EINVAL;
    }
    Ctx* c = new Ctx();
    c->S = nspecies;
    c->P = nproblems;
    c->opt = o;
    c->user_stream = (hipStream_t)stream;
    c->probs.resize(nproblems);
    c->stats.assign((size_t)nspecies * nproblems, mpm_stats{});
    const int nsys = nspecies * nproblems;
    hipError_t e = hipSuccess;
    c->own_stream = o.use_graph != 0;
    if (c->own_stream) e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    else c->stream = c->user_stream;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_status, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&c->d_probs, nproblems * sizeof(ProbDev));
    if (e == hipSuccess) e = hipMalloc(&c->d_sk, nsys * sizeof(SysK));
    if (e == hipSuccess) e = hipMalloc(&c->d_prm, sizeof(Params));
    if (e == hipSuccess) e = hipMalloc(&c->d_sysfc, 2 * kMaxSys * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&c->d_scales, kScaleCount * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&c->d_fields, nproblems * sizeof(double*));
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_fields, nproblems * sizeof(double*), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_prm, sizeof(Params), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_small, 4 * sizeof(int), hipHostMallocDefault);
    // coherent: the status heads are written there by kernels and read by the host
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&c->h_sk, nsys * sizeof(SysK), hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&c->hsk_dev, c->h_sk, 0);
    if (e == hipSuccess) std::memset(c->h_sk, 0, nsys * sizeof(SysK));
    if (e == hipSuccess) e = hipMemset(c->d_sk, 0, nsys * sizeof(SysK));
    if (e != hipSuccess) {
        int r = hip_fail(e, "mpm_create");
        destroy_ctx(c);
        return r == MPM_EHIP && e == hipErrorOutOfMemory ? MPM_ENOMEM : r;
    }
    *out = (mpm_ctx)c;
    return MPM_OK;
}

extern "C" int32_t mpm_destroy(mpm_ctx ctx) {
    destroy_ctx((Ctx*)ctx);
    return MPM_OK;
}

extern "C" int32_t mpm_fv_setup(mpm_ctx ctx, int32_t problem, const int32_t* dims, const int32_t* lo,
                                const int32_t* hi, const uint8_t* mask, const double* D, const double* k,
                                const double* src, const double* c_dirichlet, double dt, double h) {
    Ctx* c = (Ctx*)ctx;
    if (!c || !dims || !lo || !hi || !mask || !D || !k || !src || !c_dirichlet) {
        set_error("mpm_fv_setup: null pointer");
        return MPM_EINVAL;
    }
    if (problem < 0 || problem >= c->P) {
        set_error("mpm_fv_setup: problem index out of range");
        return MPM_EINVAL;
    }
    for (int d = 0; d < 3; ++d) {
        if (dims[d] <= 0 || lo[d] < 0 || hi[d] > dims[d] || lo[d] >= hi[d]) {
            set_error("mpm_fv_setup: the box must be non-empty and inside the lattice");
            return MPM_EINVAL;
        }
    }
    if ((long long)dims[0] * dims[1] * dims[2] >= 0x7fffffffLL) {
        set_error("mpm_fv_setup: lattice too large for 32-bit voxel indices");
        return MPM_EINVAL;
    }
    if (!(dt > 0.0) || !(h > 0.0) || !std::isfinite(dt) || !std::isfinite(h)) {
        set_error("mpm_fv_setup: dt and h must be positive and finite");
        return MPM_EINVAL;
    }
    for (int s = 0; s < c->S; ++s) {
        if (!std::isfinite(c_dirichlet[s])) {
            set_error("mpm_fv_setup: non-finite Dirichlet value");
            return MPM_EINVAL;
        }
    }
    if (((uintptr_t)D | (uintptr_t)k | (uintptr_t)src) % 8 != 0) {
        set_error("mpm_fv_setup: coefficient arrays must be 8-byte aligned");
        return MPM_EINVAL;
    }
    int rc = enter(c);
    if (rc != MPM_OK) return rc;
    rc = setup_problem(c, problem, dims, lo, hi, mask, D, k, src, c_dirichlet, dt, h);
    if (rc == MPM_OK) rc = leave(c);
    return rc;
}

extern "C" int32_t mpm_fv_update(mpm_ctx ctx, int32_t problem, const uint8_t* mask, const double* D, const double* k,
                                 const double* src, const double* c_dirichlet, double dt, double h) {
    Ctx* c = (Ctx*)ctx;
    if (!c || !mask || !D || !k || !src || !c_dirichlet) {
        set_error("mpm_fv_update: null pointer");
        return MPM_EINVAL;
    }
    if (problem < 0 || problem >= c->P) {
        set_error("mpm_fv_update: problem index out of range");
        return MPM_EINVAL;
    }
    if (!(dt > 0.0) || !(h > 0.0) || !std::isfinite(dt) || !std::isfinite(h)) {
        set_error("mpm_fv_update: dt and h must be positive and finite");
        return MPM_EINVAL;
    }
    for (int s = 0; s < c->S; ++s) {
        if (!std::isfinite(c_dirichlet[s])) {
            set_error("mpm_fv_update: non-finite Dirichlet value");
            return MPM_EINVAL;
        }
    }
    if (((uintptr_t)D | (uintptr_t)k | (uintptr_t)src) % 8 != 0) {
        set_error("mpm_fv_update: coefficient arrays must be 8-byte aligned");
        return MPM_EINVAL;
    }
    int rc = enter(c);
    if (rc != MPM_OK) return rc;
    rc = update_problem(c, problem, mask, D, k, src, c_dirichlet, dt, h);
    if (rc == MPM_OK) rc = leave(c);
    return rc;
}

extern "C" int32_t mpm_implicit_step(mpm_ctx ctx, double* const* fields, double tol) {
    Ctx* c = (Ctx*)ctx;
    if (!c || !fields) {
        set_error("mpm_implicit_step: null pointer");
        return MPM_EINVAL;
    }
    if (!(tol > 0.0) || !std::isfinite(tol)) {
        set_error("mpm_implicit_step: tol must be positive");
        return MPM_EINVAL;
    }
    for (int p = 0; p < c->P; ++p) {
        if (!fields[p] || ((uintptr_t)fields[p] % 8) != 0) {
            set_error("mpm_implicit_step: null or misaligned field pointer");
            return MPM_EINVAL;
        }
    }
    auto t0 = std::chrono::steady_clock::now();
    int rc = enter(c);
    if (rc != MPM_OK) return rc;
    const int st = run_step(c, fields, tol);
    if (st < 0) return st;
    rc = leave(c);
    if (rc != MPM_OK) return rc;
    const float ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (auto& s : c->stats) s.ms_total = ms;
    c->stepped = true;
    if (st == MPM_NOT_CONVERGED) set_error("mpm_implicit_step: some system did not reach the tolerance");
    return st;
}

extern "C" int32_t mpm_gmres_stats(mpm_ctx ctx, int32_t problem, int32_t species, mpm_stats* out) {
    Ctx* c = (Ctx*)ctx;
    if (!c || !out || problem < 0 || problem >= c->P || species < 0 || species >= c->S) {
        set_error("mpm_gmres_stats: bad arguments");
        return MPM_EINVAL;
    }
    if (!c->stepped) {
        set_error("mpm_gmres_stats: no step has run yet");
        return MPM_ESTATE;
    }
    // filled on the host when mpm_implicit_step returned: nothing to wait for
    *out = c->stats[(size_t)problem * c->S + species];
    return MPM_OK;
}

extern "C" int32_t mpm_debug_apply(mpm_ctx ctx, int32_t problem, const double* x_lattice, double* y_lattice,
                                   int32_t mode) {
    Ctx* c = (Ctx*)ctx;
    if (!c || !x_lattice || !y_lattice || problem < 0 || problem >= c->P || mode < 0 || mode > 2) {
        set_error("mpm_debug_apply: bad arguments");
        return MPM_EINVAL;
    }
    int rc = enter(c);
    if (rc != MPM_OK) return rc;
    rc = debug_apply(c, problem, x_lattice, y_lattice, mode);
    if (rc == MPM_OK) rc = leave(c);
    return rc;
}

extern "C" int32_t mpm_debug_krylov(mpm_ctx ctx, int32_t problem, int32_t species, int32_t kmax, int32_t* mcount,
                                    double* vs, double* basis, double* hess) {
    Ctx* c = (Ctx*)ctx;
    if (!c || !mcount || !vs || !basis || !hess || problem < 0 || problem >= c->P || species < 0 ||
        species >= c->S || kmax < 1 || kmax > c->opt.restart) {
        set_error("mpm_debug_krylov: bad arguments");
        return MPM_EINVAL;
    }
    return debug_krylov(c, problem, species, kmax, mcount, vs, basis, hess);
}

extern "C" int32_t mpm_time_kernel(mpm_ctx ctx, int32_t kind, int32_t j, int32_t repeat) {
    Ctx* c = (Ctx*)ctx;
    if (!c || kind < MPM_KERNEL_NONE || kind > MPM_KERNEL_RESIDUAL || j < 0 || j >= c->opt.restart ||
        repeat < 1 || repeat > 64) {
        set_error("mpm_time_kernel: bad arguments");
        return MPM_EINVAL;
    }
    if (kind == MPM_KERNEL_AXPY_NORM && c->opt.ortho == MPM_ORTHO_DCGS2) {
        set_error("mpm_time_kernel: the delayed Gram-Schmidt cycle has no axpy+norm kernel");
        return MPM_EINVAL;
    }
    const bool pure = kind == MPM_KERNEL_RESIDUAL || (kind == MPM_KERNEL_SPMV_DOT && c->opt.ortho == MPM_ORTHO_DCGS2);
    if (repeat > 1 && !pure) {
        set_error("mpm_time_kernel: repeat > 1 needs a kernel whose output depends on its inputs alone");
        return MPM_EINVAL;
    }
    return select_timing(c, kind, j, repeat);
}

extern "C" int32_t mpm_kernel_timing(mpm_ctx ctx, double* ms, int64_t* launches, double* bytes) {
    Ctx* c = (Ctx*)ctx;
    if (!c || !ms || !launches || !bytes) {
        set_error("mpm_kernel_timing: null pointer");
        return MPM_EINVAL;
    }
    *ms = c->time_ms;
    *launches = c->time_launches;
    *bytes = c->time_bytes;
    return MPM_OK;
}

extern "C" int32_t mpm_tile(mpm_ctx ctx, int32_t* out) {
    Ctx* c = (Ctx*)ctx;
    if (!c || !out) {
        set_error("mpm_tile: null pointer");
        return MPM_EINVAL;
    }
    if (c->layout_dirty || c->block_unknowns <= 0) {
        set_error("mpm_tile: no work split yet");
        return MPM_ESTATE;
    }
    *out = c->block_unknowns;
    return MPM_OK;
}

static int set_scales(Ctx* c, const float* in_scale, const float* out_scale) {
    const int cin = ws_channels(c->S);
    float h[kScaleCount] = {};
    for (int i = 0; i < cin; ++i) h[i] = in_scale[i];
    for (int s = 0; s < c->S; ++s) h[kScaleOut + s] = out_scale[s];
    // new values: the network input buffers are built again in full at the next warm start
    if (!c->have_scales || std::memcmp(h, c->h_scales, sizeof(h)) != 0)
        for (auto& ph : c->probs) ph.ws_ready = false;
    std::memcpy(c->h_scales, h, sizeof(h));
    MPM_HIP(hipMemcpy(c->d_scales, c->h_scales, kScaleCount * sizeof(float), hipMemcpyHostToDevice));
    c->have_scales = true;
    return MPM_OK;
}

extern "C" int32_t mpm_attach_net(mpm_ctx ctx, mpm_net net, const float* in_scale, const float* out_scale) {
    Ctx* c = (Ctx*)ctx;
    Net* n = (Net*)net;
    if (!c || !in_scale || !out_scale) {
        set_error("mpm_attach_net: null pointer");
        return MPM_EINVAL;
    }
    if (n && (n->in_ch != ws_channels(c->S) || n->out_ch != c->S)) {
        set_error("mpm_attach_net: the network must read 5 S + 1 channels and write S");
        return MPM_EINVAL;
    }
    if (!net_warm_start(c)) {
        set_error("mpm_attach_net: the context was not created with a network warm start");
        return MPM_ESTATE;
    }
    int rc = set_scales(c, in_scale, out_scale);
    if (rc != MPM_OK) return rc;
    c->net = n;
    return MPM_OK;
}

static int32_t ws_pair_call(const char* name, mpm_ctx ctx, int32_t problem, const double* c_prev, const double* c_old,
                            const double* c_new, const float* in_scale, const float* out_scale, uint16_t* in_bf16,
                            float* target) {
    Ctx* c = (Ctx*)ctx;
    if (!c || !c_old || !c_new || !in_scale || !out_scale || !in_bf16 || !target || problem < 0 || problem >= c->P) {
        set_error(std::string(name) + ": bad arguments");
        return MPM_EINVAL;
    }
    if (!net_warm_start(c) || !c->probs[problem].ready) {
        set_error(std::string(name) + ": needs a context with a network warm start and a set-up problem");
        return MPM_ESTATE;
    }
    int rc = set_scales(c, in_scale, out_scale);
    if (rc != MPM_OK) return rc;
    rc = enter(c);
    if (rc != MPM_OK) return rc;
    rc = ws_pair(c, problem, c_prev, c_old, c_new, in_bf16, target);
    if (rc == MPM_OK) rc = leave(c);
    return rc;
}

extern "C" int32_t mpm_ws_pair(mpm_ctx ctx, int32_t problem, const double* c_old, const double* c_new,
                               const float* in_scale, const float* out_scale, uint16_t* in_bf16, float* target) {
    return ws_pair_call("mpm_ws_pair", ctx, problem, nullptr, c_old, c_new, in_scale, out_scale, in_bf16, target);
}

extern "C" int32_t mpm_ws_pair_extrap(mpm_ctx ctx, int32_t problem, const double* c_prev, const double* c_old,
                                      const double* c_new, const float* in_scale, const float* out_scale,
                                      uint16_t* in_bf16, float* target) {
    if (!c_prev) {
        set_error("mpm_ws_pair_extrap: bad arguments");
        return MPM_EINVAL;
    }
    return ws_pair_call("mpm_ws_pair_extrap", ctx, problem, c_prev, c_old, c_new, in_scale, out_scale, in_bf16,
                        target);
}

extern "C" int32_t mpm_ws_loss(mpm_ctx ctx, int32_t problem, const float* out, const float* target,
                               const float* out_scale, float* grad_out, double* loss) {
    Ctx* c = (Ctx*)ctx;
    if (!c || !out || !target || !out_scale || !grad_out || !loss || problem < 0 || problem >= c->P) {
        set_error("mpm_ws_loss: bad arguments");
        return MPM_EINVAL;
    }
    if (!net_warm_start(c) || !c->probs[problem].ready) {
        set_error("mpm_ws_loss: needs a context with a network warm start and a set-up problem");
        return MPM_ESTATE;
    }
    for (int s = 0; s < c->S; ++s) {
        if (!(out_scale[s] > 0.f) || !std::isfinite(out_scale[s])) {
            set_error("mpm_ws_loss: output scales must be positive");
            return MPM_EINVAL;
        }
    }
    // the output scales go where the warm-start kernels read them; the input scales stay
    for (int s = 0; s < c->S; ++s) c->h_scales[kScaleOut + s] = out_scale[s];
    MPM_HIP(hipMemcpy(c->d_scales, c->h_scales, kScaleCount * sizeof(float), hipMemcpyHostToDevice));
    int rc = enter(c);
    if (rc != MPM_OK) return rc;
    rc = ws_loss(c, problem, out, target, grad_out, loss);
    if (rc == MPM_OK) rc = leave(c);
    return rc;
}

extern "C" int32_t mpm_ws_grid(mpm_ctx ctx, int32_t problem, int32_t* grid) {
    Ctx* c = (Ctx*)ctx;
    if (!c || !grid || problem < 0 || problem >= c->P) {
        set_error("mpm_ws_grid: bad arguments");
        return MPM_EINVAL;
    }
    if (!c->probs[problem].ready || c->probs[problem].gd[0] == 0) {
        set_error("mpm_ws_grid: no warm-start grid (set up the problem in a context with a network warm start)");
        return MPM_ESTATE;
    }
    for (int d = 0; d < 3; ++d) grid[d] = c->probs[problem].gd[d];
    return MPM_OK;
}
