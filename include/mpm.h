/*
 * libmpm - implicit-Euler finite-volume reaction-diffusion on a tumour bounding box,
 * solved by restarted GMRES on one AMD MI355X (gfx950).
 *
 * What is computed (paper: Sec. 2.2 eqs. 1-4, Sec. 2.3, Sec. 2.4).  Each species obeys
 * dc/dt = div(D grad c) - k c + s on the domain voxels (mask = 1) inside a box around
 * the tumour cells.  One step of cell-centred finite volumes with first-order implicit
 * Euler gives, for every domain voxel P with faces f toward neighbours Q,
 *     A_PP = 1 + dt k_P + dt sum_f G_f,   A_PQ = -dt G_f,
 *     b_P  = c^n_P + dt s_P + dt sum_{box faces f} G_f c_b,
 * with G_f = D_f / h^2, D_f = 2 D_P D_Q / (D_P + D_Q) (0 if both are 0) between two
 * domain voxels, G_f = 0 toward a voxel outside the mask, and G_f = 2 D_P / h^2 on a
 * box face, where the Dirichlet value c_b sits half a voxel away.  c^{n+1} = A^{-1} b
 * is written back onto the domain voxels of the box; every other lattice voxel keeps
 * its value.  The solve is restarted GMRES (Sec. 2.4) with Jacobi scaling, classical
 * Gram-Schmidt with one reorthogonalisation, and an FP64 stopping test on the true
 * residual ||b - A x||_2 / ||b||_2 per (problem, species).
 *
 * Conventions for every call:
 *  - Lattice arrays are C-ordered [z][y][x] (x fastest); multi-species lattice arrays
 *    are [S][z][y][x].  Sizes, corners and coordinates are (x, y, z) triples.
 *  - Boxes are half-open [lo, hi) per axis and lie inside the lattice.
 *  - "device" pointers are HIP device memory on the current device (for example the
 *    data_ptr() of a torch tensor); "host" pointers are ordinary CPU memory.
 *  - The caller owns every array it passes; the library keeps no pointer past the
 *    call, except the network attached with mpm_attach_net.  The library owns its
 *    own workspace and frees it in mpm_destroy / mpm_net_destroy.
 *  - 'stream' is a hipStream_t passed as void* (0 = the null stream).  All work of a
 *    context is ordered after the work already queued on that stream and before
 *    work queued on it after the call returns.
 *  - Every call returns an mpm status (int32).  Negative values are errors, the
 *    outputs are then unspecified; mpm_last_error() gives a message for the calling
 *    thread.  MPM_NOT_CONVERGED is a warning: outputs hold the best iterate.
 *  - A context is used by one host thread at a time.
 */
#ifndef MPM_H
#define MPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MPM_OK 0
#define MPM_NOT_CONVERGED 1 /* warning: fields hold the best iterate, stats are filled */
#define MPM_EINVAL (-1)     /* bad argument: sizes, box, coefficients, tolerance, pointers */
#define MPM_ENOMEM (-2)     /* device allocation failed */
#define MPM_EHIP (-3)       /* a HIP runtime call failed */
#define MPM_EEMPTY (-4)     /* no tumour voxel, or a box without any domain voxel */
#define MPM_ESTATE (-5)     /* call out of order (e.g. a step before mpm_fv_setup) */

/* precision of the Krylov inner solve */
#define MPM_FP64 0    /* FP64 everywhere (plain GMRES) */
#define MPM_FP32_IR 1 /* FP32 Krylov basis and stencil inside FP64 iterative refinement */

/* initial guess of each step */
#define MPM_WS_NONE 0   /* start from c^n */
#define MPM_WS_NET 1    /* learned warm start from the attached network, fallback c^n */
#define MPM_WS_EXTRAP 2 /* linear extrapolation 2 c^n - c^{n-1}, fallback c^n */
#define MPM_WS_NET_EXTRAP 3 /* the attached network's correction of the extrapolated start,
                               fallback c^n; no warm start while c^{n-1} is unknown */

/* orthogonalisation of the Arnoldi basis */
#define MPM_ORTHO_CGS2 0
#define MPM_ORTHO_DCGS2 1

#define MPM_MAX_SPECIES 4
#define MPM_MAX_RESTART 30

typedef struct mpm_ctx_s* mpm_ctx;

typedef struct {
    int32_t restart;     /* GMRES restart length m, 1..MPM_MAX_RESTART (default 30) */
    int32_t max_cycles;  /* restart cycles allowed per step (default 50) */
    int32_t precision;   /* MPM_FP64 or MPM_FP32_IR (default MPM_FP32_IR) */
    int32_t batched;     /* 1: every (problem, species) system in each launch (default);
                            0: one system after another */
    int32_t use_graph;   /* 1: replay each GMRES cycle from a captured hipGraph; 0 (default):
                            launch the kernels directly (measured at least as fast on MI355X
                            on every workload tried: each kernel runs longer than its launch) */
    int32_t warm_start;  /* MPM_WS_NONE, MPM_WS_NET, MPM_WS_EXTRAP or MPM_WS_NET_EXTRAP */
    int32_t tile_override; /* 0: autotuned work split; >0: unknowns per block (multiple of 1024) */
    int32_t ortho;       /* MPM_ORTHO_DCGS2 (default): classical Gram-Schmidt with delayed
                            reorthogonalisation, one global reduction and two passes per step;
                            MPM_ORTHO_CGS2: reorthogonalised classical Gram-Schmidt, three */
    double inner_rtol;   /* smallest residual reduction asked of one FP32 cycle (default 1e-6) */
} mpm_options;

typedef struct {
    int32_t iterations;      /* Arnoldi steps in the last mpm_implicit_step */
    int32_t cycles;          /* restart cycles (= refinement sweeps in MPM_FP32_IR) */
    int32_t refinements;     /* FP64 residual evaluations after the first */
    int32_t converged;       /* 1 if ||b - A x|| <= tol ||b|| */
    int32_t warm_start_used; /* 1 if the warm start was accepted */
    int32_t fallback;        /* 1 if a warm start was tried and rejected */
    double rel_res_initial;  /* ||b - A c^n|| / ||b|| */
    double rel_res_warm;     /* ||b - A x0|| / ||b|| of the warm start (0 if none) */
    double rel_res_final;    /* true FP64 relative residual of the returned fields */
    float ms_total;          /* wall time of the last mpm_implicit_step call */
    int32_t reserved;
} mpm_stats;

/* Bounding box of all tumour cells plus a margin (Sec. 2.3).
 * cell_id: device int32 [z][y][x]; a voxel belongs to a cell when its value is > 0.
 * dims: host (nx, ny, nz).  On return lo/hi (host, 3 each) hold the half-open box
 * lo_d = max(min_d - margin, 0), hi_d = min(max_d + margin + 1, n_d).
 * Synchronises 'stream'.  MPM_EEMPTY if no voxel is positive; MPM_EINVAL for
 * non-positive dims, negative margin or a null pointer.  The first call on a device
 * allocates 24.6 KB of device memory (per-block partial extremes) and 32 bytes of
 * pinned host memory, kept until the process ends; calls from several threads are
 * serialised. */
int32_t mpm_bbox_from_cells(const int32_t* cell_id, const int32_t* dims, int32_t margin,
                            int32_t* lo, int32_t* hi, void* stream);

/* mpm_bbox_from_cells for callers that cannot allocate memory (code between graph
 * launches in a tight loop, harnesses that forbid allocation): the same arguments,
 * kernels and result, but no call allocates anything.  Its scratch is a fixed
 * 24,608-byte array in device memory (the six folded extremes and the partial extremes
 * of the 1,024 blocks of the streaming pass), which the library holds on every device it
 * runs on until the process ends; its size does not depend on the lattice, so every
 * lattice mpm_bbox_from_cells accepts fits.  The result reaches the host through a copy
 * into the caller's lo/hi (pageable memory).  Every call on a device shares that
 * device's array and overwrites all of it that it reads, so no clearing is needed;
 * calls that overlap on one device (from several threads or streams) race on it and
 * must be serialised by the caller.  Synchronises 'stream'; the same error codes. */
int32_t mpm_bbox_from_cells_noalloc(const int32_t* cell_id, const int32_t* dims, int32_t margin,
                                    int32_t* lo, int32_t* hi, void* stream);

/* Fill *opt with the defaults listed in mpm_options. */
int32_t mpm_default_options(mpm_options* opt);

/* Create a solver context for 'nproblems' independent lattices, each carrying
 * 'nspecies' (1..MPM_MAX_SPECIES) uncoupled species.  opt may be NULL (defaults).
 * The context runs its work on 'stream'. */
int32_t mpm_create(mpm_ctx* ctx, int32_t nspecies, int32_t nproblems, const mpm_options* opt,
                   void* stream);

/* Discretise problem 'problem' on 'box' (Sec. 2.3-2.4).  Re-call whenever the box or
 * the coefficients change; fields live on the lattice, so a new box needs no remap.
 * dims: host (nx, ny, nz) of the lattice; lo/hi: host box corners.
 * mask: device uint8 [z][y][x] (1 = domain voxel).  D, k, src: device FP64
 * [S][z][y][x], lattice-sized (diffusivity >= 0, rate >= 0, production).
 * c_dirichlet: host FP64 [S], the value on the box faces.  dt > 0, h > 0.
 * The input arrays are read before the call returns (the stream is synchronised).
 * MPM_EINVAL for bad sizes, a box outside the lattice, negative D or k, dt <= 0 or
 * h <= 0; MPM_EEMPTY if the box holds no domain voxel. */
int32_t mpm_fv_setup(mpm_ctx ctx, int32_t problem, const int32_t* dims, const int32_t* lo,
                     const int32_t* hi, const uint8_t* mask, const double* D, const double* k,
                     const double* src, const double* c_dirichlet, double dt, double h);

/* New coefficients for problem 'problem' on the box of its last mpm_fv_setup: the
 * paper re-tracks the box only every 50 Monte Carlo steps (Sec. 2.3), while the cells,
 * and with them k and s, change every step.  The caller guarantees that the box and
 * the mask's domain voxels inside it are those of the last mpm_fv_setup (mask is read
 * for the zero-flux faces); D, k, src, c_dirichlet, dt, h as in mpm_fv_setup.  The
 * compaction, the neighbour table, the launch layout, the tuned work split and the
 * previous step's cycle lengths are kept; only the couplings, the diagonal, the
 * right-hand-side terms and the Jacobi scaling are recomputed.  Synchronises the
 * stream.  MPM_ESTATE before the first mpm_fv_setup of the problem; MPM_EINVAL as in
 * mpm_fv_setup. */
int32_t mpm_fv_update(mpm_ctx ctx, int32_t problem, const uint8_t* mask, const double* D, const double* k,
                      const double* src, const double* c_dirichlet, double dt, double h);

/* One implicit-Euler step of every problem and species (Sec. 2.4).
 * fields: host array [nproblems] of device FP64 [S][z][y][x] lattice fields; read as
 * c^n and overwritten with c^{n+1} on the domain voxels of each box.
 * tol > 0: relative FP64 residual to reach per (problem, species).
 * Returns once the outcome of every system is known (the statistics are final); the
 * writing of c^{n+1} into fields may still be running, ordered before the work the
 * caller enqueues afterwards on the stream given to mpm_create (with use_graph, the
 * context runs on a private stream which that stream is made to wait for).  At the end of each GMRES cycle the
 * calling thread reads the state of every system, which the GPU writes into pinned
 * host memory; it waits for it by polling for up to 5 ms, then blocks.  Returns MPM_NOT_CONVERGED if some
 * system did not reach tol within max_cycles (the best iterate is written). */
int32_t mpm_implicit_step(mpm_ctx ctx, double* const* fields, double tol);

/* Statistics of the last step for one (problem, species) system (host output): how the
 * solve ended, so that the caller can verify that every system completed before the
 * fields are handed on to the cell model (the paper's main process checks the
 * completion of the solve before distributing its result, Sec. 2.5).  Does not
 * synchronise: the values are final when mpm_implicit_step returns.  MPM_ESTATE
 * before the first step, MPM_EINVAL for an index out of range or a null pointer. */
int32_t mpm_gmres_stats(mpm_ctx ctx, int32_t problem, int32_t species, mpm_stats* out);

/* Free the context and all its device memory. */
int32_t mpm_destroy(mpm_ctx ctx);

/* Message for the last non-OK status returned on the calling thread. */
const char* mpm_last_error(void);

/* Measurement hook: time every launch of one kernel of the GMRES cycle with HIP
 * events recorded on the stream the kernels run on.
 * kind: MPM_KERNEL_NONE (off), MPM_KERNEL_SPMV_DOT (stencil + multi-dot: the first
 * Gram-Schmidt pass, or all dot products of the delayed scheme), MPM_KERNEL_AXPY_DOT
 * (second pass; the delayed scheme's axpy kernel), MPM_KERNEL_AXPY_NORM (third pass;
 * CGS2 only, MPM_EINVAL under MPM_ORTHO_DCGS2), MPM_KERNEL_UPDATE (x += S V y),
 * MPM_KERNEL_RESIDUAL (FP64 r = b - A x); j: Arnoldi step of kinds 1-3, ignored
 * otherwise.  repeat >= 1: each timed launch is issued 'repeat' times back to back
 * between its two events (amortises the event overhead); repeat > 1 is accepted only
 * for launches whose output depends on their inputs alone (the delayed scheme's
 * stencil + multi-dot kernel, and the residual kernel), else MPM_EINVAL.  While a
 * kernel is timed the cycle is launched directly instead of from graphs.  Selecting
 * resets the counters read by mpm_kernel_timing. */
#define MPM_KERNEL_NONE 0
#define MPM_KERNEL_SPMV_DOT 1
#define MPM_KERNEL_AXPY_DOT 2
#define MPM_KERNEL_AXPY_NORM 3
#define MPM_KERNEL_UPDATE 4
#define MPM_KERNEL_RESIDUAL 5
int32_t mpm_time_kernel(mpm_ctx ctx, int32_t kind, int32_t j, int32_t repeat);

/* Totals since mpm_time_kernel: summed event time in ms, number of launches (each
 * repeat counts), and the algorithmic bytes those launches had to move for the
 * systems that were active (domain unknowns only, padding excluded; counted per
 * unknown as stencil + multi-dot: t (j + 5) + 16 / S, CGS2 passes 2 and 3: t (j + 3),
 * delayed-scheme axpy: 3 t (j = 0) or t (j + 4), update: t m + 24, residual:
 * 56 + t + 16 / S, with t = 4 (MPM_FP32_IR) or 8 (MPM_FP64) bytes).  All outputs
 * are host pointers. */
int32_t mpm_kernel_timing(mpm_ctx ctx, double* ms, int64_t* launches, double* bytes);

/* Unknowns per block of the current work split (after autotuning, if any); *out is a
 * host int.  MPM_ESTATE before the first step or mpm_debug_apply. */
int32_t mpm_tile(mpm_ctx ctx, int32_t* out);

/* Measurement hook: the bandwidth a plain streaming kernel sustains, as the practical
 * ceiling beside the datasheet peak.  kind: MPM_PROBE_READ (sum of 'bytes' of a; c
 * receives one float per block), MPM_PROBE_COPY (c = a, 'bytes' each), MPM_PROBE_TRIAD
 * (c = a + 3 b as floats, 'bytes' each), optionally | MPM_PROBE_NONTEMPORAL
 * (nontemporal loads for READ, nontemporal stores otherwise).  a, b, c: device, 16-byte
 * aligned; bytes a positive multiple of 16; 256-thread blocks, 'blocks' of them, grid-
 * stride loops over 16-byte words.  One untimed launch, then 'repeat' launches between
 * two HIP events on 'stream'; *ms (host) = their average duration.  Bytes moved per
 * launch: bytes (READ), 2 bytes (COPY), 3 bytes (TRIAD).  Synchronises 'stream'. */
#define MPM_PROBE_READ 0
#define MPM_PROBE_COPY 1
#define MPM_PROBE_TRIAD 2
#define MPM_PROBE_NONTEMPORAL 0x100
int32_t mpm_hbm_probe(int32_t kind, const void* a, const void* b, void* c, int64_t bytes, int32_t blocks,
                      int32_t repeat, void* stream, double* ms);

/* ---- learned warm start: a 3-D U-Net on the box grid ----------------------------
 * Not part of the paper; its shape is this project's specification: 'levels' levels of
 * widths[l] channels (16, 32, 48 or 64; widths[0] = 16), two 3x3x3 convolutions + ReLU
 * per level, 2x2x2 average pooling between encoder levels, nearest x2 upsampling and
 * [upsampled, skip] concatenation in the decoder, and a 1x1x1 head.  Convolution
 * weights are W[tap][c_in][c_out] (tap = (dz+1)*9 + (dy+1)*3 + (dx+1)) followed by
 * the bias, layer by layer in forward order, FP32 master copies; compute is BF16 on
 * the matrix cores with FP32 accumulation.  Tensors are NDHWC ([n][z][y][x][c]),
 * device memory, all work on 'stream'. */
typedef struct mpm_net_s* mpm_net;

/* Create a network with He-normal weights drawn from 'seed' (host-side generator).
 * 1 <= in_ch <= 32 (16 for the warm start of three species, 21 for four), 1 <= out_ch <= 4,
 * 1 <= levels <= 6; MPM_EINVAL otherwise or for widths outside the list above. */
int32_t mpm_net_create(mpm_net* net, int32_t in_ch, int32_t out_ch, int32_t levels, const int32_t* widths,
                       uint64_t seed, void* stream);
/* Device pointers to the FP32 parameters and gradients (owned by the net) and their
 * count.  After writing parameters directly, call mpm_net_sync_weights. */
int32_t mpm_net_params(mpm_net net, float** params, float** grads, int64_t* count);
int32_t mpm_net_sync_weights(mpm_net net);
/* Copy all FP32 parameters (what = 0) or gradients (what = 1) between the net and a
 * caller device buffer of the parameter count.  Writing parameters refreshes the BF16
 * copies. */
int32_t mpm_net_read(mpm_net net, int32_t what, float* dst);
int32_t mpm_net_write(mpm_net net, int32_t what, const float* src);
/* in: device BF16 [n][d][h][w][in_ch]; out: device FP32 [n][d][h][w][out_ch]; d, h, w
 * multiples of 2^(levels-1).  Keeps the activations for mpm_net_backward.  When in_ch is
 * a multiple of 16 the input is read in place, so it must stay unchanged until the
 * backward pass; otherwise it is copied into a padded buffer. */
int32_t mpm_net_forward(mpm_net net, const uint16_t* in, int32_t n, int32_t d, int32_t h, int32_t w, float* out);
/* The same forward pass for inference (what the warm start runs): out is bit for bit
 * that of mpm_net_forward, but when the last 3x3x3 layer maps 16 channels to 16 the
 * head runs in its epilogue and that layer's output is not stored, so no
 * mpm_net_backward may follow (MPM_ESTATE) until the next mpm_net_forward.  Arguments
 * and errors as mpm_net_forward. */
int32_t mpm_net_infer(mpm_net net, const uint16_t* in, int32_t n, int32_t d, int32_t h, int32_t w, float* out);
/* Accumulate parameter gradients for dL/d(out) = grad_out (device FP32, shape of out). */
int32_t mpm_net_backward(mpm_net net, const float* grad_out);
int32_t mpm_net_zero_grad(mpm_net net);
/* Mean squared error of 'count' FP32 values: *loss (host) and grad_out = dL/d(out)
 * (device).  Synchronises the stream. */
int32_t mpm_net_mse(mpm_net net, const float* out, const float* target, int64_t count, float* grad_out,
                    double* loss);
/* One Adam step (t counts from 1) on the master parameters; refreshes the BF16 copies. */
int32_t mpm_net_adam_step(mpm_net net, float lr, float b1, float b2, float eps, int32_t t);
int32_t mpm_net_destroy(mpm_net net);

/* Test hook: one 3x3x3 layer of the net on caller tensors (device, NDHWC, one level's
 * shape n x d x h x w).  mode 0: out = conv(x) + bias (no ReLU), out FP32 [..][cout];
 * mode 1: out = input gradient of g * (gate > 0), FP32 [..][cin];
 * mode 2: out = weight gradient sum_p x[p + off] g[p] * (gate > 0), FP32 [27][cin][cout].
 * x: BF16 [..][cin rounded up to 16] (zero in the padding channels); g, gate: BF16
 * [..][cout] (gate may be NULL).  Leaves the net's accumulated gradients unchanged. */
int32_t mpm_net_debug_layer(mpm_net net, int32_t layer, int32_t mode, int32_t n, int32_t d, int32_t h,
                            int32_t w, const uint16_t* x, const uint16_t* g, const uint16_t* gate, float* out);

/* Test hook: copy a BF16 tensor the network stored in its last forward (and backward)
 * pass into dst (device, *count 16-bit values).  With dst = NULL only *count is set to
 * the element count; otherwise *count must equal it.  Tensors (index in brackets; all
 * NDHWC on the grid of their level):
 *  MPM_NT_INPUT       the input as the first layer read it, padded to a multiple of
 *                     16 channels (index ignored);
 *  MPM_NT_ACT [i]     output of 3x3x3 layer i after the ReLU (forward order);
 *  MPM_NT_ACT_GRAD [i] gradient with respect to that output (after mpm_net_backward;
 *                     for the last 3x3x3 layer see MPM_NT_HEAD_GRAD);
 *  MPM_NT_POOLED [l]  pooled input of encoder level l >= 1;
 *  MPM_NT_CAT [l]     [upsampled deeper output, skip] of decoder level l (built in the
 *                     backward pass), MPM_NT_CAT_GRAD [l] its gradient;
 *  MPM_NT_HEAD_GRAD   gradient with respect to the head's input.
 * MPM_EINVAL for an index out of range or a wrong count, MPM_ESTATE before any forward
 * pass.  Synchronises the network's stream. */
#define MPM_NT_INPUT 0
#define MPM_NT_ACT 1
#define MPM_NT_ACT_GRAD 2
#define MPM_NT_POOLED 3
#define MPM_NT_CAT 4
#define MPM_NT_CAT_GRAD 5
#define MPM_NT_HEAD_GRAD 6
int32_t mpm_net_debug_tensor(mpm_net net, int32_t kind, int32_t index, uint16_t* dst, int64_t* count);

/* Test hook: run one data-movement kernel of the network on caller tensors (device,
 * NDHWC, BF16 unless stated).  (n, d, h, w) is the finer grid, c and c2 channel counts
 * (multiples of 8 except the input of MPM_OP_PAD):
 *  MPM_OP_POOL         out [n][d/2][h/2][w/2][c] = mean of the 8 children in a [..][c];
 *  MPM_OP_POOL_BWD_ADD out [n][d][h][w][c] = a[parent][c] / 8 + the last c of the c2
 *                      channels of b (b may be NULL: no sum);
 *  MPM_OP_UP2_CAT      out [n][d][h][w][c + c2] = [nearest x2 upsampling of a (c
 *                      channels at half resolution), b (c2 channels)];
 *  MPM_OP_UP2_BWD      out [n][d/2][h/2][w/2][c] = sum over the 8 children of the first c
 *                      of the c + c2 channels of a;
 *  MPM_OP_HEAD         out FP32 [P][out_ch] = the net's 1x1x1 head on a [P][16] (c = 16);
 *  MPM_OP_HEAD_BWD     b: FP32 [P][out_ch] output gradient; out = input gradient [P][16],
 *                      out2 = FP32 head weight and bias gradient [16 out_ch + out_ch];
 *  MPM_OP_PAD          out [P][c2] = a [P][c] padded with zero channels.
 * d, h, w even for the pooling and upsampling operations.  Synchronises. */
#define MPM_OP_POOL 0
#define MPM_OP_POOL_BWD_ADD 1
#define MPM_OP_UP2_CAT 2
#define MPM_OP_UP2_BWD 3
#define MPM_OP_HEAD 4
#define MPM_OP_HEAD_BWD 5
#define MPM_OP_PAD 6
int32_t mpm_net_debug_op(mpm_net net, int32_t op, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c,
                         int32_t c2, const void* a, const void* b, void* out, void* out2);

/* Use 'net' (in_ch = 5 S + 1, out_ch = S) as the warm start of a context created with
 * warm_start = MPM_WS_NET or MPM_WS_NET_EXTRAP; net = NULL detaches.  Network input on
 * the box grid (box sizes rounded up to multiples of 8, zero beyond the box), each
 * channel times in_scale[ch] (host, exactly 5 S + 1 floats are read): c^n (S; zero off
 * the domain, which the solve never reads), k (S), D (S), s (S), the mask, and the
 * Jacobi-scaled residual d = (b - A x_b) / A_PP of the base start x_b (S; zero off the
 * domain), the first Jacobi correction of x_b, computed with the step's own residual
 * kernel.  The base start is c^n (MPM_WS_NET) or the
 * extrapolation 2 c^n - c^{n-1} (MPM_WS_NET_EXTRAP, from the second step of the context
 * on).  The prediction of species s is output * out_scale[s] (host, S floats read)
 * added to x_b.  Each step keeps the prediction of a system only if its true residual
 * is below that of c^n (mpm_stats.warm_start_used / fallback).  The net must outlive
 * its use. */
int32_t mpm_attach_net(mpm_ctx ctx, mpm_net net, const float* in_scale, const float* out_scale);

/* Training pair for the warm start of 'problem': the network input built from the
 * lattice fields c_old (device FP64 [S][z][y][x]) exactly as mpm_implicit_step builds
 * it (in_bf16: device [gz][gy][gx][5 S + 1]) and the target (c_new - c_old) / out_scale
 * on domain voxels, 0 elsewhere (target: device FP32 [gz][gy][gx][S]).  grid: see
 * mpm_ws_grid.  The residual of c_old is computed with the step's own kernels, which
 * use the context's solver workspace as scratch (the next step recomputes it).
 * Synchronises the stream. */
int32_t mpm_ws_pair(mpm_ctx ctx, int32_t problem, const double* c_old, const double* c_new,
                    const float* in_scale, const float* out_scale, uint16_t* in_bf16, float* target);

/* The same for MPM_WS_NET_EXTRAP: the base start is x_b = 2 c_old - c_prev (c_prev:
 * device FP64 lattice fields of the step before c_old) on the domain voxels of the
 * box, the input's last S channels hold the Jacobi-scaled residual of x_b, and the
 * target is (c_new - x_b) / out_scale. */
int32_t mpm_ws_pair_extrap(mpm_ctx ctx, int32_t problem, const double* c_prev, const double* c_old,
                           const double* c_new, const float* in_scale, const float* out_scale, uint16_t* in_bf16,
                           float* target);

/* Training loss of the warm start by the residual its prediction leaves.  out: device
 * FP32 [gz][gy][gx][S], the network's output for a pair of 'problem' (units of
 * out_scale); target: that pair's target (mpm_ws_pair).  With e = (out - target) *
 * out_scale on the domain voxels (the start's error) and w = S A e (S = diag(A)^(-1/2),
 * A the problem's operator), *loss (host) = sum (w / out_scale)^2 / (S N) over the
 * S species and N domain voxels, and grad_out (device FP32, shape of out) = dloss/dout
 * = 2 A S w / (S N out_scale), zero off the domain.  out_scale: host FP32 [S], positive.
 * Uses the context's solver workspace as scratch (the next step recomputes it);
 * synchronises the stream.  MPM_ESTATE without a network warm start (MPM_WS_NET or
 * MPM_WS_NET_EXTRAP) or before mpm_fv_setup. */
int32_t mpm_ws_loss(mpm_ctx ctx, int32_t problem, const float* out, const float* target, const float* out_scale,
                    float* grad_out, double* loss);

/* Grid sizes (gx, gy, gz) of the warm-start network input of 'problem' (host int[3]). */
int32_t mpm_ws_grid(mpm_ctx ctx, int32_t problem, int32_t* grid);

/* Test hook: apply the discrete operator of 'problem' to a lattice field.
 * x_lattice, y_lattice: device FP64 [S][z][y][x]; only domain voxels of the box are
 * read / written.  mode 0: y = A x (FP64, unscaled); mode 1: y = S A S x with
 * S = diag(A)^(-1/2), in FP32 (the inner operator of MPM_FP32_IR); mode 2: the same
 * scaled operator in FP64.  Synchronises the stream. */
int32_t mpm_debug_apply(mpm_ctx ctx, int32_t problem, const double* x_lattice, double* y_lattice,
                        int32_t mode);

/* Test hook: the Krylov state of one (problem, species) system after the last GMRES
 * cycle of the last step (delayed Gram-Schmidt only), for checks of orthogonality and
 * of the Arnoldi relation.  Host outputs: *mcount = columns of that cycle (m);
 * vs[k] and basis[k * N + l] (N = domain voxels of the box, compact C order) for
 * k < min(m, kmax), the orthonormal basis being v_k = vs[k] * basis[k]; hess[k *
 * (kmax + 1) + i] = H[i][k], the unrotated Hessenberg matrix (rows i <= k + 1, zero
 * elsewhere).  The caller sizes vs [kmax], basis [kmax * N], hess [kmax * (kmax + 1)].
 * 1 <= kmax <= restart.  Synchronises the stream.  MPM_ESTATE before the first step on
 * the current layout. */
int32_t mpm_debug_krylov(mpm_ctx ctx, int32_t problem, int32_t species, int32_t kmax, int32_t* mcount,
                         double* vs, double* basis, double* hess);

#ifdef __cplusplus
}
#endif

#endif /* MPM_H */
