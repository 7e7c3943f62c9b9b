#!/usr/bin/env python3
"""Implicit steps/s of the 128^3-box x 3-species reaction-diffusion workload on one MI355X.

Workload (default): 256x256x160 lattice with a synthetic pleural shell (two nested
ellipsoid pairs, 6 voxels thick), 4000 Voronoi tumour cells, the 128^3 bounding box
of the cells plus a 4-voxel margin, three species (oxygen, nutrient, cytokine), one
implicit-Euler step per "step", each solved to a relative FP64 residual of 1e-8 by
FP32 GMRES(30) inside FP64 iterative refinement, all species batched in one launch
(kernels launched directly; --graph replays each cycle from a hipGraph).  Inputs are
seeded and synthetic.

Prints ONE JSON line (rank 0).  Besides steps/s it reports the dominant kernel's
achieved algorithmic HBM bandwidth (HIP events on the library's stream), the same
workload with plain FP64 GMRES, the learned warm start against the plain solve (a
network trained on pairs this workload's solver generates), and the CPU FP64 oracle
timed on a bounded sample.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_FLOPS = 2.5e15      # dense BF16 MFMA

KERNELS = {"spmv_dot": 1, "axpy_dot": 2, "axpy_norm": 3, "update": 4, "residual": 5}
KERNEL_NAMES = {1: "k_spmv_dot", 2: "k_axpy_dot", 3: "k_axpy_norm", 4: "k_update",
                5: "k_residual"}
# delayed Gram-Schmidt: stencil + multi-dot, and the axpy that finishes q_j and forms u_{j+1}
KERNEL_NAMES_DCGS2 = {1: "k_dc_spmv_dot", 2: "k_dc_axpy", 4: "k_update", 5: "k_residual"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="config2",
                    choices=["config2", "config2-dense", "config1", "config3", "config4", "config5", "cube100",
                             "cube150", "cube200"])
    ap.add_argument("--c4-geometries", type=int, default=64, help="config4: 64^3 training geometries")
    ap.add_argument("--c4-pairs", type=int, default=10, help="config4: pairs per training geometry")
    ap.add_argument("--c4-epochs", type=int, default=4, help="config4: training epochs")
    ap.add_argument("--c4-chunk", type=int, default=16,
                    help="config4: geometries whose pairs are generated and trained on together")
    ap.add_argument("--c4-lr", type=float, default=1e-3, help="config4: Adam learning rate")
    ap.add_argument("--c4-save", default=None, help="config4: save the trained parameters and scales here")
    ap.add_argument("--c4-base", default="cn", choices=["cn", "extrap"],
                    help="config4: the network predicts the change from c^n (cn) or corrects the "
                         "extrapolated start 2 c^n - c^{n-1} (extrap, MPM_WS_NET_EXTRAP)")
    ap.add_argument("--c4-loss", default="residual", choices=["residual", "mse"],
                    help="config4: train on the Jacobi-scaled residual each prediction leaves (mpm_ws_loss), "
                         "or on the mean squared error of the predicted change")
    ap.add_argument("--c4-load", default=None,
                    help="config4: evaluate a network saved by --c4-save instead of training one")
    ap.add_argument("--c4-eval", type=int, default=4, help="config4: unseen 128^3 evaluation geometries")
    ap.add_argument("--grow", action="store_true",
                    help="lung workloads: cells grow every step; the box is recomputed and the "
                         "operator rebuilt before each step (timed with the step)")
    ap.add_argument("--track-every", type=int, default=1,
                    help="with --grow: recompute the box and set up the operator on it every K steps "
                         "(mpm_bbox_from_cells + mpm_fv_setup); in between only the coefficients of the "
                         "grown cells are updated on the standing box (mpm_fv_update)")
    ap.add_argument("--hbm-workload", default="auto",
                    help="workload of the in-run HBM roofline block (auto: config2-dense when the "
                         "headline working set fits in the 256 MB Infinity Cache; none to skip)")
    ap.add_argument("--no-probe", action="store_true", help="skip the streaming bandwidth probe")
    ap.add_argument("--species", type=int, default=3, choices=[3, 4],
                    help="4: the interleukins as separate fields (config2/config2-dense/config5/cube*)")
    ap.add_argument("--precision", default="fp32ir", choices=["fp32ir", "fp64"])
    ap.add_argument("--graph", action="store_true",
                    help="replay each GMRES cycle from a captured hipGraph (default: direct launches)")
    ap.add_argument("--unbatched", action="store_true")
    ap.add_argument("--tile", type=int, default=0, help="unknowns per block (0 = library default)")
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--start", default="cn", choices=["cn", "extrap"],
                    help="initial guess of each step: c^n, or 2 c^n - c^{n-1} kept when it lowers the residual")
    ap.add_argument("--ortho", default="dcgs2", choices=["dcgs2", "cgs2"],
                    help="Gram-Schmidt variant of the Arnoldi process")
    ap.add_argument("--time-kernel", default=None,
                    help="kernel:j timed with HIP events for the roofline ('none' to skip; default "
                         "spmv_dot:10 under dcgs2, axpy_dot:10 under cgs2)")
    ap.add_argument("--repeat", type=int, default=None,
                    help="back-to-back launches per timed event pair (default 10 for the delayed "
                         "scheme's stencil kernel, else 1)")
    ap.add_argument("--roofline-steps", type=int, default=10,
                    help="implicit steps of the roofline phase (after the headline timing)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget of the CPU oracle sample (0 = skip)")
    ap.add_argument("--learned-steps", type=int, default=20,
                    help="implicit steps of the learned-vs-plain comparison (0 = skip)")
    ap.add_argument("--train-pairs", type=int, default=16,
                    help="solver steps that produce training pairs for the warm-start network")
    ap.add_argument("--train-iters", type=int, default=600, help="Adam iterations of the network")
    ap.add_argument("--widths", default=None,
                    help="U-Net channels per level (16, 32, 48 or 64 each, the first 16); default "
                         "16,16,16 for the learned starts on the box workloads (trained on a few "
                         "pairs of the box itself), 16,32,64,64 for config4 (trained on many geometries)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy this many bytes device-to-device once (calibrates HBM counters)")
    return ap.parse_args()


def net_widths(arg, default):
    """U-Net channels per level from ``--widths`` ("16,32,64,64"), or ``default``: 1 to 6
    levels of 16, 32, 48 or 64 channels, 16 at the first (the library's network)."""
    try:
        w = [int(v) for v in (arg or default).split(",")]
    except ValueError:
        raise SystemExit(f"--widths: comma-separated channel counts expected, got {arg!r}")
    if not 1 <= len(w) <= 6 or w[0] != 16 or any(v not in (16, 32, 48, 64) for v in w):
        raise SystemExit(f"--widths: 1 to 6 levels of 16, 32, 48 or 64 channels, the first 16; got {arg!r}")
    return w


def unet_macs_per_voxel(cin, cout, widths):
    """Multiply-adds per input-grid voxel of the warm-start U-Net: per level l (1/8^l of
    the voxels) two 3x3x3 convolutions on the way down (the first from the level above,
    or the input), two on the way up (the first on the upsampled level below
    concatenated with the skip), and the 1x1x1 head."""
    L = len(widths)
    macs = 0.0
    for lv in range(L):
        c = widths[lv]
        down = (cin if lv == 0 else widths[lv - 1]) * c * 27 + c * c * 27
        up = ((widths[lv + 1] + c) * c * 27 + c * c * 27) if lv < L - 1 else 0
        macs += (down + up) / 8 ** lv
    return macs + widths[0] * cout


def alg_bytes_active(kind, j, U, precision, S, dcgs2):
    """Algorithmic bytes of one launch in which every system is active."""
    t = 4 if precision else 8
    axpy = (3 * t if j == 0 else t * (j + 4)) if dcgs2 else t * (j + 3)
    per = {1: t * (j + 5) + 16.0 / S, 2: axpy, 3: t * (j + 3), 4: None, 5: 56 + t + 16.0 / S}[kind]
    return per * U if per is not None else 0


def measured_traffic(kernel, workload, tile):
    """HBM bytes per active launch from the committed rocprofv3 counter summary of this
    kernel and workload (None if there is none for it, or for another work split)."""
    base = kernel.split("<")[0]
    path = os.path.join(ROOT, "profiles", f"{base}_{workload}_traffic.md")
    if tile or not os.path.exists(path):
        return None
    text = open(path).read()
    if f"kernel: {kernel}" not in text:
        return None
    for line in text.splitlines():
        if "traffic_bytes_per_active_launch:" in line:
            return int(line.split("traffic_bytes_per_active_launch:")[1].split("*")[0].strip().rstrip("."))
    return None


def make_workload(name, species=3):
    from synth import config1, config2, config2_dense, config5, cube
    if name == "config2":
        return config2(species=species)
    if name == "config2-dense":
        return config2_dense(species=species)
    if name == "config5":
        return config5(species=species)
    if name.startswith("cube"):
        return cube(int(name[4:]), species=species)
    return config1()


def upload(prob, torch):
    dev = torch.device("cuda")
    return {k: torch.from_numpy(getattr(prob, k)).to(dev) for k in ("mask", "D", "k", "src", "cell_id")}


def gpu_solver(m, prob, t, box, precision, graph, batched, tile=0, ortho=1, warm=0):
    s = m.Solver(prob.nspecies, 1, precision=precision, use_graph=int(graph), batched=int(batched),
                 tile_override=int(tile), ortho=int(ortho), warm_start=int(warm))
    s.setup(0, box, t["mask"], t["D"], t["k"], t["src"], prob.c_b, prob.dt, prob.h)
    return s


class Grower:
    """Cell growth between steps (the cell model's part, outside the solve): each step
    applies precomputed growth to the device arrays.  Every ``every`` steps it then
    recomputes the box (mpm_bbox_from_cells) and rebuilds the operator on it
    (mpm_fv_setup); in the steps between, the box stands and only the coefficients of
    the grown cells are updated on it (mpm_fv_update), as the paper re-tracks the box
    every 50 Monte Carlo steps only.  Cells that grow past the standing box are outside
    the solve until the next re-tracking (the margin absorbs them)."""

    def __init__(self, m, prob, t, steps, torch, every=1):
        from synth.geometry import grow_cells
        dev = torch.device("cuda")
        self.m, self.prob, self.t = m, prob, t
        self.every = max(1, int(every))
        self.events = [tuple(torch.from_numpy(a).to(dev) for a in (g.index, g.cell, g.k, g.src))
                       for g in grow_cells(prob, steps)]
        self.i = 0
        self.box = None
        self.reset()

    def reset(self):
        self.grown = 0
        self.setup_s = 0.0      # bounding box + set-up (re-tracking steps)
        self.update_s = 0.0     # coefficient updates (steps between)
        self.tracks = 0
        self.updates = 0
        self.boxes = []         # the box each step was solved on

    def __call__(self, s):
        idx, ids, kv, sv = self.events[self.i]
        S = self.prob.nspecies
        self.t["cell_id"].view(-1)[idx] = ids
        self.t["k"].view(S, -1)[:, idx] = kv
        self.t["src"].view(S, -1)[:, idx] = sv
        t0 = time.perf_counter()        # every call below waits for its result
        if self.box is None or self.i % self.every == 0:
            self.box = self.m.mpm_bbox_from_cells(self.t["cell_id"], self.prob.margin)
            s.setup(0, self.box, self.t["mask"], self.t["D"], self.t["k"], self.t["src"], self.prob.c_b,
                    self.prob.dt, self.prob.h)
            self.setup_s += time.perf_counter() - t0
            self.tracks += 1
        else:
            s.update(0, self.t["mask"], self.t["D"], self.t["k"], self.t["src"], self.prob.c_b,
                     self.prob.dt, self.prob.h)
            self.update_s += time.perf_counter() - t0
            self.updates += 1
        self.i += 1
        self.boxes.append(self.box)
        self.grown += int(idx.numel())

    def ratios(self):
        """Mean over the steps of (box voxels / lattice voxels, domain voxels in the box /
        domain voxels of the lattice), the measure of the paper's Fig. 7."""
        mask = self.prob.mask
        dom_total = float(mask.sum())
        cache = {}
        br, dr = [], []
        for b in self.boxes:
            if b not in cache:
                (x0, y0, z0), (x1, y1, z1) = b
                cache[b] = ((x1 - x0) * (y1 - y0) * (z1 - z0) / mask.size,
                            float(mask[z0:z1, y0:y1, x0:x1].sum()) / dom_total)
            br.append(cache[b][0])
            dr.append(cache[b][1])
        return float(np.mean(br)), float(np.mean(dr))


def run_steps(s, f, n, tol, torch, grow=None):
    its = []
    for _ in range(n):
        if grow is not None:
            grow(s)
        rc = s.step([f], tol)
        if rc != 0:
            raise RuntimeError(f"step did not converge (status {rc})")
        its.append(s.iterations(0))
    torch.cuda.synchronize()
    return its


def learned_vs_plain(m, prob, t, box, f0, tol, precision, ortho, args, torch):
    """Warm starts by networks trained on pairs this workload's own solver generates.

    From the state f0: ``train_pairs`` steps solved to 1e-10 give training pairs on the
    box grid, for two networks (U-Net with ``--widths`` channels per level, 16-16-16 by
    default, the library's kernels, the residual loss): one predicting the change from
    c^n (``MPM_WS_NET``), one correcting the extrapolated start 2 c^n - c^{n-1}
    (``MPM_WS_NET_EXTRAP``), each target scaled by its per-species RMS.  Then the same
    ``learned_steps`` steps are run from the state after the pair steps with each start:
    plain (c^n; in the headline's precision and in plain FP64), extrapolated, learned and
    learned correction of the extrapolation (each start kept per system only when it
    lowers the true residual), all with the launch mode of the headline, at the benchmark
    tolerance; the ratios to plain FP64 are taken on these same steps.
    """
    import numpy as np
    from paper_2505_03067_amd import train as tr
    from paper_2505_03067_amd.train import input_scales
    S = prob.nspecies
    widths = net_widths(args.widths, "16,16,16")

    def make_pairs(out_scale, extrap, keep=False):
        g = f0.clone()
        pairs = []
        s = m.Solver(S, 1, warm_start=m.MPM_WS_NET_EXTRAP if extrap else m.MPM_WS_NET)
        s.setup(0, box, t["mask"], t["D"], t["k"], t["src"], prob.c_b, prob.dt, prob.h)
        gx, gy, gz = s.ws_grid(0)
        prev = None
        for _ in range(args.train_pairs + (1 if extrap else 0)):
            old = g.clone()
            s.step([g], 1e-10)
            if extrap and prev is None:
                prev = old
                continue
            inp = torch.empty((gz, gy, gx, 5 * S + 1), dtype=torch.int16, device="cuda")
            tgt = torch.empty((gz, gy, gx, S), dtype=torch.float32, device="cuda")
            s.ws_pair(0, old, g, input_scales(S, out_scale), out_scale, inp, tgt, c_prev=prev if extrap else None)
            pairs.append((s, inp, tgt))
            prev = old
        if not keep:
            s.close()
        return pairs, g, s

    def trained(extrap):
        raw, _, _ = make_pairs([1.0] * S, extrap)
        out_scale = tr.target_rms([(inp, tgt) for _, inp, tgt in raw], S)
        del raw
        pairs, g_after, pair_solver = make_pairs(out_scale, extrap, keep=True)
        net = m.Net(5 * S + 1, S, widths, seed=7)
        rng = np.random.default_rng(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = []
        for it in range(1, args.train_iters + 1):
            # the residual each prediction leaves (mpm_ws_loss), cosine-annealed learning rate
            net.zero_grad()
            losses.append(tr.residual_step(net, [pairs[int(rng.integers(len(pairs)))]], out_scale))
            net.adam(1e-3 * 0.5 * (1.0 + np.cos(np.pi * it / args.train_iters)), it)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        pair_solver.close()
        x0 = pairs[0][1].unsqueeze(0)
        info = {"pairs": len(pairs), "iterations": args.train_iters, "seconds": round(train_s, 2),
                "loss_first": round(float(np.mean(losses[:10])), 5),
                "loss_last": round(float(np.mean(losses[-10:])), 5)}
        return net, out_scale, g_after, x0, info

    net, out_scale, f_after, x0, info_cn = trained(False)
    net_x, out_scale_x, _, _, info_x = trained(True)
    # the network's forward pass on the box grid against the dense BF16 MFMA peak
    y0 = torch.empty((1,) + tuple(x0.shape[1:4]) + (S,), dtype=torch.float32, device="cuda")
    net.forward(x0, y0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        net.forward(x0, y0)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / 5
    # the inference pass the warm start runs (head fused into the last convolution)
    net.forward(x0, y0, infer=True)
    e0.record()
    for _ in range(5):
        net.forward(x0, y0, infer=True)
    e1.record()
    torch.cuda.synchronize()
    inf_ms = e0.elapsed_time(e1) / 5
    grid = int(x0.shape[1] * x0.shape[2] * x0.shape[3])
    fwd_flop = 2.0 * unet_macs_per_voxel(5 * S + 1, S, widths) * grid
    del x0, y0
    res = {}
    for name, warm, prec in (("plain", m.MPM_WS_NONE, precision), ("plain_fp64", m.MPM_WS_NONE, m.MPM_FP64),
                             ("extrapolated", m.MPM_WS_EXTRAP, precision), ("learned", m.MPM_WS_NET, precision),
                             ("learned_correction_of_extrapolated", m.MPM_WS_NET_EXTRAP, precision)):
        g = f_after.clone()
        s = m.Solver(S, 1, precision=prec, warm_start=warm, ortho=int(ortho))
        s.setup(0, box, t["mask"], t["D"], t["k"], t["src"], prob.c_b, prob.dt, prob.h)
        if warm == m.MPM_WS_NET:
            s.attach(net, input_scales(S, out_scale), out_scale)
        if warm == m.MPM_WS_NET_EXTRAP:
            s.attach(net_x, input_scales(S, out_scale_x), out_scale_x)
        gw = g.clone()
        s.step([gw], tol)                      # allocations, tuning, graph capture
        s.step([gw], tol)                      # (the extrapolating starts need one step of history)
        torch.cuda.synchronize()
        its, acc, rw = 0, 0, []
        t1 = time.perf_counter()
        for _ in range(args.learned_steps):
            s.step([g], tol)
            st = [s.stats(0, sp) for sp in range(S)]
            its += sum(x["iterations"] for x in st)
            acc += sum(x["warm_start_used"] for x in st)
            rw += [x["rel_res_warm"] / x["rel_res_initial"] for x in st if x["warm_start_used"]]
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        s.close()
        res[name] = {"steps_per_s": round(args.learned_steps / el, 3),
                     "iterations_per_step": round(its / (args.learned_steps * S), 2)}
        if warm != m.MPM_WS_NONE:
            res[name]["accepted_fraction"] = round(acc / (args.learned_steps * S), 3)
            res[name]["residual_ratio_warm_over_cn"] = round(float(np.mean(rw)), 4) if rw else None
    net.close()
    net_x.close()
    res["network_forward"] = {"grid_voxels": grid, "ms": round(fwd_ms, 3), "flop": fwd_flop,
                              "tflops": round(fwd_flop / (fwd_ms * 1e-3) / 1e12, 1),
                              "frac_of_bf16_peak": round(fwd_flop / (fwd_ms * 1e-3) / BF16_PEAK_FLOPS, 4),
                              "inference_ms": round(inf_ms, 3)}
    res["training"] = {"learned": info_cn, "learned_correction_of_extrapolated": info_x,
                       "loss": "Jacobi-scaled residual left by the prediction (mpm_ws_loss)",
                       "network": "U-Net " + "-".join(map(str, widths)) +
                                  ", BF16 MFMA kernels, FP32 Adam, on the box grid"}
    res["learned_over_plain"] = round(res["learned"]["steps_per_s"] / res["plain"]["steps_per_s"], 3)
    res["learned_correction_over_plain"] = round(
        res["learned_correction_of_extrapolated"]["steps_per_s"] / res["plain"]["steps_per_s"], 3)
    res["extrapolated_over_plain"] = round(res["extrapolated"]["steps_per_s"] / res["plain"]["steps_per_s"], 3)
    # against plain FP64 GMRES on the same steps (the headline's own plain FP64 run starts
    # from an earlier state of the workload)
    fp64 = res["plain_fp64"]["steps_per_s"]
    res["learned_over_plain_fp64"] = round(res["learned"]["steps_per_s"] / fp64, 3)
    res["learned_correction_over_plain_fp64"] = round(res["learned_correction_of_extrapolated"]["steps_per_s"] / fp64, 3)
    res["extrapolated_over_plain_fp64"] = round(res["extrapolated"]["steps_per_s"] / fp64, 3)
    return res


def cpu_baseline(prob, box, c_start, gpu_after, tol, budget_s, threads=1):
    """The oracle (FP64 GMRES(30) + Jacobi) timed on a bounded sample, with ``threads``
    BLAS/OpenMP threads (None: every core the process may use).

    Runs consecutive steps from the same c^n the GPU started from, until the time budget
    is spent (at least one step), and compares each species with the GPU's fields.
    """
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.fv import box_slice
    from oracle.step import implicit_step

    sl = box_slice(box)
    mb = prob.mask[sl].astype(bool)
    c = c_start.copy()
    done = 0
    t0 = time.perf_counter()
    errs = []
    with threadpool_limits(limits=threads):
        while done < len(gpu_after):
            c, _ = implicit_step(c, prob.mask, prob.D, prob.k, prob.src, prob.c_b, box,
                                 prob.dt, prob.h, solver="gmres", tol=tol, restart=30)
            done += 1
            g = gpu_after[done - 1]   # the GPU's fields on the box
            errs.append([float(np.linalg.norm(g[s][mb] - c[s][sl][mb]) /
                               np.linalg.norm(c[s][sl][mb])) for s in range(prob.nspecies)])
            if time.perf_counter() - t0 >= budget_s:
                break
    dt = time.perf_counter() - t0
    return done, dt, errs


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or the platform's processor string."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def stream_probe(m, torch):
    """Rates of the library's hand-written streaming kernels (read, copy, triad) over
    buffers far larger than the 256 MB Infinity Cache: the practical ceiling of an
    HBM-bound kernel on this GPU, reported beside the 8 TB/s datasheet peak.  The best
    of a few grid sizes, with and without nontemporal accesses."""
    gib = 1 << 30
    a = torch.ones(gib // 4, dtype=torch.float32, device="cuda")        # 1 GiB each
    b = torch.ones(gib // 4, dtype=torch.float32, device="cuda")
    c = torch.empty(gib // 4, dtype=torch.float32, device="cuda")
    big = torch.ones(4 * gib // 4, dtype=torch.float32, device="cuda")  # 4 GiB for the read
    part = torch.empty(1 << 20, dtype=torch.float32, device="cuda")
    res = {}
    cases = ((m.MPM_PROBE_READ, "read", (big, None, part), 4 * gib, 1),
             (m.MPM_PROBE_COPY, "copy", (a, None, c), gib, 2),
             (m.MPM_PROBE_TRIAD, "triad", (a, b, c), gib, 3))
    for kind, name, (x, y, z), nbytes, moved in cases:
        best = None
        for blocks in (2048, 4096, 8192, 16384):
            for nt in (0, m.MPM_PROBE_NONTEMPORAL):
                ms = m.mpm_hbm_probe(kind | nt, x, y, z, nbytes, blocks, 5)
                gbs = moved * nbytes / (ms * 1e-3) / 1e9
                if best is None or gbs > best[0]:
                    best = (gbs, blocks, bool(nt))
        res[name] = {"gbs": round(best[0], 1), "bytes_per_launch": moved * nbytes, "blocks": best[1],
                     "nontemporal": best[2]}
    del a, b, c, big, part
    res["note"] = ("hand-written streaming kernels of the library (mpm_hbm_probe: 256-thread blocks, "
                   "16-byte accesses, grid-stride loops), best over 2048-16384 blocks with and without "
                   "nontemporal accesses; 4 GiB read, 1 GiB buffers for copy and triad, far past the "
                   "256 MB Infinity Cache")
    return res


def working_set_bytes(U, N, precision, restart=30):
    """Device bytes the GMRES cycle streams through: the Krylov basis and work vector,
    the FP64 iterate and right-hand side, the couplings (scaled in the Krylov type, FP64
    unscaled), diagonal, scaling and source terms, and the neighbour table."""
    t = 4 if precision else 8
    return U * (t * (restart + 2) + 16 + 3 * t + 24 + 24) + N * 20


def roofline_block(timing, kname, kj, precision, U, S, dc, repeat, names, workload, tile):
    avg_ms = timing["ms"] / timing["launches"]
    achieved = timing["bytes"] / (timing["ms"] * 1e-3) / 1e9
    kernel = f"{names[KERNELS[kname]]}<{'float' if precision else 'double'},{kj}>"
    traffic = measured_traffic(kernel, workload, tile)
    return {
        "bound": "hbm",
        "kernel": kernel,
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "traffic_source": (f"profiles/{kernel.split('<')[0]}_{workload}_traffic.md: rocprofv3 --pmc FETCH_SIZE "
                           f"and WRITE_SIZE of this kernel on this workload, scaled by the factors a device "
                           f"copy of known size reads, per active launch; taken from the committed profile, "
                           f"not counted in this run" if traffic is not None else None),
        "avg_launch_us": round(1000.0 * avg_ms, 3),
        "launches": timing["launches"],
        "launches_per_event_pair": repeat,
        "alg_bytes_per_launch": round(timing["bytes"] / timing["launches"]),
        "alg_bytes_per_active_launch": round(alg_bytes_active(KERNELS[kname], kj, U, precision, S, dc)),
    }


def hbm_roofline(m, args, torch, name, precision, ortho, dc, kname, kj, repeat):
    """The roofline kernel timed on a workload whose working set exceeds the Infinity
    Cache (so the bytes it streams come from HBM): warm-up steps, then
    ``roofline_steps`` steps with the kernel timed as for the headline."""
    prob = make_workload(name, args.species)
    t = upload(prob, torch)
    box = prob.box if prob.box is not None else m.mpm_bbox_from_cells(t["cell_id"], prob.margin)
    tol = args.tol if args.tol is not None else prob.tol
    f = torch.from_numpy(prob.c0).cuda()
    s = gpu_solver(m, prob, t, box, precision, False, True, 0, ortho)
    run_steps(s, f, 3, tol, torch)
    s.time_kernel(KERNELS[kname], kj, repeat)
    run_steps(s, f, args.roofline_steps, tol, torch)
    timing = s.kernel_timing()
    s.time_kernel(0)
    s.close()
    N = int(prob.mask[box[0][2]:box[1][2], box[0][1]:box[1][1], box[0][0]:box[1][0]].sum())
    U = N * prob.nspecies
    if not timing["launches"]:
        return None
    names = KERNEL_NAMES_DCGS2 if dc else KERNEL_NAMES
    out = roofline_block(timing, kname, kj, precision, U, prob.nspecies, dc, repeat, names, prob.name, 0)
    out["workload"] = f"{prob.name}: box {box}, {U} unknowns"
    out["working_set_bytes"] = working_set_bytes(U, N, precision)
    out["memory"] = "HBM (working set larger than the 256 MB Infinity Cache)"
    return out


def config3_run(args, m, torch):
    """Config 3: 8 tumours of different sizes in one context (one launch per kernel for
    all 24 systems), each tumour dilated by one voxel every 10 steps; after each dilation
    the boxes are recomputed (mpm_bbox_from_cells) and the problems set up again
    (mpm_fv_setup), inside the timed steps.  The dilation and the coefficients of the
    grown tumours (D halved and jittered uptake on tumour voxels) are computed with torch
    on the device: the cellular model's part, outside the library."""
    import numpy as np
    from synth import config3_tumour, species_constants
    Dc, kc, ka, sc, cb = species_constants(3)
    dev = torch.device("cuda")
    P = 8
    tum, jit, fields, mask, dims = [], [], [], [], []
    for t in range(P):
        prob, tumour = config3_tumour(t)
        dims.append(prob.dims)
        tum.append(torch.from_numpy(tumour).to(dev))
        g = torch.Generator(device=dev)
        g.manual_seed(t + 1)
        jit.append(0.8 + 0.4 * torch.rand((3,) + tumour.shape, generator=g, device=dev, dtype=torch.float64))
        fields.append(torch.from_numpy(prob.c0).to(dev))
        mask.append(torch.from_numpy(prob.mask).to(dev))
    Dt = torch.tensor(Dc, dtype=torch.float64, device=dev).view(3, 1, 1, 1)
    Kc = torch.tensor([a + b for a, b in zip(kc, ka)], dtype=torch.float64, device=dev).view(3, 1, 1, 1)
    Ka = torch.tensor(ka, dtype=torch.float64, device=dev).view(3, 1, 1, 1)
    Sc = torch.tensor(sc, dtype=torch.float64, device=dev).view(3, 1, 1, 1)
    margin, tol = 4, (args.tol if args.tol is not None else 1e-8)

    def dilate(x):
        o = x.clone()
        o[1:] |= x[:-1]
        o[:-1] |= x[1:]
        o[:, 1:] |= x[:, :-1]
        o[:, :-1] |= x[:, 1:]
        o[:, :, 1:] |= x[:, :, :-1]
        o[:, :, :-1] |= x[:, :, 1:]
        return o

    s = m.Solver(3, P, precision=m.MPM_FP32_IR if args.precision == "fp32ir" else m.MPM_FP64,
                 use_graph=int(args.graph), tile_override=int(args.tile))
    boxes = [None] * P

    def set_up(p):
        x = tum[p]
        D = torch.where(x, 0.5 * Dt, Dt).contiguous()
        k = torch.where(x, Kc * jit[p], Ka.expand_as(jit[p])).contiguous()
        src = torch.where(x, Sc.expand_as(jit[p]), torch.zeros_like(jit[p])).contiguous()
        boxes[p] = m.mpm_bbox_from_cells(x.to(torch.int32).contiguous(), margin)
        s.setup(p, boxes[p], mask[p], D, k, src, np.array(cb), 1.0, 1.0)

    step = [0]
    rounds = []                      # the boxes of each set-up round

    def advance(n):
        its = []
        for _ in range(n):
            if step[0] % 10 == 0:
                for p in range(P):
                    if step[0] > 0:
                        tum[p] = dilate(tum[p])
                    set_up(p)
                rounds.append(list(boxes))
            rc = s.step(fields, tol)
            if rc != 0:
                raise RuntimeError(f"step did not converge (status {rc})")
            its.append(sum(s.stats(p, sp)["iterations"] for p in range(P) for sp in range(3)) / (3 * P))
            step[0] += 1
        torch.cuda.synchronize()
        return its

    advance(args.warmup)
    n_before = len(rounds)
    t0 = time.perf_counter()
    its = advance(args.steps)
    elapsed = time.perf_counter() - t0
    s.close()
    vox = [int(np.prod([hi - lo for lo, hi in zip(b[0], b[1])])) for b in boxes]
    b0 = rounds[n_before - 1] if n_before else rounds[0]
    return {
        "metric": "implicit steps/s, 128^3 box x 3 species to 1e-8 resid; HBM GB/s; learned vs plain",
        "value": round(args.steps / elapsed, 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "fp32ir" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"config3: 8 tumours (lattices {dims[0]} to {dims[-1]}), all voxels in the domain, "
                        f"3 species each, 24 systems in one context, dilation every 10 steps with box "
                        f"recomputation and set-up inside the timed steps, tol {tol:g}",
            "boxes_first": [[list(b[0]), list(b[1])] for b in b0],
            "boxes_last": [[list(b[0]), list(b[1])] for b in boxes],
            "unknowns_last": 3 * sum(vox),
        },
        "iterations_per_step": round(sum(its) / len(its), 2),
        "roofline": None,
    }


def config4_run(args, m, torch):
    """Config 4: the learned warm start trained on 64^3 tumour patches and evaluated on
    unseen 128^3 boxes.  Each training geometry (``synth.config4_patch``, seeds 0, 1, ...)
    is advanced 50 steps at tol 1e-10 and a seeded choice of ``--c4-pairs`` of those steps
    gives (input, change) pairs, built on the GPU by the solver's own warm-start kernel;
    the targets are scaled by their per-species RMS.  The U-Net is trained for
    ``--c4-epochs`` epochs (batch 4, Adam, the library's kernels).  The evaluation
    geometries (seeds 10^6, 10^6 + 1, ...) run 20 steps at tol 1e-8 from c^n (plain),
    with the extrapolated start and with the learned start."""
    import numpy as np
    from paper_2505_03067_amd import train as tr
    from synth import config4_patch
    S = 3
    extrap = args.c4_base == "extrap"
    t0 = time.perf_counter()
    widths = net_widths(args.widths, "16,32,64,64")
    saved = torch.load(args.c4_load, weights_only=True) if args.c4_load else None
    if saved is not None:
        widths = [int(v) for v in saved["widths"]]
    net = m.Net(5 * S + 1, S, widths, seed=7)
    rng = np.random.default_rng(0)
    losses, gen_s, train_s, npairs, t = [], 0.0, 0.0, 0, 0
    if saved is not None:
        net.set_params(saved["params"].cuda())
        out_scale = list(saved["out_scale"])
        args.c4_epochs = 0
    elif extrap:
        # target scale: per-species RMS of the correction the extrapolated start needs, on
        # four training geometries
        raw = []
        for seed in range(4):
            sv, items = tr.solver_pairs(config4_patch(seed, 64), 10, range(1, 10), [1.0] * S, tol=1e-10, extrap=True)
            raw += items
            sv.close()
        out_scale = tr.target_rms(raw, S)
        del raw
    else:
        # target scale: per-species RMS of the one-step change on four training geometries
        out_scale = tr.estimate_out_scale([config4_patch(seed, 64) for seed in range(4)], 10)
    # streamed: every epoch regenerates the pairs of a chunk of geometries on the GPU from
    # their seeds (the solver's trajectories are deterministic), trains on them shuffled,
    # and drops them (20,000 64^3 pairs would need about 230 GB)
    for ep in range(args.c4_epochs):
        tot, nb = 0.0, 0
        order = rng.permutation(args.c4_geometries)
        for c0 in range(0, args.c4_geometries, args.c4_chunk):
            tg = time.perf_counter()
            pairs, solvers = [], []
            for seed in order[c0:c0 + args.c4_chunk]:
                seed = int(seed)
                pick = set(np.random.default_rng(seed).choice(50, size=args.c4_pairs, replace=False).tolist())
                if args.c4_loss == "residual" or extrap:
                    sv, items = tr.solver_pairs(config4_patch(seed, 64), 50, pick, out_scale, tol=1e-10,
                                                extrap=extrap)
                    solvers.append(sv)
                    pairs += [(sv, inp, tgt) for inp, tgt in items]
                else:
                    pairs += [(None, inp, tgt) for inp, tgt in
                              tr.generate_pairs([config4_patch(seed, 64)], 50, pick, out_scale, tol=1e-10)]
            torch.cuda.synchronize()
            tt = time.perf_counter()
            gen_s += tt - tg
            perm = rng.permutation(len(pairs))
            for i in range(0, len(perm), 4):
                idx = perm[i:i + 4]
                net.zero_grad()
                if args.c4_loss == "residual":
                    tot += tr.residual_step(net, [pairs[j] for j in idx], out_scale)
                else:
                    x = torch.stack([pairs[j][1] for j in idx]).contiguous()
                    y = torch.stack([pairs[j][2] for j in idx]).contiguous()
                    out = torch.empty_like(y)
                    g = torch.empty_like(y)
                    net.forward(x, out)
                    tot += net.mse(out, y, g)
                    net.backward(g)
                nb += 1
                t += 1
                # cosine decay of the learning rate over the whole run
                frac = min(1.0, t / max(1, args.c4_epochs * args.c4_geometries * args.c4_pairs // 4))
                net.adam(args.c4_lr * 0.5 * (1.0 + np.cos(np.pi * frac)), t)
            torch.cuda.synchronize()
            train_s += time.perf_counter() - tt
            if ep == 0:
                npairs += len(pairs)
            del pairs
            for sv in solvers:
                sv.close()
            print(f"config4: epoch {ep}, geometries {c0 + args.c4_chunk}/{args.c4_geometries}, "
                  f"running loss {tot / max(nb, 1):.4e}", file=sys.stderr, flush=True)
        losses.append(tot / max(nb, 1))
    pairs = None
    if args.c4_save:
        torch.save({"params": net.params().cpu(), "out_scale": list(out_scale), "widths": widths,
                    "in_ch": 5 * S + 1, "out_ch": S, "base": args.c4_base}, args.c4_save)
    del pairs
    evalp = [config4_patch(10 ** 6 + i, 128) for i in range(args.c4_eval)]
    tol = args.tol if args.tol is not None else 1e-8
    res = {}
    for name, warm, prec in (("plain", m.MPM_WS_NONE, m.MPM_FP32_IR), ("plain_fp64", m.MPM_WS_NONE, m.MPM_FP64),
                             ("extrapolated", m.MPM_WS_EXTRAP, m.MPM_FP32_IR),
                             ("learned", m.MPM_WS_NET_EXTRAP if extrap else m.MPM_WS_NET, m.MPM_FP32_IR)):
        ratios = []
        its, sps, _, acc = tr.evaluate(evalp, 20, tol, net=net, out_scale=out_scale, warm=warm, precision=prec,
                                       ratios=ratios)
        res[name] = {"steps_per_s": round(sps, 3), "iterations_per_step": round(its, 2)}
        if warm != m.MPM_WS_NONE:
            res[name]["accepted_fraction"] = round(acc, 3)
            res[name]["residual_ratio_warm_over_cn"] = round(float(np.mean(ratios)), 4) if ratios else None
    net.close()
    return {
        "metric": "implicit steps/s, 128^3 box x 3 species to 1e-8 resid; HBM GB/s; learned vs plain",
        "value": res["learned"]["steps_per_s"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": 20 * args.c4_eval,
        "warmup": args.c4_eval,
        "ms_per_step": round(1000.0 / res["learned"]["steps_per_s"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64, bf16 network",
        "data": "synthetic",
        "config": {
            "workload": f"config4: learned warm start ({'correction of the extrapolation' if extrap else 'from c^n'}), "
                        f"trained on {args.c4_geometries} x {args.c4_pairs} pairs of "
                        f"64^3 tumour patches ({args.c4_epochs} epochs), evaluated on {args.c4_eval} unseen 128^3 "
                        f"boxes x 20 steps at tol {tol:g}; value = steps/s with the learned start",
        },
        "learned_vs_plain": {
            **res,
            "learned_over_plain": round(res["learned"]["steps_per_s"] / res["plain"]["steps_per_s"], 3),
            "learned_over_plain_fp64": round(res["learned"]["steps_per_s"] / res["plain_fp64"]["steps_per_s"], 3),
            "extrapolated_over_plain": round(res["extrapolated"]["steps_per_s"] / res["plain"]["steps_per_s"], 3),
            "training": {"pairs_per_epoch": npairs, "epochs": args.c4_epochs, "batch": 4, "lr": args.c4_lr,
                         "loss": args.c4_loss, "network": "U-Net " + "-".join(map(str, widths)),
                         "base": ("the network corrects the extrapolated start 2 c^n - c^{n-1} (MPM_WS_NET_EXTRAP)"
                                  if extrap else "the network predicts the change from c^n (MPM_WS_NET)"),
                         "streamed": f"pairs of {args.c4_chunk} geometries at a time, regenerated on the GPU "
                                     f"from their seeds every epoch",
                         "generation_s": round(gen_s, 1), "training_s": round(train_s, 1),
                         "loss_by_epoch": [round(float(x), 5) for x in losses]},
        },
        "roofline": None,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the species and problems are independent within a step and would shard across "
              "GPUs with no communication)", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    if args.copy_probe:
        a = torch.empty(args.copy_probe, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}))
        return 0

    import paper_2505_03067_amd as m

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    m.lib()
    if args.workload == "config3":
        print(json.dumps(config3_run(args, m, torch)))
        return 0
    if args.workload == "config4":
        print(json.dumps(config4_run(args, m, torch)))
        return 0
    prob = make_workload(args.workload, args.species)
    tol = args.tol if args.tol is not None else prob.tol
    t = upload(prob, torch)
    if prob.box is not None:
        box = prob.box
    else:
        box = m.mpm_bbox_from_cells(t["cell_id"], prob.margin)
    precision = m.MPM_FP32_IR if args.precision == "fp32ir" else m.MPM_FP64
    ortho = m.MPM_ORTHO_DCGS2 if args.ortho == "dcgs2" else m.MPM_ORTHO_CGS2
    f = torch.from_numpy(prob.c0).cuda()

    warm = m.MPM_WS_EXTRAP if args.start == "extrap" else m.MPM_WS_NONE
    s = gpu_solver(m, prob, t, box, precision, args.graph, not args.unbatched, args.tile, ortho, warm)
    grow = None
    if args.grow:
        if prob.box is not None:
            raise SystemExit("--grow needs a workload whose box follows the cells (config2, config5)")
        grow = Grower(m, prob, t, args.warmup + args.steps, torch, args.track_every)
    run_steps(s, f, args.warmup, tol, torch, grow)
    c_start = f.clone()
    # headline: K implicit steps, nothing else on the stream (with --grow, each one after
    # the growth of the cells, the new box and the rebuilt operator)
    torch.cuda.synchronize()
    box0 = box
    if grow is not None:
        box0 = grow.boxes[-1] if grow.boxes else box
        grow.reset()
    t0 = time.perf_counter()
    its = run_steps(s, f, args.steps, tol, torch, grow)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if grow is not None:
        box = grow.boxes[-1]
    tile_used = s.tile()
    final_stats = [s.stats(0, sp) for sp in range(prob.nspecies)]
    # roofline phase: the same solver continues for a few steps with one kernel timed by
    # HIP events on the library's stream (the cycle is then launched directly)
    dc = ortho == m.MPM_ORTHO_DCGS2
    time_kernel = args.time_kernel or ("spmv_dot:10" if dc else "axpy_dot:10")
    kname, kj, timing, repeat = None, 0, None, 1
    if time_kernel != "none" and args.roofline_steps > 0:
        kname, _, kj = time_kernel.partition(":")
        kj = int(kj or 0)
        pure = KERNELS[kname] == 5 or (KERNELS[kname] == 1 and dc)
        repeat = args.repeat if args.repeat is not None else (10 if pure else 1)
        s.time_kernel(KERNELS[kname], kj, repeat)
        run_steps(s, f, args.roofline_steps, tol, torch)
        timing = s.kernel_timing()
        s.time_kernel(0)
    s.close()

    N = int(prob.mask[box[0][2]:box[1][2], box[0][1]:box[1][1], box[0][0]:box[1][0]].sum())
    U = N * prob.nspecies
    steps_per_s = args.steps / elapsed

    out = {
        "metric": "implicit steps/s, 128^3 box x 3 species to 1e-8 resid; HBM GB/s; learned vs plain",
        "value": round(steps_per_s, 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if precision == m.MPM_FP32_IR else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{prob.name}: lattice {prob.dims}, box {box}, {N} domain voxels, "
                        f"{prob.nspecies} species, {U} unknowns, tol {tol:g}, "
                        f"{'FP32 GMRES(30) in FP64 refinement' if precision else 'FP64 GMRES(30)'}, "
                        f"{'delayed CGS2' if ortho == m.MPM_ORTHO_DCGS2 else 'CGS2'} Arnoldi, "
                        f"{'extrapolated start' if warm else 'start c^n'}, "
                        f"{'batched' if not args.unbatched else 'one system at a time'}, "
                        f"{'hipGraph cycles' if args.graph else 'direct launches'}",
            "unknowns": U,
            "domain_voxels": N,
            "box": [list(box[0]), list(box[1])],
            "unknowns_per_block": tile_used,
        },
        "iterations_per_step": round(sum(its) / len(its) / prob.nspecies, 2),
        **({"growth": {
            "what": f"per step: cell growth; every {grow.every} step(s) mpm_bbox_from_cells and "
                    f"mpm_fv_setup on the new box, in the steps between mpm_fv_update of the "
                    f"coefficients on the standing box; then the step; all inside the timed steps",
            "track_every": grow.every,
            "voxels_grown_per_step": round(grow.grown / args.steps, 2),
            "box_first": [list(box0[0]), list(box0[1])],
            "box_last": [list(box[0]), list(box[1])],
            "retrackings": grow.tracks,
            "updates": grow.updates,
            "bbox_and_setup_ms_per_retracking": round(1000.0 * grow.setup_s / max(grow.tracks, 1), 4),
            "update_ms_per_update": round(1000.0 * grow.update_s / max(grow.updates, 1), 4),
            "remap_ms_per_step": round(1000.0 * (grow.setup_s + grow.update_s) / args.steps, 4),
            "box_over_lattice_voxels": round(grow.ratios()[0], 5),
            "box_domain_over_lattice_domain": round(grow.ratios()[1], 5),
        }} if grow is not None else {}),
        "cycles_last_step": [st["cycles"] for st in final_stats],
        "rel_res_final_last_step": [st["rel_res_final"] for st in final_stats],
    }
    # context for the roofline: what a plain device-to-device copy of 1 GiB sustains
    nbytes = 1 << 30
    ca = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(5):
        cb.copy_(ca)
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * nbytes / (time.perf_counter() - t2) / 1e9
    del ca, cb
    # rows a1 and a2 on this workload's lattice and box: bounding box and set-up, each
    # call waits for its result; best of 3
    lat_bytes = t["cell_id"].numel() * 4
    tb = []
    for _ in range(3):
        t3 = time.perf_counter()
        m.mpm_bbox_from_cells(t["cell_id"], prob.margin)
        tb.append(time.perf_counter() - t3)
    s4 = gpu_solver(m, prob, t, box, precision, False, True, 1024)
    ts = []
    for _ in range(3):
        t3 = time.perf_counter()
        s4.setup(0, box, t["mask"], t["D"], t["k"], t["src"], prob.c_b, prob.dt, prob.h)
        ts.append(time.perf_counter() - t3)
    s4.close()
    out["bbox_and_setup"] = {
        "bbox_us": round(1e6 * min(tb), 1),
        "bbox_lattice_bytes": lat_bytes,
        "bbox_gbs_incl_host_wait": round(lat_bytes / min(tb) / 1e9, 1),
        "setup_ms": round(1e3 * min(ts), 3),
        "note": "host wall time of mpm_bbox_from_cells / mpm_fv_setup (both wait for their result)",
    }
    if timing and timing["launches"]:
        names = KERNEL_NAMES_DCGS2 if dc else KERNEL_NAMES
        ws = working_set_bytes(U, N, precision)
        rl = roofline_block(timing, kname, kj, precision, U, prob.nspecies, dc, repeat, names, prob.name,
                            args.tile)
        rl["phase"] = f"{args.roofline_steps} steps after the headline timing (no growth), cycle launched directly"
        rl["working_set_bytes"] = ws
        rl["memory"] = ("Infinity Cache: the working set fits in the 256 MB last-level cache, so this rate is "
                        "the cache fabric's, not HBM's; see roofline_hbm" if ws < 256e6 else
                        "HBM (working set larger than the 256 MB Infinity Cache)")
        rl["copy_1gib_gbs"] = round(copy_gbs, 1)
        rl["frac_of_copy"] = round(rl["achieved"] / copy_gbs, 4)
        out["roofline"] = rl
        hbm_name = args.hbm_workload
        if hbm_name == "auto":
            hbm_name = "config2-dense" if ws < 256e6 and prob.name.startswith("config2") else "none"
        if hbm_name != "none":
            out["roofline_hbm"] = hbm_roofline(m, args, torch, hbm_name, precision, ortho, dc, kname, kj, repeat)
    if not args.no_probe:
        out["stream_probe"] = stream_probe(m, torch)
        for key in ("roofline", "roofline_hbm"):
            if out.get(key):
                out[key]["frac_of_probe_read"] = round(out[key]["achieved"] / out["stream_probe"]["read"]["gbs"], 4)
                out[key]["frac_of_probe_copy"] = round(out[key]["achieved"] / out["stream_probe"]["copy"]["gbs"], 4)

    if not args.no_plain and precision == m.MPM_FP32_IR:
        f2 = c_start.clone()
        s2 = gpu_solver(m, prob, t, box, m.MPM_FP64, args.graph, not args.unbatched, args.tile, ortho)
        run_steps(s2, f2, 2, tol, torch)
        f2.copy_(c_start)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        its2 = run_steps(s2, f2, args.steps, tol, torch)
        torch.cuda.synchronize()
        e2 = time.perf_counter() - t1
        s2.close()
        out["plain_fp64"] = {"steps_per_s": round(args.steps / e2, 3),
                             "iterations_per_step": round(sum(its2) / len(its2) / prob.nspecies, 2),
                             "speedup_of_value": round(steps_per_s / (args.steps / e2), 3)}

    if args.learned_steps > 0:
        lv = learned_vs_plain(m, prob, t, box, c_start, tol, precision, ortho, args, torch)
        out["learned_vs_plain"] = lv

    if args.cpu_seconds > 0:
        # replay the first steps of the timed run on the GPU (deterministic) to compare
        # (the fields on the box only, as many steps as about 2 GB of host memory holds, at
        # most 32: the sample ends at the time budget or there)
        s3 = gpu_solver(m, prob, t, box, precision, args.graph, not args.unbatched, args.tile, ortho)
        f3 = c_start.clone()
        after = []
        (x0, y0, z0), (x1, y1, z1) = box
        box_bytes = prob.nspecies * (x1 - x0) * (y1 - y0) * (z1 - z0) * 8
        for _ in range(max(2, min(args.steps, 32, int(2e9 // box_bytes)))):
            s3.step([f3], tol)
            after.append(f3[:, z0:z1, y0:y1, x0:x1].cpu().numpy())
        s3.close()
        done, cpu_s, errs = cpu_baseline(prob, box, c_start.cpu().numpy(), after, tol,
                                         args.cpu_seconds)
        out["cpu_baseline"] = {
            "value": round(done / cpu_s, 5),
            "unit": "steps/s",
            "cores": 1,
            "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{done} consecutive steps of the same workload from the same c^n "
                      f"(FP64 GMRES(30) + Jacobi, tol {tol:g}, scipy CSR, 1 thread), {cpu_s:.1f} s",
        }
        out["fp64_rel_err_vs_oracle"] = [max(e[sp] for e in errs) for sp in range(prob.nspecies)]
        # the same oracle with every core the process may use (scipy's sparse products stay
        # single-threaded; only numpy's BLAS-2 work spreads)
        ncores = len(os.sched_getaffinity(0))
        done2, cpu_s2, _ = cpu_baseline(prob, box, c_start.cpu().numpy(), after[:2], tol,
                                        min(args.cpu_seconds, 5.0), threads=None)
        out["cpu_baseline_all_cores"] = {
            "value": round(done2 / cpu_s2, 5),
            "unit": "steps/s",
            "cores": ncores,
            "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{done2} consecutive steps as above with {ncores} threads, {cpu_s2:.1f} s",
        }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
