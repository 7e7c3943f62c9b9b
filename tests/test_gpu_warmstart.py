"""The warm start: input/target construction, acceptance and fallback, the extrapolated
start, and what a network trained on solver-generated pairs gains over plain GMRES."""

import numpy as np
import pytest

from gpu_helpers import gpu_run, rel_err_per_species, require_gpu, to_dev
from oracle import unet
from oracle.fv import assemble, box_slice
from oracle.step import run
from synth import config1, config4_patch, random_problem

pytestmark = pytest.mark.gpu


def _torch_bf16_bits(a):
    """BF16 bit patterns from PyTorch's CPU float32 -> bfloat16 cast (an implementation
    of round-to-nearest-even independent of the library's)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16)


def _bf16_values(bits):
    return (np.asarray(bits, np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _ws_pair_case(p, S, box=None, extrap=False):
    """Network input and training target built by the library, against their
    definition: each channel (c^n on the domain voxels and zero off them, k, D, s per
    species, then the mask) times its scale, rounded to BF16 on the box grid (zero past
    the box), the Jacobi-scaled residual of the base start x_b per species; target
    (c^{n+1} - x_b) / out_scale on domain voxels, zero elsewhere.  x_b = c^n, or with
    extrap the extrapolation 2 c^n - c^{n-1}."""
    torch = require_gpu()
    import paper_2505_03067_amd as m
    from oracle.fv import assemble, box_slice
    from paper_2505_03067_amd.train import input_scales
    box = box if box is not None else p.box
    out_scale = [0.5, 0.25, 2e-3, 3e-3][:S]
    in_scale = input_scales(S, out_scale)
    d = to_dev(p)
    f = torch.from_numpy(p.c0).cuda()
    with m.Solver(S, 1, warm_start=m.MPM_WS_NET_EXTRAP if extrap else m.MPM_WS_NET) as s:
        s.setup(0, box, d["mask"], d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
        for _ in range(2):          # a c^n away from the uniform initial state
            s.step([f], 1e-10)
        prev = f.clone()
        s.step([f], 1e-10)
        old = f.clone()
        s.step([f], 1e-10)
        gx, gy, gz = s.ws_grid(0)
        ext = [hi - lo for lo, hi in zip(*box)]
        assert (gx, gy, gz) == tuple((e + 7) // 8 * 8 for e in ext)
        inp = torch.empty((gz, gy, gx, 5 * S + 1), dtype=torch.int16, device="cuda")
        tgt = torch.empty((gz, gy, gx, S), dtype=torch.float32, device="cuda")
        s.ws_pair(0, old, f, in_scale, out_scale, inp, tgt, c_prev=prev if extrap else None)
    got_in = inp.cpu().numpy().view(np.uint16)
    got_t = tgt.cpu().numpy()
    c0 = old.cpu().numpy()
    c1 = f.cpu().numpy()
    xb_all = 2.0 * c0 - prev.cpu().numpy() if extrap else c0
    sl = box_slice(box)
    chans = [c0[s] * (p.mask != 0) for s in range(S)] + [p.k[s] for s in range(S)] + \
            [p.D[s] for s in range(S)] + [p.src[s] for s in range(S)] + [p.mask.astype(np.float64)]
    ex, ey, ez = ext
    for ch, a in enumerate(chans):
        want = np.zeros((gz, gy, gx), np.uint16)
        want[:ez, :ey, :ex] = _torch_bf16_bits(a[sl].astype(np.float32) * np.float32(in_scale[ch]))
        assert np.array_equal(got_in[..., ch], want), ch
    dom = np.zeros((gz, gy, gx), bool)
    dom[:ez, :ey, :ex] = p.mask[sl] != 0
    # residual channels: d = (b - A x_b) / A_PP on the domain voxels, zero elsewhere,
    # with b = c_old + q from the oracle's assembly.  The GPU forms S (S r) with S r
    # stored in the Krylov type, so its BF16 value may differ by one unit in the last
    # place, and r carries the cancellation error of b - A x (about 1e-15 of
    # |b| + |A||x|) on both sides
    mb = p.mask[sl].astype(bool)
    for s in range(S):
        A, q = assemble(mb, p.D[s][sl], p.k[s][sl], p.src[s][sl], float(p.c_b[s]), p.dt, p.h)
        x = c0[s][sl][mb]
        xb = xb_all[s][sl][mb]
        dvals = (x + q - A @ xb) / A.diagonal()
        scale = np.float32(in_scale[4 * S + 1 + s])
        want = np.zeros((gz, gy, gx))
        want[:ez, :ey, :ex][mb] = unet.bf16(dvals.astype(np.float32) * scale)
        got = _bf16_values(got_in[..., 4 * S + 1 + s])
        assert np.all(got[~dom] == 0.0)
        atol = float(scale) * 1e-13 * (1.0 + np.abs(x).max() + np.abs(xb).max() + np.abs(q).max())
        assert np.all(np.abs(got - want) <= np.abs(want) * 2.0 ** -7 + atol), s
        big = np.abs(want) > 1e3 * atol     # values far above the cancellation error
        assert big.sum() > 1000 and np.mean(got[big] != want[big]) < 0.01, s
    for s in range(S):
        want = np.zeros((gz, gy, gx), np.float32)
        full = ((c1[s] - xb_all[s]) / np.float64(np.float32(out_scale[s])))[sl].astype(np.float32)
        want[:ez, :ey, :ex] = full
        want[~dom] = 0.0
        assert np.array_equal(got_t[..., s], want), s


def test_ws_pair_matches_definition():
    _ws_pair_case(config4_patch(3, n=32), 3)


def test_ws_pair_extrap_matches_definition():
    """The pair of the network's correction of the extrapolated start (mpm_ws_pair_extrap):
    the residual channels and the target are taken at 2 c^n - c^{n-1}."""
    _ws_pair_case(config4_patch(5, n=32), 3, extrap=True)


def test_ws_pair_matches_definition_four_species():
    """Four species: 21 input channels, the output scales after all of them (a layout
    that once let the fourth species' input scales overlap the output scales); a ragged,
    masked box whose grid is padded past it on every axis."""
    p = random_problem(91, (30, 27, 21), S=4, fill=0.7)
    _ws_pair_case(p, 4, box=((2, 3, 1), (27, 26, 18)))


@pytest.mark.parametrize("S,extrap", [(3, False), (3, True), (4, False)])
def test_in_step_input_matches_ws_pair(S, extrap):
    """The network input a warm-start step builds equals, bit for bit, the one
    mpm_ws_pair builds from the same state (itself pinned to the definition above): the
    first warm start on a grid writes every channel, later ones only the c channels of
    the box, and new scales or new coefficients must bring back a full build.  A ragged
    box whose grid is padded past it on every axis; 16 (read in place) and 21 channels."""
    torch = require_gpu()
    import paper_2505_03067_amd as m
    from paper_2505_03067_amd import mpm as mpm_mod
    from paper_2505_03067_amd.train import input_scales
    p = random_problem(97 + S, (30, 27, 21), S=S, fill=0.7)
    box = ((2, 3, 1), (27, 26, 18))
    d = to_dev(p)
    out_scale = [0.5, 0.25, 2e-3, 3e-3][:S]
    scales = [input_scales(S, out_scale), [v * 1.5 for v in input_scales(S, out_scale)]]
    C = 5 * S + 1
    net = m.Net(C, S, [16, 32], seed=11)
    f = torch.from_numpy(p.c0).cuda()
    checked = 0
    with m.Solver(S, 1, warm_start=m.MPM_WS_NET_EXTRAP if extrap else m.MPM_WS_NET) as s:
        s.setup(0, box, d["mask"], d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
        gx, gy, gz = s.ws_grid(0)
        cur = scales[0]
        s.attach(net, cur, out_scale)
        prev = None
        for n in range(7):
            if n == 3:                      # new input scales
                cur = scales[1]
                s.attach(net, cur, out_scale)
            if n == 5:                      # new coefficients on the same box
                s.update(0, d["mask"], d["D"], d["k"] * 1.25, d["src"], p.c_b, p.dt, p.h)
            old = f.clone()
            s.step([f], 1e-10)
            if extrap and prev is None:     # no c^{n-1} yet: no warm start this step
                prev = old
                continue
            got = net.debug_tensor(mpm_mod.MPM_NT_INPUT).cpu().numpy().view(np.uint16)
            got = got.reshape(gz, gy, gx, -1)[..., :C]
            inp = torch.empty((gz, gy, gx, C), dtype=torch.int16, device="cuda")
            tgt = torch.empty((gz, gy, gx, S), dtype=torch.float32, device="cuda")
            s.ws_pair(0, old, f, cur, out_scale, inp, tgt, c_prev=prev if extrap else None)
            want = inp.cpu().numpy().view(np.uint16)
            for ch in range(C):
                assert np.array_equal(got[..., ch], want[..., ch]), (n, ch)
            checked += 1
            prev = old
    net.close()
    assert checked == (6 if extrap else 7)


def _masked_problem(seed, dims, S, cut):
    """A random problem whose domain leaves many of the network's 16 x 4 x 4 tiles empty:
    no domain at x < cut[0] or z < cut[1]."""
    p = random_problem(seed, dims, S=S, fill=0.7)
    p.mask[:, :, :cut[0]] = 0
    p.mask[:cut[1]] = 0
    return p


@pytest.mark.parametrize("S,P,extrap", [(3, 1, False), (3, 1, True), (4, 2, False)])
def test_in_step_warm_start_matches_definition(S, P, extrap):
    """The whole warm start of a step against its definition: the network's full forward
    pass on the input mpm_ws_pair builds, x0 = x_b + out * out_scale on the domain voxels,
    and the true residual of x0 relative to that of c^n from the oracle's assembly,
    against the step's rel_res_warm / rel_res_initial.  The step's inference pass computes
    only the tiles of the last level that the domain's outputs read, from each problem's
    own lists; the masks leave many of the grid's 16 x 4 x 4 tiles without a domain voxel,
    so a tile skipped wrongly would leave a stale output on the domain.  Four species:
    the head with four outputs in the last convolution's epilogue, two problems in one
    context."""
    torch = require_gpu()
    import paper_2505_03067_amd as m
    from paper_2505_03067_amd.train import input_scales
    probs = [_masked_problem(123, (48, 40, 36), S, (26, 14)),
             _masked_problem(124, (40, 44, 28), S, (9, 19))][:P]
    boxes = [((0, 0, 0), p.dims) for p in probs]
    out_scale = [0.05, 0.05, 1e-3, 2e-3][:S]
    scales = input_scales(S, out_scale)
    C = 5 * S + 1
    net = m.Net(C, S, [16, 32, 64, 64], seed=31)
    fs = [torch.from_numpy(p.c0).cuda() for p in probs]
    checked = 0
    with m.Solver(S, P, warm_start=m.MPM_WS_NET_EXTRAP if extrap else m.MPM_WS_NET) as s:
        for i, (p, box) in enumerate(zip(probs, boxes)):
            d = to_dev(p)
            s.setup(i, box, d["mask"], d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
        s.attach(net, scales, out_scale)
        prev = [None] * P
        for n in range(4):
            old = [f.clone() for f in fs]
            s.step(fs, 1e-10)
            st = [[s.stats(i, sp) for sp in range(S)] for i in range(P)]
            if extrap and prev[0] is None:
                prev = old
                continue
            for i, (p, box) in enumerate(zip(probs, boxes)):
                gx, gy, gz = s.ws_grid(i)
                ex, ey, ez = p.dims
                sl = box_slice(box)
                mb = p.mask[sl].astype(bool)
                inp = torch.empty((1, gz, gy, gx, C), dtype=torch.int16, device="cuda")
                tgt = torch.empty((gz, gy, gx, S), dtype=torch.float32, device="cuda")
                s.ws_pair(i, old[i], fs[i], scales, out_scale, inp[0], tgt, c_prev=prev[i] if extrap else None)
                out = torch.empty((1, gz, gy, gx, S), dtype=torch.float32, device="cuda")
                net.forward(inp, out)
                o = out[0].cpu().numpy()[:ez, :ey, :ex]
                c = old[i].cpu().numpy()
                xb = 2.0 * c - prev[i].cpu().numpy() if extrap else c
                for sp in range(S):
                    A, q = assemble(mb, p.D[sp][sl], p.k[sp][sl], p.src[sp][sl], float(p.c_b[sp]), p.dt, p.h)
                    cn = c[sp][sl][mb]
                    b = cn + q
                    x0 = xb[sp][sl][mb] + (o[..., sp][mb].astype(np.float32) *
                                           np.float32(out_scale[sp])).astype(np.float64)
                    want = np.linalg.norm(b - A @ x0) / np.linalg.norm(b - A @ cn)
                    got = st[i][sp]["rel_res_warm"] / st[i][sp]["rel_res_initial"]
                    assert abs(got - want) <= 1e-9 * want, (n, i, sp, got, want)
            checked += 1
            prev = old
    net.close()
    assert checked == (3 if extrap else 4)


def test_four_species_network_attaches_and_falls_back():
    """A 21-channel network on a four-species context: the zero prediction is rejected
    for every system and the solve matches the oracle."""
    torch = require_gpu()
    import paper_2505_03067_amd as m
    from paper_2505_03067_amd.train import input_scales
    p = random_problem(92, (24, 20, 16), S=4, fill=0.7)
    d = to_dev(p)
    f = torch.from_numpy(p.c0).cuda()
    net = m.Net(21, 4, [16, 32], seed=4)
    with m.Solver(4, 1, warm_start=m.MPM_WS_NET) as s:
        s.setup(0, p.box, d["mask"], d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
        with pytest.raises(ValueError):
            s.attach(net, input_scales(3), [0.0] * 4)       # 16 scales for 4 species
        s.attach(net, input_scales(4), [0.0] * 4)
        for _ in range(2):
            s.step([f], 1e-10)
            assert all(s.stats(0, sp)["fallback"] == 1 for sp in range(4))
    net.close()
    _check_oracle(p, 2, f.cpu().numpy())


def _plain_and_ws(p, steps, setup_net, tile=2048):
    torch = require_gpu()
    import paper_2505_03067_amd as m
    d = to_dev(p)
    res = []
    for warm in (False, True):
        f = torch.from_numpy(p.c0).cuda()
        with m.Solver(3, 1, tile_override=tile, warm_start=m.MPM_WS_NET if warm else 0) as s:
            s.setup(0, p.box, d["mask"], d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
            net = None
            if warm:
                net = setup_net(s)
            st = []
            for _ in range(steps):
                s.step([f], 1e-10)
                st.append([s.stats(0, sp) for sp in range(3)])
            if net is not None:
                net.close()
        res.append((f.cpu().numpy(), st))
    return res


def test_zero_prediction_falls_back_to_plain():
    import paper_2505_03067_amd as m
    from paper_2505_03067_amd.train import input_scales
    p = random_problem(81, (24, 24, 16), S=3, fill=0.7)

    def setup(s):
        net = m.Net(16, 3, [16, 32], seed=1)
        s.attach(net, input_scales(3), [0.0, 0.0, 0.0])
        return net

    (f0, st0), (f1, st1) = _plain_and_ws(p, 2, setup)
    assert np.array_equal(f0, f1)
    for row in st1:
        for s in row:
            assert s["fallback"] == 1 and s["warm_start_used"] == 0
            assert s["rel_res_warm"] == s["rel_res_initial"]
    _check_oracle(p, 2, f1)


def _check_oracle(p, steps, got, tol=1e-10):
    """The fields against the oracle's CG solve to 1e-13, at the 1e-8 parity bar in the
    L2 and the max norm (the L2 error is bounded by steps kappa (tol + 1e-13) with
    kappa <= 1 + dt (k_max + 12 D_max / h^2), which is printed)."""
    want, _ = run(p, steps=steps, solver="pcg", tol=1e-13)
    mb = p.mask[box_slice(p.box)].astype(bool)
    kappa = 1 + p.dt * (p.k.max() + 12 * p.D.max() / p.h ** 2)
    bound = steps * kappa * (tol + 1e-13)
    errs = rel_err_per_species(got, want, mb, p.box)
    print(f"{p.name}: rel err vs oracle {errs}, kappa bound {bound:.2e}", flush=True)
    assert max(errs) <= 1e-8, errs


def test_poisoned_network_falls_back():
    torch = require_gpu()
    import paper_2505_03067_amd as m
    from paper_2505_03067_amd.train import input_scales
    p = random_problem(82, (24, 24, 16), S=3, fill=0.7)

    def setup(s):
        net = m.Net(16, 3, [16, 32], seed=2)
        net.set_params(torch.full((net.count,), float("nan"), device="cuda"))
        s.attach(net, input_scales(3), [1.0, 1.0, 1.0])
        return net

    (f0, _), (f1, st1) = _plain_and_ws(p, 2, setup)
    assert np.array_equal(f0, f1)
    assert all(s["fallback"] == 1 for row in st1 for s in row)
    _check_oracle(p, 2, f1)


def test_extrapolated_start_parity():
    require_gpu()
    import paper_2505_03067_amd as m
    p = config1()
    got, stats = gpu_run(p, 4, 1e-12, warm_start=m.MPM_WS_EXTRAP)
    want, _ = run(p, steps=4, solver="pcg", tol=1e-13)
    mb = p.mask[box_slice(p.box)].astype(bool)
    assert max(rel_err_per_species(got, want, mb, p.box)) <= 1e-8
    assert stats[0][0]["warm_start_used"] == 0 and stats[0][0]["fallback"] == 0   # no c^{n-1} yet
    assert stats[3][0]["warm_start_used"] + stats[3][0]["fallback"] == 1
    # the extrapolation of a smoothly decaying field is a better start than c^n
    assert stats[3][0]["rel_res_warm"] < stats[3][0]["rel_res_initial"]


def test_network_corrected_extrapolation_parity():
    """MPM_WS_NET_EXTRAP with a zero correction (out_scale 0) is the extrapolated start:
    the same fields bit for bit and the same statistics as MPM_WS_EXTRAP, no warm start
    in the first step (no c^{n-1}), and the solve within 1e-8 of the oracle."""
    torch = require_gpu()
    import paper_2505_03067_amd as m
    p = config1()
    d = to_dev(p)
    res = {}
    for mode in (m.MPM_WS_EXTRAP, m.MPM_WS_NET_EXTRAP):
        f = torch.from_numpy(p.c0).cuda()
        net = m.Net(5 * p.nspecies + 1, p.nspecies, [16, 32], seed=6) if mode == m.MPM_WS_NET_EXTRAP else None
        with m.Solver(p.nspecies, 1, warm_start=mode) as s:
            s.setup(0, p.box, d["mask"], d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
            if net is not None:
                s.attach(net, [1.0] * (5 * p.nspecies + 1), [0.0] * p.nspecies)
            st = []
            for _ in range(4):
                s.step([f], 1e-12)
                st.append([s.stats(0, sp) for sp in range(p.nspecies)])
        if net is not None:
            net.close()
        res[mode] = (f.cpu().numpy(), st)
    (fe, se), (fn, sn) = res[m.MPM_WS_EXTRAP], res[m.MPM_WS_NET_EXTRAP]
    assert np.array_equal(fe, fn)
    for a, b in zip(se, sn):
        for x, y in zip(a, b):
            for k in ("iterations", "warm_start_used", "fallback", "rel_res_warm", "rel_res_initial"):
                assert x[k] == y[k], k
    assert sn[0][0]["warm_start_used"] == 0 and sn[0][0]["fallback"] == 0
    assert sn[3][0]["warm_start_used"] == 1
    _check_oracle(p, 4, fn, tol=1e-12)


def test_network_corrected_extrapolation_two_problems_four_species():
    """Two problems of four species in one context: with a zero correction the network's
    mode reproduces the extrapolated start bit for bit for both, and both match the
    oracle."""
    torch = require_gpu()
    import paper_2505_03067_amd as m
    probs = [random_problem(94, (22, 20, 18), S=4, fill=0.7), random_problem(95, (18, 24, 20), S=4, fill=0.6)]
    res = {}
    for mode in (m.MPM_WS_EXTRAP, m.MPM_WS_NET_EXTRAP):
        fs = [torch.from_numpy(p.c0).cuda() for p in probs]
        net = m.Net(21, 4, [16, 32], seed=9) if mode == m.MPM_WS_NET_EXTRAP else None
        with m.Solver(4, 2, warm_start=mode) as s:
            for i, p in enumerate(probs):
                d = to_dev(p)
                s.setup(i, p.box, d["mask"], d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
            if net is not None:
                s.attach(net, [1.0] * 21, [0.0] * 4)
            used = 0
            for _ in range(3):
                s.step(fs, 1e-12)
                used += sum(s.stats(i, sp)["warm_start_used"] for i in range(2) for sp in range(4))
        if net is not None:
            net.close()
        res[mode] = ([f.cpu().numpy() for f in fs], used)
    for a, b in zip(res[m.MPM_WS_EXTRAP][0], res[m.MPM_WS_NET_EXTRAP][0]):
        assert np.array_equal(a, b)
    assert res[m.MPM_WS_EXTRAP][1] == res[m.MPM_WS_NET_EXTRAP][1]
    for p, f in zip(probs, res[m.MPM_WS_NET_EXTRAP][0]):
        _check_oracle(p, 3, f, tol=1e-12)


def test_learned_correction_of_extrapolation():
    """Train the network on the correction of the extrapolated start (residual loss,
    pairs from mpm_ws_pair_extrap) and evaluate on an unseen patch: the start must be
    accepted, leave a smaller residual than the extrapolation alone, and the solve to
    1e-12 must match the oracle within 1e-8."""
    torch = require_gpu()
    import paper_2505_03067_amd as m
    from paper_2505_03067_amd import train as tr
    train_probs = [config4_patch(200 + i, n=32) for i in range(3)]
    raw = []
    solvers = []
    for pr in train_probs:
        s, pairs = tr.solver_pairs(pr, 12, range(1, 12), [1.0, 1.0, 1.0], extrap=True)
        raw += pairs
        s.close()
    out_scale = tr.target_rms(raw, 3)
    del raw
    items = []
    for pr in train_probs:
        s, pairs = tr.solver_pairs(pr, 12, range(1, 12), out_scale, extrap=True)
        solvers.append(s)
        items += [(s, inp, tgt) for inp, tgt in pairs]
    net = m.Net(16, 3, [16, 32, 64, 64], seed=8)
    rng = np.random.default_rng(1)
    losses = []
    for it in range(1, 301):
        net.zero_grad()
        losses.append(tr.residual_step(net, [items[int(rng.integers(len(items)))]], out_scale))
        net.adam(1e-3 * 0.5 * (1 + np.cos(np.pi * it / 300)), it)
    for s in solvers:
        s.close()
    print(f"{len(items)} pairs, residual loss {np.mean(losses[:10]):.3e} -> {np.mean(losses[-10:]):.3e}", flush=True)
    p = config4_patch(10_010, n=32)
    d = to_dev(p)
    ratios = {}
    fields = {}
    for mode in (m.MPM_WS_EXTRAP, m.MPM_WS_NET_EXTRAP):
        f = torch.from_numpy(p.c0).cuda()
        r = []
        with m.Solver(3, 1, warm_start=mode) as s:
            s.setup(0, p.box, d["mask"], d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
            if mode == m.MPM_WS_NET_EXTRAP:
                s.attach(net, tr.input_scales(3, out_scale), out_scale)
            for _ in range(5):
                s.step([f], 1e-12)
                r += [s.stats(0, sp)["rel_res_warm"] / s.stats(0, sp)["rel_res_initial"]
                      for sp in range(3) if s.stats(0, sp)["warm_start_used"]]
        ratios[mode] = r
        fields[mode] = f.cpu().numpy()
    net.close()
    re, rn = np.mean(ratios[m.MPM_WS_EXTRAP]), np.mean(ratios[m.MPM_WS_NET_EXTRAP])
    print(f"residual ratio: extrapolated {re:.3e}, corrected {rn:.3e} ({len(ratios[m.MPM_WS_NET_EXTRAP])} accepted)",
          flush=True)
    assert len(ratios[m.MPM_WS_NET_EXTRAP]) >= 6
    assert rn < re
    _check_oracle(p, 5, fields[m.MPM_WS_NET_EXTRAP], tol=1e-12)


def test_learned_warm_start_gains_over_plain():
    """Train on pairs the solver generates (456 pairs from 24 tumour patches of 32^3) and
    evaluate on unseen patches: the learned start must be accepted and cut the GMRES
    iterations, while the solution stays within 2 kappa tol of the plain solve."""
    torch = require_gpu()
    import paper_2505_03067_amd as m
    from paper_2505_03067_amd import train as tr
    import time
    train_probs = [config4_patch(100 + i, n=32) for i in range(24)]
    out_scale = tr.estimate_out_scale(train_probs[:4], 10)
    pairs = list(tr.generate_pairs(train_probs, 20, range(1, 20), out_scale))
    net = m.Net(16, 3, [16, 32, 64, 64], seed=7)
    t0 = time.perf_counter()
    losses = tr.train(net, pairs, epochs=60, batch=4, lr=2e-3, seed=0)
    print(f"{len(pairs)} pairs, training {time.perf_counter() - t0:.1f} s, losses",
          [f"{v:.3e}" for v in losses[::5]], flush=True)
    # the normalised target has unit variance: the network must explain most of it
    assert losses[-1] < 0.1
    evalp = [config4_patch(10_000 + i, n=32) for i in range(2)]
    it_plain, sps_plain, f_plain, _ = tr.evaluate(evalp, 10, 1e-8)
    it_ws, sps_ws, f_ws, acc = tr.evaluate(evalp, 10, 1e-8, net=net, out_scale=out_scale, warm=m.MPM_WS_NET)
    print(f"iterations/step plain {it_plain:.2f} learned {it_ws:.2f}; accepted {acc:.2f}; "
          f"steps/s plain {sps_plain:.1f} learned {sps_ws:.1f}")
    assert acc > 0.5
    assert it_ws < it_plain
    kappa = 1 + 1.0 * (0.2 + 12 * 1.5)
    for a, b in zip(f_plain, f_ws):
        assert np.linalg.norm(a - b) <= 2 * kappa * 1e-8 * np.linalg.norm(a)
    # the learned-start solve itself against the oracle: one unseen patch, solved to
    # 1e-12 from the accepted learned start, every field within 1e-8 of the oracle's CG
    p = evalp[0]
    d = to_dev(p)
    f = torch.from_numpy(p.c0).cuda()
    used = 0
    with m.Solver(3, 1, warm_start=m.MPM_WS_NET) as s:
        s.setup(0, p.box, d["mask"], d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
        s.attach(net, tr.input_scales(3, out_scale), out_scale)
        for _ in range(4):
            s.step([f], 1e-12)
            used += sum(s.stats(0, sp)["warm_start_used"] for sp in range(3))
    net.close()
    print(f"learned start accepted for {used} of 12 systems at tol 1e-12", flush=True)
    assert used >= 6
    _check_oracle(p, 4, f.cpu().numpy(), tol=1e-12)


def test_ws_loss_matches_definition():
    """The residual loss of a prediction and its gradient against the oracle's
    assembly: e = (out - target) out_scale on the domain voxels, w = S A e,
    loss = sum (w / out_scale)^2 / (S N), grad = 2 A S w / (S N out_scale), zero off the
    domain; a ragged masked box whose grid is padded past it."""
    torch = require_gpu()
    import paper_2505_03067_amd as m
    from paper_2505_03067_amd.train import input_scales
    p = random_problem(93, (26, 22, 18), S=3, fill=0.7)
    box = ((1, 2, 1), (24, 21, 17))
    S = 3
    out_scale = [0.3, 0.2, 4e-3]
    d = to_dev(p)
    f = torch.from_numpy(p.c0).cuda()
    with m.Solver(S, 1, warm_start=m.MPM_WS_NET) as s:
        s.setup(0, box, d["mask"], d["D"], d["k"], d["src"], p.c_b, p.dt, p.h)
        s.step([f], 1e-10)
        old = f.clone()
        s.step([f], 1e-10)
        gx, gy, gz = s.ws_grid(0)
        inp = torch.empty((gz, gy, gx, 5 * S + 1), dtype=torch.int16, device="cuda")
        tgt = torch.empty((gz, gy, gx, S), dtype=torch.float32, device="cuda")
        s.ws_pair(0, old, f, input_scales(S, out_scale), out_scale, inp, tgt)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(5)
        out = tgt + 0.1 * torch.randn(tgt.shape, generator=gen, device="cuda")
        grad = torch.empty_like(out)
        loss = s.ws_loss(0, out, tgt, out_scale, grad)
    sl = box_slice(box)
    mb = p.mask[sl].astype(bool)
    ex, ey, ez = [hi - lo for lo, hi in zip(*box)]
    o = out.cpu().numpy().astype(np.float64)[:ez, :ey, :ex]
    t = tgt.cpu().numpy().astype(np.float64)[:ez, :ey, :ex]
    g = grad.cpu().numpy().astype(np.float64)
    N = int(mb.sum())
    want_loss = 0.0
    want_grad = np.zeros((gz, gy, gx, S))
    for sp in range(S):
        A, _ = assemble(mb, p.D[sp][sl], p.k[sp][sl], p.src[sp][sl], float(p.c_b[sp]), p.dt, p.h)
        os_ = float(np.float32(out_scale[sp]))
        e = (o[..., sp][mb] - t[..., sp][mb]) * os_
        sc = 1.0 / np.sqrt(A.diagonal())
        w = sc * (A @ e)
        want_loss += float(((w / os_) ** 2).sum())
        gv = 2.0 / (S * N * os_) * (A @ (sc * w))
        want_grad[:ez, :ey, :ex, sp][mb] = gv
    want_loss /= S * N
    print(f"loss {loss:.6e} oracle {want_loss:.6e}", flush=True)
    assert abs(loss - want_loss) <= 1e-12 * want_loss
    dom = np.zeros((gz, gy, gx), bool)
    dom[:ez, :ey, :ex] = mb
    assert np.all(g[~dom] == 0.0)
    err = np.abs(g - want_grad)
    assert np.all(err <= 2.0 ** -23 * np.abs(want_grad) + 1e-12 * np.abs(want_grad).max())
