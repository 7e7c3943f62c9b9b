"""ctypes binding of libmpm (argument marshalling only).

Every function has the name of the C entry point it wraps (see ``include/mpm.h``).
Tensors are PyTorch tensors on the GPU; the binding checks dtype, device and
contiguity, passes ``data_ptr()`` and the current HIP stream, and turns negative
status codes into ``MpmError``.  No computation happens here: if ``libmpm.so`` is
missing the import fails loudly, there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmpm.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "mpm.h")

MPM_OK = 0
MPM_NOT_CONVERGED = 1
MPM_EINVAL = -1
MPM_ENOMEM = -2
MPM_EHIP = -3
MPM_EEMPTY = -4
MPM_ESTATE = -5
MPM_FP64 = 0
MPM_FP32_IR = 1
MPM_WS_NONE = 0
MPM_WS_NET = 1
MPM_WS_EXTRAP = 2
MPM_WS_NET_EXTRAP = 3
MPM_ORTHO_CGS2 = 0
MPM_ORTHO_DCGS2 = 1

_NAMES = {MPM_EINVAL: "MPM_EINVAL", MPM_ENOMEM: "MPM_ENOMEM", MPM_EHIP: "MPM_EHIP",
          MPM_EEMPTY: "MPM_EEMPTY", MPM_ESTATE: "MPM_ESTATE"}


class MpmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class mpm_options(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("max_cycles", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("batched", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("warm_start", ctypes.c_int32),
                ("tile_override", ctypes.c_int32), ("ortho", ctypes.c_int32),
                ("inner_rtol", ctypes.c_double)]


class mpm_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("cycles", ctypes.c_int32),
                ("refinements", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("warm_start_used", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("rel_res_initial", ctypes.c_double), ("rel_res_warm", ctypes.c_double),
                ("rel_res_final", ctypes.c_double), ("ms_total", ctypes.c_float),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


_lib = None
_i32p = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p


def lib() -> ctypes.CDLL:
    """Load libmpm.so from the package directory (built by ``build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "'python -m paper_2505_03067_amd.build'")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "mpm_bbox_from_cells": [_vp, _i32p, ctypes.c_int32, _i32p, _i32p, _vp],
            "mpm_bbox_from_cells_noalloc": [_vp, _i32p, ctypes.c_int32, _i32p, _i32p, _vp],
            "mpm_default_options": [ctypes.POINTER(mpm_options)],
            "mpm_create": [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.c_int32,
                           ctypes.POINTER(mpm_options), _vp],
            "mpm_fv_setup": [_vp, ctypes.c_int32, _i32p, _i32p, _i32p, _vp, _vp, _vp, _vp,
                             ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_double],
            "mpm_fv_update": [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double),
                              ctypes.c_double, ctypes.c_double],
            "mpm_implicit_step": [_vp, ctypes.POINTER(_vp), ctypes.c_double],
            "mpm_gmres_stats": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(mpm_stats)],
            "mpm_destroy": [_vp],
            "mpm_debug_apply": [_vp, ctypes.c_int32, _vp, _vp, ctypes.c_int32],
            "mpm_debug_krylov": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _i32p,
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)],
            "mpm_time_kernel": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
            "mpm_tile": [_vp, _i32p],
            "mpm_net_create": [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                               _i32p, ctypes.c_uint64, _vp],
            "mpm_net_params": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                               ctypes.POINTER(ctypes.c_int64)],
            "mpm_net_sync_weights": [_vp],
            "mpm_net_read": [_vp, ctypes.c_int32, _vp],
            "mpm_net_write": [_vp, ctypes.c_int32, _vp],
            "mpm_net_forward": [_vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_int32, _vp],
            "mpm_net_infer": [_vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                              ctypes.c_int32, _vp],
            "mpm_net_backward": [_vp, _vp],
            "mpm_net_zero_grad": [_vp],
            "mpm_net_mse": [_vp, _vp, _vp, ctypes.c_int64, _vp, ctypes.POINTER(ctypes.c_double)],
            "mpm_net_adam_step": [_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_float, ctypes.c_int32],
            "mpm_net_destroy": [_vp],
            "mpm_net_debug_layer": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp],
            "mpm_net_debug_tensor": [_vp, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.POINTER(ctypes.c_int64)],
            "mpm_net_debug_op": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp],
            "mpm_attach_net": [_vp, _vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
            "mpm_ws_pair": [_vp, ctypes.c_int32, _vp, _vp, ctypes.POINTER(ctypes.c_float),
                            ctypes.POINTER(ctypes.c_float), _vp, _vp],
            "mpm_ws_pair_extrap": [_vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_float),
                                   ctypes.POINTER(ctypes.c_float), _vp, _vp],
            "mpm_ws_grid": [_vp, ctypes.c_int32, _i32p],
            "mpm_ws_loss": [_vp, ctypes.c_int32, _vp, _vp, ctypes.POINTER(ctypes.c_float), _vp,
                            ctypes.POINTER(ctypes.c_double)],
            "mpm_hbm_probe": [ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                              _vp, ctypes.POINTER(ctypes.c_double)],
            "mpm_kernel_timing": [_vp, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int32
        L.mpm_last_error.argtypes = []
        L.mpm_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def header_symbols() -> list:
    """Names of every function declared in include/mpm.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(mpm_[a-z_0-9]+)\s*\(", text)))


def mpm_last_error() -> str:
    return lib().mpm_last_error().decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise MpmError(rc, mpm_last_error())
    return rc


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _triple(v):
    return (ctypes.c_int32 * 3)(*[int(a) for a in v])


def mpm_default_options(**overrides) -> mpm_options:
    o = mpm_options()
    _check(lib().mpm_default_options(ctypes.byref(o)))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def mpm_bbox_from_cells(cell_id, margin: int, stream=None):
    """Box ``(lo, hi)`` ((x, y, z) triples) of the positive voxels of ``cell_id`` [z][y][x]."""
    import torch
    ptr = _dev_ptr(cell_id, torch.int32, "cell_id")
    if cell_id.dim() != 3:
        raise ValueError("cell_id must be [z][y][x]")
    nz, ny, nx = cell_id.shape
    lo = (ctypes.c_int32 * 3)()
    hi = (ctypes.c_int32 * 3)()
    _check(lib().mpm_bbox_from_cells(ptr, _triple((nx, ny, nz)), int(margin), lo, hi,
                                     _stream(stream)))
    return tuple(lo), tuple(hi)


def mpm_bbox_from_cells_noalloc(cell_id, margin: int, stream=None):
    """As mpm_bbox_from_cells, through the entry point that allocates nothing."""
    import torch
    ptr = _dev_ptr(cell_id, torch.int32, "cell_id")
    if cell_id.dim() != 3:
        raise ValueError("cell_id must be [z][y][x]")
    nz, ny, nx = cell_id.shape
    lo = (ctypes.c_int32 * 3)()
    hi = (ctypes.c_int32 * 3)()
    _check(lib().mpm_bbox_from_cells_noalloc(ptr, _triple((nx, ny, nz)), int(margin), lo, hi,
                                             _stream(stream)))
    return tuple(lo), tuple(hi)


def mpm_create(nspecies: int, nproblems: int = 1, options: Optional[mpm_options] = None,
               stream=None) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    opt = ctypes.byref(options) if options is not None else None
    _check(lib().mpm_create(ctypes.byref(ctx), int(nspecies), int(nproblems), opt,
                            _stream(stream)))
    return ctx


def mpm_fv_setup(ctx, problem: int, box, mask, D, k, src, c_dirichlet: Sequence[float],
                 dt: float, h: float):
    """Discretise ``problem`` on ``box = (lo, hi)``; lattice arrays are torch tensors."""
    import torch
    if mask.dim() != 3:
        raise ValueError("mask must be [z][y][x]")
    nz, ny, nx = mask.shape
    for name, a in (("D", D), ("k", k), ("src", src)):
        if a.dim() != 4 or tuple(a.shape[1:]) != (nz, ny, nx):
            raise ValueError(f"{name} must be [S][z][y][x] matching the mask")
    lo, hi = box
    cb = (ctypes.c_double * len(c_dirichlet))(*[float(v) for v in c_dirichlet])
    return _check(lib().mpm_fv_setup(ctx, int(problem), _triple((nx, ny, nz)), _triple(lo),
                                     _triple(hi), _dev_ptr(mask, torch.uint8, "mask"),
                                     _dev_ptr(D, torch.float64, "D"),
                                     _dev_ptr(k, torch.float64, "k"),
                                     _dev_ptr(src, torch.float64, "src"), cb, float(dt),
                                     float(h)))


def mpm_fv_update(ctx, problem: int, mask, D, k, src, c_dirichlet: Sequence[float], dt: float, h: float):
    """New coefficients on the box and domain of the last mpm_fv_setup of ``problem``."""
    import torch
    cb = (ctypes.c_double * len(c_dirichlet))(*[float(v) for v in c_dirichlet])
    return _check(lib().mpm_fv_update(ctx, int(problem), _dev_ptr(mask, torch.uint8, "mask"),
                                      _dev_ptr(D, torch.float64, "D"), _dev_ptr(k, torch.float64, "k"),
                                      _dev_ptr(src, torch.float64, "src"), cb, float(dt), float(h)))


def mpm_implicit_step(ctx, fields, tol: float) -> int:
    """One step for every problem; ``fields`` is a list of FP64 [S][z][y][x] tensors."""
    import torch
    arr = (ctypes.c_void_p * len(fields))(
        *[_dev_ptr(f, torch.float64, f"fields[{i}]").value for i, f in enumerate(fields)])
    return _check(lib().mpm_implicit_step(ctx, arr, float(tol)))


def mpm_gmres_stats(ctx, problem: int = 0, species: int = 0) -> dict:
    st = mpm_stats()
    _check(lib().mpm_gmres_stats(ctx, int(problem), int(species), ctypes.byref(st)))
    return st.as_dict()


def mpm_destroy(ctx) -> None:
    if ctx is not None and ctx.value:
        lib().mpm_destroy(ctx)


def mpm_debug_apply(ctx, problem: int, x, y, mode: int) -> None:
    import torch
    _check(lib().mpm_debug_apply(ctx, int(problem), _dev_ptr(x, torch.float64, "x"),
                                 _dev_ptr(y, torch.float64, "y"), int(mode)))


def mpm_debug_krylov(ctx, problem: int, species: int, kmax: int, n: int):
    """Krylov state of one system after the last cycle: (m, vs [k], basis [k][n], H [k][kmax+1])
    with k = min(m, kmax) columns; ``n`` = domain voxels of the problem's box."""
    import numpy as np
    m = ctypes.c_int32(0)
    vs = np.zeros(kmax)
    basis = np.zeros((kmax, n))
    hess = np.zeros((kmax, kmax + 1))
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().mpm_debug_krylov(ctx, int(problem), int(species), int(kmax), ctypes.byref(m),
                                  vs.ctypes.data_as(dp), basis.ctypes.data_as(dp), hess.ctypes.data_as(dp)))
    k = min(m.value, kmax)
    return m.value, vs[:k], basis[:k], hess[:k]


MPM_KERNEL_NONE = 0
MPM_KERNEL_SPMV_DOT = 1
MPM_KERNEL_AXPY_DOT = 2
MPM_KERNEL_AXPY_NORM = 3
MPM_KERNEL_UPDATE = 4
MPM_KERNEL_RESIDUAL = 5


def mpm_time_kernel(ctx, kind: int, j: int = 0, repeat: int = 1) -> None:
    _check(lib().mpm_time_kernel(ctx, int(kind), int(j), int(repeat)))


def mpm_kernel_timing(ctx) -> dict:
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    by = ctypes.c_double()
    _check(lib().mpm_kernel_timing(ctx, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)))
    return {"ms": ms.value, "launches": n.value, "bytes": by.value}


MPM_PROBE_READ = 0
MPM_PROBE_COPY = 1
MPM_PROBE_TRIAD = 2
MPM_PROBE_NONTEMPORAL = 0x100


def mpm_hbm_probe(kind: int, a, b, c, nbytes: int, blocks: int = 4096, repeat: int = 5, stream=None) -> float:
    """Average duration in ms of one streaming-probe launch (see include/mpm.h)."""
    ms = ctypes.c_double()
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    base = int(kind) & 0xFF
    need = {"a": int(nbytes), "b": int(nbytes) if base == MPM_PROBE_TRIAD else 0,
            "c": 4 * int(blocks) if base == MPM_PROBE_READ else int(nbytes)}
    for name, t in (("a", a), ("b", b), ("c", c)):
        if t is not None and (t.device.type != "cuda" or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous GPU tensor")
        size = 0 if t is None else t.numel() * t.element_size()
        if size < need[name]:
            raise ValueError(f"{name} holds {size} bytes, the probe needs {need[name]}")
    _check(lib().mpm_hbm_probe(int(kind), ptr(a), ptr(b), ptr(c), int(nbytes), int(blocks), int(repeat),
                               _stream(stream), ctypes.byref(ms)))
    return ms.value


def mpm_tile(ctx) -> int:
    v = ctypes.c_int32()
    _check(lib().mpm_tile(ctx, ctypes.byref(v)))
    return v.value


def mpm_net_create(in_ch: int, out_ch: int, widths, seed: int = 0, stream=None):
    net = ctypes.c_void_p()
    w = (ctypes.c_int32 * len(widths))(*[int(v) for v in widths])
    _check(lib().mpm_net_create(ctypes.byref(net), int(in_ch), int(out_ch), len(widths), w,
                                int(seed), _stream(stream)))
    return net


def mpm_net_param_count(net) -> int:
    p = ctypes.c_void_p()
    g = ctypes.c_void_p()
    n = ctypes.c_int64()
    _check(lib().mpm_net_params(net, ctypes.byref(p), ctypes.byref(g), ctypes.byref(n)))
    return n.value


def mpm_net_read(net, what: int, dst) -> None:
    import torch
    _check(lib().mpm_net_read(net, int(what), _dev_ptr(dst, torch.float32, "dst")))


def mpm_net_write(net, what: int, src) -> None:
    import torch
    _check(lib().mpm_net_write(net, int(what), _dev_ptr(src, torch.float32, "src")))


def mpm_net_forward(net, x, out, infer=False) -> None:
    """x: BF16 data as int16/uint16 tensor [n][d][h][w][c]; out: FP32 [n][d][h][w][out_ch].
    With infer, mpm_net_infer (no backward pass may follow)."""
    import torch
    if x.dtype not in (torch.int16, torch.uint16, torch.bfloat16):
        raise TypeError("x must hold BF16 bit patterns (int16/uint16/bfloat16)")
    if x.dim() != 5 or not x.is_contiguous() or x.device.type != "cuda":
        raise ValueError("x must be a contiguous 5-D GPU tensor")
    nb, d, h, w, _ = x.shape
    fn = lib().mpm_net_infer if infer else lib().mpm_net_forward
    _check(fn(net, ctypes.c_void_p(x.data_ptr()), nb, d, h, w, _dev_ptr(out, torch.float32, "out")))


def mpm_net_infer(net, x, out) -> None:
    mpm_net_forward(net, x, out, infer=True)


def mpm_net_backward(net, grad_out) -> None:
    import torch
    _check(lib().mpm_net_backward(net, _dev_ptr(grad_out, torch.float32, "grad_out")))


def mpm_net_zero_grad(net) -> None:
    _check(lib().mpm_net_zero_grad(net))


def mpm_net_mse(net, out, target, grad_out) -> float:
    import torch
    loss = ctypes.c_double()
    _check(lib().mpm_net_mse(net, _dev_ptr(out, torch.float32, "out"),
                             _dev_ptr(target, torch.float32, "target"), out.numel(),
                             _dev_ptr(grad_out, torch.float32, "grad_out"), ctypes.byref(loss)))
    return loss.value


def mpm_net_adam_step(net, lr, b1=0.9, b2=0.999, eps=1e-8, t=1) -> None:
    _check(lib().mpm_net_adam_step(net, float(lr), float(b1), float(b2), float(eps), int(t)))


def mpm_net_destroy(net) -> None:
    if net is not None and net.value:
        lib().mpm_net_destroy(net)


MPM_MAX_SPECIES = 4


def _scales(in_scale, out_scale, nspecies=None):
    """ctypes arrays of the warm-start scales.  The library reads 5 S + 1 input and S
    output scales; with ``nspecies`` the lengths must be exactly those, and the arrays
    are always at least as long as the largest S needs, so no read runs past them."""
    if nspecies is not None and (len(in_scale) != 5 * nspecies + 1 or len(out_scale) != nspecies):
        raise ValueError(f"need {5 * nspecies + 1} input scales and {nspecies} output scales, "
                         f"got {len(in_scale)} and {len(out_scale)}")
    ni = max(len(in_scale), 5 * MPM_MAX_SPECIES + 1)
    no = max(len(out_scale), MPM_MAX_SPECIES)
    a = (ctypes.c_float * ni)(*[float(v) for v in in_scale])
    b = (ctypes.c_float * no)(*[float(v) for v in out_scale])
    return a, b


def mpm_attach_net(ctx, net, in_scale, out_scale, nspecies=None) -> None:
    h = net.handle if isinstance(net, Net) else net
    a, b = _scales(in_scale, out_scale, nspecies)
    _check(lib().mpm_attach_net(ctx, h, a, b))


def mpm_ws_grid(ctx, problem: int = 0):
    g = (ctypes.c_int32 * 3)()
    _check(lib().mpm_ws_grid(ctx, int(problem), g))
    return tuple(g)


def mpm_ws_pair(ctx, problem, c_old, c_new, in_scale, out_scale, in_bf16, target, nspecies=None) -> None:
    import torch
    if in_bf16.dtype not in (torch.int16, torch.uint16, torch.bfloat16) or not in_bf16.is_contiguous():
        raise TypeError("in_bf16 must be a contiguous 16-bit tensor")
    a, b = _scales(in_scale, out_scale, nspecies)
    _check(lib().mpm_ws_pair(ctx, int(problem), _dev_ptr(c_old, torch.float64, "c_old"),
                             _dev_ptr(c_new, torch.float64, "c_new"), a, b,
                             ctypes.c_void_p(in_bf16.data_ptr()),
                             _dev_ptr(target, torch.float32, "target")))


def mpm_ws_pair_extrap(ctx, problem, c_prev, c_old, c_new, in_scale, out_scale, in_bf16, target,
                       nspecies=None) -> None:
    import torch
    if in_bf16.dtype not in (torch.int16, torch.uint16, torch.bfloat16) or not in_bf16.is_contiguous():
        raise TypeError("in_bf16 must be a contiguous 16-bit tensor")
    a, b = _scales(in_scale, out_scale, nspecies)
    _check(lib().mpm_ws_pair_extrap(ctx, int(problem), _dev_ptr(c_prev, torch.float64, "c_prev"),
                                    _dev_ptr(c_old, torch.float64, "c_old"), _dev_ptr(c_new, torch.float64, "c_new"),
                                    a, b, ctypes.c_void_p(in_bf16.data_ptr()),
                                    _dev_ptr(target, torch.float32, "target")))


MPM_NT_INPUT = 0
MPM_NT_ACT = 1
MPM_NT_ACT_GRAD = 2
MPM_NT_POOLED = 3
MPM_NT_CAT = 4
MPM_NT_CAT_GRAD = 5
MPM_NT_HEAD_GRAD = 6
MPM_OP_POOL = 0
MPM_OP_POOL_BWD_ADD = 1
MPM_OP_UP2_CAT = 2
MPM_OP_UP2_BWD = 3
MPM_OP_HEAD = 4
MPM_OP_HEAD_BWD = 5
MPM_OP_PAD = 6


def mpm_net_debug_tensor(net, kind: int, index: int = 0):
    import torch
    cnt = ctypes.c_int64(0)
    _check(lib().mpm_net_debug_tensor(net, int(kind), int(index), None, ctypes.byref(cnt)))
    t = torch.empty(cnt.value, dtype=torch.int16, device="cuda")
    _check(lib().mpm_net_debug_tensor(net, int(kind), int(index), ctypes.c_void_p(t.data_ptr()),
                                      ctypes.byref(cnt)))
    return t


def mpm_net_debug_op(net, op: int, shape, c: int, c2: int, a, b, out, out2=None) -> None:
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    for name, t in (("a", a), ("b", b), ("out", out), ("out2", out2)):
        if t is not None and (t.device.type != "cuda" or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous GPU tensor")
    nb, d, h, w = [int(v) for v in shape]
    _check(lib().mpm_net_debug_op(net, int(op), nb, d, h, w, int(c), int(c2), ptr(a), ptr(b), ptr(out),
                                  ptr(out2)))


def mpm_ws_loss(ctx, problem, out, target, out_scale, grad_out) -> float:
    import torch
    loss = ctypes.c_double()
    sc = (ctypes.c_float * max(len(out_scale), MPM_MAX_SPECIES))(*[float(v) for v in out_scale])
    _check(lib().mpm_ws_loss(ctx, int(problem), _dev_ptr(out, torch.float32, "out"),
                             _dev_ptr(target, torch.float32, "target"), sc,
                             _dev_ptr(grad_out, torch.float32, "grad_out"), ctypes.byref(loss)))
    return loss.value


class Net:
    """Owns one U-Net handle (convenience wrapper over the mpm_net_* functions)."""

    def __init__(self, in_ch=13, out_ch=3, widths=(16, 32, 64, 64), seed=0, stream=None):
        self.handle = mpm_net_create(in_ch, out_ch, widths, seed, stream)
        self.in_ch, self.out_ch, self.widths = in_ch, out_ch, tuple(widths)
        self.count = mpm_net_param_count(self.handle)

    def params(self):
        import torch
        t = torch.empty(self.count, dtype=torch.float32, device="cuda")
        mpm_net_read(self.handle, 0, t)
        return t

    def grads(self):
        import torch
        t = torch.empty(self.count, dtype=torch.float32, device="cuda")
        mpm_net_read(self.handle, 1, t)
        return t

    def set_params(self, t):
        mpm_net_write(self.handle, 0, t.contiguous())

    def set_grads(self, t):
        mpm_net_write(self.handle, 1, t.contiguous())

    def forward(self, x, out, infer=False):
        """Forward pass (mpm_net_forward); with infer the inference pass (mpm_net_infer),
        after which backward raises until the next plain forward pass."""
        if x.dim() != 5 or x.shape[-1] != self.in_ch:
            raise ValueError(f"x must be [n][d][h][w][{self.in_ch}]")
        if tuple(out.shape) != tuple(x.shape[:4]) + (self.out_ch,):
            raise ValueError(f"out must be [n][d][h][w][{self.out_ch}] matching x")
        mpm_net_forward(self.handle, x, out, infer=infer)
        self._out_numel = out.numel()

    def backward(self, grad_out):
        if grad_out.numel() != getattr(self, "_out_numel", -1):
            raise ValueError("grad_out must have the shape of the last forward pass's output")
        mpm_net_backward(self.handle, grad_out)

    def zero_grad(self):
        mpm_net_zero_grad(self.handle)

    def mse(self, out, target, grad_out):
        if target.numel() != out.numel() or grad_out.numel() != out.numel():
            raise ValueError("out, target and grad_out must have the same number of values")
        return mpm_net_mse(self.handle, out, target, grad_out)

    def adam(self, lr, t, b1=0.9, b2=0.999, eps=1e-8):
        mpm_net_adam_step(self.handle, lr, b1, b2, eps, t)

    def debug_layer(self, layer, mode, x, g, gate, out):
        """One 3x3x3 layer on caller tensors (see mpm_net_debug_layer); x, g, gate hold
        BF16 bit patterns (16-bit tensors, NDHWC) or None."""
        ref = x if x is not None else g
        nb, d, h, w = ref.shape[:4]
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        _check(lib().mpm_net_debug_layer(self.handle, int(layer), int(mode), nb, d, h, w, ptr(x), ptr(g),
                                         ptr(gate), ctypes.c_void_p(out.data_ptr())))

    def debug_tensor(self, kind, index=0):
        """A BF16 tensor stored by the last forward/backward pass (see
        mpm_net_debug_tensor), returned as a flat int16 GPU tensor of bit patterns."""
        return mpm_net_debug_tensor(self.handle, kind, index)

    def debug_op(self, op, shape, c, c2, a, b, out, out2=None):
        """One data-movement kernel on caller tensors (see mpm_net_debug_op); ``shape`` is
        the finer grid (n, d, h, w)."""
        mpm_net_debug_op(self.handle, op, shape, c, c2, a, b, out, out2)

    def close(self):
        mpm_net_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None) is not None:
                self.close()
        except Exception:
            pass


class Solver:
    """Owns one context; a convenience wrapper over the functions above."""

    def __init__(self, nspecies: int, nproblems: int = 1, stream=None, **options):
        self.options = mpm_default_options(**options)
        self.ctx = mpm_create(nspecies, nproblems, self.options, stream)
        self.nspecies = nspecies
        self.nproblems = nproblems

    def setup(self, problem, box, mask, D, k, src, c_dirichlet, dt, h):
        return mpm_fv_setup(self.ctx, problem, box, mask, D, k, src, c_dirichlet, dt, h)

    def update(self, problem, mask, D, k, src, c_dirichlet, dt, h):
        return mpm_fv_update(self.ctx, problem, mask, D, k, src, c_dirichlet, dt, h)

    def step(self, fields, tol):
        return mpm_implicit_step(self.ctx, list(fields), tol)

    def stats(self, problem=0, species=0):
        return mpm_gmres_stats(self.ctx, problem, species)

    def iterations(self, problem=0):
        """GMRES iterations of the last step summed over the species of ``problem``
        (mpm_gmres_stats into one reused record, for per-step bookkeeping)."""
        st = getattr(self, "_st", None)
        if st is None:
            st = self._st = mpm_stats()
        L = lib()
        n = 0
        for sp in range(self.nspecies):
            _check(L.mpm_gmres_stats(self.ctx, int(problem), sp, ctypes.byref(st)))
            n += st.iterations
        return n

    def time_kernel(self, kind, j=0, repeat=1):
        return mpm_time_kernel(self.ctx, kind, j, repeat)

    def tile(self):
        return mpm_tile(self.ctx)

    def kernel_timing(self):
        return mpm_kernel_timing(self.ctx)

    def attach(self, net, in_scale, out_scale):
        mpm_attach_net(self.ctx, net, in_scale, out_scale, self.nspecies)

    def ws_grid(self, problem=0):
        return mpm_ws_grid(self.ctx, problem)

    def ws_pair(self, problem, c_old, c_new, in_scale, out_scale, in_bf16, target, c_prev=None):
        """Training pair (mpm_ws_pair); with c_prev, the pair of the extrapolated base start
        (mpm_ws_pair_extrap)."""
        gx, gy, gz = self.ws_grid(problem)
        S = self.nspecies
        if in_bf16.numel() != gx * gy * gz * (5 * S + 1) or target.numel() != gx * gy * gz * S:
            raise ValueError(f"in_bf16 must hold {gx * gy * gz * (5 * S + 1)} values and target "
                             f"{gx * gy * gz * S} (grid {gx} x {gy} x {gz}, {S} species)")
        fields = [("c_old", c_old), ("c_new", c_new)] + ([("c_prev", c_prev)] if c_prev is not None else [])
        for name, f in fields:
            if f.dim() != 4 or f.shape[0] != S or f.shape != c_old.shape:
                raise ValueError(f"{name} must be [S][z][y][x] like c_old")
        if c_prev is None:
            mpm_ws_pair(self.ctx, problem, c_old, c_new, in_scale, out_scale, in_bf16, target, self.nspecies)
        else:
            mpm_ws_pair_extrap(self.ctx, problem, c_prev, c_old, c_new, in_scale, out_scale, in_bf16, target,
                               self.nspecies)

    def ws_loss(self, problem, out, target, out_scale, grad_out):
        """Residual loss of a warm-start prediction and its gradient (see mpm_ws_loss)."""
        gx, gy, gz = self.ws_grid(problem)
        n = gx * gy * gz * self.nspecies
        if out.numel() != n or target.numel() != n or grad_out.numel() != n or len(out_scale) != self.nspecies:
            raise ValueError(f"out, target and grad_out must hold {n} values, out_scale {self.nspecies}")
        return mpm_ws_loss(self.ctx, problem, out, target, out_scale, grad_out)

    def apply(self, problem, x, y, mode):
        return mpm_debug_apply(self.ctx, problem, x, y, mode)

    def krylov(self, problem, species, kmax, n):
        return mpm_debug_krylov(self.ctx, problem, species, kmax, n)

    def close(self):
        mpm_destroy(self.ctx)
        self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if getattr(self, "ctx", None) is not None:
                self.close()
        except Exception:
            pass
