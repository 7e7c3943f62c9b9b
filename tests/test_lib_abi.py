"""CPU-side checks of the C ABI: the library loads, exports every declared symbol, and
rejects bad arguments before touching a device."""

import ctypes
import os

import pytest

import paper_2505_03067_amd as m
from paper_2505_03067_amd import mpm as b


def test_library_exports_every_header_symbol():
    L = m.lib()
    names = m.header_symbols()
    assert "mpm_implicit_step" in names and "mpm_bbox_from_cells" in names
    for name in names:
        assert hasattr(L, name), name


def test_binding_argument_counts_match_header():
    """Every declaration in include/mpm.h has as many parameters as the binding passes."""
    import re
    text = open(b.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    decls = dict(re.findall(r"\b(mpm_[a-z_0-9]+)\s*\(([^)]*)\)\s*;", text))
    L = m.lib()
    for name, params in decls.items():
        params = params.strip()
        n = 0 if params in ("", "void") else params.count(",") + 1
        fn = getattr(L, name)
        if fn.argtypes is not None:
            assert len(fn.argtypes) == n, (name, n, len(fn.argtypes))


def test_default_options():
    o = m.mpm_default_options()
    assert o.restart == 30 and o.max_cycles == 50
    assert o.precision == m.MPM_FP32_IR and o.batched == 1
    assert 0 < o.inner_rtol < 1e-3


def test_struct_layouts_match_header():
    # mpm_options: 8 int32 + 1 double; mpm_stats: 6 int32 + 3 double + float + int32
    assert ctypes.sizeof(b.mpm_options) == 40
    assert ctypes.sizeof(b.mpm_stats) == 56


@pytest.mark.parametrize("ns,npb", [(0, 1), (5, 1), (1, 0), (4, 17)])
def test_create_rejects_bad_sizes(ns, npb):
    ctx = ctypes.c_void_p()
    rc = m.lib().mpm_create(ctypes.byref(ctx), ns, npb, None, None)
    assert rc == m.MPM_EINVAL
    assert "mpm_create" in m.mpm_last_error()
    assert not ctx.value


@pytest.mark.parametrize("field,value", [("restart", 0), ("restart", 31), ("precision", 7),
                                         ("max_cycles", 0), ("inner_rtol", 2.0),
                                         ("tile_override", 1000), ("warm_start", 9), ("ortho", 2)])
def test_create_rejects_bad_options(field, value):
    o = m.mpm_default_options()
    setattr(o, field, value)
    ctx = ctypes.c_void_p()
    assert m.lib().mpm_create(ctypes.byref(ctx), 3, 1, ctypes.byref(o), None) == m.MPM_EINVAL


def test_null_pointers_rejected():
    L = m.lib()
    dims = (ctypes.c_int32 * 3)(4, 4, 4)
    lo = (ctypes.c_int32 * 3)()
    hi = (ctypes.c_int32 * 3)()
    assert L.mpm_bbox_from_cells(None, dims, 1, lo, hi, None) == m.MPM_EINVAL
    assert L.mpm_implicit_step(None, None, 1e-8) == m.MPM_EINVAL
    assert L.mpm_fv_setup(None, 0, dims, lo, hi, None, None, None, None, None, 1.0, 1.0) == m.MPM_EINVAL
    st = b.mpm_stats()
    assert L.mpm_gmres_stats(None, 0, 0, ctypes.byref(st)) == m.MPM_EINVAL
    assert L.mpm_debug_apply(None, 0, None, None, 0) == m.MPM_EINVAL
    assert m.mpm_default_options().restart == 30


def test_bbox_rejects_bad_dims_without_device_access():
    L = m.lib()
    lo = (ctypes.c_int32 * 3)()
    hi = (ctypes.c_int32 * 3)()
    fake = ctypes.c_void_p(0x1000)       # never dereferenced: the size check comes first
    assert L.mpm_bbox_from_cells(fake, (ctypes.c_int32 * 3)(0, 4, 4), 1, lo, hi, None) == m.MPM_EINVAL
    assert L.mpm_bbox_from_cells(fake, (ctypes.c_int32 * 3)(4, 4, 4), -1, lo, hi, None) == m.MPM_EINVAL


def test_oracle_is_not_imported_by_the_product():
    pkg = os.path.dirname(m.__file__)
    for root, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(root, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
