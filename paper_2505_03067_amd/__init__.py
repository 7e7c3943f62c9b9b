"""MI355X-native implicit-Euler finite-volume reaction-diffusion on a tumour bounding box.

The compute path is ``libmpm.so`` (hand-written HIP for gfx950, C ABI in
``include/mpm.h``); ``mpm`` is its thin ctypes binding.  PyTorch only supplies
device memory and streams.
"""

from .mpm import (  # noqa: F401
    MPM_EEMPTY, MPM_EHIP, MPM_EINVAL, MPM_ENOMEM, MPM_ESTATE, MPM_FP32_IR, MPM_FP64,
    MPM_NOT_CONVERGED, MPM_OK, MPM_WS_EXTRAP, MPM_WS_NET, MPM_WS_NET_EXTRAP, MPM_WS_NONE, MpmError, Net, Solver,
    header_symbols, lib, mpm_bbox_from_cells, mpm_bbox_from_cells_noalloc, mpm_create, mpm_debug_apply, mpm_debug_krylov,
    mpm_default_options, mpm_destroy, mpm_fv_setup, mpm_fv_update, mpm_hbm_probe, mpm_gmres_stats, mpm_implicit_step,
    mpm_last_error, mpm_tile, mpm_ws_pair_extrap, mpm_time_kernel, mpm_kernel_timing, MPM_KERNEL_NONE, MPM_KERNEL_SPMV_DOT,
    MPM_KERNEL_AXPY_DOT, MPM_KERNEL_AXPY_NORM, MPM_KERNEL_UPDATE, MPM_KERNEL_RESIDUAL,
    MPM_ORTHO_CGS2, MPM_ORTHO_DCGS2, MPM_PROBE_READ, MPM_PROBE_COPY, MPM_PROBE_TRIAD, MPM_PROBE_NONTEMPORAL,
)
