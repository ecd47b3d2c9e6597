"""hafgpu: hafnians and loop hafnians on MI355X (gfx950) through a C-ABI HIP library.

The Python layer only marshals arguments; see ``_native`` and ``include/hafgpu.h``.
"""
from ._native import (  # noqa: F401
    KIND_HAF, KIND_LHAF, HafError, Server, batched_config, batched_dev, batched_load_cache, batched_plan,
    batched_tune, device_info, haf_dev, haf_dev_dd, haf_exact, haf_host, haf_host_dd, haf_lowrank, haf_modp,
    load, now, perm_dev, perm_host, profile_enable, profile_read, release_workspaces, set_batched_config,
    set_kernel_path, terms_dev,
)


def haf(A):
    """haf(A) of a host matrix (numpy-compatible), computed on the GPU."""
    return haf_host(A, KIND_HAF)


def lhaf(A):
    """lhaf(A) of a host matrix, computed on the GPU."""
    return haf_host(A, KIND_LHAF)
