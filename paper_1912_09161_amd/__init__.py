"""MI355X-native VELO reconstruction (arXiv:1912.09161, Sec. 2.3.1).

The computation lives in libvelo.so (hand-written HIP kernels for gfx950
behind the C ABI of include/velo.h); this package only marshals arguments.
"""
from .velo import (  # noqa: F401
    EV_BAD_OFFSETS,
    EV_BAD_WORD,
    EV_DUPLICATE,
    EV_HOLE,
    EV_LAYER_ORDER,
    EV_OVERFLOW,
    MAX_CANDIDATES,
    VeloError,
    alloc_hits,
    alloc_states,
    alloc_tracks,
    alloc_workspace,
    cluster,
    default_params,
    find_tracks,
    fit,
    lib,
    lib_path,
    reconstruct,
    workspace_bytes,
)
