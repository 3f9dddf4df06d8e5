"""CPU oracle of the VELO reconstruction path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  It wraps `libvelo_oracle.so`, built from
`velo_oracle.c` (plain C, binary32 arithmetic without contraction), and
shares no code with the HIP implementation.
"""
from .oracle import (  # noqa: F401
    DEFAULT_PARAMS,
    EV_BAD_OFFSETS,
    EV_BAD_WORD,
    EV_DUPLICATE,
    EV_HOLE,
    EV_LAYER_ORDER,
    EV_OVERFLOW,
    EV_PV_OVERFLOW,
    EV_UT_OVERFLOW,
    MAX_PVS,
    UT_MAX_HITS,
    UT_REGIONS,
    UT_SECTORS,
    UtParams,
    PvParams,
    MAX_CANDIDATES,
    N_PARAMS,
    build,
    cluster,
    features,
    find_pvs,
    find_tracks,
    fit,
    fit_momentum,
    fit_points,
    fit_points_p,
    layer_z,
    lib_path,
    mlp_forward,
    mlp_forward_bf16,
    mlp_fwd_bwd,
    pv_params,
    reconstruct,
    ut_params,
    ut_strip_u,
    ut_windows,
)
