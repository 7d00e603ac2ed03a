"""Seeded synthetic inputs shaped like the StyleBlit paper's workloads.

This package generates bytes only: exemplar textures, source and target guides
and the per-cell random jitter tables that the seed hierarchy draws from
(Sec. 3.2, SeedPoint's RandomJitterTable).  It holds none of the method's
arithmetic, so that the CPU oracle and the HIP path can both consume exactly
the same inputs without sharing any code with each other.
"""
from .gen import (  # noqa: F401
    GUIDE_U8X2,
    GUIDE_U16X2,
    GUIDE_U8X3,
    GUIDE_U8XN,
    GUIDE_U16XN,
    Frame,
    Style,
    Params,
    level_spacings,
    jitter_cells,
    jitter_table,
    value_noise_rgb,
    sphere_guide_u8,
    bump_guide_u8,
    identity_uv_guide_u16,
    warped_uv_guide_u16,
    voronoi_labels,
    animated_bump_guides,
    jitter_schedule,
    appearance_u8,
    guide_u8x3,
    appearance_target,
    APPEARANCE_PARAMS,
    texel_elements,
    guide_n,
    chroma_u8,
    features_u8,
    features_u16,
    features_target,
    FEATURE_PARAMS,
    FEATURE16_PARAMS,
    config,
    CONFIG_NAMES,
)
