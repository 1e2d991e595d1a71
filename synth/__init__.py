"""Seeded synthetic MWA-like inputs shared by the tests, the bench and the oracle checks.

This module only builds inputs (array geometry, uvw tracks, visibilities, flags and
weights).  It contains none of the gridding arithmetic: no kernel, no coordinate
snapping, no scatter or gather.
"""
from .mwa import (  # noqa: F401
    CONFIGS,
    Workload,
    antenna_positions,
    baseline_enu,
    channel_frequencies,
    make_workload,
    uvw_tracks,
)
from .polarisation import make_polconv_inputs  # noqa: F401
from .gcf import make_baseline_kernels  # noqa: F401
