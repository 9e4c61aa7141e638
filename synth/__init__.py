"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package only *draws* inputs (images, displacement fields, probe vectors).
It holds none of the registration method's arithmetic: no grid conversion, no
template interpolation, no NGF residual, no derivative.  Both sides of every
parity check receive the very same arrays produced here.
"""
from .volumes import (  # noqa: F401
    GridSpec,
    blob_pair,
    ct_pair,
    ct_warp,
    ct_inverse_target,
    smooth_field,
    quarter_nodes,
    config_c1,
    config_c2,
    config_c3,
    config_c4_sizes,
    section_pair,
    alignment_errors,
    smooth_field_2d,
    config_section,
)
