"""Seeded synthetic ensemble fields and pair lists.

This package produces INPUTS only: smoothed-Gaussian ensemble fields with
planted correlated blobs, region boxes and random point-pair lists. It holds
none of the correlation arithmetic (no standardisation, no Pearson, no KSG, no
maxima), so both the GPU library's tests and the CPU oracle may consume what it
generates without sharing any of the method's code.
"""
from .fields import (  # noqa: F401
    Ensemble,
    Region,
    make_cfg1,
    make_cfg2,
    make_cfg3,
    make_cfg4,
    make_context,
    make_two_variables,
    context_regions,
    region_pair_list,
    make_field,
    random_pairs,
    region_pairs_uniform,
    smooth_noise,
)
from .device import smooth_field_torch  # noqa: F401,E402
