"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and fixes their shapes. It holds none of the
reconstruction method's arithmetic (no spectra, FFTs, dynamics or losses): every
transformation of these draws into method inputs is done separately by the oracle
and by the product's host helpers.
"""
from .inputs import (  # noqa: F401
    white_noise,
    mlp_weights_raw,
    mlp_weights,
    halo_net_weights,
    unit_normal,
    random_positions,
    random_modes_direction,
)
