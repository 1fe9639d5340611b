"""Seeded synthetic inputs for HODLR factor/solve runs.

This package only *draws* inputs: cluster trees, leaf blocks, low-rank
generators, point sets, curve geometry and right-hand sides.  It holds none
of the factor/solve or compression arithmetic, so both the CPU oracle and the
HIP path can take their inputs from here without sharing any of the method.
"""
from .hodlr_inputs import (  # noqa: F401
    HodlrInputs,
    uniform_offsets,
    rank_prefix,
    synthetic,
    bie_star,
    kernel_matrix,
    helmholtz_matrix,
    rcb_order,
    kernel_points,
    star_curve,
    gaussian_rhs,
    CONFIGS,
    make_config,
)
