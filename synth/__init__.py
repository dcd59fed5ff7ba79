"""Seeded synthetic inputs for the ray-by-ray MGFLD transport step.

This package defines workloads only (grids, stellar profiles, opacities).  It
contains no transport arithmetic, and both the CPU oracle and the HIP path
consume the arrays it produces.
"""
from .workload import (  # noqa: F401
    C_LIGHT, SEED, TERM_DIFFUSION, TERM_EMABS, TERM_NES, TERMS_ALL,
    BC_ZERO_FLUX, BC_FREE_STREAM, BC_GEOMETRIC, LIMITER_NONE, LIMITER_INTRP, LIMITER_GEOM, R_NU_CM, CONFIGS, Workload, make, make_custom, YeInputs, ye_inputs, EadvInputs,
    eadv_inputs,
)
