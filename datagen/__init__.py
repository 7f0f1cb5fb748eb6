"""Seeded synthetic inputs for the PARAFAC2 hot path.

This package only draws inputs: sparse irregular slices {X_k} in one
concatenated CSR, initial factors, fixed serving factors and request
streams.  It holds none of the method's arithmetic, so both the FP64
oracle and the HIP path can take their inputs from it without sharing
any computation.
"""
from .synth import (  # noqa: F401
    ROOT_SEED,
    CHUNK,
    Slices,
    gen_slices,
    gen_config,
    gen_init,
    gen_planted,
    gen_batched_specs,
    gen_serving_model,
    gen_serving_requests,
    take_subjects,
    concat_slices,
    CONFIGS,
)
