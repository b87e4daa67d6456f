"""Seeded synthetic MPO inputs shared by the oracle checks, the GPU tests and the bench.

This module only draws random numbers and shapes: it holds none of the fit
method's arithmetic, so both the CPU oracle and the HIP path can consume the
same input bits without sharing any code of the method itself.
"""
from .mpo_inputs import (  # noqa: F401
    gaussian_mpo,
    uniform_alpha_mpo,
    make_pair,
    make_problem,
    multi_pair_chis,
    make_multi_pair,
    string_sum_mpo,
    reflector_product_mpo,
    CONFIGS,
)
