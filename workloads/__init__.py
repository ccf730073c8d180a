"""Seeded synthetic workloads (strain streams, filter banks, chirp targets).

This package holds no filtering arithmetic: it draws random numbers and
evaluates the leading-order chirp formula used as a fitting target. Both the
FP64 oracle and the HIP library consume what it produces.
"""
from .gen import (  # noqa: F401
    Bank,
    SEED_ROOT,
    strain,
    random_bank,
    config0,
    config1,
    config2,
    config3,
    config4,
    chirp_target,
    chirp_init_bank,
)
