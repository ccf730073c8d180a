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
    bank_4x128,
    bank_1024,
    batch_streams,
    chirp_fit,
    precision_bank,
    chirp_target,
    chirp_init_bank,
    trigger_series,
    resample_taps,
    multirate_bank,
    coloured_noise,
)
