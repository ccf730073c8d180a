"""MI355X-native summed parallel IIR (SPIIR) filter-bank library.

``libspiir.so`` (HIP, gfx950) does all the work; this package is its Python
binding. There is no CPU fallback: using the bank without the built library
raises.
"""
from ._lib import (  # noqa: F401
    EXPORTS,
    PREC_FP32,
    PREC_FP64_CARRY,
    PREC_HYBRID,
    SpiirError,
    load,
)


def __getattr__(name):
    # torch-dependent classes are imported lazily so that the ABI checks run
    # without initialising any GPU runtime
    if name in ("SpiirBank", "SpiirBatch", "SpiirFn", "SpiirMultiRate", "Tape", "TriggerClusterer", "TriggerStream", "Whitener", "autotune",
                "batch_banks", "cluster_triggers", "version"):
        from . import bank
        return getattr(bank, name)
    raise AttributeError(name)
