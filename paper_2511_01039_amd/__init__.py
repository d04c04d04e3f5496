"""MI355X (gfx950) boundary-MPS row absorption for finite PEPS-PEPO networks.

The compute lives in ``libfpeps.so`` (hand-written HIP kernels behind the C
ABI of include/fpeps.h); this package only marshals arguments.
"""
from .binding import (Context, DeviceTensor, FpepsError, make_opts, opts_for, load,
                      exported_symbols, LIB_PATH)

__all__ = ["Context", "DeviceTensor", "FpepsError", "make_opts", "opts_for", "load",
           "exported_symbols", "LIB_PATH"]
