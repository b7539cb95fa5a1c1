"""MI355X particle-mesh hot path of an electrostatic IFE-PIC step.

The compute runs in the HIP library ``libpic.so`` (gfx950 kernels behind the
C-ABI of ``include/pic.h``); this package is its Python binding.
"""
from .pic import (Batch, Config, Context, PicError, Profile, config_from_workload,  # noqa: F401
                  footprint_bytes, lib, DEPOSIT, OBJECT, REPR, SIGNATURES, LIB_PATH)
