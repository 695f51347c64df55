"""MI355X-native population-annealing molecular dynamics (PAMD) hot path.

The work runs in HIP kernels for gfx950 inside ``libpamd.so`` (C ABI in
``include/pamd.h``); ``paper_1806_06016_amd.pamd`` is its ctypes binding.
"""
from .pamd import (Pamd, PamdError, load_library, LIB_PATH, PAMD_FP32, PAMD_FP64, PAMD_OK,  # noqa: F401
                   PAMD_ERR_ARG, PAMD_ERR_HIP, PAMD_ERR_CAPACITY, PAMD_ERR_NONFINITE, PAMD_ERR_STATE,
                   EXPORTS)
