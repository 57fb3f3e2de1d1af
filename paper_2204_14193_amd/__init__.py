"""MI355X (gfx950) complex-valued Frequency Selective Extrapolation.

The compute runs in ``libfse.so`` (hand-written HIP kernels behind a C ABI,
declared in ``include/fse.h``); this package only marshals arguments. There
is no CPU fallback: if the library is not built, importing the binding
raises.
"""
from .fse import (Plan, Batch, Batch3d, extrapolate_batch, extrapolate3d, blocks_from_mask, BLOCK_DTYPE,
                  VOLUME_DTYPE, TRACE_DTYPE, BLOCK_OK, BLOCK_EMPTY_SUPPORT, BLOCK_NONFINITE, FseError,
                  measure_lds_bandwidth)

__all__ = ["Plan", "Batch", "Batch3d", "extrapolate_batch", "extrapolate3d", "blocks_from_mask", "BLOCK_DTYPE",
           "VOLUME_DTYPE", "TRACE_DTYPE",
           "BLOCK_OK", "BLOCK_EMPTY_SUPPORT", "BLOCK_NONFINITE", "FseError", "measure_lds_bandwidth"]
