"""MI355X (gfx950) echo synthesis for FMCW roadside radar (arXiv 2208.10939 hot path).

The HIP library librsim.so does all the work; `rsim` marshals arguments to it and
`pipeline` strings the calls together with torch tensors for device memory.
"""
from .rsim import (Context, RsimError, lib, LIB_PATH, RSIM_FP32_PHASE64, RSIM_FP64,
                   RSIM_MASK_COMPUTE, RSIM_MASK_INPUT)

__all__ = ["Context", "RsimError", "lib", "LIB_PATH", "RSIM_FP32_PHASE64", "RSIM_FP64",
           "RSIM_MASK_COMPUTE", "RSIM_MASK_INPUT"]
