"""MI355X-native demag + exchange + LLG hot path (HIP, gfx950).

Python surface over the C ABI in include/mmx.h.  PyTorch supplies device
memory and the stream; every step of the computation runs in libmmx.so.
"""
from ._lib import (MM_DEMAG, MM_EXCHANGE, MM_F32, MM_F64, MM_NO_GRAPH, MM_NO_RENORM, MMError, lib)
from .api import (DemagPlan, Batch, HEff, llg_run_checkpointed, llg_stability, plan_bytes, plan_scratch_bytes,
                  RK4_IMAG_LIMIT)

__all__ = ["DemagPlan", "Batch", "HEff", "llg_run_checkpointed", "llg_stability", "RK4_IMAG_LIMIT", "plan_bytes",
           "plan_scratch_bytes", "MMError", "lib",
           "MM_DEMAG", "MM_EXCHANGE", "MM_F32", "MM_F64", "MM_NO_GRAPH", "MM_NO_RENORM"]
