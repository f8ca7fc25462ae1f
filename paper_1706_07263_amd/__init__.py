"""MI355X-native haemoglobin estimation from RGB frames via Haar decomposition.

The hot path lives in the HIP/C library ``libhbgpu.so`` (C ABI in
``include/hb.h``); ``paper_1706_07263_amd.hb`` is its thin ctypes binding.
Nothing is imported eagerly so that the synthetic-input module can be used
without the GPU library.
"""
__all__ = ["hb", "synth"]
