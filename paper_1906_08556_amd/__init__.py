"""MI355X-native TV-model EM hot path (i-vector extraction and training).

The compute lives in libivx.so (hand-written HIP for gfx950 behind the C ABI
in include/ivx.h); ``paper_1906_08556_amd.ivx`` is its ctypes binding.
"""
__all__ = ["ivx", "build"]
