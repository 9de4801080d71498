"""MI355X-native higher-order delay-multiply-and-sum photoacoustic beamforming.

The compute path lives in ``libhodmas.so`` (hand-written HIP for gfx950 behind a
C ABI, declared in ``include/hodmas.h``); ``hodmas`` is its thin Python binding.
"""
__all__ = ["phantom", "hodmas"]
