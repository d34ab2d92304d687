"""MI355X-native engine for the one-loop fRG right-hand side (hp-fRG hot path).

The compute path is ``libfrg.so`` (HIP for gfx950, C ABI declared in
``include/frg.h``); :mod:`paper_1510_07799_amd.frg` is its thin ctypes binding.
Nothing is loaded at import time so that CPU-only code (input generators,
argument checks) can be used without a GPU.
"""
