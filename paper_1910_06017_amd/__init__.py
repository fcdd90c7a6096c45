"""Pyramidal Lucas-Kanade box tracking on AMD Instinct MI355X (gfx950).

The tracking stage of OmniTrack (arXiv 1910.06017, Sec. V-A: preprocessing,
feature calculation and prediction phases) as hand-written HIP kernels behind
a C ABI (``include/omnitrack.h``).  This package holds the thin ctypes binding
(`ops`), the batched/graph scheduler (`batch`), the serving loop (`serve`)
and the seeded input generators (`synth`).
"""
__all__ = ["ops", "synth", "batch", "serve"]
