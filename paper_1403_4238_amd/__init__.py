"""MI355X-native exemplar-based object removal (Criminisi-style inpainting).

The hot path -- fill front, FP64 priority, masked-SSD exemplar search and the
copy/confidence update -- runs in hand-written HIP kernels for gfx950 behind
the C ABI declared in ``include/inpaint.h``.  ``binding`` is the thin Python
layer over that library; ``synth`` draws the seeded synthetic workloads.
"""
__all__ = ["synth", "binding"]
