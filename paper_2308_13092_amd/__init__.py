"""MI355X-native explicit energy-conserving PIC (1D3V argon RF-CCP).

The particle loop of Powis & Kaganovich, "Accuracy of the explicit
energy-conserving particle-in-cell method for under-resolved simulations of
capacitively coupled plasma discharges" (Section 2a), runs as hand-written HIP
kernels for gfx950 behind the C ABI of ``include/ecpic.h``; this package is
the thin Python binding plus the batch, autotuning and serving layers above it.
"""
from ._lib import (Context, PicError, footprint, grid_refined, load, slot_bytes)  # noqa: F401
