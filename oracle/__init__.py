"""Plain, slow FP64 CPU oracle of the EC-PIC / MC-PIC time step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library never
calls it, links it or falls back to it, and it shares no code with the GPU
path: every formula here is written from the paper (Powis & Kaganovich,
"Accuracy of the explicit energy-conserving particle-in-cell method for
under-resolved simulations of capacitively coupled plasma discharges") and
from the readings stated in ``oracle/pic.py``.

Modules
-------
philox   Philox4x32-10 / 4x64-10 counter-based generator (generic in width).
physics  constants, argon cross sections, null-collision bounds.
grid     uniform and Section 3c refined grids, Eqs (11)-(12).
pic      the algorithm steps (Eqs 2-9, collisions, emission, initial load).
sim      the time loop of Section 2a and the averaged diagnostics of Section 3a.

Parity status: every function is pinned by a CPU test against closed forms,
invariants, brute force or values the paper prints (see tests/test_oracle_*.py),
except the whole-discharge profiles, which are Monte-Carlo estimates and are
"parity unpinned" against physical numbers (the paper's numbers are helium).
"""
from . import grid, philox, physics, pic, sim  # noqa: F401
from .sim import Sim  # noqa: F401
