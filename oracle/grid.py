"""Grids: uniform, and the paper's refined sheath grid.

Test infrastructure only (see ``oracle/__init__.py``).

Section 3c gives four rules for the non-uniform grid: cells within L_buff of
either electrode have size dx_min; outside that buffer cells may grow up to
dx_max; sizes change only by doubling or halving; and no two neighbouring cells
differ by more than a factor of two.  The paper does not say how the rules are
discretised.  The reading used here is a dyadic (binary-tree) refinement of the
whole gap: a cell of size s = L / 2^l is split in two while s > dx_max, or
while it overlaps a buffer region and s > dx_min; then any cell more than twice
the size of a neighbour is split until no such pair remains (a 2:1 balance).
This reading reproduces every "total number of cells" entry of Table 2 exactly
(L = 0.3 m, dx_ref = L / 2048, L_buff = 5 cm), which the tests check.

Eq (11) estimates the cell count and Eq (12) the reduction ratio CR; both are
given here as written so the tests can compare the built grids with them.
"""
from __future__ import annotations

import numpy as np


def uniform_nodes(L, n_cells):
    """Nodes of a uniform grid, x_n = n L / N (for reference; the uniform grid of
    the particle contract uses dx = L / N and never these rounded nodes)."""
    return np.arange(n_cells + 1, dtype=np.float64) * (L / n_cells)


def refined_cells(n_levels, level_min, level_max, buff_units):
    """Dyadic refinement with 2:1 balance, in integer units of the finest cell.

    The gap is 2**n_levels units.  Cells of size 2**(n_levels - level) units
    exist for level in [level_max, level_min] (level_min is the finest).  A
    cell overlaps a buffer when it starts before ``buff_units`` or ends after
    ``2**n_levels - buff_units``.  Returns the list of (start, end) unit pairs.
    """
    U = 1 << n_levels
    s_min = 1 << (n_levels - level_min)   # size of the finest cells in units
    s_max = 1 << (n_levels - level_max)
    cells = [(0, U)]
    changed = True
    while changed:
        changed = False
        out = []
        for a, b in cells:
            s = b - a
            in_buf = (a < buff_units) or (b > U - buff_units)
            if s > s_max or (in_buf and s > s_min):
                m = (a + b) // 2
                out += [(a, m), (m, b)]
                changed = True
            else:
                out.append((a, b))
        cells = out
    changed = True
    while changed:
        changed = False
        out = []
        for i, (a, b) in enumerate(cells):
            s = b - a
            neigh = [cells[j][1] - cells[j][0] for j in (i - 1, i + 1) if 0 <= j < len(cells)]
            if any(s > 2 * t for t in neigh):
                m = (a + b) // 2
                out += [(a, m), (m, b)]
                changed = True
            else:
                out.append((a, b))
        cells = out
    return cells


def refined_nodes(L, dx_min, dx_max, L_buff):
    """Node positions of the Section 3c grid.

    dx_min and dx_max must be L / 2**a and L / 2**b (b <= a), which is how the
    paper sizes them (powers-of-two multiples of dx_ref = L / 2048).
    """
    a = int(round(np.log2(L / dx_min)))
    b = int(round(np.log2(L / dx_max)))
    if not (np.isclose(L / 2 ** a, dx_min, rtol=1e-12) and np.isclose(L / 2 ** b, dx_max, rtol=1e-12)):
        raise ValueError("dx_min and dx_max must be L / 2**k")
    n_levels = a
    buff_units = L_buff / dx_min   # may be fractional: overlap is tested against it
    cells = refined_cells(n_levels, a, b, buff_units)
    unit = L / (1 << n_levels)
    starts = np.array([c[0] for c in cells] + [1 << n_levels], dtype=np.float64)
    return starts * unit


def cell_count_estimate(L, L_buff, dx_min, dx_max):
    """Eq (11): N_x ~ (L - 2 L_buff)/dx_max + 2 L_buff/dx_min."""
    return (L - 2.0 * L_buff) / dx_max + 2.0 * L_buff / dx_min


def cell_reduction(L, L_buff, R):
    """Eq (12): CR = 2 (1 - 1/R) L_buff / L + 1/R."""
    return 2.0 * (1.0 - 1.0 / R) * L_buff / L + 1.0 / R
