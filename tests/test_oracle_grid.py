"""Pins of the refined-grid builder (Section 3c) against Table 2 and Eqs 11-12."""
import math
import os

import numpy as np
import pytest

from oracle.grid import cell_count_estimate, cell_reduction, refined_nodes

HERE = os.path.dirname(os.path.abspath(__file__))
L = 0.3
DX_REF = L / 2048
L_BUFF = 0.05


def table2():
    rows = []
    with open(os.path.join(HERE, "golden", "table2_cells.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                a, b, n = line.split()
                rows.append((int(a), int(b), int(n)))
    return rows


@pytest.mark.parametrize("a,b,n", table2())
def test_table2_total_cells(a, b, n):
    nodes = refined_nodes(L, a * DX_REF, b * DX_REF, L_BUFF)
    assert len(nodes) - 1 == n


@pytest.mark.parametrize("a,b,n", table2())
def test_refinement_rules(a, b, n):
    """The four rules of Section 3c, and Eqs 11-12 up to the transition cells."""
    nodes = refined_nodes(L, a * DX_REF, b * DX_REF, L_BUFF)
    h = np.diff(nodes)
    dmin, dmax = a * DX_REF, b * DX_REF
    # Sizes are dmin times a power of two, at most dmax.
    ratio = h / dmin
    assert np.allclose(ratio, 2.0 ** np.round(np.log2(ratio)), rtol=1e-9)
    assert h.max() <= dmax * (1 + 1e-9)
    # Buffer: every cell starting within L_buff of an electrode is dmin wide.
    left = nodes[:-1] < L_BUFF
    right = nodes[1:] > L - L_BUFF
    assert np.allclose(h[left | right], dmin, rtol=1e-9)
    # Neighbours differ by at most a factor of two.
    q = h[1:] / h[:-1]
    assert np.all((q > 0.49) & (q < 2.01))
    # Symmetric about the mid-plane.
    assert np.allclose(h, h[::-1], rtol=1e-9)
    # Eq 11 ignores the transition cells: at most two extra cells per doubling per side.
    est = cell_count_estimate(L, L_BUFF, dmin, dmax)
    R = b / a
    assert abs(n - est) <= 4 * math.log2(R) + 2
    # Eq 12 is Eq 11 normalised by the unrefined count L / dx_min.
    assert cell_reduction(L, L_BUFF, R) == pytest.approx(est / (L / dmin), rel=1e-12)


def test_largest_reduction_quoted_in_text():
    # Section 3c: up to a 9.4x reduction in the number of cells (2048 -> 218).
    n = len(refined_nodes(L, 4 * DX_REF, 32 * DX_REF, L_BUFF)) - 1
    assert round(2048 / n, 1) == 9.4
