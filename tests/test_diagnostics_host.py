"""Host logic of paper_1707_00198_amd/diagnostics.py (no GPU): the Eq. 47 reading and the
interface-region helper."""
import math

import numpy as np

from paper_1707_00198_amd.diagnostics import circle_region, e_npmt


def test_e_npmt_zero_without_transfer_and_pythagorean_otherwise():
    assert e_npmt([100.0, 0.0, 0.0, 400.0]) == 0.0
    # 3 % of the red beyond the interface, 4 % of the blue inside it -> 5 %
    assert math.isclose(e_npmt([97.0, 3.0, 16.0, 384.0]), 0.05, rel_tol=1e-12)
    # the printed superscripts (red inside, blue outside) would give ~1.4 here instead
    assert e_npmt([97.0, 3.0, 16.0, 384.0]) < 0.1


def test_circle_region_counts_node_centres():
    r = circle_region((50, 80), 40.0, 25.0, 10.0)
    y, x = np.nonzero(r)
    assert ((x - 40.0) ** 2 + (y - 25.0) ** 2 <= 100.0).all()
    assert r.sum() == sum(1 for yy in range(50) for xx in range(80)
                          if (xx - 40.0) ** 2 + (yy - 25.0) ** 2 <= 100.0)
