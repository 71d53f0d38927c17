"""The NumPy input generator on the CPU: a band of rows equals the same rows of the whole
frame (the recipe is keyed by pixel index, so bands can be generated on their own)."""

import numpy as np
import pytest

from synth import numpy_gen as g


def test_rows_of_a_frame_match_the_whole_frame():
    r, f = g.make_frame(37, 23, 5, seed=3)
    for rows in ((0, 1), (4, 11), (22, 23), (0, 23)):
        r2, f2 = g.make_frame(37, 23, 5, seed=3, rows=rows)
        assert np.array_equal(r[:, :, rows[0]:rows[1]], r2) and np.array_equal(f[:, :, rows[0]:rows[1]], f2)
    R = g.make_reference(37, 23, seed=5, spp=8)
    assert np.array_equal(R[:, 20:23], g.make_reference(37, 23, seed=5, spp=8, rows=(20, 23)))
    for bad in ((5, 5), (-1, 3), (20, 24)):
        with pytest.raises(ValueError):
            g.make_frame(37, 23, 2, seed=3, rows=bad)
