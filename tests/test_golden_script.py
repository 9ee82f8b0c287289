"""The full-size golden script's parallel wall data equals the oracle's.

tests/golden/make_fullsize.py splits the oracle's wall-node local sum over
processes; every node's sum must be bitwise that of oracle.wall_data.
"""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import oracle as O  # noqa: E402
from workloads import random_case  # noqa: E402

pytestmark = pytest.mark.skipif(sys.platform != "linux", reason="fork start method")


def test_parallel_wall_data_is_bitwise_the_oracle():
    import make_fullsize as M
    c = random_case(5, 600, 10, 6.0, 1.5, 3.0, 1.0, 16, 16, 17)
    g = O.SlitGrid.from_case(c)
    xs = g.wrap(c.xs)
    f = np.asarray(c.f, dtype=np.float64)
    ref = O.wall_data(g, xs, f)
    got = M.parallel_wall_data(g, xs, f, 2)
    for a, b in zip(ref, got):
        assert a.shape == b.shape == (3, 16, 16)
        assert np.array_equal(a, b)
