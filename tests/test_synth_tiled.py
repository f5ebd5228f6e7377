"""The tiled link generator repeats the 4^4 field periodically (sampled sites) and refuses
extents that are not multiples of 4."""
import numpy as np
import pytest

import synth


def test_tiled_links_repeat_the_small_field():
    dims = (8, 4, 12, 8)
    fat, naik = synth.tiled_gauge_links(dims, 11)
    fs, ns = synth.gauge_links((4, 4, 4, 4), 11)
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(0)
    for _ in range(50):
        x, y, z, t = (int(rng.integers(d)) for d in dims)
        big = x + lx * (y + ly * (z + lz * t))
        small = (x % 4) + 4 * ((y % 4) + 4 * ((z % 4) + 4 * (t % 4)))
        assert np.array_equal(fat[big], fs[small]) and np.array_equal(naik[big], ns[small])


def test_tiled_links_need_multiples_of_4():
    with pytest.raises(ValueError):
        synth.tiled_gauge_links((6, 4, 4, 4), 1)
