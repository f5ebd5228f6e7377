"""The flop/byte accounting reproduces the paper's own arithmetic-intensity table and claims."""
import os

import numpy as np

from paper_1409_1510_amd import perfmodel as pm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_arith_intensity.txt")


def test_table1_reproduced_to_printed_digits():
    rows = np.loadtxt(GOLDEN)
    for n, full, r14 in rows:
        assert round(pm.paper_model_intensity(int(n), 18), 2) == full
        assert round(pm.paper_model_intensity(int(n), 14), 2) == r14


def test_section1_claims():
    # limit of the model for n -> infinity; the text rounds it to about 2.75
    lim = pm.paper_model_limit()
    assert 2.7 < lim < 2.85
    # n = 8 reaches about 75 % of the limit, n = 1 about 25-30 %
    assert 0.72 < pm.paper_model_intensity(8) / lim < 0.78
    assert 0.25 <= pm.paper_model_intensity(1) / lim <= 0.30
    # the r14 gain shrinks from about 10 % (n = 1) to about 3 % (n = 8)
    g1 = pm.paper_model_intensity(1, 14) / pm.paper_model_intensity(1) - 1
    g8 = pm.paper_model_intensity(8, 14) / pm.paper_model_intensity(8) - 1
    assert 0.07 < g1 < 0.11 and 0.02 < g8 < 0.04
    # going from 1 to 4 rhs more than doubles the intensity
    assert pm.paper_model_intensity(4) / pm.paper_model_intensity(1) > 2


def test_compulsory_bytes():
    assert pm.FLOP_PER_SITE_RHS == 1146
    assert pm.compulsory_bytes(1, 4, 4) == 1152 + 48
    assert pm.compulsory_bytes(16, 8, 8) == 2304 + 16 * 96
    assert pm.compulsory_bytes(8, 2, 4) == 576 + 8 * 48
    assert pm.compulsory_bytes(1, 4, 4, recon=14) == 1024 + 48
