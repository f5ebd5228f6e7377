"""Pins of the trace-estimator oracle: the SplitMix64 stream against its published reference
outputs, the Z2 noise values, unbiasedness against the exact trace of the dense inverse, and the
closed-form variance of the Z2 estimator."""
import os

import numpy as np

import synth
from oracle import trace

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed1234567.txt")


def test_splitmix64_reference_outputs():
    ref = [int(l) for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    got = [int(v) for v in trace.splitmix64(1234567, np.arange(5))]
    assert got == ref


def test_z2_noise_values_and_counter_layout():
    vh = 96
    eta = trace.z2_noise(77, 0, 3, vh)
    assert eta.shape == (3, 3, vh)
    assert np.all(eta.imag == 0) and np.all(np.abs(eta.real) == 1)
    # vectors 1 and 2 drawn on their own continue the same stream
    assert np.array_equal(trace.z2_noise(77, 1, 2, vh), eta[1:])
    # component c = (k*3 + colour)*vh + site uses output c
    k, col, s = 2, 1, 17
    c = (k * 3 + col) * vh + s
    bit = int(trace.splitmix64(77, [c])[0]) >> 63
    assert eta[k, col, s].real == (-1.0 if bit else 1.0)
    big = trace.z2_noise(5, 0, 8, 4096)
    assert abs(big.real.mean()) < 0.02


def test_estimator_is_unbiased_with_the_z2_variance():
    dims, mass = (4, 4, 4, 4), 0.5
    fat, naik = synth.gauge_links(dims, 91)
    exact = trace.trace_minv_exact(fat, naik, dims, mass)
    s = trace.trace_samples(fat, naik, dims, mass, 92, 3000)
    se = s.std(ddof=1) / np.sqrt(s.size)
    assert abs(s.mean() - exact) <= 5 * se, (s.mean(), exact, se)
    a = np.linalg.inv(trace.dense_m(fat, naik, dims, mass))
    off = a.real.copy()
    np.fill_diagonal(off, 0.0)
    var = 2 * np.sum(off ** 2)
    assert abs(s.var(ddof=1) / var - 1) < 0.15, (s.var(ddof=1), var)


def test_chiral_condensate_from_the_even_odd_trace():
    """(1/V) Tr (m + D)^-1 of the whole-lattice operator, assembled densely from Eq. 3 and
    inverted, equals (2m/V) Tr M_ee^-1 of the even-odd operator: pins the even-odd reduction
    (parity blocks, the sign of M = m^2 - D_eo D_oe, the odd block sharing the even block's
    spectrum) against an operator assembled independently of M, at two masses on random links,
    on 4^4 (where hops alias) and on 6 x 4 x 4 x 4."""
    for dims, seed in (((4, 4, 4, 4), 93), ((6, 4, 4, 4), 94)):
        fat, naik = synth.gauge_links(dims, seed)
        for mass in (0.3, 2.5):
            full = trace.chiral_condensate_exact(fat, naik, dims, mass)
            eo = trace.chiral_condensate_from_trace(trace.trace_minv_exact(fat, naik, dims, mass), dims, mass)
            assert abs(full - eo) <= 1e-10 * abs(full), (dims, mass, full, eo)
            # a dropped factor 2 (only the even block) or m (the block is m M^-1, not M^-1) fails
            assert abs(full - eo / 2) > 0.1 * abs(full) and abs(full - eo / mass) > 0.1 * abs(full)
