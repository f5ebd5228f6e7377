"""GPU stochastic trace of M^-1 (Section 1, Eq. 2) against the oracle: the counter-based Z2 noise
bit for bit, the per-vector samples eta^dag M^-1 eta against dense solves, the chiral condensate
against the dense whole-lattice operator, independence of the bundle size, and argument errors."""
import numpy as np
import pytest

from gpu_helpers import make_lattice
from oracle import trace as otrace

torch = pytest.importorskip("torch")
from paper_1409_1510_amd import hisq  # noqa: E402

pytestmark = pytest.mark.gpu


def test_noise_matches_oracle_bit_for_bit():
    dims = (8, 6, 4, 10)
    lat, fat, naik = make_lattice(dims, 500)
    got = lat.z2_noise(2024, 3, 5).cpu().numpy()
    assert np.array_equal(got, otrace.z2_noise(2024, 3, 5, lat.vh))
    lat.close()


def test_samples_match_dense_solves():
    dims, mass = (4, 4, 4, 4), 0.5
    lat, fat, naik = make_lattice(dims, 501)
    est, err, s = lat.trace_minv(mass, 24, bundle=8, seed=9, kind=hisq.HISQ_CG_F64, tol=1e-12)
    ref = otrace.trace_samples(fat, naik, dims, mass, 9, 24)
    assert np.max(np.abs(np.array(s) - ref) / np.abs(ref)) <= 1e-9
    assert abs(est - ref.mean()) <= 1e-9 * abs(ref.mean())
    assert abs(err - ref.std(ddof=1) / np.sqrt(24)) <= 1e-6 * err
    exact = otrace.trace_minv_exact(fat, naik, dims, mass)
    print(f"Tr M^-1: estimate {est:.3f} +- {err:.3f}, exact {exact:.3f}")
    lat.close()


def test_chiral_condensate_matches_the_dense_full_operator():
    """The GPU chiral condensate is (2m/V) times the GPU trace estimate from the same noise, and
    it agrees with (1/V) Tr (m + D)^-1 of the oracle's dense whole-lattice operator within the
    estimator's statistical error (Z2 noise, 4^4, two masses)."""
    dims = (4, 4, 4, 4)
    lat, fat, naik = make_lattice(dims, 503)
    vol = int(np.prod(dims))
    for mass in (0.3, 2.5):
        kw = dict(bundle=16, seed=11, kind=hisq.HISQ_CG_F64, tol=1e-12)
        est, err = lat.chiral_condensate(mass, 256, **kw)
        tr, tr_err, _ = lat.trace_minv(mass, 256, **kw)
        assert abs(est - 2 * mass / vol * tr) <= 1e-13 * abs(est)
        assert abs(err - 2 * mass / vol * tr_err) <= 1e-13 * abs(err)
        exact = otrace.chiral_condensate_exact(fat, naik, dims, mass)
        print(f"m={mass}: condensate {est:.6f} +- {err:.6f}, dense {exact:.6f}")
        assert abs(est - exact) <= 5 * err
    lat.close()


def test_bundle_size_does_not_change_the_samples():
    dims, mass = (8, 6, 4, 10), 0.2
    lat, fat, naik = make_lattice(dims, 502)
    _, _, s3 = lat.trace_minv(mass, 10, bundle=3, seed=11, kind=hisq.HISQ_CG_F64, tol=1e-10)
    _, _, s10 = lat.trace_minv(mass, 10, bundle=10, seed=11, kind=hisq.HISQ_CG_F64, tol=1e-10)
    assert s3 == s10
    _, _, sm = lat.trace_minv(mass, 10, bundle=4, seed=11, kind=hisq.HISQ_CG_MIXED, tol=1e-10,
                              link_prec=hisq.HISQ_F32)
    assert np.max(np.abs(np.array(sm) - np.array(s10)) / np.abs(np.array(s10))) <= 1e-8
    lat.close()


def test_argument_errors():
    lat, fat, naik = make_lattice((4, 4, 4, 4), 503)
    for kw in (dict(bundle=0), dict(bundle=65)):
        with pytest.raises(hisq.HisqError) as e:
            lat.trace_minv(0.5, 4, **kw)
        assert e.value.code == hisq.HISQ_ERR_ARG
    with pytest.raises(hisq.HisqError) as e:
        lat.z2_noise(1, -1, 2)
    assert e.value.code == hisq.HISQ_ERR_ARG
    lat.close()
