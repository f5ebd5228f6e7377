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


def test_naik_links_have_the_14_real_form():
    """Reading of the 14-real Naik format: for N = c U with U in SU(3), row 2 of N equals
    z conj(row0 x row1) with z = c / conj(c)^2 (z = -24 for the synthetic N = -U/24)."""
    fat, naik = synth.gauge_links((4, 4, 4, 4), 21)
    n = naik.reshape(-1, 3, 3)
    cross = np.conj(np.cross(n[:, 0, :], n[:, 1, :]))
    assert np.max(np.abs(n[:, 2, :] - (-24.0) * cross)) <= 1e-14
    u = -24.0 * n  # SU(3): unitary with determinant 1
    eye = np.eye(3)
    assert np.max(np.abs(u @ np.conj(np.transpose(u, (0, 2, 1))) - eye)) <= 1e-13
    assert np.max(np.abs(np.linalg.det(u) - 1.0)) <= 1e-13
    # fat links are not of that form (the 14-real storage must not apply to them)
    f = fat.reshape(-1, 3, 3)
    assert np.max(np.abs(f[:, 2, :] - np.conj(np.cross(f[:, 0, :], f[:, 1, :])))) > 1e-2


def test_gauge_rotated_tiled_links_lose_the_period():
    """The rotated tiled field no longer repeats with period 4, the Naik links keep the 14-real
    form (-1/24 times an SU(3) matrix), and it is the same field in another gauge: the oracle's
    D on the rotated links applied to W v equals W (D v), with W the per-site rotation drawn
    from the same seed."""
    import oracle
    dims = (8, 4, 4, 8)
    fat, naik = synth.tiled_gauge_links(dims, 11)
    rf, rn = synth.gauge_rotated(fat, naik, dims, 12)
    lx, ly, lz, lt = dims
    shift = 4 * lx * ly * lz  # one tile along t
    assert np.max(np.abs(rf[:shift] - rf[shift:2 * shift])) > 0.1
    assert np.max(np.abs(rn[:shift] - rn[shift:2 * shift])) > 0.1 / 24
    n = rn.reshape(-1, 3, 3)
    assert np.max(np.abs(n[:, 2, :] - (-24.0) * np.conj(np.cross(n[:, 0, :], n[:, 1, :])))) <= 1e-13
    # the rotation the generator draws for this seed (same stream, same order)
    vol = int(np.prod(dims))
    gen = synth._gen(12)
    w = synth.haar_su3(gen, 4096)
    which = gen.integers(0, 4096, size=vol)
    om = w[which]
    v = synth.complex_normal(np.random.default_rng(3), (vol, 3))
    dv = oracle.dslash_full(fat, naik, v, dims)
    d_rot = oracle.dslash_full(rf, rn, np.einsum("sab,sb->sa", om, v), dims)
    assert np.max(np.abs(d_rot - np.einsum("sab,sb->sa", om, dv))) <= 1e-12 * np.max(np.abs(dv))


def test_naik_links_have_the_13_and_9_real_forms():
    """Readings of the 13- and 9-real Naik formats: the synthetic N = -U/24 is a real multiple
    c = -1/24 of an SU(3) matrix (det N = c^3 is real), so row 2 = conj(row0 x row1) / c with a
    real scale (13 reals); and U is fixed by u01, u02, u10 and the phases of u00 and u20 (9 reals
    with c): |u00|^2 = 1 - |u01|^2 - |u02|^2 and |u20|^2 = |u01|^2 + |u02|^2 - |u10|^2 by the unit
    norms of row 0 and column 0, the other four entries by the orthogonality of rows 1 and 2 to
    row 0 together with row2 = conj(row0 x row1) and row1 = conj(row2 x row0)."""
    fat, naik = synth.gauge_links((4, 4, 4, 4), 22)
    n = naik.reshape(-1, 3, 3)
    det = np.linalg.det(n)
    assert np.max(np.abs(det.imag)) <= 1e-15 and np.allclose(np.cbrt(det.real), -1.0 / 24, atol=1e-14)
    c = np.cbrt(det.real)
    row2 = np.conj(np.cross(n[:, 0, :], n[:, 1, :])) / c[:, None]
    assert np.max(np.abs(row2 - n[:, 2, :])) <= 1e-15
    u = n / c[:, None, None]
    u01, u02, u10 = u[:, 0, 1], u[:, 0, 2], u[:, 1, 0]
    nn = np.abs(u01) ** 2 + np.abs(u02) ** 2
    u00 = np.sqrt(1 - nn) * np.exp(1j * np.angle(u[:, 0, 0]))
    u20 = np.sqrt(nn - np.abs(u10) ** 2) * np.exp(1j * np.angle(u[:, 2, 0]))
    cj = np.conj
    rebuilt = np.empty_like(u)
    rebuilt[:, 0] = np.stack([u00, u01, u02], -1)
    rebuilt[:, 1] = np.stack([u10, -(cj(u20 * u02) + cj(u00) * u01 * u10) / nn,
                              (cj(u01 * u20) - cj(u00) * u02 * u10) / nn], -1)
    rebuilt[:, 2] = np.stack([u20, (cj(u10 * u02) - cj(u00) * u01 * u20) / nn,
                              -(cj(u01 * u10) + cj(u00) * u02 * u20) / nn], -1)
    assert np.max(np.abs(rebuilt * c[:, None, None] - n)) <= 1e-12 / 24
