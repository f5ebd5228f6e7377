"""Seeded synthetic inputs for the HISQ multi-rhs Dslash / CG: gauge links and sources.

This module is shared by the test oracle and by the GPU path's tests and benchmark.  It holds
only input synthesis (random numbers, matrix exponentials of random Hermitian matrices, Haar
unitaries); it holds none of the Dslash or solver arithmetic.

Stand-in for the paper's HotQCD HISQ ensembles (Section 1: thousands of configurations with
~1500 random vectors each), which are not available:

* Fat links X(x, mu) = exp(i * eps * H) + pert * G, where H = (A + A^dag)/2 - tr(.)/3 is a
  Gaussian Hermitian traceless 3x3 matrix (A standard complex normal), eps = 0.4 by default
  (0.3 for the largest lattice), and G is a standard complex normal 3x3 matrix, pert = 0.05.
  The perturbation keeps the fat links away from SU(3), as smeared HISQ links are (Section 1).
* Naik links N(x, mu) = -1/24 * U with U a Haar-random SU(3) matrix (QR of a complex Ginibre
  matrix with the phase fix of Mezzadri 2007, then divided by a cube root of its determinant).
* Sources: standard complex normal per colour component (Re, Im ~ N(0, 1/2)), or Z2 noise
  (each component a real +-1 with probability 1/2), on the sites of one parity.

Conventions used throughout the project:
  dims = (Lx, Ly, Lz, Lt); lexicographic site index lex = x + Lx*(y + Ly*(z + Lz*t));
  link arrays are [V][4][3][3] complex128 (direction mu = 0..3 is x, y, z, t; row-major 3x3);
  single-parity vectors are [n][3][V/2] complex (colour-planar), the index within a parity
  being lex >> 1.

Random numbers come from numpy's Philox4x32 counter-based generator, keyed by the seed, so a
seed gives the same field on every machine with the same numpy.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 1409151 * 100

# the five workloads of the study (lattice, mass, rhs, precision recipe)
WORKLOADS = {
    "c0": dict(dims=(8, 8, 8, 8), mass=0.1, n=1, eps=0.4, tol=1e-10, source="gaussian"),
    "c1": dict(dims=(32, 32, 32, 8), mass=None, n=16, eps=0.4, tol=None, source="gaussian"),
    "c2": dict(dims=(32, 32, 32, 8), mass=0.02, n=8, eps=0.4, tol=1e-8, source="gaussian"),
    "c3": dict(dims=(48, 48, 48, 12), mass=0.01, n=16, eps=0.4, tol=1e-8, source="z2"),
    "c4": dict(dims=(64, 64, 64, 16), mass=0.005, n=32, eps=0.3, tol=1e-8, source="gaussian"),
}


def workload_seed(name: str) -> int:
    return BASE_SEED + int(name[1:])


def volume(dims) -> int:
    lx, ly, lz, lt = dims
    return lx * ly * lz * lt


def check_dims(dims) -> None:
    if len(dims) != 4 or any(int(d) < 4 or int(d) % 2 for d in dims):
        raise ValueError(f"lattice extents must be even and >= 4, got {dims}")


def _gen(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=int(seed) & ((1 << 64) - 1)))


def complex_normal(gen: np.random.Generator, shape) -> np.ndarray:
    """Standard complex normal: Re, Im independent N(0, 1/2)."""
    re = gen.standard_normal(shape)
    im = gen.standard_normal(shape)
    return (re + 1j * im) * np.sqrt(0.5)


def _dagger(a: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(a, -1, -2))


def _exp_i_hermitian(h: np.ndarray, eps: float) -> np.ndarray:
    """exp(i*eps*H) for a batch of Hermitian 3x3 matrices, by eigendecomposition."""
    lam, vec = np.linalg.eigh(h)
    phase = np.exp(1j * eps * lam)
    return (vec * phase[..., None, :]) @ _dagger(vec)


def haar_su3(gen: np.random.Generator, count: int) -> np.ndarray:
    z = complex_normal(gen, (count, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(q)
    return q / np.exp(1j * np.angle(det) / 3.0)[..., None, None]


def gauge_links(dims, seed: int, eps: float = 0.4, pert: float = 0.05, chunk: int = 1 << 20):
    """Return (X, N), each [V][4][3][3] complex128, generated in chunks of sites."""
    check_dims(dims)
    v = volume(dims)
    gen = _gen(seed)
    fat = np.empty((v, 4, 3, 3), np.complex128)
    naik = np.empty((v, 4, 3, 3), np.complex128)
    flat_f = fat.reshape(-1, 3, 3)
    flat_n = naik.reshape(-1, 3, 3)
    total = v * 4
    for lo in range(0, total, chunk):
        hi = min(total, lo + chunk)
        m = hi - lo
        a = complex_normal(gen, (m, 3, 3))
        h = 0.5 * (a + _dagger(a))
        tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
        h = h - tr[:, None, None] * np.eye(3)
        g = complex_normal(gen, (m, 3, 3))
        flat_f[lo:hi] = _exp_i_hermitian(h, eps) + pert * g
        flat_n[lo:hi] = (-1.0 / 24.0) * haar_su3(gen, m)
    return fat, naik


def tiled_gauge_links(dims, seed: int, eps: float = 0.4):
    """gauge_links on a 4^4 lattice, tiled periodically over `dims` (each extent a multiple of
    4): a fast stand-in at large volumes where only timing or sampled sites matter."""
    small = (4, 4, 4, 4)
    fat, naik = gauge_links(small, seed, eps=eps)
    lx, ly, lz, lt = dims
    if lx % 4 or ly % 4 or lz % 4 or lt % 4:
        raise ValueError("tiled links need every extent to be a multiple of 4")
    reps = (lt // 4, lz // 4, ly // 4, lx // 4, 1, 1, 1)

    def tile(u):
        return np.ascontiguousarray(np.tile(u.reshape(4, 4, 4, 4, 4, 3, 3), reps).reshape(-1, 4, 3, 3))
    return tile(fat), tile(naik)


def sources(dims, n: int, seed: int, kind: str = "gaussian") -> np.ndarray:
    """n single-parity source vectors, [n][3][V/2] complex128."""
    check_dims(dims)
    vh = volume(dims) // 2
    gen = _gen(seed)
    if kind == "gaussian":
        return complex_normal(gen, (n, 3, vh))
    if kind == "z2":
        signs = gen.integers(0, 2, size=(n, 3, vh)) * 2 - 1
        return signs.astype(np.complex128)
    raise ValueError(f"unknown source kind {kind!r}")


def workload_inputs(name: str, n: int | None = None):
    """Links and sources of a named workload: (cfg, X, N, b)."""
    cfg = dict(WORKLOADS[name])
    seed = workload_seed(name)
    fat, naik = gauge_links(cfg["dims"], seed, eps=cfg["eps"])
    nr = cfg["n"] if n is None else n
    b = sources(cfg["dims"], nr, seed + 1, cfg["source"])
    return cfg, fat, naik, b


def gauge_rotated(fat, naik, dims, seed: int, pool: int = 4096):
    """Random local SU(3) rotation of a link field (the same field in another gauge):
    X(x, mu) -> W(x) X(x, mu) W(x + mu)^dag and N(x, mu) -> W(x) N(x, mu) W(x + 3 mu)^dag, with
    W(x) drawn per site from `pool` Haar SU(3) matrices.  Applied to a tiled field it gives links
    that no longer repeat with the tile's period, so a link read from a site shifted by a multiple
    of the period shows up.  Returns new arrays; the inputs are not changed."""
    check_dims(dims)
    lx, ly, lz, lt = dims
    v = volume(dims)
    gen = _gen(seed)
    w = haar_su3(gen, pool)
    which = gen.integers(0, pool, size=v)
    wd = _dagger(w)
    ext = (lx, ly, lz, lt)
    stride = (1, lx, lx * ly, lx * ly * lz)
    out_f = np.empty_like(fat)
    out_n = np.empty_like(naik)
    chunk = 1 << 18
    for lo in range(0, v, chunk):
        lex = np.arange(lo, min(v, lo + chunk), dtype=np.int64)
        coord = (lex % lx, (lex // lx) % ly, (lex // (lx * ly)) % lz, lex // (lx * ly * lz))
        left = w[which[lex]]
        for mu in range(4):
            for src, dst, hop in ((fat, out_f, 1), (naik, out_n, 3)):
                c = coord[mu]
                nb = lex + (((c + hop) % ext[mu]) - c) * stride[mu]
                dst[lex, mu] = left @ src[lex, mu] @ wd[which[nb]]
    return out_f, out_n
