"""Stochastic estimate of Tr M^-1 on the even sites (Section 1, Eq. 2: the traces that the
multi-rhs solver exists for are estimated from random vectors), TEST INFRASTRUCTURE ONLY.

    Tr M^-1 ~ (1/N) sum_k eta_k^dag M^-1 eta_k

with Z2 noise eta_k: every colour component of every even site is +1 or -1 (real), so the
estimator is unbiased and its variance comes from the off-diagonal part only,
Var(eta^dag A eta) = 2 sum_{i != j} (Re A_ij)^2 for Hermitian A.

The noise is counter based, so that the GPU and this oracle draw the same vectors without
sharing code: component c of the noise stream (c = (k * 3 + colour) * V/2 + site for vector k)
is -1 if the top bit of the c-th SplitMix64 output for `seed` is set, else +1.  SplitMix64
(Steele, Lea and Flood, OOPSLA 2014): the c-th output (c = 0, 1, ...) is
mix(seed + (c + 1) * 0x9E3779B97F4A7C15) with mix(z) = z ^ (z >> 31) after
z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9 and z = (z ^ (z >> 27)) * 0x94D049BB133111EB, all
modulo 2^64.
"""
from __future__ import annotations

import numpy as np

from .dslash import dslash_full, m_ee

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters) -> np.ndarray:
    """Outputs number `counters` (0-based, array) of the SplitMix64 stream started at seed."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (c + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def z2_noise(seed: int, k0: int, n: int, vh: int) -> np.ndarray:
    """Noise vectors k0 .. k0+n-1 as complex128 [n][3][vh] (real +-1)."""
    c = (np.uint64(k0) * np.uint64(3 * vh)) + np.arange(n * 3 * vh, dtype=np.uint64)
    top = splitmix64(seed, c) >> np.uint64(63)
    return (1.0 - 2.0 * top.astype(np.float64)).reshape(n, 3, vh).astype(np.complex128)


def dense_m(fat, naik, dims, mass) -> np.ndarray:
    """M on the even sites as a dense (3 V/2) x (3 V/2) matrix in the [3][V/2] component order."""
    vh = int(np.prod(dims)) // 2
    eye = np.eye(3 * vh).reshape(3 * vh, 3, vh)
    return m_ee(fat, naik, eye, dims, mass).reshape(3 * vh, 3 * vh).T


def trace_minv_exact(fat, naik, dims, mass) -> float:
    """Tr M^-1 from the dense inverse (small lattices only)."""
    return float(np.trace(np.linalg.inv(dense_m(fat, naik, dims, mass))).real)


def trace_samples(fat, naik, dims, mass, seed: int, n_vec: int) -> np.ndarray:
    """eta_k^dag M^-1 eta_k for k = 0 .. n_vec-1 by dense solves (small lattices only)."""
    vh = int(np.prod(dims)) // 2
    m = dense_m(fat, naik, dims, mass)
    eta = z2_noise(seed, 0, n_vec, vh).reshape(n_vec, 3 * vh)
    x = np.linalg.solve(m, eta.T).T
    return np.einsum("ki,ki->k", np.conj(eta), x).real


def dense_d_full(fat, naik, dims) -> np.ndarray:
    """D of Eq. 3 on the whole lattice as a dense (3 V) x (3 V) matrix, assembled column by column
    from dslash_full on unit vectors (component order [site][colour], lexicographic sites)."""
    vol = int(np.prod(dims))
    eye = np.eye(3 * vol).reshape(3 * vol, vol, 3)
    cols = np.stack([dslash_full(fat, naik, e, dims).reshape(3 * vol) for e in eye])
    return cols.T


def chiral_condensate_exact(fat, naik, dims, mass) -> float:
    """(1/V) Tr (m + D)^-1 over the whole lattice (colour and sites), from the dense inverse of
    the full operator (small lattices only)."""
    vol = int(np.prod(dims))
    a = mass * np.eye(3 * vol) + dense_d_full(fat, naik, dims)
    return float(np.trace(np.linalg.inv(a)).real) / vol


def chiral_condensate_from_trace(trace_minv: float, dims, mass) -> float:
    """(1/V) Tr (m + D)^-1 from Tr M_ee^-1: the even and odd diagonal blocks of (m + D)^-1 are
    m M_ee^-1 and m M_oo^-1 (D only connects the parities), and M_oo = m^2 - D_oe D_eo has the
    spectrum of M_ee (D_eo D_oe and D_oe D_eo share their eigenvalues on equal dimensions), so
    Tr (m + D)^-1 = 2 m Tr M_ee^-1."""
    return 2.0 * mass * trace_minv / int(np.prod(dims))
