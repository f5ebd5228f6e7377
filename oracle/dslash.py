"""Oracle HISQ Dslash, its even-odd blocks and the even-even normal operator (FP64, numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition (Section 1, Eq. 3; Eq. 4 for several right-hand sides):

    w(x) = sum_{mu=0..3} [ X(x,mu) v(x+mu) - X(x-mu,mu)^dag v(x-mu)
                         + N(x,mu) v(x+3mu) - N(x-3mu,mu)^dag v(x-3mu) ]

on a periodic 4-d lattice.  Readings taken where the printed equation is silent or garbled:
  * the sum runs over the four directions mu = 0..3 (x, y, z, t); the printed upper limit 4 is
    read as a typo;
  * staggered phases and boundary signs are folded into X and N by the caller, no factor 1/2;
  * N(x,mu) sits at x and connects x to x+3mu; the backward Naik term uses N(x-3mu,mu)^dag;
  * on extents where hops alias (L = 4: x+3 == x-1; L = 6: x+3 == x-3) the contributions add;
  * Eq. 4 applies the same D to every right-hand side independently.

Even-odd blocks: parity(x) = (x+y+z+t) mod 2, D only connects sites of opposite parity (every hop
is odd), so D = [[0, D_eo], [D_oe, 0]] with D_oe mapping even to odd.  The operator solved for is
M = m^2 - D_eo D_oe on the even sites.

Layouts: links [V][4][3][3] complex128 in lexicographic order lex = x + Lx*(y + Ly*(z + Lz*t));
full-lattice vectors [V][3]; single-parity vectors [n][3][V/2], the index within a parity
being lex >> 1.
"""
from __future__ import annotations

import numpy as np

# direction mu -> numpy axis of a field reshaped to (Lt, Lz, Ly, Lx, ...)
_AXIS = (3, 2, 1, 0)


def _dag(a: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(a, -1, -2))


def _matvec(a: np.ndarray, v: np.ndarray) -> np.ndarray:
    """(A v)_a = sum_b A_ab v_b, batched over leading axes."""
    return np.einsum("...ab,...b->...a", a, v)


def site_coords(dims):
    """Coordinates (x, y, z, t) of every lexicographic site, each an int64 array of length V."""
    lx, ly, lz, lt = dims
    lex = np.arange(lx * ly * lz * lt, dtype=np.int64)
    return lex % lx, (lex // lx) % ly, (lex // (lx * ly)) % lz, lex // (lx * ly * lz)


def parity_lex(dims, parity: int) -> np.ndarray:
    """Lexicographic indices of the sites of one parity, in increasing order.

    For even Lx the pair (2k, 2k+1) holds exactly one site of each parity, so the position of a
    site in this list is lex >> 1.
    """
    x, y, z, t = site_coords(dims)
    return np.nonzero((x + y + z + t) % 2 == parity)[0]


def embed(vh: np.ndarray, dims, parity: int) -> np.ndarray:
    """Single-parity [3][V/2] -> full-lattice [V][3], zero on the other parity."""
    v = np.zeros((int(np.prod(dims)), 3), np.complex128)
    v[parity_lex(dims, parity)] = np.asarray(vh).T
    return v


def extract(v: np.ndarray, dims, parity: int) -> np.ndarray:
    """Full-lattice [V][3] -> single-parity [3][V/2]."""
    return np.ascontiguousarray(v[parity_lex(dims, parity)].T)


def dslash_full(fat: np.ndarray, naik: np.ndarray, v: np.ndarray, dims) -> np.ndarray:
    """Eq. 3 on the whole periodic lattice for one vector v [V][3]; returns w [V][3]."""
    lx, ly, lz, lt = dims
    shp = (lt, lz, ly, lx)
    xf = fat.reshape(shp + (4, 3, 3))
    nf = naik.reshape(shp + (4, 3, 3))
    vf = v.reshape(shp + (3,))
    w = np.zeros_like(vf, dtype=np.complex128)
    for mu in range(4):
        ax = _AXIS[mu]
        x_mu = xf[..., mu, :, :]
        n_mu = nf[..., mu, :, :]
        # np.roll(f, -k, ax)[x] == f[x + k mu];  np.roll(f, k, ax)[x] == f[x - k mu]
        w += _matvec(x_mu, np.roll(vf, -1, ax))
        w -= _matvec(_dag(np.roll(x_mu, 1, ax)), np.roll(vf, 1, ax))
        w += _matvec(n_mu, np.roll(vf, -3, ax))
        w -= _matvec(_dag(np.roll(n_mu, 3, ax)), np.roll(vf, 3, ax))
    return w.reshape(-1, 3)


def dslash_half(fat, naik, v_in: np.ndarray, dims, out_parity: int) -> np.ndarray:
    """The parity block of Eq. 3 applied to each rhs (Eq. 4).

    v_in: [n][3][V/2] on parity 1 - out_parity.  Returns [n][3][V/2] on out_parity.
    out_parity = 1 gives D_oe (even -> odd); out_parity = 0 gives D_eo (odd -> even).
    """
    v_in = np.asarray(v_in)
    out = np.empty(v_in.shape, np.complex128)
    for i in range(v_in.shape[0]):
        full = embed(v_in[i], dims, 1 - out_parity)
        out[i] = extract(dslash_full(fat, naik, full, dims), dims, out_parity)
    return out


def m_ee(fat, naik, v: np.ndarray, dims, mass: float) -> np.ndarray:
    """M v = m^2 v - D_eo D_oe v on even sites, for each rhs of v [n][3][V/2]."""
    t = dslash_half(fat, naik, v, dims, 1)
    return mass * mass * np.asarray(v) - dslash_half(fat, naik, t, dims, 0)


def dslash_sites(fat, naik, v_in: np.ndarray, dims, out_parity: int, sites: np.ndarray) -> np.ndarray:
    """Eq. 3 evaluated only at the given output sites, one site at a time in coordinates.

    v_in: [n][3][V/2] on parity 1 - out_parity; sites: indices within out_parity.
    Returns [n][3][len(sites)].  For checking outputs at sizes where the whole-lattice oracle is
    too slow; the neighbour arithmetic is written in coordinates, independently of dslash_full.
    """
    lx, ly, lz, lt = dims
    ext = (lx, ly, lz, lt)
    v_in = np.asarray(v_in)
    n = v_in.shape[0]
    lex_out = parity_lex(dims, out_parity)[np.asarray(sites, np.int64)]
    out = np.zeros((n, 3, len(lex_out)), np.complex128)

    def shift(c, mu, k):
        c = list(c)
        c[mu] = (c[mu] + k) % ext[mu]
        return c

    def lex_of(c):
        return c[0] + lx * (c[1] + ly * (c[2] + lz * c[3]))

    for j, l in enumerate(lex_out):
        c = [l % lx, (l // lx) % ly, (l // (lx * ly)) % lz, l // (lx * ly * lz)]
        acc = np.zeros((n, 3), np.complex128)
        for mu in range(4):
            for links, hop in ((fat, 1), (naik, 3)):
                fwd = lex_of(shift(c, mu, hop))
                bwd = lex_of(shift(c, mu, -hop))
                u_f = links[l, mu]
                u_b = links[bwd, mu]
                v_f = v_in[:, :, fwd >> 1]
                v_b = v_in[:, :, bwd >> 1]
                acc += v_f @ u_f.T            # (U v)_a = sum_b U_ab v_b, for every rhs
                acc -= v_b @ np.conj(u_b)     # (U^dag v)_a = sum_b conj(U_ba) v_b
        out[:, :, j] = acc
    return out
