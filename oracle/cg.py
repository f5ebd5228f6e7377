"""Oracle conjugate gradient for M = m^2 - D_eo D_oe on even sites, one rhs at a time (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper keeps the whole CG on the accelerator and stops each right-hand side individually
once it meets the convergence criterion (Section 2, implementation paragraph on the remaining
linear algebra).  The criterion itself is not printed; the reading taken is the relative true
residual ||b - M x||_2 / ||b||_2 <= tol in FP64, with ||b|| = 0 giving x = 0.

Textbook CG (Hestenes & Stiefel 1952) on the Hermitian positive definite M, with inner product
<a, b> = sum conj(a) b:
    r = b - M x, p = r, rho = <r, r>
    repeat: q = M p; alpha = rho / Re<p, q>; x += alpha p; r -= alpha q;
            rho' = <r, r>; stop when sqrt(rho') <= tol ||b||; beta = rho' / rho; p = r + beta p
On exit the true residual is recomputed; if it is above tol the iteration restarts from x.
"""
from __future__ import annotations

import numpy as np

from .dslash import m_ee


def _dot(a, b) -> complex:
    return complex(np.vdot(a.ravel(), b.ravel()))


def true_residual(fat, naik, x, b, dims, mass) -> np.ndarray:
    """Per-rhs ||b - M x|| / ||b|| (0 where b == 0 and x == 0)."""
    x = np.asarray(x)
    b = np.asarray(b)
    r = b - m_ee(fat, naik, x, dims, mass)
    out = np.empty(b.shape[0])
    for i in range(b.shape[0]):
        nb = np.linalg.norm(b[i])
        nr = np.linalg.norm(r[i])
        out[i] = nr / nb if nb > 0 else nr
    return out


def cg(fat, naik, b, dims, mass, tol, max_iter=100000, x0=None, max_restarts=5):
    """Solve M x = b for each rhs of b [n][3][V/2].  Returns (x, iters, true_resid)."""
    b = np.asarray(b, np.complex128)
    n = b.shape[0]
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.complex128)
    iters = np.zeros(n, np.int64)
    resid = np.zeros(n)

    def apply(v):
        return m_ee(fat, naik, v[None], dims, mass)[0]

    for i in range(n):
        bnorm = np.linalg.norm(b[i])
        if bnorm == 0.0:
            x[i] = 0.0
            continue
        xi = x[i]
        for _ in range(max_restarts + 1):
            r = b[i] - apply(xi)
            p = r.copy()
            rho = _dot(r, r).real
            while np.sqrt(rho) > tol * bnorm and iters[i] < max_iter:
                q = apply(p)
                alpha = rho / _dot(p, q).real
                xi = xi + alpha * p
                r = r - alpha * q
                rho_new = _dot(r, r).real
                iters[i] += 1
                beta = rho_new / rho
                rho = rho_new
                p = r + beta * p
            resid[i] = np.linalg.norm(b[i] - apply(xi)) / bnorm
            if resid[i] <= tol or iters[i] >= max_iter:
                break
        x[i] = xi
    return x, iters, resid


def fcg(fat, naik, b, dims, mass, tol, precond, max_iter=100000):
    """Flexible CG with truncation 1 (Notay, SIAM J. Sci. Comput. 22 (2000) 1444), the solver the
    learned preconditioner serves, with complex step sizes since a preconditioner need not be
    Hermitian.  precond(r) -> z acts on one rhs [3][V/2].  For each rhs of b [n][3][V/2], from
    x = 0:
        r = b, z = P r, p = z
        repeat: q = M p; alpha = <p, r> / <p, q>; x += alpha p; r -= alpha q;
                stop when ||r|| <= tol ||b||; z = P r; beta = -<q, z> / <p, q>; p = z + beta p
    (p is made M-orthogonal to the previous direction only).  Returns (x, iters, true_resid), the
    true residual recomputed as ||b - M x|| / ||b||; no restart."""
    b = np.asarray(b, np.complex128)
    n = b.shape[0]
    x = np.zeros_like(b)
    iters = np.zeros(n, np.int64)
    resid = np.zeros(n)

    def apply(v):
        return m_ee(fat, naik, v[None], dims, mass)[0]

    for i in range(n):
        bnorm = np.linalg.norm(b[i])
        if bnorm == 0.0:
            continue
        xi = np.zeros_like(b[i])
        r = b[i].copy()
        p = np.asarray(precond(r), np.complex128)
        while np.linalg.norm(r) > tol * bnorm and iters[i] < max_iter:
            q = apply(p)
            pq = _dot(p, q)
            alpha = _dot(p, r) / pq
            xi = xi + alpha * p
            r = r - alpha * q
            iters[i] += 1
            if np.linalg.norm(r) <= tol * bnorm:
                break
            z = np.asarray(precond(r), np.complex128)
            beta = -_dot(q, z) / pq
            p = z + beta * p
        x[i] = xi
        resid[i] = np.linalg.norm(b[i] - apply(xi)) / bnorm
    return x, iters, resid
