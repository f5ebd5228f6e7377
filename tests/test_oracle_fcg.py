"""Pins of the oracle's flexible CG (Notay's FCG with truncation 1, complex steps) against what
the method must reduce to: textbook CG for P = I and for P = a complex phase times I (the same
iterates, which fixes the conjugation convention of the complex step sizes), one step for the
exact inverse, and textbook preconditioned CG for a fixed Hermitian positive definite P."""
import numpy as np

import oracle
import synth
from oracle import trace

DIMS, MASS, TOL = (4, 4, 4, 4), 0.5, 1e-10


def _close_counts(a, b):
    """Iteration counts of recurrences that agree in exact arithmetic: rounding moves the stopping
    iteration by a step or two over ~140 iterations."""
    a, b = np.asarray(a), np.asarray(b)
    return bool(np.all(np.abs(a - b) <= np.maximum(2, 0.02 * b)))


def _case(n=2):
    fat, naik = synth.gauge_links(DIMS, 501, eps=0.4)
    b = synth.sources(DIMS, n, 502)
    return fat, naik, b


def test_identity_preconditioner_is_textbook_cg():
    fat, naik, b = _case()
    xc, ic, rc = oracle.cg(fat, naik, b, DIMS, MASS, TOL)
    xf, itf, rf = oracle.fcg(fat, naik, b, DIMS, MASS, TOL, lambda r: r)
    assert np.all(rf <= TOL) and np.all(rc <= TOL)
    assert _close_counts(itf, ic), (itf, ic)
    for i in range(b.shape[0]):
        assert np.linalg.norm(xf[i] - xc[i]) <= 1e-9 * np.linalg.norm(xc[i])


def test_phase_preconditioner_gives_the_cg_iterates():
    """P = e^{i theta} I scales every direction by the phase and every step size by its
    conjugate, so x is that of CG; swapping the arguments of <p, r> in the step would leave a
    factor e^{2 i theta} and fail."""
    fat, naik, b = _case()
    ph = np.exp(0.7j)
    xc, ic, _ = oracle.cg(fat, naik, b, DIMS, MASS, TOL)
    xf, itf, rf = oracle.fcg(fat, naik, b, DIMS, MASS, TOL, lambda r: ph * r)
    assert np.all(rf <= TOL)
    assert _close_counts(itf, ic), (itf, ic)
    for i in range(b.shape[0]):
        assert np.linalg.norm(xf[i] - xc[i]) <= 1e-9 * np.linalg.norm(xc[i])


def test_exact_inverse_converges_in_one_step():
    fat, naik, b = _case()
    m = trace.dense_m(fat, naik, DIMS, MASS)
    shape = b.shape[1:]

    def inv(r):
        return np.linalg.solve(m, r.ravel()).reshape(shape)

    x, its, res = oracle.fcg(fat, naik, b, DIMS, MASS, 1e-12, inv)
    assert np.all(its == 1), its
    assert np.all(res <= 1e-12), res


def _textbook_pcg(fat, naik, b, P, tol):
    """Preconditioned CG (Hestenes-Stiefel with the preconditioned inner product <r, P r>)."""
    x = np.zeros_like(b)
    r = b.copy()
    z = P(r)
    p = z.copy()
    rho = np.vdot(r, z)
    it = 0
    while np.linalg.norm(r) > tol * np.linalg.norm(b):
        q = oracle.m_ee(fat, naik, p[None], DIMS, MASS)[0]
        alpha = rho / np.vdot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        z = P(r)
        rho_new = np.vdot(r, z)
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, it


def test_fixed_hermitian_preconditioner_is_textbook_pcg():
    """For a fixed Hermitian positive definite P the flexible recurrence (beta from <q, z>)
    reproduces preconditioned CG (beta from <r, P r>), whose directions are M-orthogonal to all
    earlier ones, not only to the last."""
    fat, naik, b = _case()
    d = np.random.default_rng(503).uniform(0.3, 3.0, size=b.shape[1:])

    def P(r):
        return d * r

    xf, itf, rf = oracle.fcg(fat, naik, b, DIMS, MASS, TOL, P)
    assert np.all(rf <= TOL)
    for i in range(b.shape[0]):
        xp, itp = _textbook_pcg(fat, naik, b[i], P, TOL)
        assert _close_counts(int(itf[i]), itp), (itf[i], itp)
        assert np.linalg.norm(xf[i] - xp) <= 1e-9 * np.linalg.norm(xp)
    # the preconditioner changes the iteration (it is not the identity in disguise)
    _, ic, _ = oracle.cg(fat, naik, b, DIMS, MASS, TOL)
    assert np.any(itf != ic)
