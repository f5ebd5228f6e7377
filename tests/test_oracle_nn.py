"""Pins of the network oracle (forward, loss, Wirtinger gradients).

Independent facts used: central finite differences of the loss (gradients), a two-layer
one-channel closed form written with explicit site indexing (hop directions and daggers), the
fat-link part of Eq. 3 (the stencil with weights +1 forward / -1 backward is the fat Dslash),
gauge covariance and linearity.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import nn

DIMS = (4, 4, 4, 6)


def _rand_theta(c, l, seed, scale=0.5):
    g = np.random.Generator(np.random.Philox(key=seed))
    k = nn.n_params(c, l)
    return (g.standard_normal(k) + 1j * g.standard_normal(k)) * scale


def test_param_count_and_pack_roundtrip():
    assert nn.n_params(8, 4) == 496
    th = _rand_theta(3, 3, 1)
    assert np.array_equal(nn.pack(nn.unpack(th, 3, 3)), th)


@pytest.mark.parametrize("c,l,kind", [(2, 2, "solution"), (3, 3, "solution"), (2, 3, "residual")])
def test_gradient_matches_finite_differences(c, l, kind):
    fat, naik = synth.gauge_links(DIMS, 31)
    th = _rand_theta(c, l, 32)
    rs = synth.sources(DIMS, 2, 33)
    ys = synth.sources(DIMS, 2, 34)
    mass = 0.3
    kw = dict(kind=kind, naik=naik, mass=mass)
    val, grad = nn.loss_and_grad(th, fat, rs, ys, DIMS, c, l, **kw)
    assert abs(val - nn.loss(th, fat, rs, ys, DIMS, c, l, **kw)) < 1e-12 * val
    rng = np.random.default_rng(3)
    idx = rng.choice(th.size, 12, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros_like(th)
        e[k] = h
        d_re = (nn.loss(th + e, fat, rs, ys, DIMS, c, l, **kw) - nn.loss(th - e, fat, rs, ys, DIMS, c, l, **kw)) / (2 * h)
        d_im = (nn.loss(th + 1j * e, fat, rs, ys, DIMS, c, l, **kw) - nn.loss(th - 1j * e, fat, rs, ys, DIMS, c, l, **kw)) / (2 * h)
        scale = max(abs(grad[k]), 1e-3 * np.max(np.abs(grad)))
        assert abs(grad[k].real - d_re) <= 1e-6 * scale, (k, grad[k], d_re)
        assert abs(grad[k].imag - d_im) <= 1e-6 * scale, (k, grad[k], d_im)


def _coords(dims):
    lx, ly, lz, lt = dims
    lex = np.arange(lx * ly * lz * lt)
    return np.stack([lex % lx, (lex // lx) % ly, (lex // (lx * ly)) % lz, lex // (lx * ly * lz)], 1)


def _shift(dims, mu, k):
    c = _coords(dims)
    c[:, mu] = (c[:, mu] + k) % dims[mu]
    lx, ly, lz, lt = dims
    return c[:, 0] + lx * (c[:, 1] + ly * (c[:, 2] + lz * c[:, 3]))


@pytest.mark.parametrize("mu", [0, 2, 3])
def test_two_layer_closed_form(mu):
    """C = 1, layer 1 = forward hop only, layer 2 = backward hop only:
    z(x) = X(x-mu,mu)^dag X(x-mu,mu) r(x) on every even site x."""
    fat, _ = synth.gauge_links(DIMS, 35)
    p = nn.unpack(np.zeros(nn.n_params(1, 2), complex), 1, 2)
    p["W_in"][0] = 1.0
    p["W_out"][0] = 1.0
    p["W"][0][0, 0] = 1.0
    p["a"][0][1 + mu, 0] = 1.0
    p["a"][1][5 + mu, 0] = 1.0
    r = synth.sources(DIMS, 1, 36)[0]
    z = nn.forward(nn.pack(p), fat, r, DIMS, 1, 2)
    ev = oracle.parity_lex(DIMS, 0)
    back = _shift(DIMS, mu, -1)[ev]
    u = fat[back, mu]                                   # X(x - mu, mu) for even x
    expect = np.einsum("sba,sbc,cs->as", np.conj(u), u, r)  # (U^dag U r)_a
    assert np.max(np.abs(z - expect)) < 1e-13


def test_stencil_with_dslash_weights_is_fat_dslash():
    """Weights 0 (self), +1 (forward), -1 (backward) give the fat-link part of Eq. 3, so two
    layers give D_eo D_oe with the Naik links set to zero."""
    fat, _ = synth.gauge_links(DIMS, 37)
    p = nn.unpack(np.zeros(nn.n_params(1, 2), complex), 1, 2)
    p["W_in"][0] = p["W_out"][0] = p["W"][0][0, 0] = 1.0
    for l in range(2):
        p["a"][l][1:5, 0] = 1.0
        p["a"][l][5:9, 0] = -1.0
    r = synth.sources(DIMS, 1, 38)
    z = nn.forward(nn.pack(p), fat, r[0], DIMS, 1, 2)
    zero = np.zeros_like(fat)
    ref = oracle.dslash_half(fat, zero, oracle.dslash_half(fat, zero, r, DIMS, 1), DIMS, 0)[0]
    assert np.max(np.abs(z - ref)) < 1e-12 * np.max(np.abs(ref))


def test_gauge_covariance_and_linearity():
    c, l = 3, 4
    fat, _ = synth.gauge_links(DIMS, 39)
    th = _rand_theta(c, l, 40)
    vol = int(np.prod(DIMS))
    om = synth.haar_su3(np.random.Generator(np.random.Philox(key=41)), vol)
    omd = np.conj(np.swapaxes(om, -1, -2))
    fat_g = np.empty_like(fat)
    for mu in range(4):
        fat_g[:, mu] = om @ fat[:, mu] @ omd[_shift(DIMS, mu, 1)]
    ev = oracle.parity_lex(DIMS, 0)
    r = synth.sources(DIMS, 2, 42)
    rg = np.einsum("sab,bs->as", om[ev], r[0])
    z = nn.forward(th, fat, r[0], DIMS, c, l)
    zg = nn.forward(th, fat_g, rg, DIMS, c, l)
    assert np.max(np.abs(zg - np.einsum("sab,bs->as", om[ev], z))) < 1e-11 * np.max(np.abs(z))
    al, be = 0.3 - 0.7j, 1.1 + 0.2j
    z2 = nn.forward(th, fat, r[1], DIMS, c, l)
    zc = nn.forward(th, fat, al * r[0] + be * r[1], DIMS, c, l)
    assert np.max(np.abs(zc - al * z - be * z2)) < 1e-11 * np.max(np.abs(zc))


def test_init_is_near_identity():
    th = nn.init_params(8, 4, 5, scale=0.0)
    fat, _ = synth.gauge_links(DIMS, 43)
    r = synth.sources(DIMS, 1, 44)[0]
    assert np.max(np.abs(nn.forward(th, fat, r, DIMS, 8, 4) - r)) < 1e-14


def test_residual_loss_is_solution_error_in_m2_norm():
    """With y = M^-1 r exactly (from LAPACK), ||M P r - r|| = ||M (P r - y)||."""
    dims = (4, 4, 4, 4)
    fat, naik = synth.gauge_links(dims, 45)
    mass = 0.4
    th = _rand_theta(2, 2, 46)
    r = synth.sources(dims, 1, 47)
    vh = 128
    eye = np.eye(3 * vh).reshape(3 * vh, 3, vh)
    mdense = oracle.m_ee(fat, naik, eye, dims, mass).reshape(3 * vh, 3 * vh).T
    y = np.linalg.solve(mdense, r[0].ravel()).reshape(1, 3, vh)
    z = nn.forward(th, fat, r[0], dims, 2, 2)
    lhs = nn.loss(th, fat, r, y, dims, 2, 2, kind="residual", naik=naik, mass=mass)
    e = (mdense @ (z - y[0]).ravel())
    assert abs(lhs - np.linalg.norm(e) ** 2 / np.linalg.norm(r) ** 2) < 1e-10 * lhs


@pytest.mark.parametrize("kind", ["solution", "residual"])
def test_gram_gradient_matches_finite_differences(kind):
    c, l = 2, 2
    fat, naik = synth.gauge_links(DIMS, 48)
    th = _rand_theta(c, l, 49)
    rs = synth.sources(DIMS, 2, 50)
    ys = synth.sources(DIMS, 2, 51)
    kw = dict(kind=kind, naik=naik, mass=0.3)
    val, grad = nn.gram_loss_and_grad(th, fat, rs, ys, DIMS, c, l, **kw)
    assert abs(val - nn.loss(th, fat, rs, ys, DIMS, c, l, form="gram", **kw)) < 1e-12 * val
    idx = np.random.default_rng(4).choice(th.size, 12, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros_like(th)
        e[k] = h
        f = lambda t: nn.loss(t, fat, rs, ys, DIMS, c, l, form="gram", **kw)  # noqa: E731
        d_re = (f(th + e) - f(th - e)) / (2 * h)
        d_im = (f(th + 1j * e) - f(th - 1j * e)) / (2 * h)
        scale = max(abs(grad[k]), 1e-3 * np.max(np.abs(grad)))
        assert abs(grad[k].real - d_re) <= 1e-6 * scale, (k, grad[k], d_re)
        assert abs(grad[k].imag - d_im) <= 1e-6 * scale, (k, grad[k], d_im)


def test_gram_form_is_hermitian_positive_and_adjoint_is_adjoint():
    c, l = 3, 3
    fat, _ = synth.gauge_links(DIMS, 52)
    th = _rand_theta(c, l, 53)
    a, b = synth.sources(DIMS, 2, 54)
    vol = int(np.prod(DIMS))
    g = np.random.default_rng(5)
    u = g.standard_normal((vol, 3)) + 1j * g.standard_normal((vol, 3))
    # <u, N a> = <N^dag u, a>
    lhs = np.vdot(u, nn.network_full(th, fat, a, DIMS, c, l))
    rhs = np.vdot(nn.network_adjoint(th, fat, u, DIMS, c, l), a)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    pa = nn.apply(th, fat, a, DIMS, c, l, "gram")
    pb = nn.apply(th, fat, b, DIMS, c, l, "gram")
    assert abs(np.vdot(b, pa) - np.conj(np.vdot(a, pb))) < 1e-11 * abs(np.vdot(b, pa))
    assert np.vdot(a, pa).real > 0 and abs(np.vdot(a, pa).imag) < 1e-11 * abs(np.vdot(a, pa))


def test_adam_first_step_is_bias_corrected():
    """Step 1 of Adam moves every real coordinate against its gradient by lr |g| / (|g| + eps)
    (the bias corrections cancel the (1 - beta) factors); without them it would move by
    lr (1 - b1) / sqrt(1 - b2) = 3.16 lr.  Real and imaginary parts move independently."""
    g0 = np.array([3.0 - 0.5j, -2e-3 + 4.0j, 1e-9 + 0j])
    th0 = np.array([0.5 + 0.25j, -1.0 + 0.0j, 2.0 - 1.0j])
    lr = 1e-2
    th1 = nn.adam(th0, lambda th: g0, 1, lr)
    for part in (np.real, np.imag):
        g = part(g0)
        want = part(th0) - lr * g / (np.abs(g) + 1e-8)
        assert np.allclose(part(th1), want, rtol=0, atol=1e-15)


def test_adam_ignores_the_gradient_scale_and_descends_a_quadratic():
    """Adam's steps do not depend on a positive scale of the loss (up to eps), and on the
    complex quadratic L = sum |w - c|^2 (Wirtinger gradient 2 (w - c)) with coordinates of very
    different curvature it reaches the minimum."""
    c = np.array([1.0 + 2.0j, -0.5 + 0.1j, 3.0 - 1.0j])
    k = np.array([1.0, 30.0, 300.0])

    def grad(th, s=1.0):
        return s * 2.0 * k * (th - c)

    th0 = np.zeros(3, complex)
    a = nn.adam(th0, grad, 25, 0.05)
    b = nn.adam(th0, lambda th: grad(th, 1000.0), 25, 0.05)
    assert np.allclose(a, b, rtol=0, atol=1e-7)
    far = nn.adam(th0, grad, 3000, 0.01)
    assert np.max(np.abs(far - c)) < 1e-3, far
