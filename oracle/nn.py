"""Oracle of the learned gauge-covariant preconditioner: forward, loss and gradients (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no preconditioner; this network is the learned-preconditioner form the build adds
around the paper's even-odd CG.  Reading of the network (one right-hand side r on even sites):

    phi_1 = W_in (x) E(r)                      E: embed the even-site vector in the full lattice
    psi_l = S(a_l, phi_l)                      l = 1..L
    phi_l = W_l psi_{l-1}                      l = 2..L  (C x C complex channel mixing per site, colour)
    z     = R_even( sum_c W_out[c] psi_L[c] )  R_even: keep the even sites

with the per-channel gauge-covariant one-hop stencil built from the fat links X of Eq. 3:

    S(a, phi)_c(x) = a[0,c] phi_c(x) + sum_mu ( a[1+mu,c] X(x,mu) phi_c(x+mu)
                                              + a[5+mu,c] X(x-mu,mu)^dag phi_c(x-mu) ).

Every layer is linear (no activation), so z = P r for a fixed linear map P (a learned sparse
approximate inverse with a 4-hop reach for L = 4).  It is gauge covariant: with
X(x,mu) -> O(x) X(x,mu) O(x+mu)^dag and r -> O r, z -> O z.

Two forms of the preconditioner built from the same layers:
    direct: z = P r = R_even N r
    Gram:   z = N^dag N r, with N r = sum_c W_out[c] psi_L[c] on the full lattice, which is
            Hermitian positive semi-definite by construction (the form suited to CG).

Training pairs (r_j, y_j = M^-1 r_j); two losses over a minibatch of B pairs:
    solution norm: L = (1/B) sum_j ||P r_j - y_j||^2 / ||y_j||^2
    residual norm: L = (1/B) sum_j ||M (P r_j - y_j)||^2 / ||r_j||^2 = (1/B) sum_j ||M P r_j - r_j||^2 / ||r_j||^2
(the second measures the same prediction error in the norm of M^2, using M y_j = r_j).
Gradients use the Wirtinger convention grad(w) = dL/dRe(w) + i dL/dIm(w).

Parameters, canonical flat order (complex; as reals: re, im interleaved):
    W_in[C]; then for l = 1..L: (W_l[C][C] row-major [out][in], for l >= 2), a_l[9][C];
    then W_out[C].  C = 8, L = 4 gives 496 complex = 992 reals.
Hop index h: 0 self, 1+mu forward (x+mu), 5+mu backward (x-mu), mu = 0..3 = x, y, z, t.
"""
from __future__ import annotations

import numpy as np

from .dslash import _AXIS, embed, extract, m_ee


def n_params(channels: int, layers: int) -> int:
    """Number of complex parameters."""
    c = channels
    return c + layers * 9 * c + (layers - 1) * c * c + c


def unpack(theta, channels: int, layers: int) -> dict:
    """Flat complex parameter vector -> dict(W_in, W (list, index l-2), a (list), W_out)."""
    theta = np.asarray(theta, np.complex128)
    c = channels
    k = 0
    w_in = theta[k:k + c]
    k += c
    ws, as_ = [], []
    for l in range(layers):
        if l >= 1:
            ws.append(theta[k:k + c * c].reshape(c, c))
            k += c * c
        as_.append(theta[k:k + 9 * c].reshape(9, c))
        k += 9 * c
    w_out = theta[k:k + c]
    k += c
    assert k == theta.size
    return dict(W_in=w_in, W=ws, a=as_, W_out=w_out)


def pack(p: dict) -> np.ndarray:
    parts = [p["W_in"]]
    for l, a in enumerate(p["a"]):
        if l >= 1:
            parts.append(p["W"][l - 1].ravel())
        parts.append(a.ravel())
    parts.append(p["W_out"])
    return np.concatenate([np.asarray(x, np.complex128).ravel() for x in parts])


def _hops(fat, phi, dims):
    """The 9 hop images of phi [C][V][3]: list index h, each [C][V][3]."""
    lx, ly, lz, lt = dims
    shp = (lt, lz, ly, lx)
    xf = fat.reshape(shp + (4, 3, 3))
    c = phi.shape[0]
    pf = phi.reshape((c,) + shp + (3,))
    out = [None] * 9
    out[0] = phi
    for mu in range(4):
        ax = _AXIS[mu] + 1  # +1: channel axis first
        u = xf[..., mu, :, :]
        ud = np.conj(np.swapaxes(np.roll(u, 1, _AXIS[mu]), -1, -2))  # X(x-mu, mu)^dag
        fwd = np.einsum("...ab,c...b->c...a", u, np.roll(pf, -1, ax))
        bwd = np.einsum("...ab,c...b->c...a", ud, np.roll(pf, 1, ax))
        out[1 + mu] = fwd.reshape(phi.shape)
        out[5 + mu] = bwd.reshape(phi.shape)
    return out


def _adjoint_hop_index(h: int) -> int:
    """The adjoint of the forward hop along mu is the backward hop along mu and vice versa."""
    if h == 0:
        return 0
    return h + 4 if h < 5 else h - 4


def stencil(fat, a, phi, dims):
    hs = _hops(fat, phi, dims)
    return sum(a[h][:, None, None] * hs[h] for h in range(9))


def stencil_adjoint(fat, a, g, dims):
    hs = _hops(fat, g, dims)
    return sum(np.conj(a[h])[:, None, None] * hs[_adjoint_hop_index(h)] for h in range(9))


def forward(theta, fat, r, dims, channels: int, layers: int, keep: bool = False):
    """z = P r for one rhs r [3][V/2] (even sites).  keep: also return the intermediates."""
    p = unpack(theta, channels, layers)
    e = embed(r, dims, 0)                                   # [V][3]
    phi = p["W_in"][:, None, None] * e[None]                # [C][V][3]
    cache = {"e": e, "phi": [], "psi": []}
    psi = None
    for l in range(layers):
        if l >= 1:
            phi = np.einsum("oi,ivc->ovc", p["W"][l - 1], psi)
        psi = stencil(fat, p["a"][l], phi, dims)
        cache["phi"].append(phi)
        cache["psi"].append(psi)
    full = np.einsum("c,cvk->vk", p["W_out"], psi)
    z = extract(full, dims, 0)
    return (z, cache) if keep else z


def network_full(theta, fat, r, dims, channels: int, layers: int, keep: bool = False):
    """N r: the network output sum_c W_out[c] psi_L[c] on the full lattice, [V][3]."""
    p = unpack(theta, channels, layers)
    e = embed(r, dims, 0)
    phi = p["W_in"][:, None, None] * e[None]
    cache = {"e": e, "phi": [], "psi": []}
    psi = None
    for l in range(layers):
        if l >= 1:
            phi = np.einsum("oi,ivc->ovc", p["W"][l - 1], psi)
        psi = stencil(fat, p["a"][l], phi, dims)
        cache["phi"].append(phi)
        cache["psi"].append(psi)
    full = np.einsum("c,cvk->vk", p["W_out"], psi)
    return (full, cache) if keep else full


def network_adjoint(theta, fat, u, dims, channels: int, layers: int):
    """N^dag u for a full-lattice field u [V][3]: an even-site vector [3][V/2]."""
    p = unpack(theta, channels, layers)
    g = np.conj(p["W_out"])[:, None, None] * np.asarray(u)[None]
    for l in reversed(range(layers)):
        g = stencil_adjoint(fat, p["a"][l], g, dims)
        if l >= 1:
            g = np.einsum("oi,ovk->ivk", np.conj(p["W"][l - 1]), g)
    return extract(np.einsum("c,cvk->vk", np.conj(p["W_in"]), g), dims, 0)


def apply(theta, fat, r, dims, channels: int, layers: int, form: str = "direct"):
    """The preconditioner: R_even N r ("direct") or N^dag N r ("gram")."""
    if form == "direct":
        return forward(theta, fat, r, dims, channels, layers)
    return network_adjoint(theta, fat, network_full(theta, fat, r, dims, channels, layers),
                           dims, channels, layers)


def backprop(theta, fat, x, g_full, dims, channels: int, layers: int):
    """Wirtinger gradient G with dL = Re sum conj(G) dtheta of L = Re<g_full, N x> for an
    even-site input x and a full-lattice output gradient g_full."""
    p = unpack(theta, channels, layers)
    grad = {"W_in": np.zeros(channels, complex), "W": [np.zeros_like(w) for w in p["W"]],
            "a": [np.zeros_like(a) for a in p["a"]], "W_out": np.zeros(channels, complex)}
    _, cache = network_full(theta, fat, x, dims, channels, layers, keep=True)
    grad["W_out"] += np.einsum("cvk,vk->c", np.conj(cache["psi"][-1]), g_full)
    gpsi = np.conj(p["W_out"])[:, None, None] * np.asarray(g_full)[None]
    for l in reversed(range(layers)):
        phi = cache["phi"][l]
        hs = _hops(fat, phi, dims)
        for h in range(9):
            grad["a"][l][h] += np.einsum("cvk,cvk->c", np.conj(hs[h]), gpsi)
        gphi = stencil_adjoint(fat, p["a"][l], gpsi, dims)
        if l >= 1:
            grad["W"][l - 1] += np.einsum("ovk,ivk->oi", gphi, np.conj(cache["psi"][l - 1]))
            gpsi = np.einsum("oi,ovk->ivk", np.conj(p["W"][l - 1]), gphi)
        else:
            grad["W_in"] += np.einsum("vk,cvk->c", np.conj(cache["e"]), gphi)
    return pack(grad)


def gram_loss_and_grad(theta, fat, rs, ys, dims, channels: int, layers: int, kind="solution",
                       naik=None, mass=None):
    """Loss of the Gram form z = N^dag N r and its gradient.  With u = N r and G the gradient
    of the loss with respect to z, dz = (dN)^dag u + N^dag (dN) r gives
    dL = Re<u, dN G> + Re<N G, dN r>: two ordinary backward passes, one with input G and
    output gradient u, one with input r and output gradient N G."""
    nb = len(rs)
    tot = 0.0
    grad = np.zeros(n_params(channels, layers), complex)
    for r, y in zip(rs, ys):
        u = network_full(theta, fat, r, dims, channels, layers)
        z = network_adjoint(theta, fat, u, dims, channels, layers)
        lj, gz = _pair_loss(z, r, y, kind, fat, naik, dims, mass)
        tot += lj
        gz = gz / nb
        ng = network_full(theta, fat, gz, dims, channels, layers)
        grad += backprop(theta, fat, gz, u, dims, channels, layers)
        grad += backprop(theta, fat, r, ng, dims, channels, layers)
    return tot / nb, grad


def _pair_loss(z, r, y, kind, fat, naik, dims, mass):
    """(loss of one pair, Wirtinger gradient with respect to z) before the 1/B factor."""
    if kind == "solution":
        ny2 = np.linalg.norm(y) ** 2
        return np.linalg.norm(z - y) ** 2 / ny2, 2.0 * (z - y) / ny2
    mz = m_ee(fat, naik, z[None], dims, mass)[0]
    nr2 = np.linalg.norm(r) ** 2
    gw = 2.0 * (mz - r) / nr2
    return np.linalg.norm(mz - r) ** 2 / nr2, m_ee(fat, naik, gw[None], dims, mass)[0]  # M Hermitian


def loss(theta, fat, rs, ys, dims, channels: int, layers: int, kind="solution", naik=None,
         mass=None, form="direct") -> float:
    tot = 0.0
    for r, y in zip(rs, ys):
        z = apply(theta, fat, r, dims, channels, layers, form)
        tot += _pair_loss(z, r, y, kind, fat, naik, dims, mass)[0]
    return tot / len(rs)


def loss_and_grad(theta, fat, rs, ys, dims, channels: int, layers: int, kind="solution",
                  naik=None, mass=None):
    """Loss and its Wirtinger gradient (complex, canonical order) by reverse-mode adjoints.
    kind "residual" needs the Naik links and the mass of M."""
    p = unpack(theta, channels, layers)
    grad = {"W_in": np.zeros(channels, complex), "W": [np.zeros_like(w) for w in p["W"]],
            "a": [np.zeros_like(a) for a in p["a"]], "W_out": np.zeros(channels, complex)}
    nb = len(rs)
    tot = 0.0
    for r, y in zip(rs, ys):
        z, cache = forward(theta, fat, r, dims, channels, layers, keep=True)
        lj, gz = _pair_loss(z, r, y, kind, fat, naik, dims, mass)
        tot += lj
        gz = gz / nb                                        # grad of L w.r.t. z
        gout = embed(gz, dims, 0)                            # [V][3], zero on odd sites
        psi_l = cache["psi"][-1]
        grad["W_out"] += np.einsum("cvk,vk->c", np.conj(psi_l), gout)
        gpsi = np.conj(p["W_out"])[:, None, None] * gout[None]
        for l in reversed(range(layers)):
            phi = cache["phi"][l]
            hs = _hops(fat, phi, dims)
            for h in range(9):
                grad["a"][l][h] += np.einsum("cvk,cvk->c", np.conj(hs[h]), gpsi)
            gphi = stencil_adjoint(fat, p["a"][l], gpsi, dims)
            if l >= 1:
                prev = cache["psi"][l - 1]
                grad["W"][l - 1] += np.einsum("ovk,ivk->oi", gphi, np.conj(prev))
                gpsi = np.einsum("oi,ovk->ivk", np.conj(p["W"][l - 1]), gphi)
            else:
                grad["W_in"] += np.einsum("vk,cvk->c", np.conj(cache["e"]), gphi)
    return tot / nb, pack(grad)


def init_params(channels: int, layers: int, seed: int, scale: float = 0.1) -> np.ndarray:
    """Start near P = identity: channel 0 carries r through self-hops, the rest is small noise."""
    gen = np.random.Generator(np.random.Philox(key=seed))
    th = (gen.standard_normal(n_params(channels, layers)) +
          1j * gen.standard_normal(n_params(channels, layers))) * scale * np.sqrt(0.5)
    p = unpack(th, channels, layers)
    p["W_in"][0] += 1.0
    p["W_out"][0] += 1.0
    for l in range(layers):
        p["a"][l][0, 0] += 1.0
        if l >= 1:
            p["W"][l - 1][0, 0] += 1.0
    return pack(p)


def adam(theta, grad_fn, steps: int, lr: float, b1: float = 0.9, b2: float = 0.999,
         eps: float = 1e-8) -> np.ndarray:
    """`steps` Adam updates (Kingma and Ba 2014, Algorithm 1, with their default beta1, beta2,
    epsilon) of the complex parameters theta, grad_fn(theta) giving the Wirtinger gradient
    dL/dRe + i dL/dIm.  Reading for complex parameters: Adam runs on the reals (Re, Im of every
    parameter) as independent coordinates, so the gradient of coordinate Re w is Re grad(w) and
    that of Im w is Im grad(w); the moments are kept per real coordinate."""
    th = np.array(theta, complex)
    x = np.concatenate([th.real, th.imag])
    m = np.zeros_like(x)
    v = np.zeros_like(x)
    n = th.size
    for t in range(1, steps + 1):
        g = grad_fn(x[:n] + 1j * x[n:])
        gr = np.concatenate([g.real, g.imag])
        m = b1 * m + (1 - b1) * gr
        v = b2 * v + (1 - b2) * gr * gr
        mhat = m / (1 - b1 ** t)
        vhat = v / (1 - b2 ** t)
        x = x - lr * mhat / (np.sqrt(vhat) + eps)
    return x[:n] + 1j * x[n:]
