"""GPU parity of the learned preconditioner's forward pass, loss and Wirtinger gradients against
the FP64 network oracle (direct form R_even N and Gram form N^dag N), plus gauge covariance,
training and save/load on the GPU.

Tolerances: FP32 activation storage relative L2 1e-5 (forward) and 1e-4 (gradient vector);
BF16 storage (MFMA channel mixing) relative L2 5e-2 and cosine similarity >= 0.999.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import DEV, make_lattice, rel_l2
from oracle import nn as onn

torch = pytest.importorskip("torch")
from paper_1409_1510_amd import hisq  # noqa: E402

pytestmark = pytest.mark.gpu

L = 4
DIMS = (6, 4, 4, 8)


def _theta(seed, scale=0.4):
    g = np.random.Generator(np.random.Philox(key=seed))
    k = onn.n_params(8, L)
    th = (g.standard_normal(k) + 1j * g.standard_normal(k)) * scale
    return th


def _set(lat, theta):
    reals = np.empty(2 * theta.size)
    reals[0::2] = theta.real
    reals[1::2] = theta.imag
    lib = hisq.library()
    arr = (hisq.ctypes.c_double * reals.size)(*reals)
    assert lib.hisq_nn_set_params(lat.ctx, arr, reals.size) == 0


def _init(lat, bf16):
    lib = hisq.library()
    assert lib.hisq_nn_init(lat.ctx, L, 8, 7) == 0
    assert lib.hisq_nn_set_precision(lat.ctx, 1 if bf16 else 0) == 0


def _apply(lat, r):
    z = torch.empty_like(r)
    hisq._check(lat.ctx, hisq.library().hisq_nn_apply(lat.ctx, r.shape[0], hisq.HISQ_F64, hisq._ptr(r), hisq._ptr(z)))
    torch.cuda.synchronize()
    return z.cpu().numpy()


def _cos(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return abs(np.vdot(a, b)) / (np.linalg.norm(a) * np.linalg.norm(b))


@pytest.mark.parametrize("bf16", [False, True])
def test_forward_matches_oracle(bf16):
    lat, fat, naik = make_lattice(DIMS, 300)
    _init(lat, bf16)
    th = _theta(301)
    _set(lat, th)
    r = synth.sources(DIMS, 3, 302)
    z = _apply(lat, torch.from_numpy(r).to(DEV))
    ref = np.stack([onn.forward(th, fat, r[i], DIMS, 8, L) for i in range(3)])
    err = rel_l2(z, ref)
    print(f"NN forward bf16={bf16}: rel L2 {err:.3g}, cosine {_cos(z, ref):.6f}")
    if bf16:
        assert err <= 5e-2 and _cos(z, ref) >= 0.999
    else:
        assert err <= 1e-5
    lat.close()


@pytest.mark.parametrize("bf16,kind", [(False, 0), (True, 0), (False, 1), (True, 1)])
def test_loss_and_gradient_match_oracle(bf16, kind):
    """kind 0: solution-norm loss; kind 1: residual-norm loss ||M P r - r||^2 / ||r||^2."""
    lat, fat, naik = make_lattice(DIMS, 303)
    _init(lat, bf16)
    th = _theta(304)
    _set(lat, th)
    mass = 0.3
    assert hisq.library().hisq_nn_set_loss(lat.ctx, kind, mass) == 0
    r = synth.sources(DIMS, 2, 305)
    y = synth.sources(DIMS, 2, 306)
    loss = hisq.ctypes.c_double()
    grad = (hisq.ctypes.c_double * (2 * th.size))()
    tr, ty = torch.from_numpy(r).to(DEV), torch.from_numpy(y).to(DEV)
    hisq._check(lat.ctx, hisq.library().hisq_nn_loss_grad(lat.ctx, 2, hisq._ptr(tr), hisq._ptr(ty),
                                                          hisq.ctypes.byref(loss), grad))
    g = np.array(grad[0::2]) + 1j * np.array(grad[1::2])
    lref, gref = onn.loss_and_grad(th, fat, r, y, DIMS, 8, L, kind=("solution", "residual")[kind],
                                   naik=naik, mass=mass)
    err = rel_l2(g, gref)
    print(f"NN grad bf16={bf16} kind={kind}: loss {loss.value:.6g} vs {lref:.6g}; grad rel L2 {err:.3g}, cosine {_cos(g, gref):.6f}")
    if bf16:
        assert abs(loss.value - lref) <= 5e-2 * lref
        assert err <= 5e-2 and _cos(g, gref) >= 0.999
    else:
        assert abs(loss.value - lref) <= 1e-5 * lref
        assert err <= 1e-4
    lat.close()


def test_forward_gauge_covariant():
    dims = DIMS
    fat, naik = synth.gauge_links(dims, 307)
    vol = int(np.prod(dims))
    om = synth.haar_su3(np.random.Generator(np.random.Philox(key=308)), vol)
    omd = np.conj(np.swapaxes(om, -1, -2))
    lx, ly, lz, lt = dims
    lex = np.arange(vol)
    c = np.stack([lex % lx, (lex // lx) % ly, (lex // (lx * ly)) % lz, lex // (lx * ly * lz)], 1)
    fat_g = np.empty_like(fat)
    for mu in range(4):
        cc = c.copy()
        cc[:, mu] = (cc[:, mu] + 1) % dims[mu]
        fwd = cc[:, 0] + lx * (cc[:, 1] + ly * (cc[:, 2] + lz * cc[:, 3]))
        fat_g[:, mu] = om @ fat[:, mu] @ omd[fwd]
    th = _theta(309)
    r = synth.sources(dims, 1, 310)
    ev = oracle.parity_lex(dims, 0)
    rg = np.einsum("sab,bs->as", om[ev], r[0])[None]
    outs = []
    for links, rr in ((fat, r), (fat_g, rg)):
        lat = hisq.Lattice(dims, 0)
        lat.load_links(links, naik, hisq.HISQ_LINKS_F32)
        _init(lat, False)
        _set(lat, th)
        outs.append(_apply(lat, torch.from_numpy(np.ascontiguousarray(rr)).to(DEV))[0])
        lat.close()
    expect = np.einsum("sab,bs->as", om[ev], outs[0])
    assert rel_l2(outs[1], expect) <= 1e-5


def test_training_reduces_loss_and_save_load(tmp_path):
    """Pairs (b, M^-1 b) from the GPU's plain FP64 CG; a few epochs of Adam on the GPU lower the
    loss; the trained weights survive a save/load round trip bit for bit."""
    dims, mass = (8, 8, 4, 4), 0.2
    lat, fat, naik = make_lattice(dims, 311)
    b = torch.from_numpy(synth.sources(dims, 32, 312)).to(DEV)
    x, info = lat.cg(mass, b, kind=hisq.HISQ_CG_F64, tol=1e-10)
    assert info["rc"] == 0
    _init(lat, True)
    lib = hisq.library()
    hist = (hisq.ctypes.c_double * 12)()
    hisq._check(lat.ctx, lib.hisq_nn_train(lat.ctx, 32, hisq._ptr(b), hisq._ptr(x), 12, 8, 1e-2, 5, hist))
    h = list(hist)
    print("training loss per epoch:", [f"{v:.4f}" for v in h])
    assert all(np.isfinite(h)) and h[-1] < 0.9 * h[0]
    n = lib.hisq_nn_num_params(lat.ctx)
    w1 = (hisq.ctypes.c_double * (2 * n))()
    hisq._check(lat.ctx, lib.hisq_nn_get_params(lat.ctx, w1, 2 * n))
    path = str(tmp_path / "net.bin").encode()
    hisq._check(lat.ctx, lib.hisq_nn_save(lat.ctx, path))
    hisq._check(lat.ctx, lib.hisq_nn_init(lat.ctx, L, 8, 99))
    hisq._check(lat.ctx, lib.hisq_nn_load(lat.ctx, path))
    w2 = (hisq.ctypes.c_double * (2 * n))()
    hisq._check(lat.ctx, lib.hisq_nn_get_params(lat.ctx, w2, 2 * n))
    assert list(w1) == list(w2)
    lat.close()


@pytest.mark.parametrize("bf16", [False, True])
def test_gram_apply_matches_oracle(bf16):
    lat, fat, naik = make_lattice(DIMS, 320)
    _init(lat, bf16)
    th = _theta(321)
    _set(lat, th)
    assert hisq.library().hisq_nn_set_form(lat.ctx, hisq.HISQ_NN_FORM_GRAM) == 0
    r = synth.sources(DIMS, 3, 322)
    z = _apply(lat, torch.from_numpy(r).to(DEV))
    ref = np.stack([onn.apply(th, fat, r[i], DIMS, 8, L, "gram") for i in range(3)])
    err = rel_l2(z, ref)
    print(f"NN Gram apply bf16={bf16}: rel L2 {err:.3g}, cosine {_cos(z, ref):.6f}")
    if bf16:
        assert err <= 5e-2 and _cos(z, ref) >= 0.999
    else:
        assert err <= 1e-5
    lat.close()


@pytest.mark.parametrize("bf16,kind", [(False, 0), (True, 0), (False, 1), (True, 1)])
def test_gram_loss_and_gradient_match_oracle(bf16, kind):
    lat, fat, naik = make_lattice(DIMS, 323)
    _init(lat, bf16)
    th = _theta(324, scale=0.3)
    _set(lat, th)
    mass = 0.3
    lib = hisq.library()
    assert lib.hisq_nn_set_loss(lat.ctx, kind, mass) == 0
    assert lib.hisq_nn_set_form(lat.ctx, hisq.HISQ_NN_FORM_GRAM) == 0
    r = synth.sources(DIMS, 2, 325)
    y = synth.sources(DIMS, 2, 326)
    loss = hisq.ctypes.c_double()
    grad = (hisq.ctypes.c_double * (2 * th.size))()
    tr, ty = torch.from_numpy(r).to(DEV), torch.from_numpy(y).to(DEV)
    hisq._check(lat.ctx, lib.hisq_nn_loss_grad(lat.ctx, 2, hisq._ptr(tr), hisq._ptr(ty), hisq.ctypes.byref(loss), grad))
    g = np.array(grad[0::2]) + 1j * np.array(grad[1::2])
    lref, gref = onn.gram_loss_and_grad(th, fat, r, y, DIMS, 8, L, kind=("solution", "residual")[kind],
                                        naik=naik, mass=mass)
    err = rel_l2(g, gref)
    print(f"NN Gram grad bf16={bf16} kind={kind}: loss {loss.value:.6g} vs {lref:.6g}; grad rel L2 {err:.3g}, "
          f"cosine {_cos(g, gref):.6f}")
    if bf16:
        assert abs(loss.value - lref) <= 5e-2 * lref
        assert err <= 5e-2 and _cos(g, gref) >= 0.999
    else:
        assert abs(loss.value - lref) <= 1e-5 * lref
        assert err <= 1e-4
    lat.close()


def test_save_load_keeps_the_form(tmp_path):
    lat, fat, naik = make_lattice(DIMS, 327)
    lib = hisq.library()
    _init(lat, False)
    _set(lat, _theta(328))
    assert lib.hisq_nn_set_form(lat.ctx, hisq.HISQ_NN_FORM_GRAM) == 0
    r = torch.from_numpy(synth.sources(DIMS, 2, 329)).to(DEV)
    z1 = _apply(lat, r)
    path = str(tmp_path / "gram.bin").encode()
    hisq._check(lat.ctx, lib.hisq_nn_save(lat.ctx, path))
    hisq._check(lat.ctx, lib.hisq_nn_init(lat.ctx, L, 8, 99))
    assert lib.hisq_nn_set_precision(lat.ctx, 0) == 0
    hisq._check(lat.ctx, lib.hisq_nn_load(lat.ctx, path))
    z2 = _apply(lat, r)
    assert np.array_equal(z1, z2)
    assert lib.hisq_nn_set_form(lat.ctx, 2) == hisq.HISQ_ERR_ARG
    lat.close()


def test_training_steps_match_oracle_adam():
    """Two epochs of hisq_nn_train on one minibatch of two pairs (two Adam steps on the same
    pairs, FP32 activations, solution loss) against the oracle's Adam on the oracle's Wirtinger
    gradient: the recorded losses match the oracle's at the start of each step, and every real
    parameter whose starting gradient is not near zero ends where the oracle's does, to 1e-3 of
    a step.  (Near-zero gradient components take their sign from FP32 rounding on the GPU.)"""
    lat, fat, naik = make_lattice(DIMS, 330)
    _init(lat, False)
    lib = hisq.library()
    th0 = _theta(331, scale=0.3).astype(np.complex64).astype(complex)  # the FP32 master weights
    _set(lat, th0)
    r = synth.sources(DIMS, 2, 332)
    y = synth.sources(DIMS, 2, 333)
    lr = 1e-2
    hist = (hisq.ctypes.c_double * 2)()
    tr = torch.from_numpy(r).to(DEV)
    ty = torch.from_numpy(y).to(DEV)
    hisq._check(lat.ctx, lib.hisq_nn_train(lat.ctx, 2, hisq._ptr(tr), hisq._ptr(ty), 2, 2, lr, 5, hist))
    n = th0.size
    w = (hisq.ctypes.c_double * (2 * n))()
    hisq._check(lat.ctx, lib.hisq_nn_get_params(lat.ctx, w, 2 * n))
    wv = np.array(list(w))
    th_gpu = wv[0::2] + 1j * wv[1::2]

    def grad(th):
        return onn.loss_and_grad(th, fat, list(r), list(y), DIMS, 8, L)[1]

    th1 = onn.adam(th0, grad, 1, lr)
    th2 = onn.adam(th0, grad, 2, lr)
    l0 = onn.loss(th0, fat, list(r), list(y), DIMS, 8, L)
    l1 = onn.loss(th1, fat, list(r), list(y), DIMS, 8, L)
    print(f"losses GPU {hist[0]:.6f} {hist[1]:.6f}, oracle {l0:.6f} {l1:.6f}")
    assert abs(hist[0] - l0) <= 1e-5 * l0 and abs(hist[1] - l1) <= 1e-5 * l1
    g0 = grad(th0)
    g_re = np.concatenate([g0.real, g0.imag])
    d = np.concatenate([(th_gpu - th2).real, (th_gpu - th2).imag])
    keep = np.abs(g_re) > 1e-2 * np.max(np.abs(g_re))
    assert keep.mean() >= 0.7, keep.mean()
    tol = 1e-3 * lr + 2e-7 * np.max(np.abs(th0))
    print(f"Adam: {keep.sum()} of {keep.size} reals compared, max deviation {np.max(np.abs(d[keep])):.3g} "
          f"(bound {tol:.3g}); all reals {np.max(np.abs(d)):.3g} against a step of {lr}")
    assert np.max(np.abs(d[keep])) <= tol
    assert np.max(np.abs(d)) <= 2.5 * lr
    lat.close()
