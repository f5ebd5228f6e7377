"""GPU multi-rhs CG solvers against the oracle.

Check of every solve: the FP64 true residual ||b - M x|| / ||b|| recomputed on the CPU with the
oracle's M applied to the GPU's x.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import DEV, make_lattice

torch = pytest.importorskip("torch")
from paper_1409_1510_amd import hisq  # noqa: E402

pytestmark = pytest.mark.gpu


def _solve(lat, mass, b, **kw):
    x, info = lat.cg(mass, torch.from_numpy(b).to(DEV), **kw)
    return x.cpu().numpy(), info


def test_c0_plain_f64_matches_oracle_cg():
    cfg = synth.WORKLOADS["c0"]
    dims, mass, tol = cfg["dims"], cfg["mass"], cfg["tol"]
    lat, fat, naik = make_lattice(dims, synth.workload_seed("c0"))
    b = synth.sources(dims, 1, synth.workload_seed("c0") + 1)
    x, info = _solve(lat, mass, b, kind=hisq.HISQ_CG_F64, tol=tol)
    assert info["rc"] == 0 and info["converged"] == [1]
    res = oracle.true_residual(fat, naik, x, b, dims, mass)
    assert res[0] <= tol
    x_ref, it_ref, _ = oracle.cg(fat, naik, b, dims, mass, tol)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-8
    # same algorithm, same operator: the iteration counts agree to within a couple
    assert abs(info["iters"][0] - it_ref[0]) <= 3
    print(f"c0: GPU {info['iters'][0]} iterations, oracle {it_ref[0]}, true residual {res[0]:.2e}")
    lat.close()


def test_dense_lu_4444():
    dims, mass = (4, 4, 4, 4), 0.1
    lat, fat, naik = make_lattice(dims, 200)
    b = synth.sources(dims, 3, 201)
    x, info = _solve(lat, mass, b, kind=hisq.HISQ_CG_F64, tol=1e-12)
    # reference: M as a dense matrix, column j = oracle M applied to unit vector j (vectors
    # flattened in their [3][V/2] order), solved by LAPACK
    vh = lat.vh
    eye = np.eye(3 * vh).reshape(3 * vh, 3, vh)
    cols = oracle.m_ee(fat, naik, eye, dims, mass).reshape(3 * vh, 3 * vh).T
    for i in range(3):
        x_lu = np.linalg.solve(cols, b[i].ravel()).reshape(3, vh)
        assert np.linalg.norm(x[i] - x_lu) / np.linalg.norm(x_lu) < 1e-9
    lat.close()


@pytest.mark.parametrize("link_prec", [hisq.HISQ_F32, hisq.HISQ_F16])
def test_mixed_small(link_prec):
    dims, mass, tol = (8, 8, 8, 8), 0.05, 1e-8
    lat, fat, naik = make_lattice(dims, 202)
    b = synth.sources(dims, 4, 203)
    x, info = _solve(lat, mass, b, kind=hisq.HISQ_CG_MIXED, tol=tol, link_prec=link_prec,
                     reliable_every=50)
    assert info["rc"] == 0, info
    res = oracle.true_residual(fat, naik, x, b, dims, mass)
    assert np.all(res <= tol), res
    assert np.allclose(res, info["true_resid"], rtol=1e-3, atol=1e-12)
    assert info["reliable_updates"] >= 1
    print(f"mixed link_prec={link_prec}: iters {info['iters']} reps {info['reliable_updates']}")
    lat.close()


def test_per_rhs_stop_zero_rhs_and_warm_start():
    dims, mass, tol = (8, 6, 4, 10), 0.2, 1e-10
    lat, fat, naik = make_lattice(dims, 204)
    b = synth.sources(dims, 4, 205)
    b[1] = 0.0                  # zero rhs: x = 0, converged, no iterations
    b[2] *= 1e-3                # same direction scaled: same relative iteration count
    x, info = _solve(lat, mass, b, kind=hisq.HISQ_CG_F64, tol=tol)
    assert info["rc"] == 0
    assert np.all(x[1] == 0) and info["iters"][1] == 0 and info["converged"][1] == 1
    res = oracle.true_residual(fat, naik, x, b, dims, mass)
    assert np.all(res[[0, 2, 3]] <= tol)
    # warm start from the solution: converges at once
    x2, info2 = lat.cg(mass, torch.from_numpy(b).to(DEV), kind=hisq.HISQ_CG_F64, tol=1e-8,
                       x0=torch.from_numpy(x).to(DEV))
    assert info2["rc"] == 0 and max(info2["iters"]) == 0
    # iteration cap: NOCONV with valid stats
    x3, info3 = lat.cg(mass, torch.from_numpy(b).to(DEV), kind=hisq.HISQ_CG_F64, tol=1e-10,
                       max_iter=3)
    assert info3["rc"] == hisq.HISQ_ERR_NOCONV
    assert info3["converged"][1] == 1 and info3["converged"][0] == 0
    lat.close()


@pytest.mark.parametrize("kind", [hisq.HISQ_CG_F64, hisq.HISQ_CG_MIXED])
def test_max_rhs_bundle(kind):
    """A full bundle of HISQ_MAX_RHS rhs (4^4 x 6 lattice): every rhs reaches the tolerance in the
    oracle's true residual, and rhs i of the bundle gets the same iterations as the same source
    solved alone (the per-rhs scalars do not mix)."""
    dims, mass, tol = (4, 4, 4, 6), 0.1, 1e-8
    lat, fat, naik = make_lattice(dims, 210)
    n = hisq.HISQ_MAX_RHS
    b = synth.sources(dims, n, 211)
    x, info = _solve(lat, mass, b, kind=kind, tol=tol, link_prec=hisq.HISQ_F32)
    assert info["rc"] == 0 and all(info["converged"])
    res = oracle.true_residual(fat, naik, x, b, dims, mass)
    assert np.all(res <= tol)
    if kind == hisq.HISQ_CG_F64:
        for i in (0, n - 1):
            xi, infoi = _solve(lat, mass, b[i:i + 1], kind=kind, tol=tol)
            assert infoi["iters"][0] == info["iters"][i]
            assert np.array_equal(xi[0], x[i])
    lat.close()


def test_nonfinite_source_rejected():
    dims = (4, 4, 4, 4)
    lat, fat, naik = make_lattice(dims, 206)
    b = synth.sources(dims, 2, 207)
    b[1, 0, 3] = np.inf
    with pytest.raises(hisq.HisqError) as e:
        lat.cg(0.1, torch.from_numpy(b).to(DEV), kind=hisq.HISQ_CG_F64, tol=1e-8)
    assert e.value.code == hisq.HISQ_ERR_NONFINITE
    lat.close()


def test_c2_mixed_fp16_links_full_size():
    """32^3 x 8, m = 0.02, 8 complex Gaussian rhs, FP32 Dslash on FP16 links, FP64 reliable
    update every 50 iterations: every rhs to a true FP64 residual <= 1e-8 (checked with the
    oracle's M), and the plain FP64 CG on the same GPU for comparison."""
    cfg = synth.WORKLOADS["c2"]
    dims, mass, tol, n = cfg["dims"], cfg["mass"], cfg["tol"], cfg["n"]
    lat, fat, naik = make_lattice(dims, synth.workload_seed("c2"))
    b = synth.sources(dims, n, synth.workload_seed("c2") + 1)
    xm, im = _solve(lat, mass, b, kind=hisq.HISQ_CG_MIXED, tol=tol, link_prec=hisq.HISQ_F16,
                    reliable_every=50, max_iter=40000)
    assert im["rc"] == 0, im
    xd, idd = _solve(lat, mass, b, kind=hisq.HISQ_CG_F64, tol=tol, max_iter=40000)
    assert idd["rc"] == 0
    for i in (0, n - 1):  # oracle check of two rhs (the CPU M at this size takes seconds)
        res = oracle.true_residual(fat, naik, xm[i:i + 1], b[i:i + 1], dims, mass)
        assert res[0] <= tol
        res = oracle.true_residual(fat, naik, xd[i:i + 1], b[i:i + 1], dims, mass)
        assert res[0] <= tol
    assert max(im["true_resid"]) <= tol and max(idd["true_resid"]) <= tol
    print(f"c2 mixed: {im['seconds']:.3f}s iters {im['iters']} reps {im['reliable_updates']}; "
          f"fp64: {idd['seconds']:.3f}s iters {idd['iters']}")
    lat.close()


@pytest.mark.parametrize("mass", [0.01, 0.005])
def test_mixed_fp16_links_do_not_slow_ill_conditioned_solves(mass):
    """Ill-conditioned small case (8^4, m = 0.01 and 0.005): with FP16 link storage the mixed
    solver moves its inner operator to the FP32 links when the FP16 rounding dominates (true
    residual drifting from the iterated one, a stall, or a falling convergence rate), reports the
    iteration of the switch, reaches the true FP64 residual, and needs at most 25 % more
    iterations than with FP32 links throughout; with FP32 links it never switches."""
    dims, tol = (8, 8, 8, 8), 1e-8
    lat, fat, naik = make_lattice(dims, 60)
    b = synth.sources(dims, 4, 61)
    tb = torch.from_numpy(b).to(DEV)
    iters = {}
    for link_prec in (hisq.HISQ_F32, hisq.HISQ_F16):
        x, info = lat.cg(mass, tb, kind=hisq.HISQ_CG_MIXED, tol=tol, link_prec=link_prec, max_iter=60000)
        assert info["rc"] == 0, info
        res = oracle.true_residual(fat, naik, x.cpu().numpy(), b, dims, mass)
        assert np.all(res <= tol)
        sw = info["link_switch_iter"]
        iters[link_prec] = max(info["iters"])
        print(f"m {mass} link_prec {link_prec}: iters {iters[link_prec]}, FP32 links from iteration {sw}")
        if link_prec == hisq.HISQ_F32:
            assert sw == -1
        else:
            assert sw == -1 or 0 <= sw <= info["total_iters"]
    assert iters[hisq.HISQ_F16] <= 1.25 * iters[hisq.HISQ_F32]
    xf, info = lat.cg(mass, tb, kind=hisq.HISQ_CG_F64, tol=tol, max_iter=60000)
    assert info["link_switch_iter"] == -1
    lat.close()


@pytest.mark.parametrize("link_prec", [hisq.HISQ_F32, hisq.HISQ_F16])
def test_c3_mixed_full_size_true_residual(link_prec):
    """48^3 x 12, m = 0.01, Z2 rhs (2 of the 16, to keep the CPU check short): the mixed solver
    reaches a true FP64 residual <= 1e-8 as measured by the oracle's M on the GPU's solution."""
    cfg = synth.WORKLOADS["c3"]
    dims, mass, tol = cfg["dims"], cfg["mass"], cfg["tol"]
    seed = synth.workload_seed("c3")
    lat, fat, naik = make_lattice(dims, seed)
    b = synth.sources(dims, 2, seed + 1, cfg["source"])
    x, info = _solve(lat, mass, b, kind=hisq.HISQ_CG_MIXED, tol=tol, link_prec=link_prec, max_iter=40000)
    assert info["rc"] == 0, info
    res = oracle.true_residual(fat, naik, x, b, dims, mass)
    print(f"c3 mixed link_prec {link_prec}: iters {info['iters']}, oracle residual {res}")
    assert np.all(res <= tol)
    lat.close()


@pytest.mark.timeout(900)
def test_c4_mixed_full_size_true_residual():
    """64^3 x 16, m = 0.005, links with eps = 0.3, 2 complex Gaussian rhs of the 32 (the CPU
    check of the solution takes ~20 s per rhs): the mixed solver with FP16 link storage (moving to
    the FP32 links if the FP16 error dominates) reaches a true FP64 residual <= 1e-8 as measured
    by the oracle's M on the GPU's solution."""
    cfg = synth.WORKLOADS["c4"]
    dims, mass, tol = cfg["dims"], cfg["mass"], cfg["tol"]
    seed = synth.workload_seed("c4")
    lat, fat, naik = make_lattice(dims, seed, eps=cfg["eps"])
    b = synth.sources(dims, 2, seed + 1, cfg["source"])
    x, info = _solve(lat, mass, b, kind=hisq.HISQ_CG_MIXED, tol=tol, link_prec=hisq.HISQ_F16,
                     max_iter=60000)
    print(f"c4 mixed: {info['seconds']:.1f} s, iters {info['iters']}, FP32 links from iteration "
          f"{info['link_switch_iter']}, library residuals {info['true_resid']}", flush=True)
    assert info["rc"] == 0, info
    lat.close()
    res = oracle.true_residual(fat, naik, x, b, dims, mass)
    print(f"c4 mixed: oracle residual {res}")
    assert np.all(res <= tol)


@pytest.mark.parametrize("kind", [hisq.HISQ_CG_F64, hisq.HISQ_CG_MIXED])
def test_compaction_uneven_bundle_matches_single_solves(kind):
    """Rhs that converge at different iterations (6 of 8 start from an approximate solution): the
    bundle is repacked to its live rhs as they finish, every rhs meets tol in the oracle's true
    residual, and each one's solution and iteration count are those of the same rhs solved alone,
    bit for bit (a rhs's arithmetic does not depend on its slot or on the bundle size)."""
    dims, mass, tol, n = (8, 8, 8, 8), 0.05, 1e-8, 8
    lat, fat, naik = make_lattice(dims, 212)
    b = synth.sources(dims, n, 213)
    tb = torch.from_numpy(b).to(DEV)
    xa, _ = lat.cg(mass, tb, kind=hisq.HISQ_CG_F64, tol=1e-4, max_iter=20000)
    x0 = xa.clone()
    x0[6:] = 0
    kw = dict(kind=kind, tol=tol, link_prec=hisq.HISQ_F32, max_iter=20000)
    x, info = lat.cg(mass, tb, x0=x0, **kw)
    assert info["rc"] == 0, info
    print(f"kind {kind}: iterations {info['iters']}, repacks {info['compactions']}")
    assert info["compactions"] >= 1
    assert max(info["iters"][:6]) < min(info["iters"][6:])
    # the shrunk bundle ran with the launch configuration of the full one (no autotune mid-solve)
    body = hisq.HISQ_F64 if kind == hisq.HISQ_CG_F64 else hisq.HISQ_F32
    for fused in (0, 1):
        assert hisq.hisq_get_launch(lat.ctx, body, 2, fused) == hisq.hisq_get_launch(lat.ctx, body, 8, fused)
    res = oracle.true_residual(fat, naik, x.cpu().numpy(), b, dims, mass)
    assert np.all(res <= tol)
    for i in (0, 5, 7):
        xi, infoi = lat.cg(mass, tb[i:i + 1].contiguous(), x0=x0[i:i + 1].contiguous(), **kw)
        assert infoi["iters"][0] == info["iters"][i]
        assert torch.equal(xi[0], x[i])
    # the same bundle without repacking: the same solutions and iterations
    xn, infon = lat.cg(mass, tb, x0=x0, compaction=False, **kw)
    assert infon["compactions"] == 0 and infon["iters"] == info["iters"]
    assert torch.equal(xn, x)
    lat.close()


@pytest.mark.parametrize("kind", [hisq.HISQ_CG_F64, hisq.HISQ_CG_MIXED])
def test_cg_same_bits_under_every_launch_shape(kind):
    """A CG solve run with the operator forced to the register-tile form, the LDS form under each
    XCD map (0-3) and the 32-site form: the solutions and iteration counts agree bit for bit, and
    every rhs meets tol in the oracle's true residual.  (32, 32, 8, 4) admits every XCD map; half
    the rhs start from an approximate solution, so the bundle is repacked mid-solve and the shrunk
    bundles run the forced shape too."""
    dims, mass, tol, n = (32, 32, 8, 4), 0.1, 1e-8, 4
    lat, fat, naik = make_lattice(dims, 214)
    b = synth.sources(dims, n, 215)
    tb = torch.from_numpy(b).to(DEV)
    xa, _ = lat.cg(mass, tb, kind=hisq.HISQ_CG_F64, tol=1e-4)
    x0 = xa.clone()
    x0[2:] = 0
    prec = hisq.HISQ_F64 if kind == hisq.HISQ_CG_F64 else hisq.HISQ_F32
    cfgs = [(2, 64, 0, 0, 0)] + [(1, 64, 1, 1, xm) for xm in range(4)]
    if prec == hisq.HISQ_F32:
        cfgs += [(1, 32, 1, 1, 2), (2, 64, 1, 2, 3)]
    first = None
    for cfg in cfgs:
        for m in range(1, n + 1):
            hisq.hisq_set_launch(lat.ctx, prec, m, cfg)
        x, info = lat.cg(mass, tb, x0=x0, kind=kind, tol=tol, link_prec=hisq.HISQ_F32)
        assert info["rc"] == 0, (cfg, info)
        if first is None:
            first = (x, info)
            assert info["compactions"] >= 1
            res = oracle.true_residual(fat, naik, x.cpu().numpy(), b, dims, mass)
            assert np.all(res <= tol), res
        else:
            assert info["iters"] == first[1]["iters"], cfg
            assert torch.equal(x, first[0]), cfg
    print(f"kind {kind}: {len(cfgs)} launch shapes, iterations {first[1]['iters']}")
    lat.close()


@pytest.mark.parametrize("kind", [hisq.HISQ_CG_F64, hisq.HISQ_CG_MIXED])
def test_fused_reductions_same_bits(kind, monkeypatch):
    """The alpha and beta sums done inside the r and p/x passes (every workgroup of a rhs sums
    the partials itself) against the separate reduction launches: the same solutions and
    iteration counts bit for bit, through a repack of the bundle.  At 16^3 x 8 both are fused."""
    dims, mass, tol, n = (16, 16, 16, 8), 0.05, 1e-8, 4
    lat, fat, naik = make_lattice(dims, 216)
    b = synth.sources(dims, n, 217)
    tb = torch.from_numpy(b).to(DEV)
    xa, _ = lat.cg(mass, tb, kind=hisq.HISQ_CG_F64, tol=1e-4)
    x0 = xa.clone()
    x0[2:] = 0
    kw = dict(x0=x0, kind=kind, tol=tol, link_prec=hisq.HISQ_F16)
    monkeypatch.setenv("HISQ_CG_FUSED_REDUCTIONS", "0")
    xs, infos = lat.cg(mass, tb, **kw)
    monkeypatch.delenv("HISQ_CG_FUSED_REDUCTIONS")
    xf, infof = lat.cg(mass, tb, **kw)
    assert infos["rc"] == 0 and infof["rc"] == 0
    assert infof["compactions"] >= 1
    assert infof["iters"] == infos["iters"]
    assert torch.equal(xf, xs)
    res = oracle.true_residual(fat, naik, xf.cpu().numpy(), b, dims, mass)
    assert np.all(res <= tol), res
    print(f"kind {kind}: iterations {infof['iters']}")
    lat.close()
