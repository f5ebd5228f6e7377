"""The allocation-free entry point hisq_dot_mrhs_noalloc, called through the C ABI: bit-identical
to hisq_dot_mrhs on two calls in a row (the second on fewer rhs and other vectors), no device
memory allocated by it, and sizes beyond its static buffer refused with HISQ_ERR_ARG."""
import numpy as np
import pytest

import synth
from gpu_helpers import DEV

torch = pytest.importorskip("torch")
from paper_1409_1510_amd import hisq  # noqa: E402

pytestmark = pytest.mark.gpu


def _call(lat, prec, n, a, b, dots):
    hisq.hisq_set_stream(lat.ctx)  # torch's current stream, as the Lattice methods do
    rc = hisq.library().hisq_dot_mrhs_noalloc(lat.ctx, prec, n, hisq._ptr(a), hisq._ptr(b), hisq._ptr(dots))
    assert rc == hisq.HISQ_OK, hisq.hisq_last_error(lat.ctx)
    return dots


@pytest.mark.parametrize("prec", [hisq.HISQ_F64, hisq.HISQ_F32])
def test_noalloc_dot_matches_dot_on_two_calls(prec):
    dims = (8, 6, 4, 10)
    lat = hisq.Lattice(dims, 0)  # fresh context: no workspace allocated yet
    dt = torch.complex128 if prec == hisq.HISQ_F64 else torch.complex64
    cases = [(9, 150, 151), (4, 152, 153)]  # second call: fewer rhs, other vectors
    ins = [(torch.from_numpy(synth.sources(dims, n, sa)).to(DEV).to(dt),
            torch.from_numpy(synth.sources(dims, n, sb)).to(DEV).to(dt)) for n, sa, sb in cases]
    outs = [torch.full((2 * n,), float("nan"), dtype=torch.float64, device=DEV) for n, _, _ in cases]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]  # every buffer of the test exists before the calls
    got = []
    for (n, _, _), (a, b), d in zip(cases, ins, outs):
        got.append(_call(lat, prec, n, a, b, d))
        torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0  # nothing was allocated on the device
    for (n, _, _), (a, b), g in zip(cases, ins, got):
        ref = lat.dot(prec, a, b)  # the allocating entry point, same kernels
        assert torch.equal(g.view(-1, 2)[:, 0], ref.real) and torch.equal(g.view(-1, 2)[:, 1], ref.imag)
        a2, b2 = a.cpu().numpy().astype(np.complex128), b.cpu().numpy().astype(np.complex128)
        exact = np.array([np.vdot(a2[i], b2[i]) for i in range(n)])
        gc = g.cpu().numpy().view(np.complex128)
        assert np.max(np.abs(gc - exact)) <= 1e-12 * np.max(np.abs(exact))
        print(f"prec {prec} n {n}: bit-identical to hisq_dot_mrhs")
    lat.close()


def test_noalloc_dot_refuses_sizes_beyond_its_buffer():
    """64 rhs on 64^3 x 24 sites need 2 * 64 * 9216 partials, above the 2^20 of the static buffer:
    refused before anything is launched (the pointers are never read)."""
    lat = hisq.Lattice((64, 64, 64, 24), 0)
    x = torch.zeros(2, dtype=torch.complex64, device=DEV)
    dots = torch.zeros(128, dtype=torch.float64, device=DEV)
    rc = hisq.library().hisq_dot_mrhs_noalloc(lat.ctx, hisq.HISQ_F32, 64, hisq._ptr(x), hisq._ptr(x), hisq._ptr(dots))
    assert rc == hisq.HISQ_ERR_ARG
    assert "static buffer" in hisq.hisq_last_error(lat.ctx)
    lat.close()
