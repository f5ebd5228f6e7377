"""Shared helpers of the GPU parity tests (inputs from synth, expected values from oracle)."""
import numpy as np

import synth

DEV = "cuda:0"


ELEM_FLOOR = 1e-2


def rel_elem(got, ref, floor=ELEM_FLOOR):
    """max_i |got_i - ref_i| / max(|ref_i|, floor * rms(ref)): per-element relative error.

    An output element is a sum of 16 hop terms of typical size rms(ref); its rounding error is
    set by the size of those terms, not by the element itself.  An element that cancels to below
    1 % of the typical size is therefore measured against 1 % of rms(ref): the FP64 oracle itself
    reaches ~2e-14 against an 80-bit evaluation with that floor, but ~1.3e-13 with a 0.1 % floor
    (8 x 6 x 4 x 10 lattice, 5 rhs), so a tighter floor would demand more than FP64 delivers."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), floor * rms)))


def check_f64_elem(got, ref, label, tol=1e-13):
    """Assert the FP64 per-element bound and print the measured error."""
    err = rel_elem(got, ref)
    print(f"{label}: FP64 per-element error {err:.3g} (bound {tol:g})")
    assert err <= tol
    return err


def rel_l2(got, ref):
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


_LINK_CACHE = {}


def links(dims, seed, eps=0.4):
    key = (tuple(dims), seed, eps)
    if key not in _LINK_CACHE:
        _LINK_CACHE.clear()
        _LINK_CACHE[key] = synth.gauge_links(dims, seed, eps=eps)
    return _LINK_CACHE[key]


def make_lattice(dims, seed, copies=7, recon=18, eps=0.4):
    from paper_1409_1510_amd import hisq
    fat, naik = links(dims, seed, eps)
    lat = hisq.Lattice(dims, 0)
    lat.load_links(fat, naik, copies, recon)
    return lat, fat, naik
