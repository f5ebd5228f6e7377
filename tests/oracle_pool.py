"""Oracle evaluations spread over host processes (test infrastructure).

The network oracle runs one sample at a time in numpy; at batch 16 on a lattice of many
workgroups it takes minutes on one core.  The samples are independent, so the tests evaluate
them in a pool of fresh interpreter processes ("spawn": the workers import numpy, synth and
oracle only, never the GPU library or torch).  Each worker regenerates the links from their
seed once.
"""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

_W = {}


def _init(dims, seed):
    import synth
    _W["dims"] = tuple(dims)
    _W["links"] = synth.gauge_links(tuple(dims), seed)


def _nn_task(job):
    from oracle import nn as onn
    kind, theta, r, y, channels, layers, mass = job
    fat, naik = _W["links"]
    dims = _W["dims"]
    if kind == "forward":
        return onn.forward(theta, fat, r, dims, channels, layers)
    if kind == "gram":
        return onn.apply(theta, fat, r, dims, channels, layers, "gram")
    if kind == "grad_direct":
        return onn.loss_and_grad(theta, fat, r[None], y[None], dims, channels, layers, kind="residual",
                                 naik=naik, mass=mass)
    if kind == "grad_gram":
        return onn.gram_loss_and_grad(theta, fat, r[None], y[None], dims, channels, layers,
                                      kind="residual", naik=naik, mass=mass)
    raise ValueError(kind)


def workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def network_reference(dims, seed, theta, rs, ys, channels, layers, mass):
    """Per-sample oracle forward and Gram outputs, and the batch loss and Wirtinger gradient
    (mean over the pairs) of the residual-norm loss in both forms."""
    nb = len(rs)
    jobs = [(k, theta, rs[j], ys[j], channels, layers, mass)
            for k in ("grad_gram", "grad_direct", "gram", "forward") for j in range(nb)]
    ctx = mp.get_context("spawn")
    with ProcessPoolExecutor(max_workers=workers(), mp_context=ctx, initializer=_init,
                             initargs=(tuple(dims), seed)) as ex:
        res = list(ex.map(_nn_task, jobs))
    gg, gd, gram, fwd = (res[i * nb:(i + 1) * nb] for i in range(4))
    out = {"forward": np.stack(fwd), "gram": np.stack(gram)}
    for name, part in (("grad_direct", gd), ("grad_gram", gg)):
        out[name] = (float(np.mean([p[0] for p in part])), np.mean([p[1] for p in part], axis=0))
    return out
