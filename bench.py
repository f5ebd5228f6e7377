"""Benchmark of the multi-rhs HISQ Dslash and the even-odd CG solvers on one MI355X.

Workload (default): the 32^3 x 8 lattice with 16 complex Gaussian right-hand sides, FP32 Dslash
(FP32 links, complex64 vectors), seeded synthetic links (exp(i 0.4 H) + 0.05 G fat links, -1/24
Haar SU(3) Naik links).  One step = one full-lattice multi-rhs Dslash w = D v for the bundle:
the two half Dslash launches D_oe (even -> odd) and D_eo (odd -> even).
value = Gflop/s under the 1146 flop per site per rhs convention (Section 1, Table 1 model).
The timed steps follow RAMP_MS of untimed back-to-back steps and then the warmup steps: the
device needs ~30 ms of load to reach its sustained speed for this kernel.

Also reported on the same JSON line:
  roofline       : compulsory HBM bytes per half-Dslash launch / mean launch duration (HIP events
                   at the ends of the timed region on the launch stream, over its launches),
                   against 8 TB/s; the GPU clocks rocm-smi reports under the same load;
  dslash_sweep   : n = 1, 2, 4, 8, 16 in FP64, FP32 (Naik in 18, 14, 13, 9 reals), FP16 links
                   (Naik in 18, 14, 9 reals);
  volume_sweep   : the FP32 half Dslash against the lattice volume;
  cg             : seconds per rhs to a true FP64 residual 1e-8 at 32^3 x 8, m = 0.02, 8 rhs, for
                   the mixed-precision solver (FP16 and FP32 links) and the plain FP64 solver;
  trace_minv     : Tr M^-1 on the same lattice from 64 Z2 noise vectors (Eq. 2), with its error,
                   and the chiral condensate (1/V) Tr (m + D)^-1 from 16 of them;
  cg_48x48x48x12 : seconds per rhs to 1e-8 at 48^3 x 12, m = 0.01, 16 Z2 rhs: plain FP64, mixed
                   (FP16 and FP32 links) and the flexible CG with the learned preconditioner,
                   trained here on pairs harvested from plain CG, with iterations and peak memory;
  cpu_baseline   : the FP64 numpy oracle on the host's cores (a process per core): the same
                   whole-lattice Dslash per rhs, and the oracle CG (8^4 in full, 32^3 x 8 per rhs
                   extrapolated from a timed sample).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cg] [--no-c3] [--no-cpu] [--no-sweep]
       python bench.py --workload c3|c4 [--nn-variants gram:4,gram:2,...]   (solver study alone)
       python bench.py --profile [--profile-dims ..] [--profile-prec ..] | --profile-sweep |
                       --profile-nn | --profile-cg            (short runs for rocprofv3)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "k_dslash_f32_n16_32x32x32x8.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1409_1510_amd", "csrc", f)
                  for f in ("dslash_kernel.hpp", "dslash.hip", "dslash_f32.hip")]


def gpu_clocks():
    """Current GPU clocks as rocm-smi reports them (None if it cannot be read)."""
    import subprocess
    try:
        res = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True,
                             timeout=30)
        card = next(iter(json.loads(res.stdout).values()))
        return {k.strip(" :"): v for k, v in card.items() if "clock speed" in k}
    except Exception:  # reporting only: a missing tool or format leaves the field empty
        return None


def gpu_clocks_under(torch, step):
    """gpu_clocks() sampled while step() runs back to back (the clocks drop when the device idles)."""
    import threading
    res = {}
    th = threading.Thread(target=lambda: res.update(c=gpu_clocks()))
    th.start()
    t = time.perf_counter()
    while th.is_alive() and time.perf_counter() - t < 30.0:
        for _ in range(10):
            step()
        torch.cuda.synchronize()
    th.join()
    return res.get("c")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def shipped_launch(hisq, dims, prec, recon, n, fused):
    """The launch configuration the shipped tuning table holds for a case, or None."""
    if not os.path.exists(hisq.TUNING_PATH):
        return None
    key = [*dims, prec, recon, n, fused]
    for line in open(hisq.TUNING_PATH):
        f = line.split()
        if f and not f[0].startswith("#") and [int(v) for v in f[:8]] == key:
            return tuple(int(v) for v in f[8:13])
    return None


def measured_traffic(config_tuple):
    """HBM bytes per launch from the committed rocprofv3 counter summary (FETCH_SIZE and
    WRITE_SIZE, each scaled by the same counter's reading for a copy kernel of known size), if the
    summary was taken on the current kernel source and the same launch configuration."""
    if not os.path.exists(PROFILE_SUMMARY):
        return None
    fields = {}
    for line in open(PROFILE_SUMMARY):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if fields.get("launch_config") != str(tuple(config_tuple)):
        return None
    try:
        return int(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def chained_launch_ms(lat, hisq, torch, prec, v_e, w_o, w_e, steps=10):
    """Mean launch time of `steps` pairs D_oe (w_e -> w_o), D_eo (w_o -> w_e), each launch reading
    what the one before wrote, timed with HIP events on the launch stream.  The start is v_e
    scaled by 1e-25: D grows a vector by at most ~9 per application, so the 2 (steps + 2)
    launches stay within normal FP32 numbers."""
    w_e.copy_(v_e)
    w_e.mul_(1e-25)
    for _ in range(2):
        lat.dslash(1, prec, w_e, w_o)
        lat.dslash(0, prec, w_o, w_e)
    torch.cuda.synchronize()
    t0, t1 = _events(torch)
    t0.record()
    for _ in range(steps):
        lat.dslash(1, prec, w_e, w_o)
        lat.dslash(0, prec, w_o, w_e)
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / (2 * steps)


SWEEP_N = (1, 2, 4, 8, 16)


def sweep_cases(hisq):
    """(precision, Naik format, label) of the n/precision sweep."""
    return ((hisq.HISQ_F64, 18, "f64"), (hisq.HISQ_F32, 18, "f32"), (hisq.HISQ_F32, 14, "f32_r14"),
            (hisq.HISQ_F32, 13, "f32_r13"), (hisq.HISQ_F32, 9, "f32_r9"),
            (hisq.HISQ_F16, 18, "f16links"), (hisq.HISQ_F16, 14, "f16links_r14"),
            (hisq.HISQ_F16, 9, "f16links_r9"))


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


# Untimed sustained load before a measurement: under load the device takes some 30 ms to reach
# its sustained speed for this kernel, and falls back within half a second of idling (measured:
# 91-95 us per FP32 n = 16 launch at the start of a fresh process, 78 us after ~30 ms of
# back-to-back steps, 95 us again after a 0.5 s pause; a plain copy runs at the same speed
# throughout).  A CG solve runs loaded for far longer than that.
RAMP_MS = 100.0
SWEEP_RAMP_MS = 50.0


def sustain(torch, step, ms):
    """Run step() back to back, untimed, for at least `ms` milliseconds; returns the steps run."""
    t = time.perf_counter()
    k = 0
    while (time.perf_counter() - t) * 1e3 < ms:
        for _ in range(10):
            step()
        torch.cuda.synchronize()
        k += 10
    return k


def dslash_step(lat, prec, v_e, v_o, w_e, w_o):
    """One full Dslash step of the benchmark as a callable: D_oe (v_e -> w_o), D_eo (v_o -> w_e)."""
    def step():
        lat.dslash(1, prec, v_e, w_o)
        lat.dslash(0, prec, v_o, w_e)
    return step


def dslash_step_timing(lat, hisq, torch, prec, v_e, v_o, w_e, w_o, steps, warmup, isolated=True):
    """Time `steps` full Dslash applications (D_oe then D_eo) issued back to back, with one pair
    of HIP events on the launch stream at the ends of the timed region: ms per step, and the
    average launch duration as the region over its 2 * steps launches (launch gaps included).
    With `isolated`, a second, separate pass brackets every launch with its own event pair; a
    marker between kernels costs a few microseconds each, so that figure (the mean of the
    bracketed launches) is reported beside the other, not used for it."""
    for _ in range(warmup):
        lat.dslash(1, prec, v_e, w_o)
        lat.dslash(0, prec, v_o, w_e)
    torch.cuda.synchronize()
    t0, t1 = _events(torch)
    t0.record()
    for _ in range(steps):
        lat.dslash(1, prec, v_e, w_o)
        lat.dslash(0, prec, v_o, w_e)
    t1.record()
    torch.cuda.synchronize()
    ms_step = t0.elapsed_time(t1) / steps
    ms_iso = None
    if isolated:
        ev = [_events(torch) for _ in range(2 * steps)]
        for k in range(steps):
            ev[2 * k][0].record()
            lat.dslash(1, prec, v_e, w_o)
            ev[2 * k][1].record()
            ev[2 * k + 1][0].record()
            lat.dslash(0, prec, v_o, w_e)
            ev[2 * k + 1][1].record()
        torch.cuda.synchronize()
        ms_iso = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    return ms_step, ms_step / 2, ms_iso


# per-study settings: rhs of the FCG solve, training sources x snapshots (every `snap` plain-CG
# iterations, harvest tolerance), epochs, and whether the plain FP64 solve runs
STUDY = {
    # 48^3 x 12: 40 epochs, as the residual loss is still falling at 20 (0.16 there, 0.11 at 40
    # for the workload's seed, which took the flexible CG from 2720 to 1968 iterations)
    "c3": dict(n_fcg=None, nsrc=16, nsnap=16, snap=60, harvest_tol=1e-8, epochs=40, plain=True),
    # 64^3 x 16: the network and its training scale with 16 x the vector volume, so the learned
    # solve runs on 2 of the 32 rhs with 64 training pairs; the plain FP64 solve is left out
    "c4": dict(n_fcg=2, nsrc=8, nsnap=8, snap=100, harvest_tol=1e-6, epochs=20, plain=False),
}


def solver_study(name, torch, synth, hisq, pm, epochs=0, fcg_link_precs=None, variants=None,
                 plain=None, progress_tag=None, nn_seeds=None):
    """48^3x12 (16 Z2 rhs, m = 0.01) or 64^3x16 (32 Gaussian rhs, m = 0.005): CG seconds per rhs
    to a true FP64 residual 1e-8 for mixed precision (FP16 and FP32 links), plain FP64 (48^3x12)
    and the flexible CG with the learned preconditioner (trained here on pairs harvested from plain
    CG on the same links), with iterations, peak device memory, the Dslash Gflop/s inside each
    solve and the cost of one network application.  `variants`: (form, layers) of the networks to
    train and solve with (default: the Gram form with 4 layers); `fcg_link_precs`: the link copies
    the flexible CG's inner operator is run with (the faster is its result); `nn_seeds`: seeds of
    the networks' initial weights and training batches, each variant trained once per seed
    (default: the workload's seed)."""
    import ctypes
    st = STUDY[name]
    cfg = synth.WORKLOADS[name]
    dims, n, mass, tol = cfg["dims"], cfg["n"], cfg["mass"], cfg["tol"]
    seed = synth.workload_seed(name)
    fcg_link_precs = fcg_link_precs or (hisq.HISQ_F16, hisq.HISQ_F32)
    variants = variants or [("gram", 4)]
    plain = st["plain"] if plain is None else plain
    t0 = time.perf_counter()
    fat, naik = synth.gauge_links(dims, seed, eps=cfg["eps"])
    t_gen = time.perf_counter() - t0
    lat = hisq.Lattice(dims, 0)
    lat.load_links(fat, naik, hisq.HISQ_LINKS_ALL, 18)
    del fat, naik
    dev = "cuda:0"
    b = torch.from_numpy(synth.sources(dims, n, seed + 1, cfg["source"])).to(dev)
    out = {"workload": f"{'x'.join(map(str, dims))}, m={mass}, {n} {cfg['source']} rhs, tol {tol}",
           "link_generation_s": round(t_gen, 1)}
    lib = hisq.library()
    epochs = epochs or st["epochs"]
    tag = progress_tag or name

    def progress(msg):
        print(f"[{tag}] {msg}", file=sys.stderr, flush=True)

    def solve(label, rhs, max_iter=60000, **kw):
        progress(f"solve {label}")
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, info = lat.cg(mass, rhs, tol=tol, max_iter=max_iter, **kw)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        nr = rhs.shape[0]
        res = {"n_rhs": nr, "s_per_rhs": round(sec / nr, 5), "seconds": round(sec, 3),
               "iters_mean": round(float(np.mean(info["iters"])), 1),
               "iters_max": max(info["iters"]), "true_resid_max": max(info["true_resid"]),
               "converged": sum(info["converged"]), "fell_back": sum(info["fell_back"]),
               "reliable_updates": info["reliable_updates"], "compactions": info["compactions"],
               "rc": info["rc"],
               "peak_device_GB": round(info["peak_bytes"] / 1e9, 2),
               "fp32_links_from_iter": info["link_switch_iter"],
               "dslash_gflops": round(pm.FLOP_PER_SITE_RHS * info["dslash_site_rhs"] / sec / 1e9, 1)}
        progress(f"  {label}: {res['s_per_rhs']} s/rhs, {res['iters_max']} iterations")
        return res

    out["mixed_f16links"] = solve("mixed_f16links", b, kind=hisq.HISQ_CG_MIXED, link_prec=hisq.HISQ_F16)
    out["mixed_f32links"] = solve("mixed_f32links", b, kind=hisq.HISQ_CG_MIXED, link_prec=hisq.HISQ_F32)
    if plain:
        out["plain_f64"] = solve("plain_f64", b, kind=hisq.HISQ_CG_F64)
    best = min(("mixed_f16links", hisq.HISQ_F16), ("mixed_f32links", hisq.HISQ_F32),
               key=lambda kv: out[kv[0]]["seconds"])
    out["mixed_best"] = best[0]
    if plain:
        out["speedup_mixed_vs_f64"] = round(out["plain_f64"]["seconds"] / out[best[0]]["seconds"], 3)
    # training pairs along plain-CG trajectories of Gaussian sources
    nsrc, nsnap = st["nsrc"], st["nsnap"]
    bs = torch.from_numpy(synth.sources(dims, nsrc, seed + 2)).to(dev)
    r = torch.empty((nsnap * nsrc, 3, lat.vh), dtype=torch.complex128, device=dev)
    y = torch.empty_like(r)
    npairs = ctypes.c_int()
    progress("harvest training pairs")
    torch.cuda.synchronize()
    t = time.perf_counter()
    hisq._check(lat.ctx, lib.hisq_nn_harvest(lat.ctx, mass, nsrc, hisq._ptr(bs), st["harvest_tol"], nsnap,
                                             st["snap"], hisq._ptr(r), hisq._ptr(y), ctypes.byref(npairs)))
    out["harvest"] = {"pairs": npairs.value, "sources": nsrc, "snapshot_every": st["snap"],
                      "seconds": round(time.perf_counter() - t, 2)}
    del bs
    # the best multiple of the identity for the residual loss on the training residuals,
    # c = sum <r, M r> / sum ||M r||^2: the networks start there (P = c N for the direct form,
    # c N^dag N for the Gram form, whose output scales as |W_out|^2)
    r32 = r[: min(16, npairs.value)].to(torch.complex64)
    mr = lat.apply_m(hisq.HISQ_F32, mass, r32)
    c = float(torch.sum((torch.conj(r32) * mr).real) / torch.sum(torch.abs(mr) ** 2))
    del r32, mr
    bf = b if st["n_fcg"] is None else b[:st["n_fcg"]].contiguous()
    nf = bf.shape[0]
    ref_label = best[0] if nf == n else best[0] + "_fcg_bundle"
    if nf != n:
        out[ref_label] = solve(ref_label, bf, kind=hisq.HISQ_CG_MIXED, link_prec=best[1])
    out["learned"] = {}
    runs = [(form, layers, s) for s in (nn_seeds or [None]) for form, layers in variants]
    first_key = None
    for form, layers, nn_seed in runs:
        key = f"{form}_L{layers}" + ("" if nn_seed is None else f"_seed{nn_seed}")
        first_key = first_key or key
        tseed = seed if nn_seed is None else nn_seed
        hisq._check(lat.ctx, lib.hisq_nn_init(lat.ctx, layers, 8, tseed))
        hisq._check(lat.ctx, lib.hisq_nn_set_form(lat.ctx, hisq.HISQ_NN_FORM_GRAM if form == "gram"
                                                  else hisq.HISQ_NN_FORM_DIRECT))
        hisq._check(lat.ctx, lib.hisq_nn_set_loss(lat.ctx, hisq.HISQ_NN_LOSS_RESIDUAL, mass))
        nparam = lib.hisq_nn_num_params(lat.ctx)
        w = (ctypes.c_double * (2 * nparam))()
        hisq._check(lat.ctx, lib.hisq_nn_get_params(lat.ctx, w, 2 * nparam))
        scale = c ** 0.5 if form == "gram" else c
        for k in range(2 * (nparam - 8), 2 * nparam):
            w[k] *= scale
        hisq._check(lat.ctx, lib.hisq_nn_set_params(lat.ctx, w, 2 * nparam))
        hist = (ctypes.c_double * epochs)()
        batch, lr = 16, 1e-2
        progress(f"train the network {key}")
        t = time.perf_counter()
        hisq._check(lat.ctx, lib.hisq_nn_train(lat.ctx, npairs.value, hisq._ptr(r), hisq._ptr(y),
                                               epochs, batch, lr, tseed, hist))
        v = {"form": form, "layers": layers, "seed": tseed, "channels": 8, "loss": "residual",
             "init_scale": round(c, 5),
             "epochs": epochs, "batch": batch, "lr": lr, "bf16": True,
             "training_s": round(time.perf_counter() - t, 2),
             "loss_first": round(hist[0], 5), "loss_last": round(hist[epochs - 1], 5)}
        # one preconditioner application on the FCG bundle (FP32 vectors), as inside the FCG
        rv = bf.to(torch.complex64)
        zv = torch.empty_like(rv)
        for _ in range(2):
            hisq._check(lat.ctx, lib.hisq_nn_apply(lat.ctx, nf, hisq.HISQ_F32, hisq._ptr(rv), hisq._ptr(zv)))
        e0, e1 = _events(torch)
        e0.record()
        for _ in range(5):
            hisq._check(lat.ctx, lib.hisq_nn_apply(lat.ctx, nf, hisq.HISQ_F32, hisq._ptr(rv), hisq._ptr(zv)))
        e1.record()
        torch.cuda.synchronize()
        v["apply_ms"] = round(e0.elapsed_time(e1) / 5, 3)
        del rv, zv
        # a network whose flexible CG needs more than 1.5 x the mixed solver's iterations has lost
        # (and a non-Hermitian direct-form network may converge slowly): the solve stops there and
        # reports how far it got
        cap = int(1.5 * out[ref_label]["iters_max"]) if len(runs) > 1 else 60000
        for lp in fcg_link_precs:
            lab = "f16links" if lp == hisq.HISQ_F16 else "f32links"
            v["fcg_" + lab] = solve(f"fcg_{key}_{lab}", bf, max_iter=cap, kind=hisq.HISQ_FCG_NN, link_prec=lp)
        fbest = min((k for k in v if k.startswith("fcg_")), key=lambda k: v[k]["seconds"])
        v["fcg_best"] = fbest
        v["speedup_vs_mixed"] = round(out[ref_label]["seconds"] / v[fbest]["seconds"], 3)
        v["iteration_ratio_vs_mixed"] = round(v[fbest]["iters_mean"] / out[ref_label]["iters_mean"], 3)
        out["learned"][key] = v
    lead = out["learned"][first_key]
    out["fcg_learned"] = dict(lead[lead["fcg_best"]], network=first_key, link_copy=lead["fcg_best"][4:])
    out["fcg_reference"] = ref_label
    out["speedup_fcg_vs_mixed"] = lead["speedup_vs_mixed"]
    out["iteration_ratio_fcg_vs_mixed"] = lead["iteration_ratio_vs_mixed"]
    lat.close()
    return out


def volume_sweep(hisq, torch, synth, pm):
    """Half-Dslash time against the lattice volume (the paper reads its performance against the
    lattice size at 4 rhs, Section 4), with 64^3 x 16 as the case no cache level holds: FP32 at
    n = 4 and 16 on every lattice, FP16 links at n = 8 and 32 on 64^3 x 16."""
    out = []
    for dims in ((16, 16, 16, 16), (24, 24, 24, 24), (32, 32, 32, 8), (48, 48, 48, 12), (64, 64, 64, 16)):
        fat, naik = synth.tiled_gauge_links(dims, 7)
        lat = hisq.Lattice(dims, 0)
        lat.load_links(fat, naik, hisq.HISQ_LINKS_F32 | hisq.HISQ_LINKS_F16, 18)
        del fat, naik
        cases = [(hisq.HISQ_F32, 4), (hisq.HISQ_F32, 16)]
        if dims == (64, 64, 64, 16):
            cases += [(hisq.HISQ_F16, 8), (hisq.HISQ_F16, 32)]
        for prec, nn in cases:
            a = torch.randn(nn, 3, lat.vh, dtype=torch.complex64, device="cuda:0")
            b = torch.randn(nn, 3, lat.vh, dtype=torch.complex64, device="cuda:0")
            c, d = torch.empty_like(a), torch.empty_like(b)
            sustain(torch, dslash_step(lat, prec, a, b, c, d), SWEEP_RAMP_MS)
            _, ml, _ = dslash_step_timing(lat, hisq, torch, prec, a, b, c, d, 10, 3, isolated=False)
            byt = pm.half_dslash_bytes(lat.vh, nn, prec, 18)
            out.append({"lattice": "x".join(map(str, dims)), "prec": "f32" if prec == hisq.HISQ_F32 else "f16links",
                        "n": nn, "ms_per_launch": round(ml, 5),
                        "gflops": round(pm.half_dslash_flops(lat.vh, nn) / (ml * 1e-3) / 1e9, 1),
                        "compulsory_GBps": round(byt / (ml * 1e-3) / 1e9, 1),
                        "launch": list(hisq.hisq_get_launch(lat.ctx, prec, nn, 0))})
            del a, b, c, d
        lat.close()
    return out


# ---- CPU baseline: the FP64 oracle on the host's cores ----------------------------------------

def _host_cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    # one GPU's share of a shared host is 16 CPUs on the machines this runs on, whatever the
    # affinity mask reports
    return max(1, min(16, n))


_CPU = {}


def _cpu_init(dims, seed, nrhs):
    # workers: numpy only, one thread each (the pool supplies the parallelism)
    import synth
    _CPU["dims"] = tuple(dims)
    _CPU["links"] = synth.gauge_links(tuple(dims), seed)
    _CPU["v"] = synth.sources(tuple(dims), nrhs, seed + 1)


def _cpu_dslash(job):
    """Whole-lattice Eq. 3 for rhs i, `reps` times; returns the seconds taken."""
    import oracle
    i, reps = job
    fat, naik = _CPU["links"]
    dims = _CPU["dims"]
    full = oracle.embed(_CPU["v"][i], dims, 0) + oracle.embed(_CPU["v"][(i + 1) % len(_CPU["v"])], dims, 1)
    t = time.perf_counter()
    for _ in range(reps):
        oracle.dslash_full(fat, naik, full, dims)
    return time.perf_counter() - t


def _cpu_cg(job):
    """Oracle CG on one rhs: (iterations, seconds, true residual)."""
    import oracle
    i, mass, tol, max_iter = job
    fat, naik = _CPU["links"]
    dims = _CPU["dims"]
    t = time.perf_counter()
    x, it, res = oracle.cg(fat, naik, _CPU["v"][i:i + 1], dims, mass, tol, max_iter=max_iter, max_restarts=0)
    return int(it[0]), time.perf_counter() - t, float(res[0])


def cpu_baseline(dims, nrhs, gpu_cg_iters, gpu_c3_iters=None):
    """The FP64 numpy oracle timed on the host's cores (a process per core, one thread each):
    the whole-lattice Dslash of the benchmark step (Eq. 3 on both parities, 1146 flop per site and
    rhs) over the benchmark's rhs, the oracle CG on the 8^4 workload solved in full, and the
    oracle CG on the 32^3 x 8 and 48^3 x 12 workloads per rhs, extrapolated from a timed sample
    of iterations to the iteration count of the GPU's plain FP64 solve."""
    import multiprocessing as mp
    import platform
    from concurrent.futures import ProcessPoolExecutor

    import synth
    from paper_1409_1510_amd import perfmodel as pm
    cores = _host_cores()
    env_threads = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env_threads:
        os.environ[k] = "1"
    ctx = mp.get_context("spawn")
    out = {"kind": "oracle", "cores": cores}
    try:
        # 1. whole-lattice Dslash, every worker on its own rhs, ~12 s of wall time
        c1 = synth.WORKLOADS["c1"]
        with ProcessPoolExecutor(cores, mp_context=ctx, initializer=_cpu_init,
                                 initargs=(dims, synth.workload_seed("c1"), nrhs)) as ex:
            probe = list(ex.map(_cpu_dslash, [(i, 1) for i in range(cores)]))
            per = float(np.median(probe))
            reps = max(1, int(12.0 / per))
            t = time.perf_counter()
            secs = list(ex.map(_cpu_dslash, [(i % nrhs, reps) for i in range(cores)]))
            wall = time.perf_counter() - t
        flops = cores * reps * pm.half_dslash_flops(int(np.prod(dims)) // 2, 1) * 2
        out["value"] = round(flops / wall / 1e9, 3)
        out["unit"] = "Gflop/s"
        out["sample"] = (f"{cores * reps} whole-lattice FP64 oracle Dslash applications (Eq. 3 on both "
                         f"parities, 1 rhs each, rhs of the {'x'.join(map(str, dims))} benchmark bundle) "
                         f"in {cores} processes of one thread, {wall:.1f} s wall; the same work unit as "
                         f"one benchmark step per rhs")
        out["dslash_s_per_rhs"] = round(float(np.median(secs)) / reps, 4)
        # 2. oracle CG: 8^4 solved in full; 32^3 x 8 sampled per rhs
        c0, c2, c3 = synth.WORKLOADS["c0"], synth.WORKLOADS["c2"], synth.WORKLOADS["c3"]
        with ProcessPoolExecutor(1, mp_context=ctx, initializer=_cpu_init,
                                 initargs=(c0["dims"], synth.workload_seed("c0"), 1)) as ex0, \
                ProcessPoolExecutor(2, mp_context=ctx, initializer=_cpu_init,
                                    initargs=(c2["dims"], synth.workload_seed("c2"), 2)) as ex2, \
                ProcessPoolExecutor(1, mp_context=ctx, initializer=_cpu_init,
                                    initargs=(c3["dims"], synth.workload_seed("c3"), 1)) as ex3:
            f0 = ex0.submit(_cpu_cg, (0, c0["mass"], c0["tol"], 100000))
            k, k3 = 8, 2
            f2 = [ex2.submit(_cpu_cg, (i, c2["mass"], c2["tol"], k)) for i in range(2)]
            f3 = ex3.submit(_cpu_cg, (0, c3["mass"], c3["tol"], k3))
            it0, s0, r0 = f0.result()
            samples = [f.result() for f in f2]
            sample3 = f3.result()
        out["cg_8x8x8x8"] = {"iters": it0, "seconds": round(s0, 3), "true_resid": r0, "tol": c0["tol"],
                             "mass": c0["mass"], "s_per_rhs": round(s0, 3)}
        # k iterations plus the initial and the final residual: k + 2 applications of M
        s_it = float(np.mean([s for _, s, _ in samples])) / (k + 2)
        c2_out = {"sample": f"{k} CG iterations on each of 2 rhs (one process each), plus the initial "
                            "and final residual: s per iteration = time / (k + 2)",
                  "s_per_iteration": round(s_it, 4), "mass": c2["mass"], "tol": c2["tol"]}
        if gpu_cg_iters:
            c2_out["gpu_plain_f64_iterations"] = gpu_cg_iters
            c2_out["s_per_rhs_extrapolated"] = round(s_it * gpu_cg_iters, 1)
        out["cg_32x32x32x8_per_rhs"] = c2_out
        s_it3 = sample3[1] / (k3 + 2)
        c3_out = {"sample": f"{k3} CG iterations on 1 rhs (one process), plus the initial and final "
                            "residual: s per iteration = time / (k + 2)",
                  "s_per_iteration": round(s_it3, 4), "mass": c3["mass"], "tol": c3["tol"]}
        if gpu_c3_iters:
            c3_out["gpu_plain_f64_iterations"] = gpu_c3_iters
            c3_out["s_per_rhs_extrapolated"] = round(s_it3 * gpu_c3_iters, 1)
        out["cg_48x48x48x12_per_rhs"] = c3_out
        out["host"] = {"cores_used": cores, "os_cpu_count": os.cpu_count(), "machine": platform.machine(),
                       "cpu_model": _cpu_model()}
    finally:
        for k, v in env_threads.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return out


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--nrhs", type=int, default=16)
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--workload", default="c1", choices=["c1", "c3", "c4"],
                    help="c1: Dslash throughput at 32^3x8 (default, the timed steps); c3/c4: the "
                         "solver comparison at 48^3x12 / 64^3x16 (plain FP64, mixed, learned FCG)")
    ap.add_argument("--epochs", type=int, default=0,
                    help="training epochs of the solver study (0: 20)")
    ap.add_argument("--fcg-links", default="both", choices=["both", "f32", "f16"],
                    help="--workload c3|c4: the link copies the flexible CG's inner operator runs with")
    ap.add_argument("--nn-variants", default="",
                    help="solver study: networks to train and solve with, as form:layers pairs, e.g. "
                         "gram:4,gram:2,direct:4 (default gram:4)")
    ap.add_argument("--nn-seeds", default="",
                    help="--workload c3|c4: train each network once per seed (comma-separated) to see "
                         "how the learned preconditioner varies with its initial weights and batches")
    ap.add_argument("--no-c3", action="store_true",
                    help="leave out the 48^3x12 solver comparison of the default run")
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: one 256 MiB read + 256 MiB write elementwise "
                         "kernel (counter calibration), 100 ms of untimed steps with another "
                         "rhs_per_thread, then --steps FP32 Dslash steps")
    ap.add_argument("--profile-dims", default="32,32,32,8",
                    help="--profile: lattice extents (other than 32,32,32,8: tiled links, which the "
                         "timing does not depend on)")
    ap.add_argument("--profile-prec", default="f32", choices=["f32", "f16links"],
                    help="--profile: FP32 links or FP16 link storage (FP32 vectors either way)")
    ap.add_argument("--profile-launch", default="",
                    help="--profile: launch configuration rt,spb,nt,lds,xm to time (default: the "
                         "shipped table's entry for the case, else the autotuner's choice), so that "
                         "separate counter runs profile the same launch")
    ap.add_argument("--profile-sweep", action="store_true",
                    help="short run for rocprofv3: the counter-calibration kernel, then for every "
                         "case of the n/precision sweep 50 ms of untimed steps, 1 warm-up step and "
                         "3 steps")
    ap.add_argument("--profile-nn", action="store_true",
                    help="only the learned preconditioner's Gram application at 48^3x12 on 16 rhs, "
                         "2 + --steps times (for a rocprofv3 run)")
    ap.add_argument("--profile-cg-workload", default="c2", choices=["c2", "c3", "c4"],
                    help="--profile-cg: the 32^3x8 CG to convergence (c2), or --steps iterations of "
                         "the 48^3x12 mixed CG on 16 rhs (c3) or the 64^3x16 one on 32 rhs (c4)")
    ap.add_argument("--cg-naik-recon", type=int, default=18, choices=[18, 14, 13, 9],
                    help="reals per stored Naik link of the FP32 and FP16 copies in the 32^3x8 CG "
                         "(default run and --profile-cg)")
    ap.add_argument("--profile-cg", action="store_true",
                    help="short run for rocprofv3: the 32^3x8 mixed CG (FP16 links, 8 rhs) of the "
                         "benchmark, solved twice")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solver works on a single device (the multi-GPU "
              "design is rhs-bundle sharding, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1409_1510_amd import hisq
    from paper_1409_1510_amd import perfmodel as pm

    torch.cuda.set_device(0)
    if args.profile_cg or args.profile:
        # counter calibration for the summaries: an elementwise kernel that reads 256 MiB and
        # writes 256 MiB
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if args.profile_cg and args.profile_cg_workload in ("c3", "c4"):
        # the mixed CG's kernels where no cache level holds the vectors: 48^3 x 12 with 16 rhs or
        # 64^3 x 16 with 32 rhs, FP32 links, a fixed number of iterations (tiled links: the
        # per-kernel traffic does not depend on the link values or on convergence)
        c4 = synth.WORKLOADS[args.profile_cg_workload]
        fat4, naik4 = synth.tiled_gauge_links(c4["dims"], 7)
        lat4 = hisq.Lattice(c4["dims"], 0)
        lat4.load_links(fat4, naik4, hisq.HISQ_LINKS_ALL, 18)
        del fat4, naik4
        b = torch.randn(c4["n"], 3, lat4.vh, dtype=torch.complex128, device="cuda:0")
        for _ in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            x, info = lat4.cg(c4["mass"], b, tol=1e-12, max_iter=args.steps, kind=hisq.HISQ_CG_MIXED,
                              link_prec=hisq.HISQ_F32)
            torch.cuda.synchronize()
            print(f"profile-cg solve: {time.perf_counter() - t:.3f} s, {max(info['iters'])} iterations "
                  f"(stopped at the cap), {c4['n']} rhs", flush=True)
        lat4.close()
        return
    if args.profile_cg:
        c2 = synth.WORKLOADS["c2"]
        fat2, naik2 = synth.gauge_links(c2["dims"], synth.workload_seed("c2"), eps=c2["eps"])
        lat2 = hisq.Lattice(c2["dims"], 0)
        lat2.load_links(fat2, naik2, hisq.HISQ_LINKS_ALL, args.cg_naik_recon)
        b = torch.from_numpy(synth.sources(c2["dims"], c2["n"], synth.workload_seed("c2") + 1)).to("cuda:0")
        for _ in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            x, info = lat2.cg(c2["mass"], b, tol=c2["tol"], max_iter=40000, kind=hisq.HISQ_CG_MIXED,
                              link_prec=hisq.HISQ_F16)
            torch.cuda.synchronize()
            print(f"profile-cg solve: {time.perf_counter() - t:.3f} s, {max(info['iters'])} iterations",
                  flush=True)
        lat2.close()
        return
    if args.profile_nn:
        # the learned preconditioner's Gram application (two network passes, BF16 activations,
        # FP16 links) on 16 rhs at 48^3 x 12, as inside the flexible CG; the kernels' time does
        # not depend on the weights, so the network keeps its initial ones
        dims3 = synth.WORKLOADS["c3"]["dims"]
        fat3, naik3 = synth.tiled_gauge_links(dims3, 7)
        lat3 = hisq.Lattice(dims3, 0)
        lat3.load_links(fat3, naik3, hisq.HISQ_LINKS_F32 | hisq.HISQ_LINKS_F16, 18)
        del fat3, naik3
        lib = hisq.library()
        hisq._check(lat3.ctx, lib.hisq_nn_init(lat3.ctx, 4, 8, 5))
        hisq._check(lat3.ctx, lib.hisq_nn_set_form(lat3.ctx, hisq.HISQ_NN_FORM_GRAM))
        r = torch.randn(16, 3, lat3.vh, dtype=torch.complex64, device="cuda:0")
        z = torch.empty_like(r)
        for k in range(2 + args.steps):
            hisq._check(lat3.ctx, lib.hisq_nn_apply(lat3.ctx, 16, hisq.HISQ_F32, hisq._ptr(r), hisq._ptr(z)))
        torch.cuda.synchronize()
        print(f"profile-nn done: {2 + args.steps} Gram applications on 16 rhs, lattice {dims3}", flush=True)
        lat3.close()
        return
    if args.workload in ("c3", "c4"):
        variants = None
        if args.nn_variants:
            variants = [(f.split(":")[0], int(f.split(":")[1])) for f in args.nn_variants.split(",")]
        links = {"both": None, "f32": (hisq.HISQ_F32,), "f16": (hisq.HISQ_F16,)}[args.fcg_links]
        seeds = [int(v) for v in args.nn_seeds.split(",")] if args.nn_seeds else None
        print(json.dumps(solver_study(args.workload, torch, synth, hisq, pm, epochs=args.epochs,
                                      fcg_link_precs=links, variants=variants, nn_seeds=seeds)))
        return
    cfg = synth.WORKLOADS["c1"]
    dims, n = cfg["dims"], args.nrhs
    seed = synth.workload_seed("c1")
    fat, naik = synth.gauge_links(dims, seed, eps=cfg["eps"])
    lat = hisq.Lattice(dims, 0)
    lat.load_links(fat, naik, hisq.HISQ_LINKS_ALL, 18)
    vh = lat.vh
    v = synth.sources(dims, n, seed + 1)
    v_e = torch.from_numpy(v).to("cuda:0").to(torch.complex64)
    v_o = torch.from_numpy(synth.sources(dims, n, seed + 2)).to("cuda:0").to(torch.complex64)
    w_e = torch.empty_like(v_e)
    w_o = torch.empty_like(v_o)

    if args.profile_sweep:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)  # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        srcs = {nn: (torch.from_numpy(synth.sources(dims, nn, 9)).to("cuda:0"),
                     torch.from_numpy(synth.sources(dims, nn, 10)).to("cuda:0")) for nn in SWEEP_N}
        marker = torch.ones(64, device="cuda:0")
        for prec, recon, name in sweep_cases(hisq):
            if recon != 18:
                lat.load_links(fat, naik, hisq.HISQ_LINKS_F32 | hisq.HISQ_LINKS_F16, recon)
            for nn in SWEEP_N:
                dt = torch.complex128 if prec == hisq.HISQ_F64 else torch.complex64
                a, b = srcs[nn][0].to(dt), srcs[nn][1].to(dt)
                c, d = torch.empty_like(a), torch.empty_like(b)
                k = sustain(torch, dslash_step(lat, prec, a, b, c, d), SWEEP_RAMP_MS)
                dslash_step_timing(lat, hisq, torch, prec, a, b, c, d, 3, 1, isolated=False)
                # the trace holds, per case, any autotune trials, 2 k untimed launches, 2 warmup and
                # 6 timed launches, then a marker kernel (a negation of a small tensor) that closes
                # the case for the summary
                marker.neg_()
                torch.cuda.synchronize()
                print(f"profile-sweep case {name} n {nn} launch {hisq.hisq_get_launch(lat.ctx, prec, nn, 0)} "
                      f"ramp {k}", flush=True)
            if recon != 18:
                lat.load_links(fat, naik, hisq.HISQ_LINKS_ALL, 18)
        lat.close()
        return
    if args.profile:
        pdims = tuple(int(d) for d in args.profile_dims.split(","))
        prec = hisq.HISQ_F32 if args.profile_prec == "f32" else hisq.HISQ_F16
        if pdims != dims:
            lat.close()
            fat_p, naik_p = synth.tiled_gauge_links(pdims, 7)
            lat = hisq.Lattice(pdims, 0)
            lat.load_links(fat_p, naik_p, hisq.HISQ_LINKS_F32 | hisq.HISQ_LINKS_F16, 18)
            del fat_p, naik_p
            v_e = torch.randn(n, 3, lat.vh, dtype=torch.complex64, device="cuda:0")
            v_o = torch.randn(n, 3, lat.vh, dtype=torch.complex64, device="cuda:0")
            w_e, w_o = torch.empty_like(v_e), torch.empty_like(v_o)
        # the launch a solve on this lattice would use: the shipped table's, else the tuner's
        if args.profile_launch:
            tuned = tuple(int(v) for v in args.profile_launch.split(","))
        else:
            tuned = shipped_launch(hisq, pdims, prec, 18, n, 0)
            if tuned is None:
                hisq.hisq_autotune(lat.ctx, prec, n, 0)
                tuned = hisq.hisq_get_launch(lat.ctx, prec, n, 0)
        # the sustained load runs the same kernel with another rhs_per_thread (another kernel
        # symbol), so that the trace's statistics of the timed kernel hold the timed launches only
        hisq.hisq_set_launch(lat.ctx, prec, n, (1 if tuned[0] > 1 else 2,) + tuned[1:])
        sustain(torch, dslash_step(lat, prec, v_e, v_o, w_e, w_o), RAMP_MS)
        hisq.hisq_set_launch(lat.ctx, prec, n, tuned)
        _, ms_launch, _ = dslash_step_timing(lat, hisq, torch, prec, v_e, v_o, w_e, w_o,
                                             args.steps, 0, isolated=False)
        print(f"profile run done: {args.steps} steps, {n} rhs, lattice {pdims}, {args.profile_prec}, launch "
              f"{tuple(hisq.hisq_get_launch(lat.ctx, prec, n, 0))}, source {kernel_source_hash()}, "
              f"region-timed average {ms_launch * 1e3:.1f} us per launch, algorithmic bytes per launch "
              f"{pm.half_dslash_bytes(lat.vh, n, prec, 18)}")
        lat.close()
        return

    step = dslash_step(lat, hisq.HISQ_F32, v_e, v_o, w_e, w_o)
    # context beside the value: the same steps on a device that has been idle for 0.5 s (it takes
    # ~30 ms of load to reach its sustained speed), 1 warmup step and 10 timed steps
    torch.cuda.synchronize()
    time.sleep(0.5)
    _, ms_idle, _ = dslash_step_timing(lat, hisq, torch, hisq.HISQ_F32, v_e, v_o, w_e, w_o, 10, 1,
                                       isolated=False)
    ramp_steps = sustain(torch, step, RAMP_MS)
    ms_step, ms_launch, ms_iso = dslash_step_timing(lat, hisq, torch, hisq.HISQ_F32, v_e, v_o, w_e, w_o,
                                                    args.steps, args.warmup)
    ms_chain = chained_launch_ms(lat, hisq, torch, hisq.HISQ_F32, v_e, w_o, w_e)
    clocks = gpu_clocks_under(torch, step)
    launch_cfg = hisq.hisq_get_launch(lat.ctx, hisq.HISQ_F32, n, 0)
    flops_step = 2 * pm.half_dslash_flops(vh, n)
    gflops = flops_step / (ms_step * 1e-3) / 1e9
    bytes_launch = pm.half_dslash_bytes(vh, n, hisq.HISQ_F32)
    achieved = bytes_launch / (ms_launch * 1e-3) / 1e9
    result = {
        "metric": "multi-rhs Dslash HBM GB/s & Gflop/s; CG s/rhs to 1e-8 vs plain FP64 CG",
        "value": round(gflops, 1),
        "unit": "Gflop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"Dslash-only throughput, {'x'.join(map(str, dims))} lattice, "
                               f"{n} complex Gaussian rhs, FP32 links and vectors, full 18-real "
                               "Naik links; step = D_oe + D_eo (whole-lattice D on the bundle)",
                   "lattice": list(dims), "n_rhs": n, "flop_per_site_rhs": pm.FLOP_PER_SITE_RHS},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(launch_cfg),
                     "kernel": ("k_dslash_lds" if launch_cfg[3] else "k_dslash") + " (half Dslash, FP32)",
                     "launch_config": {"rhs_per_thread": launch_cfg[0], "sites_per_block": launch_cfg[1],
                                       "nontemporal_links": launch_cfg[2], "lds_links": launch_cfg[3],
                                       "xcd_map": launch_cfg[4]},
                     "kernel_source_sha256_16": kernel_source_hash(),
                     "bytes_per_launch": bytes_launch, "ms_per_launch": round(ms_launch, 5),
                     "ms_per_launch_event_bracketed": round(ms_iso, 5)},
        # untimed back-to-back steps before the warmup steps (the device's sustained speed)
        "sustained_load_before_warmup": {"ms": RAMP_MS, "steps": ramp_steps},
        "from_idle": {"ms_per_launch": round(ms_idle, 5),
                      "compulsory_GBps": round(bytes_launch / (ms_idle * 1e-3) / 1e9, 1),
                      "frac_of_peak": round(bytes_launch / (ms_idle * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "note": "10 steps after 0.5 s idle and 1 warmup step, before the sustained load"},
        "gpu_clocks_under_load": clocks,
        # context, not the value: the same launches with each input written by the launch before
        # (D_oe then D_eo of its result, as the CG applies M), where the input is still cached
        "dslash_chained_as_in_cg": {
            "ms_per_launch": round(ms_chain, 5),
            "compulsory_GBps": round(bytes_launch / (ms_chain * 1e-3) / 1e9, 1),
            "frac_of_peak": round(bytes_launch / (ms_chain * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
    }

    if not args.no_sweep:
        srcs = {nn: (torch.from_numpy(synth.sources(dims, nn, 9)).to("cuda:0"),
                     torch.from_numpy(synth.sources(dims, nn, 10)).to("cuda:0")) for nn in SWEEP_N}
        sweep = []
        for prec, recon, name in sweep_cases(hisq):
            if recon != 18:
                lat.load_links(fat, naik, hisq.HISQ_LINKS_F32 | hisq.HISQ_LINKS_F16, recon)
            for nn in SWEEP_N:
                dt = torch.complex128 if prec == hisq.HISQ_F64 else torch.complex64
                a, b = srcs[nn][0].to(dt), srcs[nn][1].to(dt)
                c, d = torch.empty_like(a), torch.empty_like(b)
                sustain(torch, dslash_step(lat, prec, a, b, c, d), SWEEP_RAMP_MS)
                ms, ml, _ = dslash_step_timing(lat, hisq, torch, prec, a, b, c, d, 10, 3, isolated=False)
                byt = pm.half_dslash_bytes(vh, nn, prec, recon)
                lb, vb = pm.PREC_BYTES[prec]
                paper_b = vh * (pm.link_reals(recon if prec else 18) * lb + nn * 17 * 6 * vb)
                sweep.append({"prec": name, "n": nn, "ms_per_launch": round(ml, 5),
                              "gflops": round(pm.half_dslash_flops(vh, nn) / (ml * 1e-3) / 1e9, 1),
                              "compulsory_GBps": round(byt / (ml * 1e-3) / 1e9, 1),
                              "paper_model_GBps": round(paper_b / (ml * 1e-3) / 1e9, 1)})
            if recon != 18:
                lat.load_links(fat, naik, hisq.HISQ_LINKS_ALL, 18)
        result["dslash_sweep"] = sweep
        del srcs
        result["volume_sweep"] = volume_sweep(hisq, torch, synth, pm)
        # the same kernel's roofline where no cache level holds the working set (per parity: links
        # 2.4 GB, input bundle 0.8 GB against the 256 MB last-level cache)
        big = [e for e in result["volume_sweep"]
               if e["lattice"] == "64x64x64x16" and e["prec"] == "f32" and e["n"] == 16]
        if big:
            e = big[0]
            result["roofline_64x64x64x16"] = {
                "bound": "hbm", "achieved": e["compulsory_GBps"], "peak": 8000.0, "unit": "GB/s",
                "frac": round(e["compulsory_GBps"] / 8000.0, 4),
                "kernel": "k_dslash_lds (half Dslash, FP32, 16 rhs)", "launch": e["launch"],
                "counters": "profiles/k_dslash_f32_n16_64x64x64x16.txt"}

    if not args.no_cg:
        c2 = synth.WORKLOADS["c2"]
        fat2, naik2 = synth.gauge_links(c2["dims"], synth.workload_seed("c2"), eps=c2["eps"])
        lat2 = hisq.Lattice(c2["dims"], 0)
        lat2.load_links(fat2, naik2, hisq.HISQ_LINKS_ALL, args.cg_naik_recon)
        b = torch.from_numpy(synth.sources(c2["dims"], c2["n"], synth.workload_seed("c2") + 1)).to("cuda:0")
        cg = {"workload": "32x32x32x8, m=0.02, 8 complex Gaussian rhs, tol 1e-8 (true FP64 residual)",
              "naik_reals": args.cg_naik_recon}
        for name, kw in (("mixed_f16links", dict(kind=hisq.HISQ_CG_MIXED, link_prec=hisq.HISQ_F16)),
                         ("mixed_f32links", dict(kind=hisq.HISQ_CG_MIXED, link_prec=hisq.HISQ_F32)),
                         ("plain_f64", dict(kind=hisq.HISQ_CG_F64))):
            x, info = lat2.cg(c2["mass"], b, tol=c2["tol"], max_iter=40000, **kw)
            torch.cuda.synchronize()
            t = time.perf_counter()
            x, info = lat2.cg(c2["mass"], b, tol=c2["tol"], max_iter=40000, **kw)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t
            cg[name] = {"s_per_rhs": round(sec / c2["n"], 5), "seconds": round(sec, 4),
                        "iters_max": max(info["iters"]), "iters_min": min(info["iters"]),
                        "reliable_updates": info["reliable_updates"],
                        "fp32_links_from_iter": info["link_switch_iter"],
                        "true_resid_max": max(info["true_resid"]), "rc": info["rc"],
                        "dslash_gflops": round(pm.FLOP_PER_SITE_RHS * info["dslash_site_rhs"] / sec / 1e9, 1)}
        cg["speedup_mixed_vs_f64"] = round(cg["plain_f64"]["seconds"] / min(cg["mixed_f16links"]["seconds"],
                                                                          cg["mixed_f32links"]["seconds"]), 3)
        # repacking a bundle whose rhs finish at different iterations: 16 rhs, 12 of them started
        # from a solution to 1e-5, against the same solve with the finished rhs only masked
        b16 = torch.from_numpy(synth.sources(c2["dims"], 16, synth.workload_seed("c2") + 4)).to("cuda:0")
        xa, _ = lat2.cg(c2["mass"], b16, tol=1e-5, max_iter=40000, kind=hisq.HISQ_CG_MIXED,
                        link_prec=hisq.HISQ_F32)
        x0 = xa.clone()
        x0[12:] = 0
        uneven = {"workload": "32x32x32x8, m=0.02, 16 complex Gaussian rhs, 12 of them started from a "
                              "solution to 1e-5; mixed CG, FP16 links, tol 1e-8"}
        for label, comp in (("repacked", True), ("masked", False)):
            for rep in range(2):  # the first run tunes the launches of the smaller bundles
                torch.cuda.synchronize()
                t = time.perf_counter()
                x, info = lat2.cg(c2["mass"], b16, tol=c2["tol"], max_iter=40000, kind=hisq.HISQ_CG_MIXED,
                                  link_prec=hisq.HISQ_F16, x0=x0, compaction=comp)
                torch.cuda.synchronize()
                sec = time.perf_counter() - t
            uneven[label] = {"seconds": round(sec, 4), "iters_min": min(info["iters"]),
                             "iters_max": max(info["iters"]), "repacks": info["compactions"],
                             "true_resid_max": max(info["true_resid"]), "rc": info["rc"]}
        uneven["speedup_repacked_vs_masked"] = round(uneven["masked"]["seconds"] / uneven["repacked"]["seconds"], 3)
        cg["uneven_bundle"] = uneven
        del b16, xa, x0, x
        result["cg"] = cg
        # the paper's multi-rhs CG figure, on other hardware (context, not a comparison target)
        result["paper_context"] = {
            "cg_gflops_fp32": ">250 on Xeon Phi 5110P and Kepler Tesla GPUs (abstract, Section 4)",
            "mixed_cg_dslash_gflops_here": cg["mixed_f16links"]["dslash_gflops"],
            "note": "Dslash flops per second of the whole mixed solve (BLAS-1 flops not counted)"}
        # Eq. 2: Tr M^-1 from Z2 noise bundles through the mixed solver
        nvec, bundle = 64, 16
        torch.cuda.synchronize()
        t = time.perf_counter()
        est, err, smp = lat2.trace_minv(c2["mass"], nvec, bundle=bundle, seed=synth.workload_seed("c2") + 3,
                                        kind=hisq.HISQ_CG_MIXED, tol=c2["tol"], link_prec=hisq.HISQ_F16)
        sec = time.perf_counter() - t
        smp = np.array(smp)
        result["trace_minv"] = {
            "workload": "32x32x32x8, m=0.02, Z2 noise, bundles of 16, mixed CG (FP16 links) to 1e-8",
            "vectors": nvec, "estimate": round(est, 3), "std_error": round(err, 3),
            "std_error_vs_n": {str(k): round(float(smp[:k].std(ddof=1) / np.sqrt(k)), 3) for k in (16, 32, 64)},
            "seconds": round(sec, 3), "s_per_vector": round(sec / nvec, 5)}
        # the chiral condensate (1/V) Tr (m + D)^-1 from the library, on the first 16 of the same
        # noise vectors (one bundle)
        pbp, pbp_err = lat2.chiral_condensate(c2["mass"], 16, bundle=bundle, seed=synth.workload_seed("c2") + 3,
                                              kind=hisq.HISQ_CG_MIXED, tol=c2["tol"], link_prec=hisq.HISQ_F16)
        result["trace_minv"]["chiral_condensate_16_vectors"] = {"estimate": round(pbp, 6),
                                                                "std_error": round(pbp_err, 6)}
        lat2.close()

    if not args.no_c3 and not args.no_cg:
        # the 48^3 x 12 solver comparison: plain FP64, mixed (FP16 and FP32 links) and the
        # flexible CG with the learned preconditioner (its inner operator on the FP32 links)
        # (a failure here is recorded in the line rather than losing the Dslash figures above)
        t = time.perf_counter()
        try:
            c3 = solver_study("c3", torch, synth, hisq, pm, fcg_link_precs=(hisq.HISQ_F32,))
            c3["study_seconds"] = round(time.perf_counter() - t, 1)
        except Exception as e:  # noqa: BLE001 - reported, not hidden
            c3 = {"error": f"{type(e).__name__}: {e}"}
            print(f"[c3] failed: {c3['error']}", file=sys.stderr, flush=True)
        result["cg_48x48x48x12"] = c3

    if not args.no_cpu:
        cg_iters = None
        if "cg" in result:
            cg_iters = result["cg"]["plain_f64"]["iters_max"]
        c3_iters = None
        if "cg_48x48x48x12" in result and "plain_f64" in result["cg_48x48x48x12"]:
            c3_iters = result["cg_48x48x48x12"]["plain_f64"]["iters_max"]
        try:
            result["cpu_baseline"] = cpu_baseline(dims, n, cg_iters, c3_iters)
        except Exception as e:  # noqa: BLE001 - reported, not hidden
            result["cpu_baseline"] = {"kind": "oracle", "error": f"{type(e).__name__}: {e}"}
            print(f"[cpu_baseline] failed: {result['cpu_baseline']['error']}", file=sys.stderr, flush=True)
    lat.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
