"""Benchmark of the multi-rhs HISQ Dslash and the even-odd CG solvers on one MI355X.

Workload (default): the 32^3 x 8 lattice with 16 complex Gaussian right-hand sides, FP32 Dslash
(FP32 links, complex64 vectors), seeded synthetic links (exp(i 0.4 H) + 0.05 G fat links, -1/24
Haar SU(3) Naik links).  One step = one full-lattice multi-rhs Dslash w = D v for the bundle:
the two half Dslash launches D_oe (even -> odd) and D_eo (odd -> even).
value = Gflop/s under the 1146 flop per site per rhs convention (Section 1, Table 1 model).

Also reported on the same JSON line:
  roofline      : compulsory HBM bytes per half-Dslash launch / mean launch duration (HIP events
                  at the ends of the timed region on the launch stream, over its launches),
                  against 8 TB/s; the GPU clocks rocm-smi reports under the same load;
The timed steps follow RAMP_MS of untimed back-to-back steps and then the warmup steps: the
device needs ~30 ms of load to reach its sustained speed for this kernel.
  dslash_sweep  : n = 1, 2, 4, 8, 16 in FP64, FP32, FP32 with 14-real Naik, FP16 links;
  cg            : seconds per rhs to a true FP64 residual 1e-8 at 32^3 x 8, m = 0.02, 8 rhs, for
                  the mixed-precision solver (FP16 and FP32 links) and the plain FP64 solver;
  trace_minv    : Tr M^-1 on the same lattice from 64 Z2 noise vectors (Eq. 2), with its error;
  volume_sweep  : the FP32 half Dslash against the lattice volume;
  cpu_baseline  : the FP64 numpy oracle's half Dslash on a bounded sample of the same lattice.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cg] [--no-cpu] [--no-sweep]
       python bench.py --workload c3|c4          (solver study at 48^3x12 / 64^3x16)
       python bench.py --profile|--profile-sweep|--profile-nn|--profile-cg   (short runs for rocprofv3)
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
            (hisq.HISQ_F16, 18, "f16links"), (hisq.HISQ_F16, 14, "f16links_r14"))


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
    "c3": dict(n_fcg=None, nsrc=16, nsnap=16, snap=60, harvest_tol=1e-8, epochs=20, plain=True),
    # 64^3 x 16: the network and its training scale with 16 x the vector volume, so the learned
    # solve runs on 2 of the 32 rhs with 64 training pairs; the plain FP64 solve is left out
    "c4": dict(n_fcg=2, nsrc=8, nsnap=8, snap=100, harvest_tol=1e-6, epochs=20, plain=False),
}


def solver_study(args, torch, synth, hisq, pm):
    """48^3x12 (16 Z2 rhs, m = 0.01) or 64^3x16 (32 Gaussian rhs, m = 0.005): CG seconds per rhs
    to a true FP64 residual 1e-8 for mixed precision (FP16 links), plain FP64 (48^3x12) and the
    flexible CG with the learned preconditioner (trained here on pairs harvested from plain CG on
    the same links), with iterations, peak device memory, the Dslash Gflop/s inside each solve
    and the cost of one network application."""
    import ctypes
    name = args.workload
    st = STUDY[name]
    cfg = synth.WORKLOADS[name]
    dims, n, mass, tol = cfg["dims"], cfg["n"], cfg["mass"], cfg["tol"]
    seed = synth.workload_seed(name)
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
    epochs = args.epochs if args.epochs else st["epochs"]

    def progress(msg):
        print(f"[{name}] {msg}", file=sys.stderr, flush=True)

    def solve(label, rhs, **kw):
        progress(f"solve {label}")
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, info = lat.cg(mass, rhs, tol=tol, max_iter=60000, **kw)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        nr = rhs.shape[0]
        out[label] = {"n_rhs": nr, "s_per_rhs": round(sec / nr, 5), "seconds": round(sec, 3),
                      "iters_mean": round(float(np.mean(info["iters"])), 1),
                      "iters_max": max(info["iters"]), "true_resid_max": max(info["true_resid"]),
                      "converged": sum(info["converged"]), "fell_back": sum(info["fell_back"]),
                      "reliable_updates": info["reliable_updates"], "rc": info["rc"],
                      "peak_device_GB": round(info["peak_bytes"] / 1e9, 2),
                      "fp32_links_from_iter": info["link_switch_iter"],
                      "dslash_gflops": round(pm.FLOP_PER_SITE_RHS * info["dslash_site_rhs"] / sec / 1e9, 1)}
        return x, info

    solve("mixed_f16links", b, kind=hisq.HISQ_CG_MIXED, link_prec=hisq.HISQ_F16)
    solve("mixed_f32links", b, kind=hisq.HISQ_CG_MIXED, link_prec=hisq.HISQ_F32)
    if st["plain"]:
        solve("plain_f64", b, kind=hisq.HISQ_CG_F64)
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
    # Gram form N^dag N (Hermitian positive semi-definite) trained on the residual-norm loss
    hisq._check(lat.ctx, lib.hisq_nn_init(lat.ctx, 4, 8, seed))
    hisq._check(lat.ctx, lib.hisq_nn_set_form(lat.ctx, hisq.HISQ_NN_FORM_GRAM))
    hisq._check(lat.ctx, lib.hisq_nn_set_loss(lat.ctx, hisq.HISQ_NN_LOSS_RESIDUAL, mass))
    # start from the best multiple of the identity for the residual loss on the training
    # residuals, c = sum <r, M r> / sum ||M r||^2 (P = N^dag N scales as |W_out|^2)
    r32 = r[: min(16, npairs.value)].to(torch.complex64)
    mr = lat.apply_m(hisq.HISQ_F32, mass, r32)
    c = float(torch.sum((torch.conj(r32) * mr).real) / torch.sum(torch.abs(mr) ** 2))
    del r32, mr
    nparam = lib.hisq_nn_num_params(lat.ctx)
    w = (ctypes.c_double * (2 * nparam))()
    hisq._check(lat.ctx, lib.hisq_nn_get_params(lat.ctx, w, 2 * nparam))
    for k in range(2 * (nparam - 8), 2 * nparam):
        w[k] *= c ** 0.5
    hisq._check(lat.ctx, lib.hisq_nn_set_params(lat.ctx, w, 2 * nparam))
    hist = (ctypes.c_double * epochs)()
    batch, lr = 16, 1e-2
    progress("train the network")
    t = time.perf_counter()
    hisq._check(lat.ctx, lib.hisq_nn_train(lat.ctx, npairs.value, hisq._ptr(r), hisq._ptr(y),
                                           epochs, batch, lr, seed, hist))
    out["training"] = {"form": "gram", "loss": "residual", "init_scale": round(c, 5), "epochs": epochs, "batch": batch,
                       "lr": lr, "bf16": True, "seconds": round(time.perf_counter() - t, 2),
                       "loss_first": round(hist[0], 5), "loss_last": round(hist[epochs - 1], 5)}
    del r, y
    bf = b if st["n_fcg"] is None else b[:st["n_fcg"]].contiguous()
    nf = bf.shape[0]
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
    out["network_apply_ms"] = {"n_rhs": nf, "ms": round(e0.elapsed_time(e1) / 5, 3)}
    del rv, zv
    # the faster mixed solver is the reference of the learned one (on the same bundle)
    best = min(("mixed_f16links", hisq.HISQ_F16), ("mixed_f32links", hisq.HISQ_F32),
               key=lambda kv: out[kv[0]]["seconds"])
    if nf != n:
        solve(best[0] + "_fcg_bundle", bf, kind=hisq.HISQ_CG_MIXED, link_prec=best[1])
    # the flexible CG's inner operator with either link copy (the network reads the FP16 copy in
    # both); the faster of the two is the learned solver's result
    solve("fcg_learned_f16links", bf, kind=hisq.HISQ_FCG_NN, link_prec=hisq.HISQ_F16)
    solve("fcg_learned_f32links", bf, kind=hisq.HISQ_FCG_NN, link_prec=hisq.HISQ_F32)
    fcg = min(("fcg_learned_f16links", "fcg_learned_f32links"), key=lambda k: out[k]["seconds"])
    ref = out[best[0] if nf == n else best[0] + "_fcg_bundle"]
    out["fcg_reference"] = best[0]
    out["fcg_best"] = fcg
    if st["plain"]:
        out["speedup_mixed_vs_f64"] = round(out["plain_f64"]["seconds"] / out[best[0]]["seconds"], 3)
    out["speedup_fcg_vs_mixed"] = round(ref["seconds"] / out[fcg]["seconds"], 3)
    out["iteration_ratio_fcg_vs_mixed"] = round(out[fcg]["iters_mean"] / ref["iters_mean"], 3)
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
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: one 256 MiB read + 256 MiB write elementwise "
                         "kernel (counter calibration), 100 ms of untimed steps with another "
                         "rhs_per_thread, then --steps FP32 Dslash steps")
    ap.add_argument("--profile-sweep", action="store_true",
                    help="short run for rocprofv3: the counter-calibration kernel, then for every "
                         "case of the n/precision sweep 50 ms of untimed steps, 1 warm-up step and "
                         "3 steps")
    ap.add_argument("--profile-nn", action="store_true",
                    help="only the learned preconditioner's Gram application at 48^3x12 on 16 rhs, "
                         "2 + --steps times (for a rocprofv3 run)")
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
    if args.profile_cg:
        c2 = synth.WORKLOADS["c2"]
        fat2, naik2 = synth.gauge_links(c2["dims"], synth.workload_seed("c2"), eps=c2["eps"])
        lat2 = hisq.Lattice(c2["dims"], 0)
        lat2.load_links(fat2, naik2)
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
        print(json.dumps(solver_study(args, torch, synth, hisq, pm)))
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
        for prec, recon, name in sweep_cases(hisq):
            if recon == 14:
                lat.load_links(fat, naik, hisq.HISQ_LINKS_F32 | hisq.HISQ_LINKS_F16, 14)
            for nn in SWEEP_N:
                dt = torch.complex128 if prec == hisq.HISQ_F64 else torch.complex64
                a, b = srcs[nn][0].to(dt), srcs[nn][1].to(dt)
                c, d = torch.empty_like(a), torch.empty_like(b)
                k = sustain(torch, dslash_step(lat, prec, a, b, c, d), SWEEP_RAMP_MS)
                dslash_step_timing(lat, hisq, torch, prec, a, b, c, d, 3, 1, isolated=False)
                # the trace holds 2 k untimed launches, then 2 warmup and 6 timed launches per case
                print(f"profile-sweep case {name} n {nn} launch {hisq.hisq_get_launch(lat.ctx, prec, nn, 0)} "
                      f"ramp {k}", flush=True)
            if recon == 14:
                lat.load_links(fat, naik, hisq.HISQ_LINKS_ALL, 18)
        lat.close()
        return
    if args.profile:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)  # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        # the sustained load runs the same kernel with another rhs_per_thread (another kernel
        # symbol), so that the trace's statistics of the timed kernel hold the timed launches only
        tuned = hisq.hisq_get_launch(lat.ctx, hisq.HISQ_F32, n, 0)
        hisq.hisq_set_launch(lat.ctx, hisq.HISQ_F32, n, (1 if tuned[0] > 1 else 2,) + tuned[1:])
        sustain(torch, dslash_step(lat, hisq.HISQ_F32, v_e, v_o, w_e, w_o), RAMP_MS)
        hisq.hisq_set_launch(lat.ctx, hisq.HISQ_F32, n, tuned)
        _, ms_launch, _ = dslash_step_timing(lat, hisq, torch, hisq.HISQ_F32, v_e, v_o, w_e, w_o,
                                             args.steps, 0, isolated=False)
        print(f"profile run done: {args.steps} steps, {n} rhs, lattice {dims}, launch "
              f"{hisq.hisq_get_launch(lat.ctx, hisq.HISQ_F32, n, 0)}, source {kernel_source_hash()}, "
              f"region-timed average {ms_launch * 1e3:.1f} us per launch")
        lat.close()
        return

    step = dslash_step(lat, hisq.HISQ_F32, v_e, v_o, w_e, w_o)
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
            if recon == 14:
                lat.load_links(fat, naik, hisq.HISQ_LINKS_F32 | hisq.HISQ_LINKS_F16, 14)
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
            if recon == 14:
                lat.load_links(fat, naik, hisq.HISQ_LINKS_ALL, 18)
        result["dslash_sweep"] = sweep
        del srcs
        result["volume_sweep"] = volume_sweep(hisq, torch, synth, pm)

    if not args.no_cg:
        c2 = synth.WORKLOADS["c2"]
        fat2, naik2 = synth.gauge_links(c2["dims"], synth.workload_seed("c2"), eps=c2["eps"])
        lat2 = hisq.Lattice(c2["dims"], 0)
        lat2.load_links(fat2, naik2)
        b = torch.from_numpy(synth.sources(c2["dims"], c2["n"], synth.workload_seed("c2") + 1)).to("cuda:0")
        cg = {"workload": "32x32x32x8, m=0.02, 8 complex Gaussian rhs, tol 1e-8 (true FP64 residual)"}
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
        lat2.close()

    if not args.no_cpu:
        import oracle
        nthreads = 1
        vs = v[:1]
        t = time.perf_counter()
        reps = 0
        while time.perf_counter() - t < 12.0 or reps < 1:
            oracle.dslash_half(fat, naik, vs, dims, 1)
            reps += 1
        sec = time.perf_counter() - t
        result["cpu_baseline"] = {
            "value": round(reps * pm.half_dslash_flops(vh, 1) / sec / 1e9, 3), "unit": "Gflop/s",
            "cores": nthreads, "kind": "oracle",
            "sample": f"{reps} FP64 numpy-oracle half Dslash applications (1 rhs) on the same "
                      f"32^3x8 links, {sec:.1f} s; single-threaded numpy"}
    lat.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
