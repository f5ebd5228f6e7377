"""Tune the Dslash launch configurations for the study lattices on this GPU and save them to
paper_1409_1510_amd/tuning/<arch>.txt (loaded by hisq.Lattice.load_links).

Usage (on the GPU): python -m paper_1409_1510_amd.tune_study [--out PATH] [--lattices c1,c3,c4]
                                                         [--precs 0,1,2]
The timing does not depend on the link values, so the links are a small random field tiled over
the lattice.
"""
from __future__ import annotations

import argparse
import os
import sys


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from paper_1409_1510_amd import hisq  # noqa: E402

RHS = {"c1": (1, 2, 4, 8, 16), "c2": (8,), "c3": (8, 16), "c4": (8, 16, 32)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=hisq.TUNING_PATH)
    ap.add_argument("--lattices", default="c1,c3,c4")
    ap.add_argument("--precs", default="0,1,2",
                    help="precisions to re-tune (the others keep the entries of the shipped table)")
    args = ap.parse_args()
    retune = {int(p) for p in args.precs.split(",")}
    os.environ["HISQ_AUTOTUNE"] = "1"
    for name in args.lattices.split(","):
        dims = synth.WORKLOADS[name]["dims"]
        fat, naik = synth.tiled_gauge_links(dims, 7)
        for recon in (18, 14):
            lat = hisq.Lattice(dims, 0)
            lat.load_links(fat, naik, hisq.HISQ_LINKS_ALL if recon == 18 else
                           hisq.HISQ_LINKS_F32 | hisq.HISQ_LINKS_F16, recon)
            precs = (0, 1, 2) if recon == 18 else (1, 2)
            for prec in precs:
                if prec not in retune:
                    continue
                for n in RHS[name]:
                    hisq.hisq_set_launch(lat.ctx, prec, n, None)  # clears both forms
                    for fused in (0, 1):
                        cfg, ms = hisq.hisq_autotune(lat.ctx, prec, n, fused)
                        print(f"{name} r{recon} prec {prec} n {n} fused {fused}: {cfg} {ms:.5f} ms", flush=True)
            hisq._check(lat.ctx, hisq.library().hisq_save_tuning(lat.ctx, args.out.encode()))
            lat.close()
    print(f"saved {args.out}")


if __name__ == "__main__":
    main()
