"""Build libhisq.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libhisq.so")

SOURCES = ["context.cpp", "links.hip", "dslash.hip", "dslash_f64.hip", "dslash_f32.hip",
           "dslash_f32c.hip", "dslash_f16.hip", "dslash_f16c.hip", "blas.hip", "cg.cpp", "nn.hip",
           "trace.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # explicit fma() only: per-rhs results must not depend on how the compiler contracts
    "-ffp-contract=off",
    # no packed FP32 (v_pk_*_f32) instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


# per-unit scheduler: the FP64 Dslash instances are scheduled for instruction-level parallelism
# (LLVM's max-ilp strategy), which issues their 16-byte gathers earlier: measured 11-19 % faster
# FP64 LDS launches at 8 and 16 rhs (32^3 x 8) and within 1 % at 1-4 rhs.  The FP32 and FP16-link
# units keep the default strategy, under which their 16-rhs launches are 8-10 % faster than with
# max-ilp.  Scheduling only orders instructions: every output stays bit-identical.
EXTRA_FLAGS = {"dslash_f64.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]}


def _compile(src: str) -> str:
    obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *EXTRA_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def hip_runtime_dir() -> str:
    """Directory of the HIP runtime PyTorch loads (torch/lib ships its own libamdhip64.so).

    libhisq links that same runtime: two HIP runtimes in one process do not share the device,
    and the one initialised second finds no GPU."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or spec.origin is None:
        raise RuntimeError("torch is required: libhisq links the HIP runtime that PyTorch loads")
    d = os.path.join(os.path.dirname(spec.origin), "lib")
    if not os.path.exists(os.path.join(d, "libamdhip64.so")):
        raise RuntimeError(f"no libamdhip64.so in {d}")
    return d


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    rt = hip_runtime_dir()
    # plain host link (the device code is already embedded in the objects); the HIP runtime is
    # PyTorch's, found through the rpath whether or not torch is imported first
    cmd = ["g++", "-shared", "-fPIC", *objs, "-o", tmp, f"-L{rt}", "-l:libamdhip64.so",
           f"-Wl,-rpath,{rt}", "-Wl,--no-undefined"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
