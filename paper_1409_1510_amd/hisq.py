"""ctypes binding of libhisq (the C ABI in include/hisq.h): argument marshalling only.

Every computation runs in the HIP kernels of libhisq.so; this module checks tensor shapes,
dtypes and devices, passes raw pointers and the current torch stream, and turns error codes into
exceptions.  There is no fallback: if the library is missing, importing this module raises.

The functions keep the C names (hisq_create, hisq_dslash_mrhs, ...).  `Lattice` bundles a
context with torch conveniences for tests and benchmarks.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhisq.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "hisq.h")
# launch configurations tuned on MI355X for the study lattices (loaded by Lattice.load_links)
TUNING_PATH = os.path.join(_HERE, "tuning", "gfx950.txt")

HISQ_OK = 0
HISQ_ERR_ARG = -1
HISQ_ERR_STATE = -2
HISQ_ERR_HIP = -3
HISQ_ERR_OOM = -4
HISQ_ERR_NOCONV = -5
HISQ_ERR_NONFINITE = -6
HISQ_ERR_IO = -7

HISQ_F64, HISQ_F32, HISQ_F16 = 0, 1, 2
HISQ_LINKS_F64, HISQ_LINKS_F32, HISQ_LINKS_F16, HISQ_LINKS_ALL = 1, 2, 4, 7
HISQ_CG_F64, HISQ_CG_MIXED, HISQ_FCG_NN = 0, 1, 2
HISQ_MAX_RHS = 64
HISQ_NN_LOSS_SOLUTION, HISQ_NN_LOSS_RESIDUAL = 0, 1
HISQ_NN_FORM_DIRECT, HISQ_NN_FORM_GRAM = 0, 1

_ERR_NAMES = {
    HISQ_ERR_ARG: "HISQ_ERR_ARG", HISQ_ERR_STATE: "HISQ_ERR_STATE", HISQ_ERR_HIP: "HISQ_ERR_HIP",
    HISQ_ERR_OOM: "HISQ_ERR_OOM", HISQ_ERR_NOCONV: "HISQ_ERR_NOCONV",
    HISQ_ERR_NONFINITE: "HISQ_ERR_NONFINITE", HISQ_ERR_IO: "HISQ_ERR_IO",
}


class HisqError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class hisq_launch(ctypes.Structure):
    _fields_ = [("rhs_per_thread", ctypes.c_int), ("sites_per_block", ctypes.c_int),
                ("nontemporal_links", ctypes.c_int), ("lds_links", ctypes.c_int),
                ("xcd_map", ctypes.c_int)]

    def as_tuple(self):
        return (self.rhs_per_thread, self.sites_per_block, self.nontemporal_links, self.lds_links,
                self.xcd_map)


class hisq_cg_params(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("reliable_every", ctypes.c_int), ("link_prec", ctypes.c_int),
                ("use_x0", ctypes.c_int), ("check_every", ctypes.c_int),
                ("no_compaction", ctypes.c_int)]


class hisq_cg_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.POINTER(ctypes.c_int)),
                ("true_resid", ctypes.POINTER(ctypes.c_double)),
                ("converged", ctypes.POINTER(ctypes.c_int)),
                ("fell_back", ctypes.POINTER(ctypes.c_int)),
                ("total_iters", ctypes.c_int), ("reliable_updates", ctypes.c_int),
                ("dslash_site_rhs", ctypes.c_longlong), ("seconds", ctypes.c_double),
                ("peak_bytes", ctypes.c_size_t), ("link_switch_iter", ctypes.c_int),
                ("compactions", ctypes.c_int)]


def header_functions() -> list[str]:
    """Names of the functions declared in include/hisq.h."""
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"\b(hisq_\w+)\s*\(", text)


def _preload_hip_runtime():
    """Load PyTorch's HIP runtime (torch/lib/libamdhip64.so, soname libamdhip64.so.7) before
    libhisq, so that libhisq binds to the same runtime as torch whatever the import order: a
    second HIP runtime in the process would not see the GPU."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or spec.origin is None:
        raise ImportError("torch is required (libhisq uses PyTorch's HIP runtime)")
    path = os.path.join(os.path.dirname(spec.origin), "lib", "libamdhip64.so")
    ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    _preload_hip_runtime()
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, dp, cint, cd = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_double
    sig = {
        "hisq_create": (cint, [ctypes.POINTER(vp), ip, cint, vp]),
        "hisq_destroy": (cint, [vp]),
        "hisq_last_error": (ctypes.c_char_p, [vp]),
        "hisq_set_stream": (cint, [vp, vp]),
        "hisq_load_links": (cint, [vp, vp, vp, cint, cint]),
        "hisq_dslash_mrhs": (cint, [vp, cint, cint, cint, vp, vp]),
        "hisq_apply_m": (cint, [vp, cint, cd, cint, vp, vp, vp]),
        "hisq_dot_mrhs": (cint, [vp, cint, cint, vp, vp, vp]),
        "hisq_dot_mrhs_noalloc": (cint, [vp, cint, cint, vp, vp, vp]),
        "hisq_set_launch": (cint, [vp, cint, cint, ctypes.POINTER(hisq_launch)]),
        "hisq_get_launch": (cint, [vp, cint, cint, cint, ctypes.POINTER(hisq_launch)]),
        "hisq_autotune": (cint, [vp, cint, cint, cint, ctypes.POINTER(hisq_launch), dp]),
        "hisq_save_tuning": (cint, [vp, ctypes.c_char_p]),
        "hisq_load_tuning": (cint, [vp, ctypes.c_char_p, ip]),
        "hisq_cg_mrhs": (cint, [vp, cd, cint, vp, vp, ctypes.POINTER(hisq_cg_params),
                                ctypes.POINTER(hisq_cg_stats)]),
    }
    optional = {
        "hisq_nn_init": (cint, [vp, cint, cint, ctypes.c_ulonglong]),
        "hisq_nn_get_params": (cint, [vp, dp, cint]),
        "hisq_nn_set_params": (cint, [vp, dp, cint]),
        "hisq_nn_num_params": (cint, [vp]),
        "hisq_nn_apply": (cint, [vp, cint, cint, vp, vp]),
        "hisq_nn_loss_grad": (cint, [vp, cint, vp, vp, dp, dp]),
        "hisq_nn_train": (cint, [vp, cint, vp, vp, cint, cint, cd, ctypes.c_ulonglong, dp]),
        "hisq_nn_set_precision": (cint, [vp, cint]),
        "hisq_nn_set_form": (cint, [vp, cint]),
        "hisq_nn_set_loss": (cint, [vp, cint, cd]),
        "hisq_nn_harvest": (cint, [vp, cd, cint, vp, cd, cint, cint, vp, vp, ip]),
        "hisq_z2_noise": (cint, [vp, ctypes.c_ulonglong, ctypes.c_longlong, cint, vp]),
        "hisq_trace_minv": (cint, [vp, cd, cint, cint, ctypes.c_ulonglong, ctypes.POINTER(hisq_cg_params),
                                   dp, dp, dp]),
        "hisq_chiral_condensate": (cint, [vp, cd, cint, cint, ctypes.c_ulonglong,
                                          ctypes.POINTER(hisq_cg_params), dp, dp]),
        "hisq_nn_save": (cint, [vp, ctypes.c_char_p]),
        "hisq_nn_load": (cint, [vp, ctypes.c_char_p]),
    }
    for name, (res, args) in list(sig.items()) + list(optional.items()):
        if not hasattr(lib, name):
            if name in sig:
                raise ImportError(f"{LIB_PATH} does not export {name}")
            continue
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def library():
    return _lib


def _check(ctx, rc: int) -> int:
    if rc != HISQ_OK:
        msg = _lib.hisq_last_error(ctx)
        raise HisqError(rc, msg.decode() if msg else "")
    return rc


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(0)
    if isinstance(t, np.ndarray):
        return ctypes.c_void_p(t.ctypes.data)
    return ctypes.c_void_p(t.data_ptr())


# ---- the C functions, same names -------------------------------------------------------------

def hisq_create(dims, device: int = 0, stream=0):
    """stream: a torch stream, a raw hipStream_t as int, 0 for the null stream, or None for
    torch's current stream."""
    ctx = ctypes.c_void_p()
    arr = (ctypes.c_int * 4)(*[int(d) for d in dims])
    rc = _lib.hisq_create(ctypes.byref(ctx), arr, int(device), _stream_ptr(stream))
    if rc != HISQ_OK:
        raise HisqError(rc, _lib.hisq_last_error(None).decode())
    return ctx


def hisq_destroy(ctx) -> None:
    _lib.hisq_destroy(ctx)


def hisq_last_error(ctx) -> str:
    m = _lib.hisq_last_error(ctx)
    return m.decode() if m else ""


def hisq_set_stream(ctx, stream=None) -> None:
    _check(ctx, _lib.hisq_set_stream(ctx, _stream_ptr(stream)))


def hisq_load_links(ctx, fat, naik, copies: int = HISQ_LINKS_ALL, naik_recon: int = 18) -> None:
    for a in (fat, naik):
        if isinstance(a, np.ndarray):
            if a.dtype != np.complex128 or not a.flags.c_contiguous:
                raise ValueError("links must be C-contiguous complex128 [V][4][3][3]")
        elif str(a.dtype) != "torch.complex128" or not a.is_contiguous():
            raise ValueError("links must be contiguous complex128 [V][4][3][3]")
    _check(ctx, _lib.hisq_load_links(ctx, _ptr(fat), _ptr(naik), int(copies), int(naik_recon)))


def hisq_dslash_mrhs(ctx, out_parity: int, prec: int, n: int, inp, out) -> None:
    _check(ctx, _lib.hisq_dslash_mrhs(ctx, int(out_parity), int(prec), int(n), _ptr(inp), _ptr(out)))


def hisq_apply_m(ctx, prec: int, mass: float, n: int, inp, out, pq_out=None) -> None:
    _check(ctx, _lib.hisq_apply_m(ctx, int(prec), float(mass), int(n), _ptr(inp), _ptr(out), _ptr(pq_out)))


def hisq_dot_mrhs(ctx, prec: int, n: int, a, b, dots) -> None:
    _check(ctx, _lib.hisq_dot_mrhs(ctx, int(prec), int(n), _ptr(a), _ptr(b), _ptr(dots)))


def hisq_dot_mrhs_noalloc(ctx, prec: int, n: int, a, b, dots) -> None:
    _check(ctx, _lib.hisq_dot_mrhs_noalloc(ctx, int(prec), int(n), _ptr(a), _ptr(b), _ptr(dots)))


def hisq_set_launch(ctx, prec: int, n: int, cfg=None) -> None:
    """cfg: (rhs_per_thread, sites_per_block, nontemporal_links, lds_links[, xcd_map]), a
    hisq_launch, or None."""
    if cfg is not None and not isinstance(cfg, hisq_launch):
        cfg = hisq_launch(*(tuple(cfg) + (0,) * (5 - len(cfg))))
    _check(ctx, _lib.hisq_set_launch(ctx, int(prec), int(n), ctypes.byref(cfg) if cfg is not None else None))


def hisq_get_launch(ctx, prec: int, n: int, fused_m: int = 0) -> tuple:
    c = hisq_launch()
    _check(ctx, _lib.hisq_get_launch(ctx, int(prec), int(n), int(fused_m), ctypes.byref(c)))
    return c.as_tuple()


def hisq_autotune(ctx, prec: int, n: int, fused_m: int = 0):
    c = hisq_launch()
    ms = ctypes.c_double()
    _check(ctx, _lib.hisq_autotune(ctx, int(prec), int(n), int(fused_m), ctypes.byref(c), ctypes.byref(ms)))
    return c.as_tuple(), ms.value


def hisq_save_tuning(ctx, path: str) -> None:
    _check(ctx, _lib.hisq_save_tuning(ctx, os.fsencode(path)))


def hisq_load_tuning(ctx, path: str) -> int:
    """Entries of the file that match this context's lattice and link formats; returns how many
    were taken."""
    cnt = ctypes.c_int()
    _check(ctx, _lib.hisq_load_tuning(ctx, os.fsencode(path), ctypes.byref(cnt)))
    return cnt.value


def hisq_cg_mrhs(ctx, mass: float, n: int, b, x, params: hisq_cg_params, stats: hisq_cg_stats):
    rc = _lib.hisq_cg_mrhs(ctx, float(mass), int(n), _ptr(b), _ptr(x), ctypes.byref(params),
                           ctypes.byref(stats))
    if rc not in (HISQ_OK, HISQ_ERR_NOCONV):
        _check(ctx, rc)
    return rc


# ---- convenience wrapper -----------------------------------------------------------------------

_VEC_DTYPE = {HISQ_F64: "torch.complex128", HISQ_F32: "torch.complex64", HISQ_F16: "torch.complex64"}


class Lattice:
    """A libhisq context on one GPU for one lattice, with torch tensors for vectors."""

    def __init__(self, dims, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.dims = tuple(int(d) for d in dims)
        self.volume = int(np.prod(self.dims))
        self.vh = self.volume // 2
        self.device = torch.device("cuda", device)
        self.ctx = None
        self.ctx = hisq_create(self.dims, device, stream)

    def close(self):
        if self.ctx is not None:
            hisq_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def vec_dtype(self, prec):
        return self.torch.complex128 if prec == HISQ_F64 else self.torch.complex64

    def empty(self, n, prec=HISQ_F64):
        return self.torch.empty((n, 3, self.vh), dtype=self.vec_dtype(prec), device=self.device)

    def _vec(self, v, prec, name="vector", n=None):
        """Check a vector argument: device, dtype of the precision, contiguous [n][3][V/2] (with
        the given n if any: the library reads or writes exactly that many rhs)."""
        if not v.is_cuda or v.device != self.device:
            raise ValueError(f"{name} must live on {self.device}")
        if str(v.dtype) != _VEC_DTYPE[prec]:
            raise ValueError(f"{name} must be {_VEC_DTYPE[prec]} for precision {prec}, got {v.dtype}")
        if v.dim() != 3 or v.shape[1] != 3 or v.shape[2] != self.vh or not v.is_contiguous():
            raise ValueError(f"{name} must be contiguous [n][3][{self.vh}], got {tuple(v.shape)}")
        if n is not None and v.shape[0] != n:
            raise ValueError(f"{name} must hold {n} right-hand sides, got {v.shape[0]}")
        return v

    def load_links(self, fat, naik, copies=HISQ_LINKS_ALL, naik_recon=18):
        if isinstance(fat, np.ndarray):
            fat = np.ascontiguousarray(fat, np.complex128)
            naik = np.ascontiguousarray(naik, np.complex128)
            if fat.shape != (self.volume, 4, 3, 3) or naik.shape != fat.shape:
                raise ValueError(f"links must be [{self.volume}][4][3][3]")
        else:  # device tensors: the library reads V * 36 complex128 from each
            for name, t in (("fat", fat), ("naik", naik)):
                if (str(t.dtype) != "torch.complex128" or tuple(t.shape) != (self.volume, 4, 3, 3)
                        or not t.is_contiguous()):
                    raise ValueError(f"{name} links must be contiguous complex128 [{self.volume}][4][3][3]")
        hisq_load_links(self.ctx, fat, naik, copies, naik_recon)
        if os.path.exists(TUNING_PATH) and os.environ.get("HISQ_AUTOTUNE", "1") != "0":
            hisq_load_tuning(self.ctx, TUNING_PATH)

    def dslash(self, out_parity, prec, v_in, out=None):
        self._vec(v_in, prec, "in")
        n = v_in.shape[0]
        out = self.empty(n, prec) if out is None else self._vec(out, prec, "out", n)
        hisq_set_stream(self.ctx)
        hisq_dslash_mrhs(self.ctx, out_parity, prec, n, v_in, out)
        return out

    def apply_m(self, prec, mass, v_in, out=None, with_pq=False):
        self._vec(v_in, prec, "in")
        n = v_in.shape[0]
        out = self.empty(n, prec) if out is None else self._vec(out, prec, "out", n)
        pq = self.torch.empty(n, dtype=self.torch.float64, device=self.device) if with_pq else None
        hisq_set_stream(self.ctx)
        hisq_apply_m(self.ctx, prec, mass, n, v_in, out, pq)
        return (out, pq) if with_pq else out

    def dot(self, prec, a, b):
        self._vec(a, prec, "a")
        n = a.shape[0]
        self._vec(b, prec, "b", n)
        d = self.torch.empty(2 * n, dtype=self.torch.float64, device=self.device)
        hisq_set_stream(self.ctx)
        hisq_dot_mrhs(self.ctx, prec, n, a, b, d)
        return self.torch.complex(d[0::2], d[1::2])

    def z2_noise(self, seed, k0, n):
        out = self.empty(n, HISQ_F64)
        hisq_set_stream(self.ctx)
        _check(self.ctx, _lib.hisq_z2_noise(self.ctx, seed, k0, n, _ptr(out)))
        return out

    def trace_minv(self, mass, n_vec, bundle=16, seed=1, kind=HISQ_CG_MIXED, tol=1e-8, max_iter=40000,
                   reliable_every=50, link_prec=HISQ_F32):
        """(estimate, std_error, samples) of Tr M^-1 from n_vec Z2 noise vectors."""
        p = hisq_cg_params(kind, tol, max_iter, reliable_every, link_prec, 0, 0)
        samples = (ctypes.c_double * n_vec)()
        est, err = ctypes.c_double(), ctypes.c_double()
        hisq_set_stream(self.ctx)
        _check(self.ctx, _lib.hisq_trace_minv(self.ctx, mass, n_vec, bundle, seed, ctypes.byref(p), samples,
                                              ctypes.byref(est), ctypes.byref(err)))
        return est.value, err.value, list(samples)

    def chiral_condensate(self, mass, n_vec, bundle=16, seed=1, kind=HISQ_CG_MIXED, tol=1e-8,
                          max_iter=40000, reliable_every=50, link_prec=HISQ_F32):
        """(estimate, std_error) of (1/V) Tr (m + D)^-1 from n_vec Z2 noise vectors."""
        p = hisq_cg_params(kind, tol, max_iter, reliable_every, link_prec, 0, 0)
        est, err = ctypes.c_double(), ctypes.c_double()
        hisq_set_stream(self.ctx)
        _check(self.ctx, _lib.hisq_chiral_condensate(self.ctx, mass, n_vec, bundle, seed, ctypes.byref(p),
                                                     ctypes.byref(est), ctypes.byref(err)))
        return est.value, err.value

    def cg(self, mass, b, kind=HISQ_CG_F64, tol=1e-10, max_iter=20000, reliable_every=50,
           link_prec=HISQ_F32, x0=None, check_every=0, compaction=True):
        self._vec(b, HISQ_F64, "b")
        n = b.shape[0]
        x = self.empty(n, HISQ_F64) if x0 is None else self._vec(x0.clone(), HISQ_F64, "x0", n)
        p = hisq_cg_params(kind, tol, max_iter, reliable_every, link_prec, 0 if x0 is None else 1,
                           check_every, 0 if compaction else 1)
        iters = (ctypes.c_int * n)()
        res = (ctypes.c_double * n)()
        conv = (ctypes.c_int * n)()
        fb = (ctypes.c_int * n)()
        st = hisq_cg_stats(iters, res, conv, fb, 0, 0, 0, 0.0, 0, -1, 0)
        hisq_set_stream(self.ctx)
        rc = hisq_cg_mrhs(self.ctx, mass, n, b, x, p, st)
        info = dict(rc=rc, iters=list(iters), true_resid=list(res), converged=list(conv),
                    fell_back=list(fb), total_iters=st.total_iters,
                    reliable_updates=st.reliable_updates, dslash_site_rhs=st.dslash_site_rhs,
                    seconds=st.seconds, peak_bytes=st.peak_bytes, link_switch_iter=st.link_switch_iter,
                    compactions=st.compactions)
        return x, info
