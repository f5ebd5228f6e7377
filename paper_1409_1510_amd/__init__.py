"""MI355X (gfx950) multi-right-hand-side HISQ Dslash and even-odd CG solvers.

Kaczmarek, Schmidt, Steinbrecher, Mukherjee, Wagner, "HISQ inverter on Intel Xeon Phi and NVIDIA
GPUs" (PoS LATTICE2014): the staggered HISQ Dslash (fat links, +-1 hops; Naik links, +-3 hops,
Section 1 Eq. 3) applied to a bundle of right-hand sides at once (Eq. 4) inside an even-odd CG.

The compute path is the HIP library libhisq.so (C ABI in include/hisq.h); `hisq` is its thin
ctypes binding and `perfmodel` the flop/byte accounting.
"""
__all__ = ["hisq", "perfmodel"]
