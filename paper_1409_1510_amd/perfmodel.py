"""Flop and byte accounting of the multi-rhs HISQ half Dslash and the CG (host-side helpers).

Flops (Section 1, the arithmetic-intensity model behind Table 1): per output site and rhs,
16 SU(3) matrix-vector products (66 flop each: 9 complex multiplies and 6 complex adds) and 15
colour-vector additions (6 flop each) to sum the 16 hop results: 16*66 + 15*6 = 1146 flop.

Bytes, two models per output site:
  * the paper's model, which reproduces Table 1: every link read once (16 links of 18 reals, or
    8 fat links of 18 reals plus 8 Naik links of 14 reals), and per rhs 16 neighbour vectors plus
    one output vector (17 vectors of 6 reals) with no reuse between sites;
  * the compulsory traffic of one half Dslash on a device: every link read once, and per rhs the
    input vector and the output vector each touched once (in a half Dslash every input site is
    a neighbour of 16 output sites; an ideal cache reads it once).
"""
from __future__ import annotations

FLOP_PER_SITE_RHS = 16 * 66 + 15 * 6  # 1146

REAL_BYTES = {"f64": 8, "f32": 4, "f16": 2}


def link_reals(recon: int = 18) -> int:
    """Reals stored for the 16 links an output site reads: 8 fat links of 18 reals and 8 Naik
    links of `recon` reals (18, 14, 13 or 9)."""
    if recon not in (18, 14, 13, 9):
        raise ValueError(f"Naik storage format {recon}: 18, 14, 13 or 9")
    return 8 * 18 + 8 * recon


def paper_model_bytes(n: int, recon: int = 18, real_bytes: int = 4) -> int:
    return link_reals(recon) * real_bytes + n * 17 * 6 * real_bytes


def paper_model_intensity(n: int, recon: int = 18, real_bytes: int = 4) -> float:
    return FLOP_PER_SITE_RHS * n / paper_model_bytes(n, recon, real_bytes)


def paper_model_limit(real_bytes: int = 4) -> float:
    """n -> infinity limit of the paper model: 1146 / (17 * 6 * b)."""
    return FLOP_PER_SITE_RHS / (17 * 6 * real_bytes)


def compulsory_bytes(n: int, link_bytes: int, vec_bytes: int, recon: int = 18) -> int:
    """Compulsory bytes per output site of a half Dslash with n rhs.

    link_bytes: bytes per stored link real (8 FP64, 4 FP32, 2 FP16); vec_bytes: bytes per vector
    real (8 FP64, 4 FP32)."""
    return link_reals(recon) * link_bytes + n * 2 * 6 * vec_bytes


PREC_BYTES = {0: (8, 8), 1: (4, 4), 2: (2, 4)}  # HISQ_F64, HISQ_F32, HISQ_F16 -> (link, vector)


def half_dslash_bytes(vh: int, n: int, prec: int, recon: int = 18) -> int:
    lb, vb = PREC_BYTES[prec]
    return vh * compulsory_bytes(n, lb, vb, 18 if prec == 0 else recon)


def half_dslash_flops(vh: int, n: int) -> int:
    return FLOP_PER_SITE_RHS * vh * n
