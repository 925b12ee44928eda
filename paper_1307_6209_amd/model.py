"""Code-balance (roofline) performance model of SELL-C-sigma spMVM.

Sect. 4 of Kreutzer et al. (arXiv:1307.6209): with FP64 values, 4-byte
indices and y updated in memory, the SELL-C-sigma spMVM moves
    B(alpha, beta, N_nzr) = 6/beta + 4*alpha + 8/N_nzr  bytes per flop
(Eq. (sellbalance)); its performance bound is P = b / B (Eq.
(roof_general)), in the ideal-RHS case alpha = 1/N_nzc (Eq. (roof_alpha)),
and P_bar = b*beta/6 for long rows (Eq. (best_veccache)). alpha follows from
a measured data volume V by solving B = V / (2 N_nz) (Eq. (eq:sellalpha)).

The general form below extends the same byte count to the kernels of this
library: value/index/x/y element sizes s_v, s_i, s_x, s_y; y written once
(not read); a row permutation read (4 bytes per row) when sigma > 1; the
chunk metadata cl (4 B) and cs (8 B) per chunk; and k right-hand sides per
matrix pass. With s = (8, 4, 8, 16) (y read and written), no permutation,
no metadata and k = 1 it reduces to Eq. (sellbalance).
"""
from __future__ import annotations

from dataclasses import dataclass


def sell_balance(alpha: float, beta: float, nnzr: float) -> float:
    """Eq. (sellbalance): bytes per flop of FP64 SELL-C-sigma."""
    return 6.0 / beta + 4.0 * alpha + 8.0 / nnzr


def crs_balance(alpha: float, nnzr: float) -> float:
    """Eq. (crsbalance): the beta = 1 case."""
    return sell_balance(alpha, 1.0, nnzr)


def roofline(b: float, alpha: float, beta: float, nnzr: float) -> float:
    """Eq. (roof_general): performance bound (flop/s if b is in B/s)."""
    return b / sell_balance(alpha, beta, nnzr)


def roofline_ideal(b: float, beta: float, nnzr: float, nnzc: float | None = None) -> float:
    """Eq. (roof_alpha): alpha = 1/N_nzc."""
    return roofline(b, 1.0 / (nnzc if nnzc else nnzr), beta, nnzr)


def best_attainable(b: float, beta: float = 1.0) -> float:
    """Eq. (best_veccache): P_bar = b*beta/6."""
    return b * beta / 6.0


def alpha_from_volume(V: float, nnz: int, beta: float, nnzr: float) -> float:
    """Eq. (eq:sellalpha) with its byte unit read as bytes: solve
    6/beta + 4 alpha + 8/N_nzr = V / (2 N_nz) for alpha."""
    return 0.25 * (V / (2.0 * nnz) - 6.0 / beta - 8.0 / nnzr)


@dataclass
class Sizes:
    """Element sizes in bytes of one kernel variant."""
    sv: int = 8   # matrix value
    si: int = 4   # column index
    sx: int = 8   # x element
    sy: int = 8   # y element traffic per row (8: written once; 16: read and written)
    sp: int = 0   # permutation bytes per row (4 when sigma > 1)
    meta: float = 12  # cl (4) + cs (8) per chunk (+ window tables with the x window)


def general_balance(alpha: float, beta: float, nnzr: float, C: int, k: int = 1, s: Sizes = Sizes()) -> float:
    """Bytes per flop, per nonzero and right-hand side:
    [(s_v+s_i)/(k beta) + s_x alpha + (s_y + s_p/k)/N_nzr + meta/(k C N_nzr)] / 2."""
    return ((s.sv + s.si) / (k * beta) + s.sx * alpha + (s.sy + s.sp / k) / nnzr + s.meta / (k * C * nnzr)) / 2.0


def general_alpha_from_volume(V: float, nnz: int, beta: float, nnzr: float, C: int, k: int = 1,
                              s: Sizes = Sizes()) -> float:
    """Solve general_balance(alpha, ...) = V / (2 N_nz k) for alpha. Here
    alpha counts x traffic in units of s_x bytes per nonzero and right-hand
    side (alpha = 1/N_nzc: every x element loaded once)."""
    per_nnz = V / (nnz * k)
    return (per_nnz - (s.sv + s.si) / (k * beta) - (s.sy + s.sp / k) / nnzr - s.meta / (k * C * nnzr)) / s.sx


def algorithmic_bytes(nrows: int, ncols: int, padded: int, nchunks: int, k: int = 1, s: Sizes = Sizes()) -> int:
    """Data the method must move in one product when every x element is
    loaded once (alpha = 1/N_nzc): the padded matrix, x, y, the permutation
    and the chunk metadata."""
    return int((s.sv + s.si) * padded + s.sx * ncols * k + s.sy * nrows * k + s.sp * nrows + s.meta * nchunks)


def sizes_for(val_dtype: str, acc_dtype: str, sigma_gt_1: bool, xwindow: bool = False,
              segments_per_chunk: float = 0.0, group_chunks: int = 4) -> Sizes:
    """Element sizes of a product. With the x window staged in LDS the
    streamed index is the 2-byte window position, and each chunk also moves
    its share of the window tables: 8 bytes of group offsets per group of
    group_chunks chunks and 12 bytes per segment."""
    sv = {"f64": 8, "f32": 4, "bf16": 2}[val_dtype]
    sx = 8 if val_dtype == "f64" else 4
    sy = 8 if acc_dtype == "f64" else 4
    if xwindow:
        return Sizes(sv=sv, si=2, sx=sx, sy=sy, sp=4 if sigma_gt_1 else 0, meta=12 + 8 / group_chunks + 12 * segments_per_chunk)
    return Sizes(sv=sv, si=4, sx=sx, sy=sy, sp=4 if sigma_gt_1 else 0)
