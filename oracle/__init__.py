"""CPU oracle for SELL-C-sigma spMVM (see ``oracle.c`` for the definitions).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``. The GPU library never imports,
links or calls it, and it shares no code with the GPU library.

All arrays are numpy. Matrices are ``synth.CRS``-like objects with fields
``nrows, ncols, rpt (int64), col (int32), val (float64)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

# CFLAGS of the oracle: no contraction into fused multiply-add, so the CRS
# sums are reproducible bit for bit on any x86-64 host.
CFLAGS = ["-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc."""
    global _lib
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = configure(ctypes.CDLL(_LIB))
    return _lib


def configure(lib):
    """Declare the C signatures on a loaded oracle library."""
    if True:
        i64, i32, p, d = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double
        lib.or_crs_validate.argtypes = [i64, i64, i64, p, p]
        lib.or_crs_validate.restype = ctypes.c_int
        lib.or_crs_spmv.argtypes = [i64, p, p, p, p, p, ctypes.c_int, ctypes.c_int]
        lib.or_crs_spmv_ld.argtypes = [i64, p, p, p, p, p]
        lib.or_crs_absmv.argtypes = [i64, p, p, p, p, p]
        lib.or_crs_spmmv_ld.argtypes = [i64, p, p, p, p, i64, p, p]
        lib.or_sell_layout.argtypes = [i64, p, i32, i64, p, p, p]
        lib.or_sell_layout.restype = ctypes.c_int
        lib.or_sell_fill.argtypes = [i64, p, p, p, i32, p, p, p, p, p]
        lib.or_crs_symperm.argtypes = [i64, p, p, p, p, p, p, p]
        lib.or_crs_symperm.restype = ctypes.c_int
        lib.or_sell_beta.argtypes = [i64, i64]
        lib.or_sell_beta.restype = d
        lib.or_row_zeta.argtypes = [i64, p]
        lib.or_row_zeta.restype = d
        lib.or_sell_spmv.argtypes = [i64, i32, p, p, p, p, p, p, p]
        lib.or_round_f32.argtypes = [i64, p, p]
        lib.or_round_bf16.argtypes = [i64, p, p]
        lib.or_bf16_to_f64.argtypes = [i64, p, p]
    return lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _arrays(A):
    """Contiguous (rpt int64, col int32, val float64) views/copies of A. The
    caller keeps them in locals for the duration of the C call."""
    return _c(A.rpt, np.int64), _c(A.col, np.int32), _c(A.val, np.float64)


# ------------------------------------------------------------------ CRS
def crs_validate(A) -> int:
    """0 if the CRS arrays are well formed, else a nonzero reason code."""
    rpt, col = _c(A.rpt, np.int64), _c(A.col, np.int32)
    return int(_L().or_crs_validate(A.nrows, A.ncols, int(col.size), _p(rpt), _p(col)))


def schedule_for(A) -> int:
    """OpenMP schedule of the paper's CPU runs (Sect. 5): STATIC (0) when the
    coefficient of variation of the row lengths is below 0.4, else GUIDED,1
    (1). (The paper also uses STATIC when the matrix fits the last-level
    cache; the workloads here do not.)"""
    return 0 if row_zeta(A) < 0.4 else 1


def crs_spmv(A, x, nthreads: int = 1, sched: int | None = None) -> np.ndarray:
    """y = A x in double, CRS order, no fused multiply-add (Listing CRS)."""
    x = _c(x, np.float64)
    rpt, col, val = _arrays(A)
    y = np.empty(A.nrows, np.float64)
    if sched is None:
        sched = schedule_for(A)
    _L().or_crs_spmv(A.nrows, _p(rpt), _p(col), _p(val), _p(x), _p(y), nthreads, sched)
    return y


def crs_spmv_hi(A, x, val=None) -> np.ndarray:
    """y = A x accumulated in long double, rounded once. ``val`` overrides
    the matrix values (e.g. values already rounded to a narrower format)."""
    x = _c(x, np.float64)
    v = _c(A.val if val is None else val, np.float64)
    y = np.empty(A.nrows, np.float64)
    rpt, col, _ = _arrays(A)
    _L().or_crs_spmv_ld(A.nrows, _p(rpt), _p(col), _p(v), _p(x), _p(y))
    return y


def crs_absmv(A, x, val=None) -> np.ndarray:
    """(|A| |x|)_i, the scale of componentwise error bounds."""
    x = _c(x, np.float64)
    v = _c(A.val if val is None else val, np.float64)
    y = np.empty(A.nrows, np.float64)
    rpt, col, _ = _arrays(A)
    _L().or_crs_absmv(A.nrows, _p(rpt), _p(col), _p(v), _p(x), _p(y))
    return y


def crs_spmmv_hi(A, X, val=None):
    """(Y, |A||X|) for row-major X (ncols x k): column v of Y is the CRS
    product with column v of X, accumulated in long double."""
    X = _c(X, np.float64)
    k = X.shape[1]
    v = _c(A.val if val is None else val, np.float64)
    Y = np.empty((A.nrows, k), np.float64)
    aY = np.empty((A.nrows, k), np.float64)
    rpt, col, _ = _arrays(A)
    _L().or_crs_spmmv_ld(A.nrows, _p(rpt), _p(col), _p(v), _p(X), k, _p(Y), _p(aY))
    return Y, aY


# ------------------------------------------------------------------ SELL
def sell_layout(A, C: int, sigma: int):
    """(perm, cl, cs): the sigma-window row order, chunk widths and chunk
    start offsets of SELL-C-sigma."""
    n = A.nrows
    nc = (n + C - 1) // C
    perm = np.empty(n, np.int32)
    cl = np.empty(nc, np.int32)
    cs = np.empty(nc + 1, np.int64)
    rpt = _c(A.rpt, np.int64)
    rc = _L().or_sell_layout(n, _p(rpt), C, sigma, _p(perm), _p(cl), _p(cs))
    if rc != 0:
        raise ValueError("or_sell_layout failed (C=%d sigma=%d)" % (C, sigma))
    return perm, cl, cs


def crs_symperm(A, perm):
    """P A P^T: row p is row perm[p] of A with columns renamed by the inverse
    permutation (square matrices)."""
    if A.nrows != A.ncols:
        raise ValueError("symmetric permutation needs a square matrix")
    rpt, col, val = _arrays(A)
    perm = _c(perm, np.int32)
    rpt2 = np.empty(A.nrows + 1, np.int64)
    col2 = np.empty(col.size, np.int32)
    val2 = np.empty(col.size, np.float64)
    rc = _L().or_crs_symperm(A.nrows, _p(rpt), _p(col), _p(val), _p(perm), _p(rpt2), _p(col2), _p(val2))
    if rc != 0:
        raise MemoryError("or_crs_symperm")
    return type(A)(A.nrows, A.ncols, rpt2, col2, val2)


def sell_build(A, C: int, sigma: int, val_dtype: str = "f64", permute_columns: bool = False) -> dict:
    """The full SELL-C-sigma representation of A as a dict of numpy arrays:
    perm, cl, cs, col, val (float64, or float32, or bfloat16 bits as uint16),
    plus nchunks, padded, beta, zeta. With permute_columns the stored matrix
    is P A P^T in sorted row order (its own row order is the identity) and
    perm is the sort of A."""
    if permute_columns:
        perm, _, _ = sell_layout(A, C, sigma)
        S = sell_build(crs_symperm(A, perm), C, 1, val_dtype)
        S["perm"] = perm
        S["sigma"] = sigma
        S["zeta"] = row_zeta(A)
        return S
    perm, cl, cs = sell_layout(A, C, sigma)
    padded = int(cs[-1])
    scol = np.empty(padded, np.int32)
    sval = np.empty(padded, np.float64)
    rpt, col, val = _arrays(A)
    _L().or_sell_fill(A.nrows, _p(rpt), _p(col), _p(val), C, _p(perm), _p(cl), _p(cs), _p(scol), _p(sval))
    out = dict(perm=perm, cl=cl, cs=cs, col=scol, val_f64=sval, nchunks=cl.size, padded=padded, C=C, sigma=sigma,
               beta=beta(A.nnz, padded), zeta=row_zeta(A))
    if val_dtype == "f64":
        out["val"] = sval
    elif val_dtype == "f32":
        out["val"] = round_f32(sval)
    elif val_dtype == "bf16":
        out["val"] = round_bf16(sval)
    else:
        raise ValueError(val_dtype)
    return out


def sell_spmv(S: dict, nrows: int, x) -> np.ndarray:
    """y = A x from the SELL arrays (double values), y in original row order."""
    x = _c(x, np.float64)
    y = np.empty(nrows, np.float64)
    _L().or_sell_spmv(nrows, S["C"], _p(S["perm"]), _p(S["cl"]), _p(S["cs"]), _p(S["col"]), _p(S["val_f64"]),
                      _p(x), _p(y))
    return y


def beta(nnz: int, padded: int) -> float:
    """Chunk occupancy, Eq. (beta)."""
    return float(_L().or_sell_beta(int(nnz), int(padded)))


def row_zeta(A) -> float:
    """Coefficient of variation of the row lengths, Eq. (eq:cv)."""
    rpt = _c(A.rpt, np.int64)
    return float(_L().or_row_zeta(A.nrows, _p(rpt)))


# ------------------------------------------------------------- rounding
def round_f32(a) -> np.ndarray:
    a = _c(a, np.float64)
    out = np.empty(a.shape, np.float32)
    _L().or_round_f32(a.size, _p(a), _p(out))
    return out


def round_bf16(a) -> np.ndarray:
    """bfloat16 bit patterns (uint16) of a, round to nearest even."""
    a = _c(a, np.float64)
    out = np.empty(a.shape, np.uint16)
    _L().or_round_bf16(a.size, _p(a), _p(out))
    return out


def bf16_to_f64(b) -> np.ndarray:
    b = _c(b, np.uint16)
    out = np.empty(b.shape, np.float64)
    _L().or_bf16_to_f64(b.size, _p(b), _p(out))
    return out
