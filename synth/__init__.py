"""Seeded synthetic inputs: CRS matrices and dense vectors.

This package produces inputs only. It holds none of the SELL-C-sigma
arithmetic and imports neither the oracle nor the GPU library; both of
those consume what it returns. The numbers come from a counter-based
splitmix64 (see ``gen.c``), so every array is a pure function of its seed.

Workload shapes follow the regimes the paper evaluates (Sect. 2.2, Table of
test matrices): a small cache-resident stencil, a large regular stencil with
many entries per row, and an irregular matrix with few entries per row and a
high coefficient of variation of the row lengths. The paper's own test
matrices are not reproduced; these generators stand in for them.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None

# Seeds of the standard workloads (structure / values / x / batch sizes).
SEED_STRUCT, SEED_VAL, SEED_X, SEED_BATCH = 1001, 1002, 1003, 1004


def build(force: bool = True) -> str:
    """Compile gen.c into libsynth.so with gcc."""
    global _lib
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, u64, d, p = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
        lib.synth_draw_u64.argtypes = [u64, u64, u64]
        lib.synth_draw_u64.restype = u64
        lib.synth_u64.argtypes = [u64, u64, u64, i64, p]
        lib.synth_uniform.argtypes = [u64, u64, d, d, i64, p]
        lib.synth_lap5_size.argtypes = [i64, p, p]
        lib.synth_lap5.argtypes = [i64, p, p, p]
        lib.synth_stencil27_size.argtypes = [i64, p, p]
        lib.synth_stencil27.argtypes = [i64, u64, d, d, ctypes.c_int, p, p, p]
        lib.synth_powerlaw_lengths.argtypes = [i64, u64, d, i64, i64, p]
        lib.synth_powerlaw_fill.argtypes = [i64, u64, i64, p, p, p]
        lib.synth_powerlaw_fill.restype = ctypes.c_int
        lib.synth_uniform_fill.argtypes = [i64, i64, u64, p, p, p]
        lib.synth_uniform_fill.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


@dataclass
class CRS:
    """A sparse matrix in CRS form: row i holds val[rpt[i]:rpt[i+1]] at
    columns col[rpt[i]:rpt[i+1]]."""
    nrows: int
    ncols: int
    rpt: np.ndarray  # int64[nrows + 1]
    col: np.ndarray  # int32[nnz]
    val: np.ndarray  # float64[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rpt[-1]) if self.rpt.size else 0

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.rpt)


# ---------------------------------------------------------------- vectors
def u64(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    if count:
        _L().synth_u64(seed, stream, start, count, _ptr(out))
    return out


def uniform(count: int, seed: int = SEED_X, stream: int = 0, a: float = -1.0, b: float = 1.0) -> np.ndarray:
    """count values a + (b - a) * U[0,1) (float64)."""
    out = np.empty(count, dtype=np.float64)
    if count:
        _L().synth_uniform(seed, stream, a, b, count, _ptr(out))
    return out


def block_vector(nrows: int, k: int, seed: int = SEED_X, stream: int = 0) -> np.ndarray:
    """Row-major nrows x k block of U[-1,1) values."""
    return uniform(nrows * k, seed, stream).reshape(nrows, k)


# --------------------------------------------------------------- matrices
def lap5(m: int) -> CRS:
    """2D 5-point Laplacian over an m x m grid (diagonal 4, neighbours -1)."""
    n, nnz = ctypes.c_int64(), ctypes.c_int64()
    _L().synth_lap5_size(m, ctypes.byref(n), ctypes.byref(nnz))
    rpt = np.zeros(n.value + 1, np.int64)
    col = np.empty(nnz.value, np.int32)
    val = np.empty(nnz.value, np.float64)
    _L().synth_lap5(m, _ptr(rpt), _ptr(col), _ptr(val))
    return CRS(n.value, n.value, rpt, col, val, name="lap5_m%d" % m)


def stencil27(m: int, seed: int = SEED_VAL, lo: float = 0.5, hi: float = 1.5, ones: bool = False) -> CRS:
    """3D 27-point stencil over an m^3 grid, values U[lo,hi) (or all ones)."""
    n, nnz = ctypes.c_int64(), ctypes.c_int64()
    _L().synth_stencil27_size(m, ctypes.byref(n), ctypes.byref(nnz))
    rpt = np.zeros(n.value + 1, np.int64)
    col = np.empty(nnz.value, np.int32)
    val = np.empty(nnz.value, np.float64)
    _L().synth_stencil27(m, seed, lo, hi, 1 if ones else 0, _ptr(rpt), _ptr(col), _ptr(val))
    return CRS(n.value, n.value, rpt, col, val, name="stencil27_m%d" % m)


def powerlaw_lengths(n: int, seed: int = SEED_STRUCT, expo: float = 2.1, lmin: int = 1, lmax: int = 10000) -> np.ndarray:
    out = np.empty(n, np.int64)
    if n:
        _L().synth_powerlaw_lengths(n, seed, expo, lmin, lmax, _ptr(out))
    return out


def powerlaw(n: int, seed: int = SEED_STRUCT, expo: float = 2.1, lmin: int = 1, lmax: int = 10000,
             band: int = 1000) -> CRS:
    """Square n x n matrix with truncated power-law row lengths; half of the
    entries in a band around the diagonal, half uniform; values N(0,1)."""
    lens = powerlaw_lengths(n, seed, expo, lmin, lmax)
    rpt = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=rpt[1:])
    nnz = int(rpt[-1])
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    rc = _L().synth_powerlaw_fill(n, seed, band, _ptr(rpt), _ptr(col), _ptr(val))
    if rc != 0:
        raise RuntimeError("powerlaw generator could not place distinct columns")
    return CRS(n, n, rpt, col, val, name="powerlaw_n%d_s%d" % (n, seed))


def random_crs(nrows: int, ncols: int, seed: int, max_len: int, empty_frac: float = 0.2,
               duplicates: bool = False, unsorted: bool = False, integer_values: bool = False) -> CRS:
    """Small random CRS matrix for tests: lengths U{0..max_len} (a fraction
    of rows forced empty), columns uniform (optionally with repeated column
    ids and unsorted), values U[-1,1) or small integers in [-4, 4]."""
    r_len = u64(seed, 11, nrows)
    r_empty = u64(seed, 12, nrows)
    lens = (r_len % np.uint64(max_len + 1)).astype(np.int64)
    lens[(r_empty >> np.uint64(11)).astype(np.float64) * 2.0**-53 < empty_frac] = 0
    if not duplicates:
        lens = np.minimum(lens, ncols)
    rpt = np.zeros(nrows + 1, np.int64)
    np.cumsum(lens, out=rpt[1:])
    nnz = int(rpt[-1])
    col = np.empty(nnz, np.int32)
    for i in range(nrows):
        a, b = int(rpt[i]), int(rpt[i + 1])
        if b == a:
            continue
        r = u64(seed, 13, b - a, start=a)
        if duplicates:
            c = (r % np.uint64(ncols)).astype(np.int32)
        else:
            # distinct columns: rank the row's draws against a seeded key per column
            keys = u64(seed + i + 1, 14, ncols)
            c = np.argsort(keys, kind="stable")[: b - a].astype(np.int32)
        if not unsorted:
            c = np.sort(c)
        col[a:b] = c
    if integer_values:
        val = ((u64(seed, 15, nnz) % np.uint64(9)).astype(np.int64) - 4).astype(np.float64)
    else:
        val = uniform(nnz, seed, 16)
    return CRS(nrows, ncols, rpt, col, val, name="random_%dx%d_s%d" % (nrows, ncols, seed))


def worst_case_beta(C: int, nchunks: int) -> CRS:
    """Matrix of the occupancy worst case (Sect. 3.4, Eq. betaworst): N =
    nchunks*C rows and columns; the first row of every chunk is full (N
    entries), every other row holds one entry (on its diagonal)."""
    n = C * nchunks
    lens = np.ones(n, np.int64)
    lens[::C] = n
    rpt = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=rpt[1:])
    col = np.empty(int(rpt[-1]), np.int32)
    for i in range(n):
        a, b = int(rpt[i]), int(rpt[i + 1])
        col[a:b] = np.arange(n, dtype=np.int32) if b - a == n else i
    val = uniform(int(rpt[-1]), 7, 17)
    return CRS(n, n, rpt, col, val, name="worstbeta_C%d_x%d" % (C, nchunks))


def rail_like(nrows: int = 4284, ncols: int = 1_092_610, mean_len: float = 2633.0, zeta: float = 1.6,
              seed: int = SEED_STRUCT + 5) -> CRS:
    """Few rows, very many columns (the shape of an LP constraint matrix such
    as the paper's rail4284): row lengths lognormal with the given mean and
    coefficient of variation zeta (capped at ncols/2, at least 1), columns
    uniform without repetition, values N(0,1)."""
    s2 = math.log(1.0 + zeta * zeta)
    mu = math.log(mean_len) - s2 / 2.0
    u1 = 1.0 - uniform(nrows, seed, 20, 0.0, 1.0)
    u2 = uniform(nrows, seed, 21, 0.0, 1.0)
    g = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    lens = np.clip(np.round(np.exp(mu + math.sqrt(s2) * g)), 1, ncols // 2).astype(np.int64)
    rpt = np.zeros(nrows + 1, np.int64)
    np.cumsum(lens, out=rpt[1:])
    nnz = int(rpt[-1])
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    if _L().synth_uniform_fill(nrows, ncols, seed, _ptr(rpt), _ptr(col), _ptr(val)) != 0:
        raise RuntimeError("rail_like generator could not place distinct columns")
    return CRS(nrows, ncols, rpt, col, val, name="rail_like_%dx%d" % (nrows, ncols))


def dense(nrows: int, ncols: int, seed: int = SEED_VAL) -> CRS:
    """Fully populated nrows x ncols matrix in CRS, values U[-1,1)."""
    rpt = np.arange(nrows + 1, dtype=np.int64) * ncols
    col = np.tile(np.arange(ncols, dtype=np.int32), nrows)
    val = uniform(nrows * ncols, seed, 18)
    return CRS(nrows, ncols, rpt, col, val, name="dense_%dx%d" % (nrows, ncols))


def batch_sizes(count: int, seed: int = SEED_BATCH, lo: float = 1e3, hi: float = 2e5) -> np.ndarray:
    """count sizes floor(exp(U[ln lo, ln hi)))."""
    u = uniform(count, seed, 19, 0.0, 1.0)
    return np.floor(np.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * u)).astype(np.int64)


# ------------------------------------------------------- standard workloads
def workload(name: str):
    """The standard workloads by name. Returns a CRS matrix."""
    if name == "lap5_128":
        return lap5(128)
    if name == "powerlaw_2m":
        return powerlaw(2_000_000, seed=SEED_STRUCT + 1)
    if name == "stencil27_160":
        return stencil27(160, seed=SEED_VAL + 2)
    if name == "powerlaw_1m":
        return powerlaw(1_000_000, seed=SEED_STRUCT + 3)
    if name == "dense_8000":
        return dense(8000, 8000, seed=SEED_VAL + 5)
    if name == "rail_like":
        return rail_like()
    raise KeyError(name)


def batch_workload(count: int = 64, seed: int = SEED_BATCH + 3):
    """count power-law matrices with log-uniform sizes in [1e3, 2e5)."""
    sizes = batch_sizes(count, seed)
    return [powerlaw(int(nb), seed=SEED_STRUCT + 100 + b) for b, nb in enumerate(sizes)]
