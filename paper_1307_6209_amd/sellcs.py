"""Python binding of the SELL-C-sigma C ABI (include/sellcs.h).

Argument marshalling only: every step of the build and of the products runs
in the HIP kernels of libsellcs.so. torch supplies device memory (tensors)
and streams (``torch.cuda.current_stream()`` unless one is given). There is
no CPU path: if the shared library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsellcs.so")
_lib = None

SELL_OK, SELL_ERR_INVALID_ARG, SELL_ERR_BAD_CRS, SELL_ERR_OOM, SELL_ERR_UNSUPPORTED, SELL_ERR_HIP = range(6)
DTYPES = {"f64": 0, "f32": 1, "bf16": 2}
DTYPE_NAMES = {v: k for k, v in DTYPES.items()}


class SellError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__("%s: %s (%s)" % (where, detail, _status_name(status)))


c_i32, c_i64, c_p, c_d = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_double


class SellCrs(ctypes.Structure):
    _fields_ = [("nrows", c_i64), ("ncols", c_i64), ("nnz", c_i64), ("rpt", c_p), ("col", c_p), ("val", c_p)]


class SellAllocator(ctypes.Structure):
    _fields_ = [("alloc", c_p), ("free", c_p), ("ctx", c_p)]


class SellBuildOpts(ctypes.Structure):
    _fields_ = [("val_dtype", ctypes.c_int), ("acc_dtype", ctypes.c_int), ("unroll", c_i32), ("vec", c_i32),
                ("seg_cols", c_i32), ("ktile", c_i32), ("kmax", c_i32), ("permute_columns", c_i32),
                ("xwindow", c_i32), ("alloc", ctypes.POINTER(SellAllocator)), ("xwindow_chunks", c_i32),
                ("row_lengths", c_i32)]


class SellInfo(ctypes.Structure):
    _fields_ = [("nrows", c_i64), ("ncols", c_i64), ("nnz", c_i64), ("C", c_i32), ("sigma", c_i64),
                ("nchunks", c_i64), ("padded", c_i64), ("beta", c_d), ("zeta", c_d), ("max_row_len", c_i64),
                ("val_dtype", ctypes.c_int), ("x_dtype", ctypes.c_int), ("acc_dtype", ctypes.c_int),
                ("lanes_per_row", c_i32), ("unroll", c_i32), ("vec", c_i32), ("seg_cols", c_i32), ("nunits", c_i64),
                ("nsplit", c_i64), ("has_perm", c_i32), ("permuted_columns", c_i32), ("device_bytes", c_i64),
                ("xwindow", c_i32), ("xwindow_max", c_i32), ("xsegments", c_i64), ("xwindow_group_chunks", c_i32),
                ("row_lengths", c_i32)]


class SellTuneSpace(ctypes.Structure):
    _fields_ = [("C", ctypes.POINTER(c_i32)), ("nC", c_i32), ("sigma", ctypes.POINTER(c_i64)), ("nsigma", c_i32),
                ("unroll", ctypes.POINTER(c_i32)), ("nunroll", c_i32), ("ktile", ctypes.POINTER(c_i32)),
                ("nktile", c_i32), ("vec", ctypes.POINTER(c_i32)), ("nvec", c_i32),
                ("seg_cols", ctypes.POINTER(c_i32)), ("nseg_cols", c_i32), ("val_dtype", ctypes.c_int),
                ("acc_dtype", ctypes.c_int), ("reps", c_i32), ("model_guided", c_i32),
                ("xwindow", ctypes.POINTER(c_i32)), ("nxwindow", c_i32),
                ("xwindow_chunks", ctypes.POINTER(c_i32)), ("nxwindow_chunks", c_i32),
                ("row_lengths", ctypes.POINTER(c_i32)), ("nrow_lengths", c_i32)]


class SellTuned(ctypes.Structure):
    _fields_ = [("C", c_i32), ("sigma", c_i64), ("unroll", c_i32), ("ktile", c_i32), ("vec", c_i32),
                ("seg_cols", c_i32), ("gflops", c_d),
                ("us_per_call", c_d), ("beta", c_d), ("candidates", c_i32), ("predicted", c_i32),
                ("xwindow", c_i32), ("xwindow_chunks", c_i32), ("row_lengths", c_i32)]


class SellBatchTuned(ctypes.Structure):
    _fields_ = [("C", c_i32), ("candidates", c_i32), ("gflops", c_d), ("us_per_call", c_d)]


# Every entry point the header declares: name -> (restype, argtypes).
SIGNATURES = {
    "sell_build": (ctypes.c_int, [ctypes.POINTER(SellCrs), c_i32, c_i64, ctypes.POINTER(SellBuildOpts), c_p,
                                  ctypes.POINTER(c_p)]),
    "sell_spmv": (ctypes.c_int, [c_p, c_p, c_p, c_p]),
    "sell_spmmv": (ctypes.c_int, [c_p, c_p, c_p, c_i32, c_p]),
    "sell_spmmv_noalloc": (ctypes.c_int, [c_p, c_p, c_p, c_i32, c_p]),
    "sell_info": (ctypes.c_int, [c_p, ctypes.POINTER(SellInfo)]),
    "sell_export": (ctypes.c_int, [c_p, c_p, c_p, c_p, c_p, c_p]),
    "sell_export_xwindow": (ctypes.c_int, [c_p, c_p, c_p, c_p]),
    "sell_destroy": (ctypes.c_int, [c_p]),
    "sell_batch_create": (ctypes.c_int, [ctypes.POINTER(c_p), c_i32, ctypes.POINTER(c_p)]),
    "sell_batch_create_persistent": (ctypes.c_int, [ctypes.POINTER(c_p), c_i32, ctypes.POINTER(c_p)]),
    "sell_batch_autotune": (ctypes.c_int, [ctypes.POINTER(SellCrs), c_i32, ctypes.POINTER(SellTuneSpace), c_p,
                                           ctypes.POINTER(SellBatchTuned), ctypes.POINTER(c_i64)]),
    "sell_batch_spmv": (ctypes.c_int, [c_p, ctypes.POINTER(c_p), ctypes.POINTER(c_p), c_p]),
    "sell_batch_destroy": (ctypes.c_int, [c_p]),
    "sell_autotune": (ctypes.c_int, [ctypes.POINTER(SellCrs), c_i32, ctypes.POINTER(SellTuneSpace), c_p,
                                     ctypes.POINTER(SellTuned)]),
    "sell_probe_bandwidth": (ctypes.c_int, [c_i32, ctypes.c_size_t, c_i32, c_p, ctypes.POINTER(c_d)]),
    "sell_permute": (ctypes.c_int, [c_p, c_p, c_p, c_p]),
    "sell_unpermute": (ctypes.c_int, [c_p, c_p, c_p, c_p]),
    "sell_crs_spmv": (ctypes.c_int, [ctypes.POINTER(SellCrs), c_i32, c_p, c_p, c_p]),
    "sell_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sell_last_error": (ctypes.c_char_p, []),
}


def hip_runtimes() -> list:
    """Paths of the HIP runtime libraries mapped into this process."""
    found = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                path = line.split()[-1] if line.strip() else ""
                if "libamdhip64.so" in os.path.basename(path):
                    found.add(os.path.realpath(path))
    except OSError:
        pass
    return sorted(found)


def lib():
    """The loaded libsellcs.so (raises if it has not been built).

    torch is imported first: it loads the HIP runtime it ships with, and the
    library then binds to that same runtime (same soname) instead of loading
    a second one from the ROCm install. Two HIP runtimes in one process do
    not share device state, and allocations through the second one fail."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsellcs.so is not built (run: python -m paper_1307_6209_amd._build)")
        import torch  # noqa: F401  (loads torch's HIP runtime before the library)
        L = ctypes.CDLL(LIB_PATH)
        rts = hip_runtimes()
        if len(rts) > 1:
            raise RuntimeError("two HIP runtimes are loaded (%s); import torch before loading libsellcs.so"
                               % ", ".join(rts))
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _status_name(s: int) -> str:
    try:
        return lib().sell_status_string(s).decode()
    except Exception:
        return str(s)


def _check(status: int, where: str):
    if status != SELL_OK:
        raise SellError(status, where, lib().sell_last_error().decode())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dptr(t, dtype, name, numel=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements, got %d" % (name, numel, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


def _torch_dtype(code: int):
    import torch
    return {0: torch.float64, 1: torch.float32}[code]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class TorchAllocator:
    """Device memory for a handle from torch's caching allocator: every block
    the library asks for is a uint8 tensor kept alive until the library frees
    it (sell_destroy synchronises the device before freeing)."""

    def __init__(self, fail_after: int | None = None):
        self.live = {}
        self.calls = 0
        self.frees = 0
        self.fail_after = fail_after  # return NULL from this allocation on (tests)
        self._alloc = ALLOC_FN(self._on_alloc)
        self._free = FREE_FN(self._on_free)
        self.struct = SellAllocator(ctypes.cast(self._alloc, c_p), ctypes.cast(self._free, c_p), None)

    def _on_alloc(self, nbytes, ctx):
        import torch
        self.calls += 1
        if self.fail_after is not None and self.calls > self.fail_after:
            return None
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        except RuntimeError:
            return None
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _on_free(self, ptr, ctx):
        self.frees += 1
        self.live.pop(ptr, None)


class SellMatrix:
    """A device-resident SELL-C-sigma matrix (wraps a sell_handle)."""

    def __init__(self, handle: ctypes.c_void_p, allocator: TorchAllocator | None = None):
        self._h = handle
        self.allocator = allocator  # keeps the callbacks and the blocks alive
        self.info = sell_info(self)

    @property
    def handle(self):
        if not self._h:
            raise ValueError("matrix already destroyed")
        return self._h

    @property
    def x_dtype(self):
        return _torch_dtype(self.info["x_dtype"])

    @property
    def y_dtype(self):
        return _torch_dtype(self.info["acc_dtype"])

    def close(self):
        if self._h:
            _check(lib().sell_destroy(self._h), "sell_destroy")
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None) and not sys.is_finalizing():
                lib().sell_destroy(self._h)
        except Exception:
            pass
        self._h = None


def sell_build(rpt, col, val, ncols: int, C: int, sigma: int, val_dtype: str = "f64", acc_dtype: str | None = None,
               unroll: int = 0, vec: int = 0, seg_cols: int = 0, ktile: int = 0, kmax: int = 0,
               permute_columns: bool = False, xwindow: int = 0, allocator: TorchAllocator | None = None,
               stream=None, xwindow_chunks: int = 0, row_lengths: bool = False) -> SellMatrix:
    """Build SELL-C-sigma from device CRS tensors (rpt int64, col int32, val float64).
    xwindow: 0 stage x windows in LDS when they fit, -1 never, 1 required.
    xwindow_chunks: chunks per window group, 0 auto (8 at C = 32 when they fit), 4 or 8.
    row_lengths: keep every row's length; sell_spmv's lanes then stop at
    their rows' ends (global-index product, C in 8..64; same result bit for bit).
    allocator: a TorchAllocator to take the handle's device memory from
    torch's caching allocator (default: the library's hipMalloc)."""
    import torch
    nrows = rpt.numel() - 1
    nnz = col.numel()
    A = SellCrs(nrows, int(ncols), nnz, _dptr(rpt, torch.int64, "rpt"), _dptr(col, torch.int32, "col"),
                _dptr(val, torch.float64, "val", nnz))
    if acc_dtype is None:
        acc_dtype = "f64" if val_dtype == "f64" else "f32"
    o = SellBuildOpts(DTYPES[val_dtype], DTYPES[acc_dtype], unroll, vec, seg_cols, ktile, kmax,
                      1 if permute_columns else 0, xwindow,
                      ctypes.pointer(allocator.struct) if allocator else None, xwindow_chunks,
                      1 if row_lengths else 0)
    h = c_p()
    _check(lib().sell_build(ctypes.byref(A), C, sigma, ctypes.byref(o), _stream(stream), ctypes.byref(h)), "sell_build")
    return SellMatrix(h, allocator)


def sell_spmv(h: SellMatrix, x, y, stream=None):
    """y = A x on the stream (asynchronous)."""
    xp = _dptr(x, h.x_dtype, "x", h.info["ncols"])
    yp = _dptr(y, h.y_dtype, "y", h.info["nrows"])
    _check(lib().sell_spmv(h.handle, xp, yp, _stream(stream)), "sell_spmv")
    return y


def _block_args(h: SellMatrix, X, Y):
    if X.dim() != 2 or Y.dim() != 2 or X.shape[1] != Y.shape[1]:
        raise ValueError("X and Y must be 2-D with the same number of columns")
    if X.shape[0] != h.info["ncols"] or Y.shape[0] != h.info["nrows"]:
        raise ValueError("X must be ncols x k and Y nrows x k")
    return _dptr(X, h.x_dtype, "X"), _dptr(Y, h.y_dtype, "Y"), X.shape[1]


def sell_spmmv(h: SellMatrix, X, Y, stream=None):
    """Y = A X for row-major X (ncols x k) and Y (nrows x k)."""
    xp, yp, k = _block_args(h, X, Y)
    _check(lib().sell_spmmv(h.handle, xp, yp, k, _stream(stream)), "sell_spmmv")
    return Y


def sell_spmmv_noalloc(h: SellMatrix, X, Y, stream=None):
    """sell_spmmv with the segment sums of split chunks in the library's
    static per-device scratch (no device allocation; k not bounded by the
    kmax given at build; overlapping calls on one device race)."""
    xp, yp, k = _block_args(h, X, Y)
    _check(lib().sell_spmmv_noalloc(h.handle, xp, yp, k, _stream(stream)), "sell_spmmv_noalloc")
    return Y


def sell_info(h: SellMatrix) -> dict:
    info = SellInfo()
    _check(lib().sell_info(h.handle, ctypes.byref(info)), "sell_info")
    return {name: getattr(info, name) for name, _ in SellInfo._fields_}


def sell_export(h: SellMatrix, parts=("perm", "cl", "cs", "col", "val")) -> dict:
    """Host copies (numpy) of perm, cl, cs, col and val (bf16 as uint16 bits);
    only the arrays named in parts are copied."""
    inf = h.info
    vdt = {0: np.float64, 1: np.float32, 2: np.uint16}[inf["val_dtype"]]
    shapes = {"perm": (inf["nrows"], np.int32), "cl": (inf["nchunks"], np.int32), "cs": (inf["nchunks"] + 1, np.int64),
              "col": (inf["padded"], np.int32), "val": (inf["padded"], vdt)}
    out = {k: np.empty(shapes[k][0], shapes[k][1]) for k in parts}
    p = lambda k: ctypes.c_void_p(out[k].ctypes.data) if k in out else None  # noqa: E731
    _check(lib().sell_export(h.handle, p("perm"), p("cl"), p("cs"), p("col"), p("val")), "sell_export")
    return out


def sell_export_xwindow(h: SellMatrix) -> dict:
    """Host copies (numpy) of the x-window tables: segoff (ngroups + 1),
    seg (xsegments x 3: first column, window position, length) and lcol
    (window position of every slot)."""
    inf = h.info
    if not inf["xwindow"]:  # the library reports the error
        _check(lib().sell_export_xwindow(h.handle, None, None, None), "sell_export_xwindow")
    G = inf["xwindow_group_chunks"]
    ngroups = (inf["nchunks"] + G - 1) // G
    out = {"segoff": np.empty(ngroups + 1, np.int64), "seg": np.empty((inf["xsegments"], 3), np.int32),
           "lcol": np.empty(inf["padded"], np.uint16), "group_chunks": G}
    p = lambda k: ctypes.c_void_p(out[k].ctypes.data)  # noqa: E731
    _check(lib().sell_export_xwindow(h.handle, p("segoff"), p("seg"), p("lcol")), "sell_export_xwindow")
    return out


def sell_permute(h: SellMatrix, x, xp, stream=None):
    """xp[p] = x[perm[p]]: caller's order -> sorted order."""
    n = h.info["nrows"]
    _check(lib().sell_permute(h.handle, _dptr(x, h.x_dtype, "x", n), _dptr(xp, h.x_dtype, "xp", n), _stream(stream)),
           "sell_permute")
    return xp


def sell_unpermute(h: SellMatrix, yp, y, stream=None):
    """y[perm[p]] = yp[p]: sorted order -> caller's order."""
    n = h.info["nrows"]
    _check(lib().sell_unpermute(h.handle, _dptr(yp, h.y_dtype, "yp", n), _dptr(y, h.y_dtype, "y", n),
                                _stream(stream)), "sell_unpermute")
    return y


def sell_crs_spmv(rpt, col, val, x, y, ncols: int, lanes_per_row: int = 0, stream=None):
    """y = A x straight from device CRS (FP64), the comparison kernel."""
    import torch
    nrows = rpt.numel() - 1
    nnz = col.numel()
    A = SellCrs(nrows, int(ncols), nnz, _dptr(rpt, torch.int64, "rpt"), _dptr(col, torch.int32, "col"),
                _dptr(val, torch.float64, "val", nnz))
    _check(lib().sell_crs_spmv(ctypes.byref(A), lanes_per_row, _dptr(x, torch.float64, "x", int(ncols)),
                               _dptr(y, torch.float64, "y", nrows), _stream(stream)), "sell_crs_spmv")
    return y


def sell_destroy(h: SellMatrix):
    h.close()


class SellBatch:
    def __init__(self, handle, mats):
        self._h = handle
        self.mats = list(mats)  # keep the matrices alive

    def close(self):
        if self._h:
            _check(lib().sell_batch_destroy(self._h), "sell_batch_destroy")
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None) and not sys.is_finalizing():
                lib().sell_batch_destroy(self._h)
        except Exception:
            pass
        self._h = None


def sell_batch_create(mats) -> SellBatch:
    """One graph-captured launch over all matrices, one wave per work unit."""
    arr = (c_p * len(mats))(*[m.handle for m in mats])
    b = c_p()
    _check(lib().sell_batch_create(arr, len(mats), ctypes.byref(b)), "sell_batch_create")
    return SellBatch(b, mats)


def sell_batch_create_persistent(mats) -> SellBatch:
    """The same batch as one persistent launch (resident waves, equal-cost slices)."""
    arr = (c_p * len(mats))(*[m.handle for m in mats])
    b = c_p()
    _check(lib().sell_batch_create_persistent(arr, len(mats), ctypes.byref(b)), "sell_batch_create_persistent")
    return SellBatch(b, mats)


class BatchVectors:
    """The x and y vectors of a batch, checked and marshalled once: passing
    it to sell_batch_spmv (as xs, with ys None) costs one ctypes call instead
    of checking 2 x count tensors per launch. Keeps the tensors alive."""

    def __init__(self, b: SellBatch, xs, ys):
        n = len(b.mats)
        if len(xs) != n or len(ys) != n:
            raise ValueError("need one x and one y per matrix")
        self.batch = b
        self.tensors = (list(xs), list(ys))
        self.xa = (c_p * n)(*[_dptr(x, m.x_dtype, "xs[%d]" % i, m.info["ncols"]).value
                             for i, (x, m) in enumerate(zip(xs, b.mats))])
        self.ya = (c_p * n)(*[_dptr(y, m.y_dtype, "ys[%d]" % i, m.info["nrows"]).value
                             for i, (y, m) in enumerate(zip(ys, b.mats))])


def sell_batch_spmv(b: SellBatch, xs, ys=None, stream=None):
    """y_i = A_i x_i for every matrix of the batch, one graph launch. xs, ys:
    lists of tensors, or xs a BatchVectors of this batch (ys None)."""
    if isinstance(xs, BatchVectors):
        if xs.batch is not b or ys is not None:
            raise ValueError("a BatchVectors of this batch, and no ys")
        v = xs
    else:
        v = BatchVectors(b, xs, ys)
    _check(lib().sell_batch_spmv(b._h, v.xa, v.ya, _stream(stream)), "sell_batch_spmv")
    return v.tensors[1]


def sell_batch_destroy(b: SellBatch):
    b.close()


def sell_autotune(rpt, col, val, ncols: int, k: int = 1, C=(), sigma=(), unroll=(), ktile=(), vec=(), seg_cols=(),
                  val_dtype: str = "f64", acc_dtype: str | None = None, reps: int = 0, model_guided: int = 0,
                  xwindow=(), stream=None, xwindow_chunks=(), row_lengths=()) -> dict:
    """Time the configurations of the search space (all of them, or the
    model_guided best by the code-balance model); return the fastest.
    row_lengths: values of the row_lengths build option to try (0, 1)."""
    import torch
    nrows = rpt.numel() - 1
    nnz = col.numel()
    A = SellCrs(nrows, int(ncols), nnz, _dptr(rpt, torch.int64, "rpt"), _dptr(col, torch.int32, "col"),
                _dptr(val, torch.float64, "val", nnz))
    if acc_dtype is None:
        acc_dtype = "f64" if val_dtype == "f64" else "f32"
    arrs = [(c_i32 * len(C))(*C), (c_i64 * len(sigma))(*sigma), (c_i32 * len(unroll))(*unroll),
            (c_i32 * len(ktile))(*ktile), (c_i32 * len(vec))(*vec), (c_i32 * len(seg_cols))(*seg_cols)]
    xa = (c_i32 * len(xwindow))(*xwindow)
    wa = (c_i32 * len(xwindow_chunks))(*xwindow_chunks)
    ra = (c_i32 * len(row_lengths))(*[int(v) for v in row_lengths])
    sp = SellTuneSpace(arrs[0], len(C), arrs[1], len(sigma), arrs[2], len(unroll), arrs[3], len(ktile),
                       arrs[4], len(vec), arrs[5], len(seg_cols), DTYPES[val_dtype], DTYPES[acc_dtype], reps,
                       model_guided, xa, len(xwindow), wa, len(xwindow_chunks), ra, len(row_lengths))
    r = SellTuned()
    _check(lib().sell_autotune(ctypes.byref(A), k, ctypes.byref(sp), _stream(stream), ctypes.byref(r)), "sell_autotune")
    return {name: getattr(r, name) for name, _ in SellTuned._fields_}


def sell_batch_autotune(mats, C=(), sigma=(), val_dtype: str = "f64", acc_dtype: str | None = None, reps: int = 0,
                        stream=None) -> dict:
    """One C for the batch and a sigma per matrix (fewest model bytes), the
    fastest C by timing the batched launch. mats: list of (rpt, col, val,
    ncols) device tensors. Returns C, sigmas (per matrix), gflops,
    us_per_call and candidates."""
    import torch
    n = len(mats)
    arr = (SellCrs * n)()
    for i, (rpt, col, val, ncols) in enumerate(mats):
        nnz = col.numel()
        arr[i] = SellCrs(rpt.numel() - 1, int(ncols), nnz, _dptr(rpt, torch.int64, "rpt"),
                         _dptr(col, torch.int32, "col"), _dptr(val, torch.float64, "val", nnz))
    if acc_dtype is None:
        acc_dtype = "f64" if val_dtype == "f64" else "f32"
    ca, sa = (c_i32 * len(C))(*C), (c_i64 * len(sigma))(*sigma)
    empty = (c_i32 * 0)()
    sp = SellTuneSpace(ca, len(C), sa, len(sigma), empty, 0, empty, 0, empty, 0, empty, 0, DTYPES[val_dtype],
                       DTYPES[acc_dtype], reps, 0, empty, 0)
    r = SellBatchTuned()
    sig = (c_i64 * n)()
    _check(lib().sell_batch_autotune(arr, n, ctypes.byref(sp), _stream(stream), ctypes.byref(r), sig),
           "sell_batch_autotune")
    out = {name: getattr(r, name) for name, _ in SellBatchTuned._fields_}
    out["sigmas"] = list(sig)
    return out


def sell_probe_bandwidth(kind: int, nbytes: int, reps: int = 10, stream=None) -> float:
    """Read-only (kind 0) or copy (kind 1) bandwidth in GB/s; kind 2: random
    8-byte gathers over an nbytes array, in gathered GB/s (8 B per gather);
    kinds 3, 4, 5: random rows of 128, 256, 512 bytes, in GB/s of rows;
    kind 6: write-only (16-byte non-temporal stores); kinds 7, 8, 9: rows of
    128, 256, 512 bytes written in order, each the sum of four random rows
    read, in GB/s of rows read and written."""
    g = c_d()
    _check(lib().sell_probe_bandwidth(kind, nbytes, reps, _stream(stream), ctypes.byref(g)), "sell_probe_bandwidth")
    return g.value
