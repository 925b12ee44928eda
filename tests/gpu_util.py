"""Helpers of the GPU tests: move synthetic CRS matrices to the device, call
the library through its binding, and compare with the oracle."""
import sys

import numpy as np

import oracle
import synth

U = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch():
    import torch as t
    return t


def dev_crs(A):
    t = torch()
    return (t.from_numpy(np.ascontiguousarray(A.rpt)).cuda(), t.from_numpy(np.ascontiguousarray(A.col)).cuda(),
            t.from_numpy(np.ascontiguousarray(A.val)).cuda())


def build(A, C, sigma, **kw):
    from paper_1307_6209_amd import sellcs
    rpt, col, val = dev_crs(A)
    h = sellcs.sell_build(rpt, col, val, A.ncols, C, sigma, **kw)
    torch().cuda.synchronize()
    return h


def assert_layout_equal(A, h, C, sigma, val_dtype="f64"):
    """Bit-exact comparison of perm, cl, cs, col and the value bits."""
    from paper_1307_6209_amd import sellcs
    got = sellcs.sell_export(h)
    want = oracle.sell_build(A, C, sigma, val_dtype)
    for key in ["perm", "cl", "cs", "col"]:
        assert np.array_equal(got[key], want[key]), key
    wv = want["val"]
    assert got["val"].dtype.itemsize == wv.dtype.itemsize
    gb = got["val"].view(np.uint64 if wv.itemsize == 8 else np.uint32 if wv.itemsize == 4 else np.uint16)
    wb = wv.view(gb.dtype)
    assert np.array_equal(gb, wb), "val bits"
    inf = h.info
    assert inf["padded"] == want["padded"] and inf["nchunks"] == want["nchunks"]
    assert inf["beta"] == want["beta"]
    return want


def gamma(m, u):
    m = np.asarray(m, np.float64)
    return m * u / (1 - m * u)


def spmv_gpu(h, x_np, dtype=None):
    t = torch()
    xd = t.from_numpy(np.ascontiguousarray(x_np)).cuda().to(h.x_dtype)
    y = t.full((h.info["nrows"],), float("nan"), dtype=h.y_dtype, device="cuda")
    from paper_1307_6209_amd import sellcs
    sellcs.sell_spmv(h, xd, y)
    t.cuda.synchronize()
    return y.double().cpu().numpy()


def check_fp64(A, y, x, tol=1e-13):
    """|y - y_ref|_i <= tol * (|A||x|)_i, y_ref from the long double oracle."""
    yh = oracle.crs_spmv_hi(A, x)
    ax = oracle.crs_absmv(A, x)
    err = np.abs(y - yh)
    ok = err <= tol * ax
    assert np.all(np.isfinite(y))
    assert np.all(ok), "max rel err %g at %d" % (np.max(err / np.where(ax > 0, ax, 1)), int(np.argmax(~ok)))
    return float(np.max(err / np.where(ax > 0, ax, 1)))


def chunk_width_per_row(A, lay, C):
    """Width cl of the chunk that stores each original row."""
    inv = np.empty(A.nrows, np.int64)
    inv[lay["perm"]] = np.arange(A.nrows)
    return lay["cl"][inv // C].astype(np.int64)


def rounded_values(A, val_dtype):
    if val_dtype == "f32":
        return oracle.round_f32(A.val).astype(np.float64)
    if val_dtype == "bf16":
        return oracle.bf16_to_f64(oracle.round_bf16(A.val))
    return A.val


def check_reduced(A, h, x, val_dtype, acc, C, nseg_max=1):
    """Reduced-precision forms. Kernel check against y_q (the exact product of
    the rounded values and rounded x, in long double):
        |y - y_q|_i <= gamma_acc(m_i) (|A^||x^|)_i,
    m_i = chunk width + log2(64) + nseg + 1 (a bound on the summation chain).
    Against the double product of A and x^:
        |y - A x^|_i <= [u_v + (1 + u_v) gamma_acc(m_i)] (|A||x^|)_i.
    Returns (max componentwise, normwise) error against A x^."""
    xr = oracle.round_f32(x).astype(np.float64)
    return check_reduced_y(A, spmv_gpu(h, xr), h, x, val_dtype, acc, C, nseg_max)


def check_reduced_y(A, y, h, x, val_dtype, acc, C, nseg_max=1):
    """The bounds of check_reduced for a result y computed elsewhere (the
    batched launch) from the layout of handle h."""
    from paper_1307_6209_amd import sellcs
    xr = oracle.round_f32(x).astype(np.float64)
    vr = rounded_values(A, val_dtype)
    yq = oracle.crs_spmv_hi(A, xr, val=vr)
    aq = oracle.crs_absmv(A, xr, val=vr)
    lay = sellcs.sell_export(h)
    m = chunk_width_per_row(A, lay, C) + 8 + nseg_max
    ua = 2.0 ** -53 if acc == "f64" else 2.0 ** -24
    g = gamma(m, ua)
    assert np.all(np.isfinite(y))
    assert np.all(np.abs(y - yq) <= g * aq * 1.0001 + 1e-300)
    yref = oracle.crs_spmv_hi(A, xr)
    aref = oracle.crs_absmv(A, xr)
    uv = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8}[val_dtype]
    assert np.all(np.abs(y - yref) <= (uv + (1 + uv) * g) * aref * 1.0001 + 1e-300)
    comp = float(np.max(np.abs(y - yref) / np.where(aref > 0, aref, 1)))
    norm = float(np.linalg.norm(y - yref) / max(np.linalg.norm(yref), 1e-300))
    return comp, norm
