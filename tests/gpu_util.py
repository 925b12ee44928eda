"""Helpers of the GPU tests: move synthetic CRS matrices to the device, call
the library through its binding, and compare with the oracle."""
import sys

import numpy as np

import oracle

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


def check_fp64(A, y, x, tol=1e-13, m=None):
    """|y - y_ref|_i <= tol * (|A||x|)_i, y_ref from the long double oracle.
    With m (per-row bound on the roundings a term goes through on the GPU,
    see chain_per_row) the bound is the smaller of tol and the one the
    summation chain guarantees: gamma_{m_i+1} (the +1 covers the rounding of
    y_ref to double) plus the oracle's own long double chain."""
    yh = oracle.crs_spmv_hi(A, x)
    ax = oracle.crs_absmv(A, x)
    err = np.abs(y - yh)
    bound = tol * ax
    if m is not None:
        lens = A.row_lengths()
        g = gamma(np.asarray(m) + 1, U["f64"]) * 1.0001 + gamma(lens, 2.0 ** -64)
        bound = np.minimum(tol, g) * ax
    ok = err <= bound
    assert np.all(np.isfinite(y))
    assert np.all(ok), "max rel err %g at %d" % (np.max(err / np.where(ax > 0, ax, 1)), int(np.argmax(~ok)))
    return float(np.max(err / np.where(ax > 0, ax, 1)))


def chunk_width_per_row(A, lay, C):
    """Width cl of the chunk that stores each original row."""
    inv = np.empty(A.nrows, np.int64)
    inv[lay["perm"]] = np.arange(A.nrows)
    return lay["cl"][inv // C].astype(np.int64)


def chain_per_row(A, h, C, block=False):
    """Per-row bound m_i on the roundings one product term goes through in
    the GPU product of handle h (FMA: one rounding per term added):
      * the terms one lane adds in turn: its share ceil(w / T) of the row's
        chunk width w, T the lanes per row (the block-form kernels keep a
        whole row in one lane, T = 1); of the segment width S instead where
        the chunk is split into segments on different waves;
      * log2(T) cross-lane additions;
      * the additions of a split row's segment sums, in segment order."""
    from paper_1307_6209_amd import sellcs
    inf = h.info
    w = chunk_width_per_row(A, sellcs.sell_export(h, parts=("perm", "cl")), C)
    T = 1 if block else int(inf["lanes_per_row"])
    S = int(inf["seg_cols"])
    split = (inf["nsplit"] > 0) & (w > S)
    nseg = np.where(split, -(-w // S), 0)
    width = np.where(split, S, w)
    return -(-width // T) + (T.bit_length() - 1) + nseg


def batch_chain_per_row(A, h, C):
    """chain_per_row for the batched launch, which loads one slot per lane
    (T = 64 / min(C, 64)) and cuts chunks at a segment width S of its own (a
    multiple of 64, so of T). For a split row S/T + ceil(w/S) <= w/T + 2
    whatever S is (the left side is convex in S and equals w/T + 1 at S = T
    and S = w), so the bound holds without knowing S."""
    from paper_1307_6209_amd import sellcs
    w = chunk_width_per_row(A, sellcs.sell_export(h, parts=("perm", "cl")), C)
    T = 64 // min(C, 64)
    return -(-w // T) + (T.bit_length() - 1) + 2


def rounded_values(A, val_dtype):
    if val_dtype == "f32":
        return oracle.round_f32(A.val).astype(np.float64)
    if val_dtype == "bf16":
        return oracle.bf16_to_f64(oracle.round_bf16(A.val))
    return A.val


def check_reduced(A, h, x, val_dtype, acc, C):
    """Reduced-precision forms, with m_i the per-row chain of chain_per_row
    and u_acc the unit roundoff of the accumulation type. Kernel check
    against y_q (the exact product of the rounded values and rounded x, in
    long double, rounded once to double):
        |y - y_q|_i <= gamma_acc(m_i + 1) (|A^||x^|)_i.
    Against the double product of A and x^:
        |y - A x^|_i <= [u_v + (1 + u_v) gamma_acc(m_i + 1)] (|A||x^|)_i.
    Returns (max componentwise, normwise) error against A x^."""
    xr = oracle.round_f32(x).astype(np.float64)
    return check_reduced_y(A, spmv_gpu(h, xr), h, x, val_dtype, acc, C)


def check_reduced_y(A, y, h, x, val_dtype, acc, C, m=None):
    """The bounds of check_reduced for a result y computed elsewhere (the
    batched launch passes its own chain m) from the layout of handle h."""
    xr = oracle.round_f32(x).astype(np.float64)
    vr = rounded_values(A, val_dtype)
    yq = oracle.crs_spmv_hi(A, xr, val=vr)
    aq = oracle.crs_absmv(A, xr, val=vr)
    if m is None:
        m = chain_per_row(A, h, C)
    ua = U[acc]
    g = gamma(np.asarray(m) + 1, ua) + gamma(A.row_lengths(), 2.0 ** -64)
    assert np.all(np.isfinite(y))
    assert np.all(np.abs(y - yq) <= g * aq * 1.0001 + 1e-300)
    yref = oracle.crs_spmv_hi(A, xr)
    aref = oracle.crs_absmv(A, xr)
    uv = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8}[val_dtype]
    assert np.all(np.abs(y - yref) <= (uv + (1 + uv) * g) * aref * 1.0001 + 1e-300)
    comp = float(np.max(np.abs(y - yref) / np.where(aref > 0, aref, 1)))
    norm = float(np.linalg.norm(y - yref) / max(np.linalg.norm(yref), 1e-300))
    return comp, norm
