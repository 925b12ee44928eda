"""The x window staged in LDS (xwindow build option): the product equals the
global-index product bit for bit (same lanes, same order of the multiply-adds;
padding reads x[0] through the window as it does directly), stays within the
oracle's bound, leaves the exported layout unchanged, falls back silently
when a window does not fit, and is refused with an error when required but
impossible."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_layout_equal, build, check_fp64, check_reduced, say, spmv_gpu
from xwindow_def import window_tables

pytestmark = pytest.mark.gpu


def banded(n, seed, half=40, max_len=30):
    """Random rows whose columns lie within +-half of the diagonal."""
    A = synth.random_crs(n, n, seed=seed, max_len=max_len, empty_frac=0.15)
    lens = np.diff(A.rpt)
    rows = np.repeat(np.arange(n), lens)
    col = np.clip(rows + (A.col.astype(np.int64) % (2 * half + 1)) - half, 0, n - 1)
    # keep each row's columns sorted and distinct enough for a CRS
    out = []
    for i in range(n):
        c = np.unique(col[A.rpt[i]:A.rpt[i + 1]])
        out.append(c)
    rpt = np.zeros(n + 1, np.int64)
    np.cumsum([len(c) for c in out], out=rpt[1:])
    cc = np.concatenate(out).astype(np.int32) if rpt[-1] else np.zeros(0, np.int32)
    val = synth.uniform(int(rpt[-1]), seed, 3)
    return synth.CRS(n, n, rpt, cc, val)


def fits_group(A, C, sigma, gc, x_bytes=8):
    """Whether the required window of groups of gc chunks can be built: every
    group holds at most 8,192 slots and 1,024 runs of consecutive columns,
    and its window at most 16 KiB per chunk of the group."""
    lay = oracle.sell_build(A, C, sigma)
    cs = lay["cs"]
    nc = cs.size - 1
    starts = np.arange(0, nc, gc)
    if int(np.max(cs[np.minimum(starts + gc, nc)] - cs[starts])) > 8192:
        return False
    segoff, seg, _ = window_tables(lay["col"], cs, gc)
    runs = np.diff(segoff)
    win = np.add.reduceat(seg[:, 2], segoff[:-1][runs > 0]) if seg.shape[0] else np.zeros(1, np.int64)
    return int(runs.max()) <= 1024 and int(win.max()) * x_bytes <= (16 << 10) * gc


def build_or_refused(A, C, sigma, gc, **kw):
    """The window build with groups of gc chunks, or None after checking that
    it is refused because a group holds too many slots."""
    from paper_1307_6209_amd import sellcs
    if fits_group(A, C, sigma, gc):
        return build(A, C, sigma, xwindow=1, xwindow_chunks=gc, **kw)
    with pytest.raises(sellcs.SellError) as e:
        build(A, C, sigma, xwindow=1, xwindow_chunks=gc, **kw)
    assert e.value.status == sellcs.SELL_ERR_UNSUPPORTED
    return None


MATS = [
    ("stencil27_24", lambda: synth.stencil27(24)),
    ("lap5_96", lambda: synth.lap5(96)),
    ("banded_3000", lambda: banded(3000, 7)),
]


@pytest.mark.parametrize("gc", [4, 8])
@pytest.mark.parametrize("name,make", MATS, ids=[m[0] for m in MATS])
@pytest.mark.parametrize("C,sigma,vec", [(32, 1, 0), (32, 1, 1), (8, 1, 2), (16, 64, 0), (64, 1, 0), (64, 4096, 1),
                                         (32, 10**9, 2)])
def test_window_equals_global_index_product(name, make, C, sigma, vec, gc):
    """Groups of 4 and of 8 chunks (one workgroup of 4 or 8 waves)."""
    A = make()
    x = synth.uniform(A.ncols, 31, 1)
    on = build_or_refused(A, C, sigma, gc, vec=vec)
    if on is None:
        return
    off = build(A, C, sigma, vec=vec, xwindow=-1)
    inf = on.info
    say("xwindow", name, "C", C, "sigma", sigma, "vec", inf["vec"], "chunks", gc, "window", inf["xwindow_max"],
        "segments", inf["xsegments"])
    assert inf["xwindow"] == 1 and off.info["xwindow"] == 0 and inf["xwindow_group_chunks"] == gc
    y_on, y_off = spmv_gpu(on, x), spmv_gpu(off, x)
    assert np.array_equal(y_on.view(np.uint64), y_off.view(np.uint64))
    check_fp64(A, y_on, x)
    assert_layout_equal(A, on, C, sigma)


@pytest.mark.parametrize("val_dtype,acc", [("f32", "f32"), ("f32", "f64"), ("bf16", "f32"), ("bf16", "f64")])
@pytest.mark.parametrize("C", [32, 64])
@pytest.mark.parametrize("vec", [1, 2, 4])
def test_window_reduced_precision_bitwise(val_dtype, acc, C, vec):
    A = synth.stencil27(20)
    x = oracle.round_f32(synth.uniform(A.ncols, 32, 1)).astype(np.float64)
    on = build(A, C, 1, val_dtype=val_dtype, acc_dtype=acc, vec=vec, xwindow=1)
    off = build(A, C, 1, val_dtype=val_dtype, acc_dtype=acc, vec=vec, xwindow=-1)
    assert on.info["xwindow"] == 1 and on.info["vec"] == vec
    y_on, y_off = spmv_gpu(on, x), spmv_gpu(off, x)
    assert np.array_equal(y_on, y_off)
    comp, norm = check_reduced(A, on, x, val_dtype, acc, C)
    say("window", val_dtype, acc, "C", C, "vec", vec, "componentwise %.3g normwise %.3g" % (comp, norm))


def test_window_default_slots_per_lane():
    """With the window, FP32/BF16 values default to two slots per lane; the
    plain kernel keeps one. With two slots per lane the window kernel keeps
    sixteen in flight (eight wave steps) by default; the plain kernel takes
    an unroll of 16 as 8."""
    A = synth.stencil27(64)
    on = build(A, 64, 1, val_dtype="bf16", acc_dtype="f32").info
    assert on["vec"] == 2 and on["unroll"] == 16
    off = build(A, 64, 1, val_dtype="bf16", acc_dtype="f32", xwindow=-1).info
    assert off["vec"] == 1 and off["unroll"] == 8
    assert build(A, 32, 1).info["vec"] == 2 and build(A, 32, 1).info["unroll"] == 16
    assert build(A, 32, 1, unroll=16, xwindow=-1).info["unroll"] == 8
    assert build(A, 32, 1, unroll=16, vec=1).info["unroll"] == 8
    assert build(A, 32, 1, unroll=4).info["unroll"] == 4


@pytest.mark.parametrize("C", [8, 16, 32, 64])
@pytest.mark.parametrize("unroll", [4, 8, 16])
@pytest.mark.parametrize("val_dtype,acc", [("f64", "f64"), ("bf16", "f32")])
def test_window_unroll_equals_global_index_product(C, unroll, val_dtype, acc):
    """Every batch depth of the window kernel (two slots per lane) against
    the global-index product: the same multiply-adds in the same order, so
    the results agree bit for bit; a banded matrix with ragged rows leaves
    partial last steps and chunks shorter than one batch."""
    A = banded(2500, 11, half=30, max_len=30)
    x = synth.uniform(A.ncols, 35, 1)
    if val_dtype != "f64":
        x = oracle.round_f32(x).astype(np.float64)
    on = build(A, C, 1, val_dtype=val_dtype, acc_dtype=acc, vec=2, unroll=unroll, xwindow=1)
    off = build(A, C, 1, val_dtype=val_dtype, acc_dtype=acc, vec=2, xwindow=-1)
    assert on.info["xwindow"] == 1 and on.info["unroll"] == unroll
    y_on, y_off = spmv_gpu(on, x), spmv_gpu(off, x)
    assert np.array_equal(y_on, y_off)
    if val_dtype == "f64":
        check_fp64(A, y_on, x)


def test_window_symmetric_mode():
    import torch
    from paper_1307_6209_amd import sellcs
    A = synth.stencil27(16)
    x = synth.uniform(A.ncols, 33, 1)
    hs = [build(A, 32, 256, permute_columns=True, xwindow=w) for w in (1, -1)]
    assert hs[0].info["xwindow"] == 1
    ys = []
    for h in hs:
        xd = torch.from_numpy(x).cuda()
        xp, yp = torch.empty_like(xd), torch.empty_like(xd)
        y = torch.empty_like(xd)
        sellcs.sell_permute(h, xd, xp)
        sellcs.sell_spmv(h, xp, yp)
        sellcs.sell_unpermute(h, yp, y)
        torch.cuda.synchronize()
        ys.append(y.cpu().numpy())
    assert np.array_equal(ys[0], ys[1])
    check_fp64(A, ys[0], x)


def test_window_auto_falls_back_and_required_is_refused():
    from paper_1307_6209_amd import sellcs
    P = synth.powerlaw(40_000, seed=8)  # uniform half of the columns: windows far too large
    h = build(P, 32, 1)
    assert h.info["xwindow"] == 0
    with pytest.raises(sellcs.SellError) as e:
        build(P, 32, 1, xwindow=1)
    assert e.value.status == sellcs.SELL_ERR_UNSUPPORTED
    S = synth.stencil27(12)
    for kw in ({"C": 128}, {"C": 32, "vec": 4}, {"C": 4}):
        C = kw.pop("C")
        with pytest.raises(sellcs.SellError):
            build(S, C, 1, xwindow=1, **kw)
        assert build(S, C, 1, **kw).info["xwindow"] == 0  # auto: the plain kernel
    # the default build uses the window on a banded matrix with enough groups
    # of chunks (two per compute unit), not on a small one; at C = 32 groups
    # of 8 chunks when there are two of those per compute unit, else of 4
    assert build(S, 32, 1).info["xwindow"] == 0
    inf = build(synth.stencil27(64), 32, 1).info  # 8,192 chunks
    assert inf["xwindow"] == 1 and inf["xwindow_group_chunks"] == 8
    for C in (16, 64):  # the wide groups only at C = 32
        inf = build(synth.stencil27(64), C, 1).info
        assert inf["xwindow"] == 1 and inf["xwindow_group_chunks"] == 4
    inf = build(synth.stencil27(48), 32, 1).info  # 3,456 chunks: 432 groups of 8, 864 of 4
    assert inf["xwindow"] == 1 and inf["xwindow_group_chunks"] == 4
    # an explicit size is built as asked, or refused when required
    assert build(synth.stencil27(48), 32, 1, xwindow_chunks=8).info["xwindow_group_chunks"] == 8
    with pytest.raises(sellcs.SellError):
        build(scattered_runs(n=3000), 32, 1, xwindow=1, xwindow_chunks=8)  # 15,360 slots per group


def test_window_ragged_groups_and_empty_rows():
    """Row counts that leave the last group of chunks short, empty rows and
    empty chunks."""
    for n in (1, 31, 33, 129, 1000):
        A = banded(n, n, half=5, max_len=8)
        x = synth.uniform(A.ncols, 34, 1)
        if A.nnz == 0:
            continue
        for C in (8, 32, 64):
            off = build(A, C, 1, xwindow=-1)
            for gc in (4, 8):
                on = build(A, C, 1, xwindow=1, xwindow_chunks=gc)
                assert on.info["xwindow"] == 1, (n, C, gc)
                assert np.array_equal(spmv_gpu(on, x).view(np.uint64), spmv_gpu(off, x).view(np.uint64))


def blocks_with_empty_runs(seed):
    """Banded rows with runs of empty rows long enough to empty whole chunks
    and whole groups of chunks, in the middle and at the end."""
    A = banded(1400, seed, half=12, max_len=14)
    lens = np.diff(A.rpt)
    keep = np.ones(A.nrows, bool)
    keep[300:760] = False      # 14+ chunks of 32 rows: several whole groups
    keep[1100:1400] = False    # empty tail
    keep[905] = False
    rpt = np.zeros(A.nrows + 1, np.int64)
    np.cumsum(np.where(keep, lens, 0), out=rpt[1:])
    sel = np.repeat(keep, lens)
    return synth.CRS(A.nrows, A.ncols, rpt, A.col[sel], A.val[sel])


@pytest.mark.parametrize("gc", [4, 8])
@pytest.mark.parametrize("C", [8, 32, 64])
@pytest.mark.parametrize("unroll", [4, 16])
def test_window_empty_chunks_and_groups(C, unroll, gc):
    """Live waves whose chunk holds no column read nothing and store zeros;
    groups without a slot stage an empty window; the rest of the product is
    untouched (bit-exact against the global-index product)."""
    A = blocks_with_empty_runs(41)
    x = synth.uniform(A.ncols, 36, 1)
    assert fits_group(A, C, 1, gc)
    on = build(A, C, 1, vec=2, unroll=unroll, xwindow=1, xwindow_chunks=gc)
    off = build(A, C, 1, vec=2, xwindow=-1)
    assert on.info["xwindow"] == 1
    y_on, y_off = spmv_gpu(on, x), spmv_gpu(off, x)
    assert np.array_equal(y_on.view(np.uint64), y_off.view(np.uint64))
    assert np.all(y_on[300:760] == 0.0) and np.all(y_on[1100:] == 0.0) and y_on[905] == 0.0
    check_fp64(A, y_on, x)


def scattered_runs(n=66_000, run=60, ncols=1_000_000, seed=77):
    """Each row holds `run` consecutive columns at a random offset: a group
    of 4 chunks of 32 rows has a window of ~7,700 columns in 128 runs
    (61 KB in FP64, above the automatic 16 KiB limit of 4 chunks); 516
    groups, more than two per compute unit, so the window size alone decides
    the default. A group of 8 such chunks holds 15,360 slots, more than a
    group may hold."""
    off = (synth.uniform(n, seed, 1, 0.0, 1.0) * (ncols - run)).astype(np.int64)
    rpt = np.arange(n + 1, dtype=np.int64) * run
    col = (off[:, None] + np.arange(run)[None, :]).reshape(-1).astype(np.int32)
    val = synth.uniform(n * run, seed, 2)
    return synth.CRS(n, ncols, rpt, col, val)


@pytest.mark.parametrize("val_dtype,acc", [("f64", "f64"), ("f32", "f32")])
def test_window_largest_required(val_dtype, acc):
    """Windows beyond the automatic limit: the default build falls back to
    the global-index product; xwindow = 1 builds them (groups of 4 chunks, up
    to 64 KiB of LDS) and the product still equals the global-index one bit
    for bit."""
    A = scattered_runs()
    x = synth.uniform(A.ncols, 37, 1)
    if val_dtype != "f64":
        x = oracle.round_f32(x).astype(np.float64)
    auto = build(A, 32, 1, val_dtype=val_dtype, acc_dtype=acc)
    assert auto.info["xwindow"] == 0
    on = build(A, 32, 1, val_dtype=val_dtype, acc_dtype=acc, vec=2, xwindow=1)
    inf = on.info
    say("largest window", val_dtype, inf["xwindow_max"], "segments", inf["xsegments"])
    assert inf["xwindow"] == 1 and inf["xwindow_max"] > 7000 and inf["xwindow_group_chunks"] == 4
    off = build(A, 32, 1, val_dtype=val_dtype, acc_dtype=acc, vec=2, xwindow=-1)
    y_on, y_off = spmv_gpu(on, x), spmv_gpu(off, x)
    assert np.array_equal(y_on, y_off)
    if val_dtype == "f64":
        check_fp64(A, y_on, x)


def span_matrix():
    """Three groups of four 32-row chunks over 600,000 columns. Group 0: rows
    of one or two entries at columns 2..51 and 262,145 -- the span 2..262,145
    is exactly 32 * 8192 values (the builder's bitmap), with column 0 from
    padding kept apart in front. Group 1: columns 5..34 and 262,150, one value
    more (the builder sorts). Group 2: columns 1, 3 and the row index, with
    padding: column 0 joins the first run."""
    rows = []
    for i in range(384):
        if i < 128:
            c = [2 + i % 50] + ([262_145] if i % 2 == 0 else [])
        elif i < 256:
            c = [5 + i % 30] + ([262_150] if i % 3 == 0 else [])
        else:
            c = sorted({1, 3, i}) if i % 4 else [1]
        rows.append(c)
    rpt = np.zeros(len(rows) + 1, np.int64)
    np.cumsum([len(c) for c in rows], out=rpt[1:])
    col = np.concatenate([np.array(c, np.int32) for c in rows])
    return synth.CRS(len(rows), 600_000, rpt, col, synth.uniform(col.size, 88, 1))


TABLE_CASES = [
    ("stencil27_24_C32", lambda: synth.stencil27(24), 32, 1, 0),
    ("stencil27_24_C16_vec2", lambda: synth.stencil27(24), 16, 64, 2),
    ("lap5_96_C8", lambda: synth.lap5(96), 8, 1, 0),
    ("banded_3000_C64", lambda: banded(3000, 7), 64, 4096, 1),
    ("powerlaw_5000_C8", lambda: synth.powerlaw(5000, seed=12, lmax=100), 8, 1, 0),
    ("powerlaw_5000_C16_sorted", lambda: synth.powerlaw(5000, seed=13, lmax=20), 16, 10**9, 1),
    ("ragged_1000_C32", lambda: blocks_with_empty_runs(43), 32, 1, 0),
    ("span_limit_C32", span_matrix, 32, 1, 0),
]


@pytest.mark.parametrize("gc", [4, 8])
@pytest.mark.parametrize("name,make,C,sigma,vec", TABLE_CASES, ids=[c[0] for c in TABLE_CASES])
def test_window_tables_match_definition(name, make, C, sigma, vec, gc):
    """The window tables the builder stores (run offsets per group, the runs,
    the 16-bit position of every slot) against their plain definition --
    sorted distinct columns of each group of chunks, position = rank -- taken
    from the oracle's layout, for every group; groups of 4 and of 8 chunks."""
    from paper_1307_6209_amd import sellcs
    A = make()
    h = build_or_refused(A, C, sigma, gc, vec=vec)
    if h is None:
        return
    assert h.info["xwindow"] == 1 and h.info["xwindow_group_chunks"] == gc
    got = sellcs.sell_export_xwindow(h)
    lay = oracle.sell_build(A, C, sigma)
    segoff, seg, lcol = window_tables(lay["col"], lay["cs"], got["group_chunks"])
    say("window tables", name, "groups", segoff.size - 1, "runs", seg.shape[0], "largest", h.info["xwindow_max"])
    assert np.array_equal(got["segoff"], segoff)
    assert np.array_equal(got["seg"].astype(np.int64), seg)
    assert np.array_equal(got["lcol"].astype(np.int64), lcol)
    assert h.info["xsegments"] == seg.shape[0]
    assert h.info["xwindow_max"] == max(int(seg[a:b, 2].sum()) for a, b in zip(segoff[:-1], segoff[1:]))
    check_fp64(A, spmv_gpu(h, synth.uniform(A.ncols, 38, 1)), synth.uniform(A.ncols, 38, 1))


def test_window_tables_without_window_refused():
    from paper_1307_6209_amd import sellcs
    h = build(synth.stencil27(10), 32, 1, xwindow=-1)
    with pytest.raises(sellcs.SellError) as e:
        sellcs.sell_export_xwindow(h)
    assert e.value.status == sellcs.SELL_ERR_UNSUPPORTED
