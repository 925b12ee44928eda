"""Bandwidth probes and the autotuner."""
import pytest

import synth
from gpu_util import build, check_fp64, dev_crs, say, spmv_gpu

pytestmark = pytest.mark.gpu


def test_probes_plausible():
    from paper_1307_6209_amd import sellcs
    r = sellcs.sell_probe_bandwidth(0, 2 << 30, 5)
    c = sellcs.sell_probe_bandwidth(1, 2 << 30, 5)
    w = sellcs.sell_probe_bandwidth(6, 2 << 30, 5)
    say("read GB/s", r, "copy GB/s", c, "write GB/s", w)
    assert 1000 < r < 8000 * 1.02
    assert 1000 < c < 8000 * 1.02
    assert 1000 < w < 8000 * 1.02


def test_gather_probe_plausible():
    """Random 8-byte gathers: a small (L2-sized) array serves them faster than
    one far beyond the 256 MB MALL, and neither beats the streaming read."""
    from paper_1307_6209_amd import sellcs
    small = sellcs.sell_probe_bandwidth(2, 2 << 20, 3)
    big = sellcs.sell_probe_bandwidth(2, 2 << 30, 3)
    read = sellcs.sell_probe_bandwidth(0, 2 << 30, 3)
    say("gather GB/s (8 B per gather): 2 MiB", small, "2 GiB", big, "read", read)
    assert 0 < big < small
    assert big < read


@pytest.mark.parametrize("kind", [3, 4, 5, 7, 8, 9])
def test_row_probes_plausible(kind):
    """Random rows (kinds 3-5) and random rows read with rows written (7-9)
    over 256 MiB: positive, and neither beats 8 TB/s by more than rounding."""
    from paper_1307_6209_amd import sellcs
    g = sellcs.sell_probe_bandwidth(kind, 256 << 20, 3)
    say("row probe", kind, "GB/s", g)
    assert 100 < g < 8000 * 1.02


def test_autotune_small():
    from paper_1307_6209_amd import sellcs
    A = synth.powerlaw(100_000, seed=71)
    rpt, col, val = dev_crs(A)
    r = sellcs.sell_autotune(rpt, col, val, A.ncols, k=1, C=(16, 32, 64), sigma=(1, 64, 4096), unroll=(4, 8), reps=5)
    say("autotune", r)
    assert r["C"] in (16, 32, 64) and r["sigma"] in (1, 64, 4096) and r["unroll"] in (4, 8, 16)
    assert r["candidates"] == 18 and r["gflops"] > 0


def test_autotune_block():
    from paper_1307_6209_amd import sellcs
    A = synth.powerlaw(50_000, seed=72)
    rpt, col, val = dev_crs(A)
    r = sellcs.sell_autotune(rpt, col, val, A.ncols, k=8, C=(16, 32), sigma=(1, 256), unroll=(8,), ktile=(0, 4, 8),
                             reps=3)
    assert r["candidates"] == 12 and r["ktile"] in (0, 4, 8)


def test_autotune_model_guided():
    """Model-guided search ranks all (C, sigma) by the model's bytes from a
    layout-only build and times only the best few; on the power-law matrix
    the global sort has the fewest bytes."""
    from paper_1307_6209_amd import sellcs
    A = synth.powerlaw(200_000, seed=73)
    rpt, col, val = dev_crs(A)
    r = sellcs.sell_autotune(rpt, col, val, A.ncols, k=1, C=(16, 32, 64), sigma=(1, 64, 4096, 200_000),
                             unroll=(8,), reps=5, model_guided=2)
    say("model guided", r)
    assert r["predicted"] == 12 and r["candidates"] == 2
    assert r["sigma"] == 200_000 and r["C"] in (16, 32, 64)


def test_autotune_lanes_per_row_and_split_width():
    """vec (lanes per row = 64 vec / C) and the split width of long rows are
    searched too; unsupported combinations are skipped."""
    from paper_1307_6209_amd import sellcs
    A = synth.powerlaw(100_000, seed=74)
    rpt, col, val = dev_crs(A)
    r = sellcs.sell_autotune(rpt, col, val, A.ncols, k=1, C=(32, 128), sigma=(100_000,), unroll=(8,), vec=(1, 2, 4),
                             seg_cols=(64, 256), reps=5)
    say("autotune vec/seg", r)
    # C = 128 accepts vec 1 only: 3*2 builds for C = 32, 1*2 for C = 128
    assert r["candidates"] == 8
    assert r["vec"] in (1, 2, 4) and r["seg_cols"] in (64, 256)


def test_spmv_in_captured_graph():
    """sell_spmv launches can be captured in a graph (no allocation or
    synchronisation inside); replays with eager work between them match
    the eager result bit for bit."""
    import numpy as np
    import torch
    from paper_1307_6209_amd import sellcs
    A = synth.lap5(128)
    rpt, col, val = dev_crs(A)
    h = sellcs.sell_build(rpt, col, val, A.ncols, 32, 1)
    hs = sellcs.sell_build(rpt, col, val, A.ncols, 16, A.nrows, seg_cols=64)
    hw = sellcs.sell_build(rpt, col, val, A.ncols, 32, 1, xwindow=1)  # the x-window product
    assert hw.info["xwindow"] == 1
    x = torch.from_numpy(synth.uniform(A.ncols, 75, 1)).cuda()
    y = torch.empty(A.nrows, dtype=torch.float64, device="cuda")
    y2 = torch.empty_like(y)
    y3 = torch.empty_like(y)
    sellcs.sell_spmv(h, x, y)
    sellcs.sell_spmv(hs, x, y2)
    sellcs.sell_spmv(hw, x, y3)
    torch.cuda.synchronize()
    want, want2, want3 = y.cpu().numpy().copy(), y2.cpu().numpy().copy(), y3.cpu().numpy().copy()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for _ in range(5):
                sellcs.sell_spmv(h, x, y)
                sellcs.sell_spmv(hs, x, y2)
                sellcs.sell_spmv(hw, x, y3)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        y.fill_(float("nan"))
        y2.fill_(float("nan"))
        y3.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), want) and np.array_equal(y2.cpu().numpy(), want2)
        assert np.array_equal(y3.cpu().numpy(), want3)
        sellcs.sell_spmv(hs, x, y2)  # eager work between replays
        sellcs.sell_spmv(hw, x, y3)
        torch.cuda.synchronize()


def test_autotune_x_path():
    """The x path (LDS window or L2 gathers) is searched too; on a banded
    matrix large enough for the window the window wins."""
    from paper_1307_6209_amd import sellcs
    A = synth.stencil27(64)
    rpt, col, val = dev_crs(A)
    r = sellcs.sell_autotune(rpt, col, val, A.ncols, k=1, C=(32,), sigma=(1,), unroll=(8,), xwindow=(-1, 0), reps=10)
    say("autotune x path", r)
    assert r["candidates"] == 2 and r["xwindow"] in (0, 1)


def test_autotune_window_workgroup_size():
    """The window product's workgroup size (4 or 8 chunks, one wave each) is
    searched too: every window size is timed once, the global-index product
    once (the size does not change it), and the result names the size of
    the window that won."""
    from paper_1307_6209_amd import sellcs
    A = synth.stencil27(64)
    rpt, col, val = dev_crs(A)
    r = sellcs.sell_autotune(rpt, col, val, A.ncols, k=1, C=(32,), sigma=(1,), unroll=(8,), xwindow=(-1, 0),
                             xwindow_chunks=(4, 8), reps=10)
    say("autotune window workgroup size", r)
    assert r["candidates"] == 3
    assert (r["xwindow"], r["xwindow_chunks"]) in ((0, 0), (1, 4), (1, 8))


def test_autotune_row_lengths():
    """The row_lengths build option is searched too: both values timed where
    they apply (C in 8..64, single vector, no x window), the option skipped
    elsewhere; the winner, rebuilt as reported, gives the oracle's product."""
    from paper_1307_6209_amd import sellcs
    A = synth.powerlaw(60_000, seed=31)
    rpt, col, val = dev_crs(A)
    r = sellcs.sell_autotune(rpt, col, val, A.ncols, k=1, C=(4, 32), sigma=(1024,), unroll=(8,), xwindow=(-1,),
                             row_lengths=(0, 1), reps=10)
    say("autotune row lengths", r)
    assert r["candidates"] == 3  # C = 4 without row lengths only
    assert r["row_lengths"] in (0, 1) and (r["row_lengths"] == 0 or r["C"] == 32)
    h = build(A, r["C"], r["sigma"], unroll=r["unroll"], vec=r["vec"], xwindow=-1, row_lengths=bool(r["row_lengths"]))
    x = synth.uniform(A.ncols, 31, 1)
    check_fp64(A, spmv_gpu(h, x), x)
    # a window layout does not time the row-length product
    S = synth.stencil27(64)
    rs, cs_, vs = dev_crs(S)
    r2 = sellcs.sell_autotune(rs, cs_, vs, S.ncols, k=1, C=(32,), sigma=(1,), unroll=(8,), xwindow=(1,),
                              row_lengths=(0, 1), reps=10)
    assert r2["candidates"] == 1 and r2["row_lengths"] == 0 and r2["xwindow"] == 1
