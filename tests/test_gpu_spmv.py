"""GPU FP64 SELL-C-sigma spMVM against the long double oracle:
|y - y_ref|_i <= 1e-13 (|A||x|)_i for every row."""
import numpy as np
import pytest

import synth
from gpu_util import build, check_fp64, say, spmv_gpu

pytestmark = pytest.mark.gpu

MATS = {
    "random": lambda: synth.random_crs(301, 90, seed=1, max_len=30, empty_frac=0.3, duplicates=True, unsorted=True),
    "nonsquare_wide": lambda: synth.random_crs(77, 5000, seed=2, max_len=300, empty_frac=0.1),
    "nonsquare_tall": lambda: synth.random_crs(3000, 17, seed=3, max_len=12, empty_frac=0.2, duplicates=True),
    "lap5_128": lambda: synth.lap5(128),
    "powerlaw_50k": lambda: synth.powerlaw(50_000, seed=3),
    "stencil27_24": lambda: synth.stencil27(24),
    "dense_300": lambda: synth.dense(300, 257),
}
CS = [(1, 1), (2, 1), (4, 7), (8, 1), (16, 1), (16, 256), (32, 1), (32, 10**9), (64, 1), (64, 4096), (128, 1),
      (128, 64)]


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("C,sigma", CS)
@pytest.mark.parametrize("unroll,vec", [(4, 1), (8, 1), (4, 2), (8, 2), (4, 4), (8, 4), (0, 0)])
def test_spmv_fp64(name, C, sigma, unroll, vec):
    if vec > 1 and (C > 64 or vec > C):
        pytest.skip("vec > 1 needs C <= 64 and vec <= C")
    A = MATS[name]()
    x = synth.uniform(A.ncols, 11, 1)
    say("spmv", name, "C", C, "sigma", sigma, "U", unroll, "V", vec)
    h = build(A, C, sigma, unroll=unroll, vec=vec)
    y = spmv_gpu(h, x)
    check_fp64(A, y, x)


@pytest.mark.parametrize("seg", [64, 128, 448, 4096])
@pytest.mark.parametrize("C,vec", [(1, 1), (8, 1), (8, 4), (32, 1), (32, 2), (64, 4), (128, 1)])
def test_split_chunks(seg, C, vec):
    """Chunks cut into segments of `seg` chunk columns: segment sums added in
    order by the combining kernel; identical bits on repeated calls."""
    A = synth.powerlaw(40_000, seed=8)
    x = synth.uniform(A.ncols, 12, 1)
    say("split", "C", C, "seg", seg, "V", vec)
    h = build(A, C, 1, seg_cols=seg, vec=vec)
    assert h.info["nsplit"] > 0
    y1 = spmv_gpu(h, x)
    check_fp64(A, y1, x)
    for _ in range(3):
        assert np.array_equal(spmv_gpu(h, x), y1)


def test_auto_split_on_long_rows():
    A = synth.powerlaw(200_000, seed=9)
    h = build(A, 32, 1)
    inf = h.info
    say("auto split", inf["seg_cols"], inf["nsplit"], inf["nunits"])
    x = synth.uniform(A.ncols, 13, 1)
    check_fp64(A, spmv_gpu(h, x), x)


def test_empty_rows_give_zero_and_nothing_else_written():
    A = synth.random_crs(500, 40, seed=14, max_len=6, empty_frac=0.7)
    x = synth.uniform(40, 14, 1)
    for C, sigma in [(32, 1), (16, 64)]:
        h = build(A, C, sigma)
        y = spmv_gpu(h, x)
        assert np.all(y[A.row_lengths() == 0] == 0.0)
        check_fp64(A, y, x)


def test_nnz_zero():
    A = synth.CRS(100, 30, np.zeros(101, np.int64), np.zeros(0, np.int32), np.zeros(0))
    h = build(A, 32, 1)
    assert np.array_equal(spmv_gpu(h, np.ones(30)), np.zeros(100))


def test_laplacian_row_sums_exact():
    """A 1 for the 5-point Laplacian is exact integer arithmetic: 0 inside,
    1 on edges, 2 at corners, whatever the summation order."""
    m = 128
    A = synth.lap5(m)
    for C, sigma in [(32, 1), (64, A.nrows), (4, 16)]:
        h = build(A, C, sigma)
        y = spmv_gpu(h, np.ones(A.nrows))
        g = y.reshape(m, m)
        want = np.zeros((m, m))
        want[0, :] += 1
        want[-1, :] += 1
        want[:, 0] += 1
        want[:, -1] += 1
        assert np.array_equal(g, want)


@pytest.mark.parametrize("vec", [1, 2, 4])
def test_misaligned_y_and_zero_entries(vec):
    """y one element off a vector boundary (row stores fall back to scalar),
    and explicit zero values among the stored entries."""
    import torch
    from paper_1307_6209_amd import sellcs
    A = synth.stencil27(12)
    A.val[::7] = 0.0
    x = synth.uniform(A.ncols, 15, 1)
    h = build(A, 32, 1, vec=vec)
    yb = torch.full((A.nrows + 1,), float("nan"), dtype=torch.float64, device="cuda")
    sellcs.sell_spmv(h, torch.from_numpy(x).cuda(), yb[1:])
    torch.cuda.synchronize()
    check_fp64(A, yb[1:].cpu().numpy(), x)
