"""Symmetric-permutation mode with the sorted-order helpers, and the CRS
comparison kernels, against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import build, check_fp64, dev_crs, say

pytestmark = pytest.mark.gpu


def t():
    import torch
    return torch


@pytest.mark.parametrize("C,sigma", [(1, 1), (8, 1), (8, 64), (32, 1000), (64, 10**9), (128, 4096)])
def test_symmetric_layout_and_product(C, sigma):
    from paper_1307_6209_amd import sellcs
    torch = t()
    A = synth.powerlaw(30_000, seed=51)
    x = synth.uniform(A.ncols, 52, 1)
    say("symmetric C", C, "sigma", sigma)
    h = build(A, C, sigma, permute_columns=True)
    assert h.info["permuted_columns"] == 1
    got = sellcs.sell_export(h)
    want = oracle.sell_build(A, C, sigma, permute_columns=True)
    for key in ("perm", "cl", "cs", "col"):
        assert np.array_equal(got[key], want[key]), key
    assert np.array_equal(got["val"].view(np.uint64), want["val"].view(np.uint64))
    xd = torch.from_numpy(x).cuda()
    xp = torch.empty_like(xd)
    sellcs.sell_permute(h, xd, xp)
    yp = torch.empty(A.nrows, dtype=torch.float64, device="cuda")
    sellcs.sell_spmv(h, xp, yp)
    y = torch.empty_like(yp)
    sellcs.sell_unpermute(h, yp, y)
    torch.cuda.synchronize()
    perm = want["perm"]
    assert np.array_equal(xp.cpu().numpy(), x[perm])
    ypn = yp.cpu().numpy()
    assert np.array_equal(y.cpu().numpy()[perm], ypn)
    check_fp64(A, y.cpu().numpy(), x)


def test_symmetric_needs_square():
    from paper_1307_6209_amd import sellcs
    A = synth.random_crs(50, 40, seed=53, max_len=5)
    with pytest.raises(sellcs.SellError) as ei:
        build(A, 8, 16, permute_columns=True)
    assert ei.value.status == sellcs.SELL_ERR_UNSUPPORTED


def test_symmetric_block_and_reduced():
    """The block form and FP32 storage run unchanged in sorted order."""
    from paper_1307_6209_amd import sellcs
    torch = t()
    A = synth.powerlaw(20_000, seed=54)
    perm, _, _ = oracle.sell_layout(A, 32, 512)
    B = oracle.crs_symperm(A, perm)
    h = build(A, 32, 512, permute_columns=True)
    X = synth.block_vector(A.ncols, 8, seed=55)
    Xp = np.ascontiguousarray(X[perm])
    Y = torch.empty(A.nrows, 8, dtype=torch.float64, device="cuda")
    sellcs.sell_spmmv(h, torch.from_numpy(Xp).cuda(), Y)
    torch.cuda.synchronize()
    Yh, aY = oracle.crs_spmmv_hi(B, Xp)
    assert np.all(np.abs(Y.cpu().numpy() - Yh) <= 1e-13 * aY)


@pytest.mark.parametrize("L", [0, 1, 2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("name,make", [
    ("powerlaw", lambda: synth.powerlaw(50_000, seed=56)),
    ("stencil27", lambda: synth.stencil27(20)),
    ("random", lambda: synth.random_crs(999, 300, seed=57, max_len=80, empty_frac=0.3, duplicates=True, unsorted=True)),
])
def test_crs_kernels(L, name, make):
    from paper_1307_6209_amd import sellcs
    torch = t()
    A = make()
    x = synth.uniform(A.ncols, 58, 1)
    rpt, col, val = dev_crs(A)
    y = torch.full((A.nrows,), float("nan"), dtype=torch.float64, device="cuda")
    sellcs.sell_crs_spmv(rpt, col, val, torch.from_numpy(x).cuda(), y, A.ncols, lanes_per_row=L)
    torch.cuda.synchronize()
    check_fp64(A, y.cpu().numpy(), x)


@pytest.mark.parametrize("C,sigma", [(32, 1), (64, 1), (128, 1)])
def test_dense_2000(C, sigma):
    """Dense 2000 x 2000 in SELL (few rows, every row 2000 long)."""
    A = synth.dense(2000, 2000)
    x = synth.uniform(A.ncols, 59, 1)
    from gpu_util import spmv_gpu
    h = build(A, C, sigma)
    say("dense 2000 C", C, "nsplit", h.info["nsplit"])
    check_fp64(A, spmv_gpu(h, x), x)


@pytest.mark.parametrize("C,sigma", [(8, 1), (32, 1), (32, 4284), (128, 4284)])
def test_rail_like(C, sigma):
    """Few rows, ~2,650 entries per row, 1.09M columns, zeta ~ 1.5."""
    from gpu_util import spmv_gpu
    A = synth.workload("rail_like")
    x = synth.uniform(A.ncols, 60, 1)
    h = build(A, C, sigma)
    say("rail_like C", C, "sigma", sigma, "beta", h.info["beta"], "nsplit", h.info["nsplit"])
    check_fp64(A, spmv_gpu(h, x), x)
