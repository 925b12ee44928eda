"""Block form Y = A X (k right-hand sides, row-major) against the oracle:
every column within 1e-13 (|A||X|)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import build, say

pytestmark = pytest.mark.gpu


def run_spmmv(h, X):
    import torch
    from paper_1307_6209_amd import sellcs
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    Y = torch.full((h.info["nrows"], X.shape[1]), float("nan"), dtype=torch.float64, device="cuda")
    sellcs.sell_spmmv(h, Xd, Y)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


def check(A, Y, X, tol=1e-13):
    Yh, aY = oracle.crs_spmmv_hi(A, X)
    assert np.all(np.isfinite(Y))
    assert np.all(np.abs(Y - Yh) <= tol * aY)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8, 16, 32])
@pytest.mark.parametrize("C,sigma", [(8, 1), (16, 1), (32, 64), (64, 1), (128, 1000)])
def test_spmmv(k, C, sigma):
    A = synth.powerlaw(30_000, seed=41)
    X = synth.block_vector(A.ncols, k, seed=42)
    say("spmmv k", k, "C", C, "sigma", sigma)
    h = build(A, C, sigma, seg_cols=-1)
    check(A, run_spmmv(h, X), X)


@pytest.mark.parametrize("ktile", [1, 2, 4, 8, 16, 32, 64])
def test_spmmv_ktile(ktile):
    A = synth.random_crs(700, 900, seed=43, max_len=60, empty_frac=0.1, duplicates=True, unsorted=True)
    X = synth.block_vector(A.ncols, 16, seed=44)
    h = build(A, 16, 1, ktile=ktile)
    check(A, run_spmmv(h, X), X)


@pytest.mark.parametrize("k", [2, 8, 32])
@pytest.mark.parametrize("C", [16, 32, 128])
def test_spmmv_split(k, C):
    A = synth.powerlaw(30_000, seed=45)
    X = synth.block_vector(A.ncols, k, seed=46)
    h = build(A, C, 1, seg_cols=64)
    assert h.info["nsplit"] > 0
    Y1 = run_spmmv(h, X)
    check(A, Y1, X)
    assert np.array_equal(run_spmmv(h, X), Y1)


def test_spmmv_k_above_kmax_rejected():
    from paper_1307_6209_amd import sellcs
    A = synth.powerlaw(30_000, seed=47)
    h = build(A, 32, 1, seg_cols=64, kmax=8)
    with pytest.raises(sellcs.SellError):
        run_spmmv(h, synth.block_vector(A.ncols, 16))
    check(A, run_spmmv(h, synth.block_vector(A.ncols, 8)), synth.block_vector(A.ncols, 8))


def test_spmmv_columns_equal_spmv():
    """Column v of Y equals the single-vector product of column v of X
    within the FP64 bound (summation orders differ)."""
    from gpu_util import spmv_gpu, check_fp64
    A = synth.stencil27(16)
    X = synth.block_vector(A.ncols, 4, seed=48)
    h = build(A, 32, 1)
    Y = run_spmmv(h, X)
    for v in range(4):
        y = spmv_gpu(h, X[:, v].copy())
        check_fp64(A, y, X[:, v].copy())
        check_fp64(A, Y[:, v].copy(), X[:, v].copy())


def test_spmmv_misaligned_block():
    """X and Y one element off a 16-byte boundary: the vector gathers fall
    back to narrower accesses and the results are unchanged."""
    import torch
    from paper_1307_6209_amd import sellcs
    A = synth.powerlaw(20_000, seed=49)
    k = 8
    X = synth.block_vector(A.ncols, k, seed=50)
    h = build(A, 32, 64)
    Xb = torch.zeros(A.ncols * k + 1, dtype=torch.float64, device="cuda")
    Xb[1:] = torch.from_numpy(X.ravel()).cuda()
    Yb = torch.zeros(A.nrows * k + 1, dtype=torch.float64, device="cuda")
    Xv, Yv = Xb[1:].view(A.ncols, k), Yb[1:].view(A.nrows, k)
    sellcs.sell_spmmv(h, Xv, Yv)
    torch.cuda.synchronize()
    check(A, Yv.cpu().numpy(), X)


@pytest.mark.parametrize("k", [16, 32, 64])
@pytest.mark.parametrize("C,sigma,seg", [(16, 1, 64), (32, 30_000, 64), (64, 1, -1), (128, 1000, 32)])
def test_spmmv_rows_kernel_equals_pass_kernel(k, C, sigma, seg):
    """With the automatic pass width k = 16, 32 and 64 run the one-pass
    kernel with 8 lanes per row (4 for k = 16), on padding-heavy (sigma = 1)
    and dense (sigma = n) layouts; an explicit k-tile runs the pass kernel. Both add each row's products in column order: equal bit for
    bit, and within the oracle's bound (split rows included)."""
    A = synth.powerlaw(30_000, seed=51)
    X = synth.block_vector(A.ncols, k, seed=52)
    h_rows = build(A, C, sigma, seg_cols=seg, kmax=64)
    h_pass = build(A, C, sigma, seg_cols=seg, kmax=64, ktile=16)
    say("spmmv rows k", k, "C", C, "sigma", sigma, "nsplit", h_rows.info["nsplit"])
    Y_rows, Y_pass = run_spmmv(h_rows, X), run_spmmv(h_pass, X)
    check(A, Y_rows, X)
    assert np.array_equal(Y_rows, Y_pass)


def test_spmmv_rows_kernel_misaligned_falls_back():
    """X and Y 8 bytes off a 16-byte boundary at k = 32: the pass kernel
    runs (narrower gathers) and the result is unchanged."""
    import torch
    from paper_1307_6209_amd import sellcs
    A = synth.powerlaw(20_000, seed=53)
    k = 32
    X = synth.block_vector(A.ncols, k, seed=54)
    h = build(A, 32, A.nrows)
    Xb = torch.zeros(A.ncols * k + 1, dtype=torch.float64, device="cuda")
    Xb[1:] = torch.from_numpy(X.ravel()).cuda()
    Yb = torch.zeros(A.nrows * k + 1, dtype=torch.float64, device="cuda")
    Xv, Yv = Xb[1:].view(A.ncols, k), Yb[1:].view(A.nrows, k)
    sellcs.sell_spmmv(h, Xv, Yv)
    torch.cuda.synchronize()
    Y = Yv.cpu().numpy()
    check(A, Y, X)
    assert np.array_equal(Y, run_spmmv(h, X))


@pytest.mark.parametrize("k,ktile", [(4, 0), (16, 0), (32, 0), (64, 0), (32, 8)])
@pytest.mark.parametrize("sigma", [1, 10**9])
def test_spmmv_explicit_zero_entries(k, ktile, sigma):
    """Explicit zero values (a quarter of the entries, whole rows among them)
    with finite X: the block kernels skip the gather of every zero slot, and
    the result still matches the oracle, where those terms add exactly 0.
    Both the pass kernel and the one-pass row kernels (k = 16, 32, 64 with
    the automatic pass width), dense and padding-heavy layouts."""
    A = synth.powerlaw(20_000, seed=47)
    zero = (synth.u64(48, 1, A.nnz) % np.uint64(4)) == 0
    lens = A.row_lengths()
    zero |= np.repeat((synth.u64(48, 2, A.nrows) % np.uint64(10)) == 0, lens)  # whole rows of zeros
    val = np.where(zero, 0.0, A.val)
    B = synth.CRS(A.nrows, A.ncols, A.rpt, A.col, val)
    X = synth.block_vector(B.ncols, k, seed=49)
    h = build(B, 32, sigma, ktile=ktile, kmax=64)
    say("explicit zeros k", k, "ktile", ktile, "sigma", sigma, "beta", round(h.info["beta"], 3),
        "zero entries", int(zero.sum()))
    Y = run_spmmv(h, X)
    check(B, Y, X)
    allzero = np.array([not np.any(~zero[A.rpt[i]:A.rpt[i + 1]]) for i in range(A.nrows)])
    assert np.all(Y[allzero] == 0.0)


@pytest.mark.parametrize("k", [32, 64])
def test_spmmv_rows_kernel_16_byte_aligned(k):
    """X and Y 16 bytes off a 32-byte boundary: the one-pass kernel reads and
    writes 16-byte pairs of right-hand sides, so it still runs; the result
    equals the aligned call's bit for bit and the oracle within its bound."""
    import torch
    from paper_1307_6209_amd import sellcs
    A = synth.powerlaw(20_000, seed=55)
    X = synth.block_vector(A.ncols, k, seed=56)
    h = build(A, 32, A.nrows, kmax=64)
    Xb = torch.zeros(A.ncols * k + 2, dtype=torch.float64, device="cuda")
    Xb[2:] = torch.from_numpy(X.ravel()).cuda()
    Yb = torch.zeros(A.nrows * k + 2, dtype=torch.float64, device="cuda")
    Xv, Yv = Xb[2:].view(A.ncols, k), Yb[2:].view(A.nrows, k)
    assert Xv.data_ptr() % 32 == 16 and Yv.data_ptr() % 32 == 16
    sellcs.sell_spmmv(h, Xv, Yv)
    torch.cuda.synchronize()
    Y = Yv.cpu().numpy()
    check(A, Y, X)
    assert np.array_equal(Y, run_spmmv(h, X))
