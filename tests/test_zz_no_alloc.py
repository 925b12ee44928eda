"""sell_spmmv_noalloc (segment sums in the library's static per-device
scratch) against sell_spmmv on the same handles: the same kernels, so the
same bits. Two calls in a row, the second on a smaller input; block widths
beyond the kmax given at build; sizes beyond the scratch refused."""
import numpy as np
import pytest

import synth
from gpu_util import build, say

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20


def run(fn, h, X):
    import torch
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    Y = torch.full((h.info["nrows"], X.shape[1]), float("nan"), dtype=torch.float64, device="cuda")
    fn(h, Xd, Y)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


def same_bits(a, b):
    return np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_noalloc_equals_spmmv_twice_second_smaller():
    from paper_1307_6209_amd import sellcs
    big = synth.powerlaw(200_000, seed=71)
    small = synth.powerlaw(30_000, seed=72)
    hb = build(big, 32, big.nrows, kmax=64)
    hs = build(small, 16, 1024, kmax=64)
    assert hb.info["nsplit"] > 0 and hs.info["nsplit"] > 0
    for (h, A, k, seed) in ((hb, big, 64, 1), (hs, small, 8, 2)):
        X = synth.block_vector(A.ncols, k, seed=700 + seed)
        want = run(sellcs.sell_spmmv, h, X)
        got = run(sellcs.sell_spmmv_noalloc, h, X)
        say("noalloc n", A.nrows, "k", k, "nsplit", h.info["nsplit"])
        assert np.all(np.isfinite(got)) and same_bits(got, want)


@pytest.mark.parametrize("k", [1, 2, 4, 16, 32])
def test_noalloc_each_kernel_path(k):
    """k = 1 (the single-vector kernels), the pass kernel (k = 2, 4) and the
    one-pass row kernels (k = 16, 32 at beta >= 0.5), on a split layout, then
    again on a layout without split chunks (no scratch used)."""
    from paper_1307_6209_amd import sellcs
    A = synth.powerlaw(50_000, seed=73)
    for h in (build(A, 32, A.nrows, kmax=32, seg_cols=64), build(A, 32, 1, seg_cols=-1)):
        X = synth.block_vector(A.ncols, k, seed=710 + k)
        assert same_bits(run(sellcs.sell_spmmv_noalloc, h, X), run(sellcs.sell_spmmv, h, X))


def test_noalloc_k_beyond_kmax():
    """The handle's buffer holds the segment sums of kmax = 8 right-hand
    sides; the scratch takes k = 48 on the same layout. Reference: the same
    layout built with kmax = 64 (same kernels, same order)."""
    from paper_1307_6209_amd import sellcs
    A = synth.powerlaw(60_000, seed=74)
    h8 = build(A, 32, A.nrows, kmax=8)
    h64 = build(A, 32, A.nrows, kmax=64)
    assert h8.info["nsplit"] > 0
    X = synth.block_vector(A.ncols, 48, seed=720)
    with pytest.raises(sellcs.SellError):
        run(sellcs.sell_spmmv, h8, X)
    assert same_bits(run(sellcs.sell_spmmv_noalloc, h8, X), run(sellcs.sell_spmmv, h64, X))


def test_noalloc_refuses_sizes_beyond_the_scratch():
    import torch
    from paper_1307_6209_amd import sellcs
    A = synth.powerlaw(200_000, seed=77)
    h = build(A, 32, A.nrows, kmax=32, seg_cols=64)
    k = 1024  # pass kernel, 16 per pass: the segment sums need more than 64 MiB
    rows = 32 * h.info["nsplit"]
    assert h.info["nsplit"] > 0
    X = torch.zeros((A.ncols, k), dtype=torch.float64, device="cuda")
    Y = torch.zeros((A.nrows, k), dtype=torch.float64, device="cuda")
    with pytest.raises(sellcs.SellError) as e:
        sellcs.sell_spmmv_noalloc(h, X, Y)
    assert e.value.status == sellcs.SELL_ERR_UNSUPPORTED and "scratch" in str(e.value)
    say("refused:", str(e.value), "split slices", rows // 32)
    # a width that fits still runs, after the refusal
    X = synth.block_vector(A.ncols, 16, seed=730)
    assert np.all(np.isfinite(run(sellcs.sell_spmmv_noalloc, h, X)))
