"""Error behaviour of the library on the device (malformed CRS detected by
the validation kernels, bad dtype/size combinations)."""
import pytest

import synth
from gpu_util import build, dev_crs, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("breakage", ["rpt0", "decr", "rptn", "colhi", "colneg"])
def test_bad_crs(breakage):
    from paper_1307_6209_amd import sellcs
    A = synth.random_crs(300, 200, seed=11, max_len=5, empty_frac=0.0)
    rpt, col = A.rpt.copy(), A.col.copy()
    if breakage == "rpt0":
        rpt[0] = 1
    elif breakage == "decr":
        rpt[5], rpt[6] = rpt[6], rpt[5] - 1
    elif breakage == "rptn":
        rpt[-1] -= 1
    elif breakage == "colhi":
        col[3] = 200
    else:
        col[77] = -1
    B = synth.CRS(A.nrows, A.ncols, rpt, col, A.val)
    say("bad crs", breakage)
    with pytest.raises(sellcs.SellError) as ei:
        build(B, 32, 1)
    assert ei.value.status == sellcs.SELL_ERR_BAD_CRS


def test_unsupported_and_invalid():
    from paper_1307_6209_amd import sellcs
    import torch
    A = synth.random_crs(100, 50, seed=3, max_len=5)
    rpt, col, val = dev_crs(A)
    with pytest.raises(sellcs.SellError) as ei:
        sellcs.sell_build(rpt, col, val, A.ncols, 24, 1)
    assert ei.value.status == sellcs.SELL_ERR_UNSUPPORTED
    with pytest.raises(sellcs.SellError) as ei:
        sellcs.sell_build(rpt, col, val, A.ncols, 32, 0)
    assert ei.value.status == sellcs.SELL_ERR_INVALID_ARG
    with pytest.raises(sellcs.SellError):
        sellcs.sell_build(rpt, col, val, A.ncols, 32, 1, val_dtype="f64", acc_dtype="f32")
    h = sellcs.sell_build(rpt, col, val, A.ncols, 32, 1, val_dtype="f32")
    X = torch.zeros(A.ncols, 4, dtype=torch.float32, device="cuda")
    Y = torch.zeros(A.nrows, 4, dtype=torch.float32, device="cuda")
    with pytest.raises(sellcs.SellError) as ei:
        sellcs.sell_spmmv(h, X, Y)
    assert ei.value.status == sellcs.SELL_ERR_UNSUPPORTED
    with pytest.raises(TypeError):
        sellcs.sell_spmv(h, torch.zeros(A.ncols, dtype=torch.float64, device="cuda"),
                         torch.zeros(A.nrows, dtype=torch.float32, device="cuda"))


@pytest.mark.parametrize("fail_after", [0, 1, 2, 3, 4, 5, 6, 7])
def test_allocation_failure_midway_frees_everything(fail_after):
    """The n-th device allocation fails: sell_build returns SELL_ERR_OOM and
    every block it had obtained is given back to the allocator."""
    from paper_1307_6209_amd import sellcs
    A = synth.powerlaw(20_000, seed=12)
    rpt, col, val = dev_crs(A)
    al = sellcs.TorchAllocator(fail_after=fail_after)
    with pytest.raises(sellcs.SellError) as ei:
        sellcs.sell_build(rpt, col, val, A.ncols, 32, 1, seg_cols=64, allocator=al)
    assert ei.value.status == sellcs.SELL_ERR_OOM
    assert not al.live and al.frees == min(fail_after, al.calls)


def test_torch_allocator_build_and_destroy():
    from paper_1307_6209_amd import sellcs
    import torch
    A = synth.powerlaw(20_000, seed=13)
    rpt, col, val = dev_crs(A)
    al = sellcs.TorchAllocator()
    h = sellcs.sell_build(rpt, col, val, A.ncols, 32, 256, seg_cols=64, allocator=al)
    assert al.live and h.info["device_bytes"] > 0
    x = synth.uniform(A.ncols, 14, 1)
    from gpu_util import spmv_gpu, check_fp64
    check_fp64(A, spmv_gpu(h, x), x)
    h.close()
    assert not al.live and al.frees == al.calls
