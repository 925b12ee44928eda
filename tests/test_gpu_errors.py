"""Error behaviour of the library on the device (malformed CRS detected by
the validation kernels, bad dtype/size combinations)."""
import numpy as np
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
