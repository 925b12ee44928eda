"""Reduced-precision forms: values stored in FP32 or BF16 (rounded to nearest
even from FP64 at build), x in FP32, accumulation in FP32 or FP64, with
componentwise error bounds against the oracle."""
import pytest

import synth
from gpu_util import build, check_reduced, say

pytestmark = pytest.mark.gpu

FORMS = [("f32", "f32"), ("f32", "f64"), ("bf16", "f32"), ("bf16", "f64")]


@pytest.mark.parametrize("val_dtype,acc", FORMS)
@pytest.mark.parametrize("vec", [0, 1, 2, 4])
@pytest.mark.parametrize("name,make,C,sigma", [
    ("stencil27_24", lambda: synth.stencil27(24), 32, 1),
    ("powerlaw_60k", lambda: synth.powerlaw(60_000, seed=21), 32, 1024),
    ("powerlaw_60k_c128", lambda: synth.powerlaw(60_000, seed=21), 128, 60_000),
    ("random", lambda: synth.random_crs(500, 300, seed=5, max_len=40, empty_frac=0.2, duplicates=True), 8, 16),
])
def test_reduced_precision_bounds(val_dtype, acc, vec, name, make, C, sigma):
    if vec > 1 and (C > 64 or vec > C):
        pytest.skip("vec > 1 needs C <= 64 and vec <= C")
    A = make()
    x = synth.uniform(A.ncols, 31, 1)
    h = build(A, C, sigma, val_dtype=val_dtype, acc_dtype=acc, vec=vec)
    comp, norm = check_reduced(A, h, x, val_dtype, acc, C)
    say("precision", name, val_dtype, acc, "componentwise %.3g normwise %.3g" % (comp, norm))


@pytest.mark.parametrize("val_dtype,acc", FORMS)
def test_reduced_precision_split(val_dtype, acc):
    A = synth.powerlaw(40_000, seed=22)
    x = synth.uniform(A.ncols, 32, 1)
    h = build(A, 16, 1, val_dtype=val_dtype, acc_dtype=acc, seg_cols=64)
    assert h.info["nsplit"] > 0
    check_reduced(A, h, x, val_dtype, acc, 16)
