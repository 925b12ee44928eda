"""The product whose lanes stop at their rows' ends (build option
row_lengths; the GPU form of the kernel that Sect. 3.4 describes): on every
layout the same bits as the plain product of the same layout, and the
oracle's bound, over chunk heights, sorting scopes, slots per lane, steps in
flight, value types, split chunks, groups of short chunks and empty rows;
the full-size power-law matrix at the sorting scopes the benchmark times."""
import numpy as np
import pytest

import synth
from gpu_util import build, check_fp64, check_reduced, say, spmv_gpu

pytestmark = pytest.mark.gpu

MATS = {
    "random": lambda: synth.random_crs(301, 90, seed=1, max_len=30, empty_frac=0.3, duplicates=True, unsorted=True),
    "nonsquare_wide": lambda: synth.random_crs(77, 5000, seed=2, max_len=300, empty_frac=0.1),
    "powerlaw_50k": lambda: synth.powerlaw(50_000, seed=3),
    "stencil27_24": lambda: synth.stencil27(24),
}
CS = [(8, 1), (16, 1), (16, 256), (32, 1), (32, 10**9), (64, 1), (64, 4096)]


def bits(y):
    return np.ascontiguousarray(y, np.float64).view(np.uint64)


def pair(A, C, sigma, **kw):
    """The plain handle and the one with row lengths, same layout."""
    h0 = build(A, C, sigma, xwindow=-1, **kw)
    h1 = build(A, C, sigma, xwindow=-1, row_lengths=True, **kw)
    i0, i1 = h0.info, h1.info
    assert i1["row_lengths"] == 1 and i0["row_lengths"] == 0
    assert i1["padded"] == i0["padded"] and i1["nunits"] == i0["nunits"]
    assert i1["device_bytes"] >= i0["device_bytes"] + 4 * i0["nchunks"] * C
    return h0, h1


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("C,sigma", CS)
@pytest.mark.parametrize("unroll,vec", [(4, 1), (8, 1), (4, 2), (8, 2), (4, 4), (8, 4), (0, 0)])
def test_same_bits_as_plain_product(name, C, sigma, unroll, vec):
    if vec > C:
        pytest.skip("vec <= C")
    A = MATS[name]()
    x = synth.uniform(A.ncols, 21, 1)
    say("row lengths", name, "C", C, "sigma", sigma, "U", unroll, "V", vec)
    h0, h1 = pair(A, C, sigma, unroll=unroll, vec=vec)
    y0, y1 = spmv_gpu(h0, x), spmv_gpu(h1, x)
    assert np.array_equal(bits(y1), bits(y0))
    check_fp64(A, y1, x)


@pytest.mark.parametrize("val_dtype,acc", [("f32", "f32"), ("f32", "f64"), ("bf16", "f32"), ("bf16", "f64")])
@pytest.mark.parametrize("C,sigma", [(16, 1), (32, 1024), (32, 10**9), (64, 1)])
@pytest.mark.parametrize("vec", [1, 2, 4])
def test_reduced_precision(val_dtype, acc, C, sigma, vec):
    A = synth.powerlaw(50_000, seed=4)
    x = synth.uniform(A.ncols, 22, 1)
    say("row lengths", val_dtype, acc, "C", C, "sigma", sigma, "V", vec)
    h0, h1 = pair(A, C, sigma, val_dtype=val_dtype, acc_dtype=acc, vec=vec)
    xr = x.astype(np.float32).astype(np.float64)
    assert np.array_equal(bits(spmv_gpu(h1, xr)), bits(spmv_gpu(h0, xr)))
    check_reduced(A, h1, x, val_dtype, acc, C)


@pytest.mark.parametrize("seg", [64, 448])
@pytest.mark.parametrize("C,vec", [(8, 1), (8, 4), (32, 1), (32, 2), (64, 4)])
@pytest.mark.parametrize("sigma", [1, 4096])
def test_split_chunks(seg, C, vec, sigma):
    """Long chunks cut into segments: each segment's lanes stop at their rows'
    ends; the combining kernel adds the same sums."""
    A = synth.powerlaw(40_000, seed=8)
    x = synth.uniform(A.ncols, 23, 1)
    say("row lengths split", "C", C, "seg", seg, "V", vec, "sigma", sigma)
    h0, h1 = pair(A, C, sigma, seg_cols=seg, vec=vec)
    assert h1.info["nsplit"] > 0
    y1 = spmv_gpu(h1, x)
    assert np.array_equal(bits(y1), bits(spmv_gpu(h0, x)))
    check_fp64(A, y1, x)
    for _ in range(2):
        assert np.array_equal(bits(spmv_gpu(h1, x)), bits(y1))


def test_empty_rows_and_no_nonzeros():
    A = synth.random_crs(500, 40, seed=14, max_len=6, empty_frac=0.7)
    x = synth.uniform(40, 24, 1)
    for C, sigma in [(32, 1), (16, 64), (8, 500)]:
        h0, h1 = pair(A, C, sigma)
        y1 = spmv_gpu(h1, x)
        assert np.all(y1[A.row_lengths() == 0] == 0.0)
        assert np.array_equal(bits(y1), bits(spmv_gpu(h0, x)))
        check_fp64(A, y1, x)
    E = synth.CRS(100, 30, np.zeros(101, np.int64), np.zeros(0, np.int32), np.zeros(0))
    h = build(E, 32, 1, row_lengths=True)
    assert np.array_equal(spmv_gpu(h, np.ones(30)), np.zeros(100))


def test_window_layout_keeps_the_window():
    """With an x window the window product runs (it does not read the row
    lengths); the result is still the plain product's."""
    A = synth.stencil27(40)
    x = synth.uniform(A.ncols, 25, 1)
    h0 = build(A, 32, 1, xwindow=1)
    h1 = build(A, 32, 1, xwindow=1, row_lengths=True)
    assert h1.info["xwindow"] == 1 and h1.info["row_lengths"] == 1
    assert np.array_equal(bits(spmv_gpu(h1, x)), bits(spmv_gpu(h0, x)))


@pytest.fixture(scope="module")
def powerlaw_2m():
    A = synth.workload("powerlaw_2m")
    return A, synth.uniform(A.ncols, synth.SEED_X + 1)


@pytest.mark.parametrize("sigma", [1, 1024, 16384])
def test_powerlaw_2m_full_size(powerlaw_2m, sigma):
    A, x = powerlaw_2m
    say("row lengths powerlaw_2m C 32 sigma", sigma)
    h0, h1 = pair(A, 32, sigma)
    y1 = spmv_gpu(h1, x)
    assert np.array_equal(bits(y1), bits(spmv_gpu(h0, x)))
    check_fp64(A, y1, x)
