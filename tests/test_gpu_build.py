"""GPU construction (row lengths, sigma-window sort, chunk widths, offsets,
padded fill) against the oracle, bit for bit."""
import numpy as np
import pytest

import synth
from gpu_util import assert_layout_equal, build, say

pytestmark = pytest.mark.gpu

SMALL = [
    ("random", lambda: synth.random_crs(301, 90, seed=1, max_len=30, empty_frac=0.3, duplicates=True, unsorted=True)),
    ("random_wide", lambda: synth.random_crs(77, 5000, seed=2, max_len=300, empty_frac=0.1)),
    ("lap5_128", lambda: synth.lap5(128)),
    ("powerlaw_50k", lambda: synth.powerlaw(50_000, seed=3)),
    ("stencil27_24", lambda: synth.stencil27(24)),
    ("worst_beta", lambda: synth.worst_case_beta(4, 64)),
]
CS = [(1, 1), (2, 3), (4, 1), (8, 16), (16, 1), (16, 10**9), (32, 1), (32, 32), (32, 1000), (64, 1), (64, 4096),
      (64, 4097), (128, 1), (128, 20000), (32, 2**14)]


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
@pytest.mark.parametrize("C,sigma", CS)
def test_layout_bit_exact(name, make, C, sigma):
    A = make()
    say("build", name, A.nrows, A.nnz, "C", C, "sigma", sigma)
    h = build(A, C, sigma)
    assert_layout_equal(A, h, C, sigma)
    h.close()


@pytest.mark.parametrize("val_dtype,acc", [("f32", "f32"), ("f32", "f64"), ("bf16", "f32"), ("bf16", "f64")])
@pytest.mark.parametrize("C,sigma", [(32, 1), (16, 256), (128, 50_000)])
def test_converted_values_bit_exact(val_dtype, acc, C, sigma):
    A = synth.powerlaw(60_000, seed=4)
    # spread magnitudes over the whole binary32 / bfloat16 range, subnormals included
    e = (synth.u64(4, 9, A.nnz) % np.uint64(300)).astype(np.int64) - 150
    A.val = np.ldexp(A.val, e)
    say("convert", val_dtype, acc, C, sigma)
    h = build(A, C, sigma, val_dtype=val_dtype, acc_dtype=acc)
    assert_layout_equal(A, h, C, sigma, val_dtype)


def test_empty_and_degenerate():
    for A in [synth.CRS(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0)),
              synth.CRS(7, 3, np.zeros(8, np.int64), np.zeros(0, np.int32), np.zeros(0)),
              synth.CRS(1, 1, np.array([0, 1], np.int64), np.zeros(1, np.int32), np.ones(1))]:
        for C, sigma in [(1, 1), (32, 1), (4, 100)]:
            say("degenerate", A.nrows, A.nnz, C, sigma)
            h = build(A, C, sigma)
            if A.nrows:
                assert_layout_equal(A, h, C, sigma)
            assert h.info["beta"] == (1.0 if A.nnz == 0 else A.nnz / h.info["padded"])


def test_info_fields():
    A = synth.powerlaw(20_000, seed=6)
    h = build(A, 32, 64)
    inf = h.info
    assert inf["nrows"] == A.nrows and inf["nnz"] == A.nnz and inf["C"] == 32 and inf["sigma"] == 64
    assert inf["has_perm"] == 1 and inf["lanes_per_row"] == 64 * inf["vec"] // 32
    assert inf["max_row_len"] == int(A.row_lengths().max())
    L = A.row_lengths().astype(np.float64)
    assert abs(inf["zeta"] - L.std() / L.mean()) < 1e-9
