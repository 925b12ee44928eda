"""Seeded random sweep over the build and product options: matrix shape
(random, banded, power-law, stencil, Laplacian), C, sigma, value and
accumulation types, slots per lane, unroll, split width, x path, row
lengths (every third case with C in 8..64; then also bit for bit against
the plain product) and, for FP64 handles, the block form. Every result is checked against the oracle
with the bound of the summation chain of each row (the terms one lane adds,
the cross-lane sum and the segments of a split row), capped at
1e-13 (|A||x|)_i for FP64."""
import numpy as np
import pytest

import synth
from gpu_util import build, chain_per_row, check_fp64, check_reduced, say, spmv_gpu

pytestmark = pytest.mark.gpu

COMBOS = [("f64", "f64"), ("f32", "f32"), ("f32", "f64"), ("bf16", "f32"), ("bf16", "f64")]


def banded(n, seed, half, max_len):
    A = synth.random_crs(n, n, seed=seed, max_len=max_len, empty_frac=0.1)
    lens = np.diff(A.rpt)
    rows = np.repeat(np.arange(n), lens)
    col = np.clip(rows + (A.col.astype(np.int64) % (2 * half + 1)) - half, 0, n - 1)
    out = [np.unique(col[A.rpt[i]:A.rpt[i + 1]]) for i in range(n)]
    rpt = np.zeros(n + 1, np.int64)
    np.cumsum([len(c) for c in out], out=rpt[1:])
    cc = np.concatenate(out).astype(np.int32) if rpt[-1] else np.zeros(0, np.int32)
    return synth.CRS(n, n, rpt, cc, synth.uniform(int(rpt[-1]), seed, 3))


def matrix(rng, case):
    kind = case % 5
    if kind == 0:
        nr, nc = int(rng.integers(1, 3000)), int(rng.integers(1, 5000))
        return "random", synth.random_crs(nr, nc, seed=100 + case, max_len=int(rng.integers(1, 80)),
                                          empty_frac=float(rng.uniform(0, 0.5)), duplicates=bool(rng.integers(2)),
                                          unsorted=bool(rng.integers(2)))
    if kind == 1:
        return "banded", banded(int(rng.integers(50, 6000)), 200 + case, int(rng.integers(2, 60)),
                                int(rng.integers(2, 40)))
    if kind == 2:
        return "powerlaw", synth.powerlaw(int(rng.integers(1000, 20000)), seed=300 + case)
    if kind == 3:
        return "stencil27", synth.stencil27(int(rng.integers(3, 22)))
    return "lap5", synth.lap5(int(rng.integers(4, 70)))


@pytest.mark.parametrize("case", range(160))
def test_random_configuration(case):
    from paper_1307_6209_amd import sellcs
    import torch
    rng = np.random.default_rng(9000 + case)
    name, A = matrix(rng, case)
    C = int(rng.choice([1, 2, 4, 8, 16, 32, 64, 128]))
    sigma = int(rng.choice([1, C, int(rng.integers(1, max(2, A.nrows + 1))), max(1, A.nrows), A.nrows + 7]))
    val_dtype, acc = COMBOS[int(rng.integers(len(COMBOS)))]
    vecs = [0, 1] + [v for v in (2, 4) if C <= 64 and v <= C]
    vec = int(rng.choice(vecs))
    unroll = int(rng.choice([0, 4, 8, 16]))
    seg = int(rng.choice([0, -1, 64, 256]))
    xw = int(rng.choice([-1, 0, 1]))
    rl = 8 <= C <= 64 and case % 3 == 1  # outside the random draws: they stay those of every case
    say("sweep case", case, name, "n", A.nrows, "m", A.ncols, "nnz", A.nnz, "C", C, "sigma", sigma, val_dtype, acc,
        "vec", vec, "unroll", unroll, "seg", seg, "xwindow", xw, "row_lengths", rl)
    kw = dict(val_dtype=val_dtype, acc_dtype=acc, vec=vec, unroll=unroll, seg_cols=seg, xwindow=xw, kmax=64,
              row_lengths=rl)
    try:
        h = build(A, C, sigma, **kw)
    except sellcs.SellError as e:
        # the x window is refused where it cannot be built (C outside 8..64,
        # split chunks, vec 4, windows too large): then the global-index path
        assert xw == 1 and e.status == sellcs.SELL_ERR_UNSUPPORTED, (e.status, str(e))
        kw["xwindow"] = 0
        h = build(A, C, sigma, **kw)
    inf = h.info
    say("  built: vec", inf["vec"], "unroll", inf["unroll"], "xwindow", inf["xwindow"], "nsplit", inf["nsplit"],
        "beta", round(inf["beta"], 4))
    x = synth.uniform(A.ncols, 500 + case, 1)
    if rl:  # lanes stopped at their rows' ends: the plain product's bits
        plain = build(A, C, sigma, **dict(kw, row_lengths=False))
        xr = x if val_dtype == "f64" else x.astype(np.float32).astype(np.float64)
        assert np.array_equal(spmv_gpu(h, xr).view(np.uint64), spmv_gpu(plain, xr).view(np.uint64))
    if val_dtype == "f64":
        y = spmv_gpu(h, x)
        check_fp64(A, y, x, m=chain_per_row(A, h, C))
        assert np.array_equal(spmv_gpu(h, x).view(np.uint64), y.view(np.uint64))
        if C >= 8 and A.nrows > 0:
            k = int(rng.choice([2, 3, 8, 16, 32, 40, 64, 100]))
            X = synth.block_vector(A.ncols, k, seed=600 + case)
            Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
            Y = torch.full((A.nrows, k), float("nan"), dtype=torch.float64, device="cuda")
            say("  block form k", k)
            if inf["nsplit"] > 0 and k > 64:  # beyond the kmax the partial sums were sized for
                with pytest.raises(sellcs.SellError):
                    sellcs.sell_spmmv(h, Xd, Y)
                return
            sellcs.sell_spmmv(h, Xd, Y)
            torch.cuda.synchronize()
            Yc = Y.cpu().numpy()
            m = chain_per_row(A, h, C, block=True)
            for v in range(k):
                check_fp64(A, Yc[:, v].copy(), X[:, v].copy(), m=m)
    else:
        check_reduced(A, h, x, val_dtype, acc, C)
