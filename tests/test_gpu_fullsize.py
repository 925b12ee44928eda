"""Parity at the full workload sizes, in the launch configurations the
benchmark times: 5-point Laplacian 128^2, power-law n = 2,000,000 (C and
sigma sweep), 27-point stencil 160^3, the block form on the power-law
n = 1,000,000 matrix (pass kernel and one-pass row kernels), 64 uneven
matrices in one batched launch (one wave per unit and persistent), and the
reduced-precision forms (x window and global indices). Every result is
compared element by element with the oracle; FP64 within the smaller of
1e-13 (|A||x|)_i and the bound of each row's summation chain."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import (assert_layout_equal, batch_chain_per_row, build, chain_per_row, check_fp64, check_reduced,
                      say, spmv_gpu)

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def powerlaw_2m():
    A = synth.workload("powerlaw_2m")
    x = synth.uniform(A.ncols, synth.SEED_X + 1)
    return A, x


@pytest.fixture(scope="module")
def stencil_160():
    A = synth.workload("stencil27_160")
    x = synth.uniform(A.ncols, synth.SEED_X + 2)
    return A, x


def test_lap5_128():
    A = synth.workload("lap5_128")
    x = synth.uniform(A.ncols, synth.SEED_X)
    h = build(A, 32, 1)
    want = assert_layout_equal(A, h, 32, 1)
    assert want["padded"] == 81_664
    check_fp64(A, spmv_gpu(h, x), x, m=chain_per_row(A, h, 32))


SWEEP = [(C, s) for C in (16, 32, 64, 128) for s in (1, C, 2**10, 2**14, 2_000_000)]
FULL_LAYOUT = {(16, 2_000_000), (32, 1), (128, 2**14), (64, 2**10)}


@pytest.mark.parametrize("C,sigma", SWEEP)
def test_powerlaw_2m_sweep(powerlaw_2m, C, sigma):
    from paper_1307_6209_amd import sellcs
    A, x = powerlaw_2m
    say("powerlaw_2m C", C, "sigma", sigma)
    h = build(A, C, sigma)
    if (C, sigma) in FULL_LAYOUT:
        assert_layout_equal(A, h, C, sigma)
    else:
        perm, cl, cs = oracle.sell_layout(A, C, sigma)
        got = sellcs.sell_export(h)
        assert np.array_equal(got["perm"], perm) and np.array_equal(got["cl"], cl) and np.array_equal(got["cs"], cs)
    say("beta", h.info["beta"], "nsplit", h.info["nsplit"])
    check_fp64(A, spmv_gpu(h, x), x, m=chain_per_row(A, h, C))
    h.close()


@pytest.mark.parametrize("sigma", [1, 2**10, 2**17])
def test_stencil27_160(stencil_160, sigma):
    A, x = stencil_160
    say("stencil27_160 sigma", sigma)
    h = build(A, 32, sigma)
    if sigma == 1:
        want = assert_layout_equal(A, h, 32, 1)
        assert want["padded"] == 109_672_320
    else:
        from paper_1307_6209_amd import sellcs
        perm, cl, cs = oracle.sell_layout(A, 32, sigma)
        got = sellcs.sell_export(h)
        assert np.array_equal(got["perm"], perm) and np.array_equal(got["cl"], cl) and np.array_equal(got["cs"], cs)
    check_fp64(A, spmv_gpu(h, x), x, m=chain_per_row(A, h, 32))
    h.close()


PRECISION = [("f32", "f32"), ("f32", "f64"), ("bf16", "f32"), ("bf16", "f64")]


# the benchmark's reduced-precision forms on the stencil: the x window (16-bit
# window positions) at C = 32 and at C = 64 with two slots per lane, and the
# global int32 column indices at C = 32
@pytest.mark.parametrize("C,xwindow,vec", [(32, 0, 0), (64, 0, 2), (32, -1, 0)])
@pytest.mark.parametrize("val_dtype,acc", PRECISION)
def test_precision_stencil_160(stencil_160, val_dtype, acc, C, xwindow, vec):
    A, x = stencil_160
    say("stencil27_160", val_dtype, acc, "C", C, "xwindow", xwindow, "vec", vec)
    h = build(A, C, 1, val_dtype=val_dtype, acc_dtype=acc, xwindow=xwindow, vec=vec)
    inf = h.info
    assert inf["xwindow"] == (1 if xwindow == 0 else 0)
    if vec:
        assert inf["vec"] == vec
    comp, norm = check_reduced(A, h, x, val_dtype, acc, C)
    say("  componentwise %.3g normwise %.3g" % (comp, norm))
    h.close()


@pytest.mark.parametrize("val_dtype,acc", PRECISION)
def test_precision_powerlaw_2m(powerlaw_2m, val_dtype, acc):
    A, x = powerlaw_2m
    h = build(A, 32, 2_000_000, val_dtype=val_dtype, acc_dtype=acc)
    comp, norm = check_reduced(A, h, x, val_dtype, acc, 32)
    say("powerlaw_2m", val_dtype, acc, "componentwise %.3g normwise %.3g" % (comp, norm))
    h.close()


@pytest.fixture(scope="module")
def powerlaw_1m():
    return synth.workload("powerlaw_1m")


def spmmv_check(A, h, C, k, seed, **kw):
    import torch
    from paper_1307_6209_amd import sellcs
    X = synth.block_vector(A.ncols, k, seed=seed)
    Xd = torch.from_numpy(X).cuda()
    Y = torch.full((A.nrows, k), float("nan"), dtype=torch.float64, device="cuda")
    sellcs.sell_spmmv(h, Xd, Y)
    torch.cuda.synchronize()
    Yg = Y.cpu().numpy()
    del Xd, Y
    Yh, aY = oracle.crs_spmmv_hi(A, X)
    assert np.all(np.isfinite(Yg))
    m = chain_per_row(A, h, C, block=k > 1)
    g = np.minimum(1e-13, gamma_rows(m, A))
    err = np.abs(Yg - Yh)
    ok = err <= g[:, None] * aY
    assert np.all(ok), "k %d: max rel err %g" % (k, float(np.max(err / np.where(aY > 0, aY, 1))))
    return float(np.max(err / np.where(aY > 0, aY, 1)))


def gamma_rows(m, A):
    from gpu_util import gamma
    return gamma(np.asarray(m) + 1, 2.0 ** -53) * 1.0001 + gamma(A.row_lengths(), 2.0 ** -64)


def test_spmmv_powerlaw_1m_sigma1024(powerlaw_1m):
    A = powerlaw_1m
    h = build(A, 32, 1024, kmax=64)
    for k in (1, 4, 8, 16, 32, 64):
        say("spmmv SELL-32-1024 k", k, "max rel err %.3g" % spmmv_check(A, h, 32, k, synth.SEED_X + 3))
    h.close()


# SELL-32-n with the automatic pass width: k = 16, 32 and 64 run the one-pass
# row kernel (beta >= 0.5) and add the segment sums of the split rows with
# the block-form combine, as in the benchmark
def test_spmmv_powerlaw_1m_sigma_n(powerlaw_1m):
    A = powerlaw_1m
    h = build(A, 32, A.nrows, kmax=64)
    assert h.info["beta"] >= 0.5 and h.info["nsplit"] > 0
    for k in (1, 4, 8, 16, 32, 64):
        say("spmmv SELL-32-n k", k, "max rel err %.3g" % spmmv_check(A, h, 32, k, synth.SEED_X + 4))
    h.close()


# the pass kernel's best shape at k = 32 (C = 16, sigma = n, 16 right-hand
# sides per pass; the autotuner's winner before the one-pass kernel took
# k = 32)
def test_spmmv_powerlaw_1m_tuned_k32(powerlaw_1m):
    A = powerlaw_1m
    h = build(A, 16, A.nrows, kmax=32, ktile=16)
    say("spmmv SELL-16-n ktile 16 k 32", "max rel err %.3g" % spmmv_check(A, h, 16, 32, synth.SEED_X + 5))
    h.close()


@pytest.mark.parametrize("C", [16, 32])
@pytest.mark.parametrize("form", ["sell_batch_create", "sell_batch_create_persistent"])
@pytest.mark.parametrize("sigma", ["mixed", "n"])
def test_batch_64(form, sigma, C):
    """The 64-matrix batch in both launch forms, at C = 32 and at the batch
    autotuner's choice on this workload, C = 16."""
    import torch
    from paper_1307_6209_amd import sellcs
    mats = synth.batch_workload(64)
    say("batch", form, "C", C, "sigma", sigma, "rows", sum(A.nrows for A in mats), "nnz", sum(A.nnz for A in mats))
    sig = [1, 32, 1024, 16384]
    hs = [build(A, C, sig[i % 4] if sigma == "mixed" else A.nrows) for i, A in enumerate(mats)]
    b = getattr(sellcs, form)(hs)
    xs = [synth.uniform(A.ncols, synth.SEED_X + 10 + i) for i, A in enumerate(mats)]
    xd = [torch.from_numpy(x).cuda() for x in xs]
    yd = [torch.full((A.nrows,), float("nan"), dtype=torch.float64, device="cuda") for A in mats]
    sellcs.sell_batch_spmv(b, xd, yd)
    torch.cuda.synchronize()
    for A, h, x, y in zip(mats, hs, xs, yd):
        check_fp64(A, y.cpu().numpy(), x, m=batch_chain_per_row(A, h, C))
    b.close()
