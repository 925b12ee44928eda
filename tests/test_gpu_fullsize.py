"""Parity at the full workload sizes, in the launch configuration the
benchmark times: 5-point Laplacian 128^2, power-law n = 2,000,000 (C and
sigma sweep), 27-point stencil 160^3, the block form on the power-law
n = 1,000,000 matrix, 64 uneven matrices in one batched launch, and the
reduced-precision forms."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_layout_equal, build, check_fp64, check_reduced, say, spmv_gpu

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
    check_fp64(A, spmv_gpu(h, x), x)


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
    check_fp64(A, spmv_gpu(h, x), x)
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
    check_fp64(A, spmv_gpu(h, x), x)
    h.close()


@pytest.mark.parametrize("val_dtype,acc", [("f32", "f32"), ("f32", "f64"), ("bf16", "f32"), ("bf16", "f64")])
def test_precision_stencil_160(stencil_160, val_dtype, acc):
    A, x = stencil_160
    h = build(A, 32, 1, val_dtype=val_dtype, acc_dtype=acc)
    comp, norm = check_reduced(A, h, x, val_dtype, acc, 32)
    say("stencil27_160", val_dtype, acc, "componentwise %.3g normwise %.3g" % (comp, norm))
    h.close()


@pytest.mark.parametrize("val_dtype,acc", [("f32", "f32"), ("bf16", "f64")])
def test_precision_powerlaw_2m(powerlaw_2m, val_dtype, acc):
    A, x = powerlaw_2m
    h = build(A, 32, 2_000_000, val_dtype=val_dtype, acc_dtype=acc)
    comp, norm = check_reduced(A, h, x, val_dtype, acc, 32, nseg_max=200)
    say("powerlaw_2m", val_dtype, acc, "componentwise %.3g normwise %.3g" % (comp, norm))
    h.close()


def test_spmmv_powerlaw_1m():
    import torch
    from paper_1307_6209_amd import sellcs
    A = synth.workload("powerlaw_1m")
    h = build(A, 32, 1024)
    for k in (1, 4, 8, 16, 32):
        X = synth.block_vector(A.ncols, k, seed=synth.SEED_X + 3)
        Xd = torch.from_numpy(X).cuda()
        Y = torch.full((A.nrows, k), float("nan"), dtype=torch.float64, device="cuda")
        sellcs.sell_spmmv(h, Xd, Y)
        torch.cuda.synchronize()
        Yh, aY = oracle.crs_spmmv_hi(A, X)
        Yg = Y.cpu().numpy()
        say("spmmv k", k)
        assert np.all(np.abs(Yg - Yh) <= 1e-13 * aY)


def test_batch_64():
    import torch
    from paper_1307_6209_amd import sellcs
    mats = synth.batch_workload(64)
    say("batch rows", sum(A.nrows for A in mats), "nnz", sum(A.nnz for A in mats))
    sig = [1, 32, 1024, 16384]
    hs = [build(A, 32, sig[i % 4]) for i, A in enumerate(mats)]
    b = sellcs.sell_batch_create(hs)
    xs = [synth.uniform(A.ncols, synth.SEED_X + 10 + i) for i, A in enumerate(mats)]
    xd = [torch.from_numpy(x).cuda() for x in xs]
    yd = [torch.full((A.nrows,), float("nan"), dtype=torch.float64, device="cuda") for A in mats]
    sellcs.sell_batch_spmv(b, xd, yd)
    torch.cuda.synchronize()
    for A, x, y in zip(mats, xs, yd):
        check_fp64(A, y.cpu().numpy(), x)
