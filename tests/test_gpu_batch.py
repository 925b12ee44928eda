"""One hipGraph-captured launch over many matrices of uneven
size: each result against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import batch_chain_per_row, build, check_fp64, check_reduced_y, say

pytestmark = pytest.mark.gpu

# both forms of the batched launch: one wave per unit, and persistent
FORMS = ["sell_batch_create", "sell_batch_create_persistent"]


def create(form, hs):
    from paper_1307_6209_amd import sellcs
    return getattr(sellcs, form)(hs)


def make_batch(count, seed, lo=1000, hi=20000):
    sizes = synth.batch_sizes(count, seed, lo, hi)
    return [synth.powerlaw(int(n), seed=seed * 100 + b) for b, n in enumerate(sizes)]


def run(b, mats, xs, dtype):
    import torch
    from paper_1307_6209_amd import sellcs
    xd = [torch.from_numpy(np.ascontiguousarray(x)).cuda().to(dtype[0]) for x in xs]
    yd = [torch.full((A.nrows,), float("nan"), dtype=dtype[1], device="cuda") for A in mats]
    sellcs.sell_batch_spmv(b, xd, yd)
    torch.cuda.synchronize()
    return [y.double().cpu().numpy() for y in yd]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("C", [16, 32, 64, 128])
def test_batch_fp64(C, form):
    import torch
    from paper_1307_6209_amd import sellcs
    mats = make_batch(12, 3)
    sigmas = [1, C, 256, 4096, 10**9, 1, 512, 1, 2048, C, 1, 100000]
    hs = [build(A, C, s) for A, s in zip(mats, sigmas)]
    b = create(form, hs)
    xs = [synth.uniform(A.ncols, 50 + i, 1) for i, A in enumerate(mats)]
    say("batch C", C, "rows", sum(A.nrows for A in mats))
    ys = run(b, mats, xs, (torch.float64, torch.float64))
    short = wide = False
    for A, h, x, y in zip(mats, hs, xs, ys):
        check_fp64(A, y, x, m=batch_chain_per_row(A, h, C))
    # a second call with new vectors (the pointer table is rewritten)
    xs2 = [synth.uniform(A.ncols, 80 + i, 1) for i, A in enumerate(mats)]
    ys2 = run(b, mats, xs2, (torch.float64, torch.float64))
    for A, h, x, y in zip(mats, hs, xs2, ys2):
        check_fp64(A, y, x, m=batch_chain_per_row(A, h, C))
    b.close()


@pytest.mark.parametrize("form", FORMS)
def test_batch_repeat_same_pointers_is_deterministic(form):
    import torch
    from paper_1307_6209_amd import sellcs
    mats = make_batch(20, 4, 1000, 50000)
    hs = [build(A, 32, 64) for A in mats]
    b = create(form, hs)
    xd = [torch.from_numpy(synth.uniform(A.ncols, 9, 1)).cuda() for A in mats]
    yd = [torch.empty(A.nrows, dtype=torch.float64, device="cuda") for A in mats]
    sellcs.sell_batch_spmv(b, xd, yd)
    torch.cuda.synchronize()
    first = [y.cpu().numpy().copy() for y in yd]
    for _ in range(5):
        sellcs.sell_batch_spmv(b, xd, yd)
    torch.cuda.synchronize()
    for f, y in zip(first, yd):
        assert np.array_equal(f, y.cpu().numpy())
    for A, x, y in zip(mats, xd, first):
        check_fp64(A, y, x.cpu().numpy())


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("val_dtype,acc", [("f32", "f32"), ("bf16", "f64")])
def test_batch_reduced(val_dtype, acc, form):
    import torch
    from paper_1307_6209_amd import sellcs
    mats = make_batch(6, 5)
    hs = [build(A, 32, 128, val_dtype=val_dtype, acc_dtype=acc) for A in mats]
    b = create(form, hs)
    xs = [oracle.round_f32(synth.uniform(A.ncols, 60 + i, 1)).astype(np.float64) for i, A in enumerate(mats)]
    ys = run(b, mats, xs, (torch.float32, torch.float64 if acc == "f64" else torch.float32))
    for A, h, x, y in zip(mats, hs, xs, ys):
        comp, norm = check_reduced_y(A, y, h, x, val_dtype, acc, 32, m=batch_chain_per_row(A, h, 32))
        say("batch", form, val_dtype, acc, "componentwise %.3g normwise %.3g" % (comp, norm))


@pytest.mark.parametrize("form", FORMS)
def test_batch_mixed_C_rejected(form):
    from paper_1307_6209_amd import sellcs
    mats = make_batch(2, 6)
    hs = [build(mats[0], 32, 1), build(mats[1], 64, 1)]
    with pytest.raises(sellcs.SellError):
        create(form, hs)


@pytest.mark.parametrize("form", FORMS)
def test_batch_graph_replays_with_eager_work_between(form):
    """Replay the captured launch several times with other eager launches and
    synchronisations in between: every replay gives the same bits, and they
    match the oracle."""
    import torch
    from paper_1307_6209_amd import sellcs
    mats = make_batch(10, 7, 1000, 60000)
    hs = [build(A, 32, [1, 64, 4096][i % 3]) for i, A in enumerate(mats)]
    b = create(form, hs)
    xs = [torch.from_numpy(synth.uniform(A.ncols, 90 + i, 1)).cuda() for i, A in enumerate(mats)]
    ys = [torch.empty(A.nrows, dtype=torch.float64, device="cuda") for A in mats]
    other = build(synth.powerlaw(30_000, seed=99), 64, 1)
    xo = torch.from_numpy(synth.uniform(30_000, 98, 1)).cuda()
    yo = torch.empty(30_000, dtype=torch.float64, device="cuda")
    first = None
    for rep in range(4):
        for y in ys:
            y.fill_(float("nan"))
        sellcs.sell_batch_spmv(b, xs, ys)
        torch.cuda.synchronize()
        got = [y.cpu().numpy().copy() for y in ys]
        if first is None:
            first = got
            for A, x, g in zip(mats, xs, got):
                check_fp64(A, g, x.cpu().numpy())
        else:
            for f, g in zip(first, got):
                assert np.array_equal(f, g)
        for hh, xx, yy in zip(hs[:3], xs[:3], ys[:3]):  # eager single-matrix work in between
            sellcs.sell_spmv(hh, xx, yy)
        sellcs.sell_spmv(other, xo, yo)
        torch.cuda.synchronize()


def test_batch_autotune_picks_model_sigmas_and_a_working_C():
    """The batch autotuner gives every matrix the sigma whose layout has the
    fewest model bytes (checked against the oracle's layouts) and returns a C
    whose batch matches the oracle."""
    import torch
    from paper_1307_6209_amd import sellcs
    from gpu_util import dev_crs
    mats = make_batch(8, 11, 1000, 30000)
    dev = [dev_crs(A) for A in mats]
    Cs, sigmas = (16, 32), (1, 256, 1 << 40)
    r = sellcs.sell_batch_autotune([(rp, cc, vv, A.ncols) for (rp, cc, vv), A in zip(dev, mats)], C=Cs,
                                   sigma=sigmas, reps=5)
    say("batch autotune", r)
    assert r["C"] in Cs and r["candidates"] == len(Cs) and r["gflops"] > 0
    for A, sg in zip(mats, r["sigmas"]):
        def model_bytes(s):
            L = oracle.sell_build(A, r["C"], s)
            return 12.0 * L["padded"] + (4.0 * A.nrows if min(s, A.nrows) > 1 else 0.0)
        best = min(sigmas, key=lambda s: (model_bytes(s), sigmas.index(s)))
        assert model_bytes(sg) == model_bytes(best)
    hs = [sellcs.sell_build(rp, cc, vv, A.ncols, r["C"], sg) for (rp, cc, vv), A, sg in zip(dev, mats, r["sigmas"])]
    b = sellcs.sell_batch_create(hs)
    xs = [synth.uniform(A.ncols, 120 + i, 1) for i, A in enumerate(mats)]
    ys = run(b, mats, xs, (torch.float64, torch.float64))
    for A, x, y in zip(mats, xs, ys):
        check_fp64(A, y, x)
    b.close()


def short_rows(n, m, seed):
    """Rows of length 0 or 1 and a few longer ones (values U[-1,1))."""
    rng = np.random.default_rng(seed)
    lens = (rng.random(n) >= 0.3).astype(np.int64)
    lens[rng.random(n) < 0.2] = 2
    lens[rng.random(n) < 0.05] = 3
    lens[rng.integers(0, n, max(1, n // 500))] = 9
    rpt = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=rpt[1:])
    col = np.concatenate([np.sort(rng.choice(m, int(L), replace=False)) for L in lens if L] or
                         [np.zeros(0, np.int64)]).astype(np.int32)
    return synth.CRS(n, m, rpt, col, synth.uniform(int(rpt[-1]), seed, 2))


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("C", [16, 32])
def test_batch_width1_groups(form, C):
    """Chunks of at most 64 / C columns run 64 / C to a wave in the batched
    kernel (and in the single-vector product on split layouts): every row
    equals the single-matrix product with one slot per lane bit for bit (the
    same products, added in the same tree), is within the oracle's bound,
    and the ragged ends (matrix sizes not multiples of the group) are
    covered."""
    import torch
    from paper_1307_6209_amd import sellcs
    mats = [short_rows(n, 3000 + 7 * n % 977, 70 + i) for i, n in enumerate((997, 4096, 1, 77, 12_345, 64))]
    hs = [build(A, C, 10**9, vec=1) for A in mats]
    b = create(form, hs)
    xs = [synth.uniform(A.ncols, 90 + i, 1) for i, A in enumerate(mats)]
    ys = run(b, mats, xs, (torch.float64, torch.float64))
    short = wide = False
    for A, h, x, y in zip(mats, hs, xs, ys):
        check_fp64(A, y, x, m=batch_chain_per_row(A, h, C))
        lay = sellcs.sell_export(h, parts=("perm", "cl"))
        w = np.empty(A.nrows, np.int64)
        w[lay["perm"]] = np.repeat(lay["cl"], C)[:A.nrows]
        single = torch.full((A.nrows,), float("nan"), dtype=torch.float64, device="cuda")
        sellcs.sell_spmv(h, torch.from_numpy(x).cuda(), single)
        torch.cuda.synchronize()
        assert np.array_equal(y.view(np.uint64), single.cpu().numpy().view(np.uint64))
        short |= bool(((w > 1) & (w <= 64 // C)).any())
        wide |= bool((w > 64 // C).any())
    assert short and wide
    b.close()
