"""The seeded input generators: determinism and the shapes the workloads
are meant to have."""
import numpy as np

import synth


def test_counter_rng_is_addressable():
    a = synth.u64(7, 3, 100)
    b = synth.u64(7, 3, 60, start=40)
    assert np.array_equal(a[40:], b)
    assert not np.array_equal(a, synth.u64(8, 3, 100))


def test_splitmix64_reference_value():
    """Output 0 of splitmix64 with state 0 is 0xE220A8397B1DCDAF (Vigna's
    reference implementation); stream_key(seed, stream) = mix64(seed*G +
    stream + 1) so state 0 is reached by no simple seed -- check the mixer
    through synth_draw_u64 on a key we can form: seed 0, stream -1 gives
    key mix64(0) = 0."""
    v = synth._L().synth_draw_u64(0, 2**64 - 1, 0)
    assert v == 0xE220A8397B1DCDAF


def test_lap5_shape():
    A = synth.lap5(128)
    assert A.nrows == 16384 and A.nnz == 81408
    assert np.all(np.diff(A.col[A.rpt[100]:A.rpt[101]]) > 0)


def test_stencil27_shape():
    A = synth.stencil27(20)
    assert A.nnz == 58 ** 3
    v = A.val
    assert v.min() >= 0.5 and v.max() < 1.5


def test_powerlaw_statistics():
    A = synth.powerlaw(300_000, seed=5)
    L = A.row_lengths()
    assert abs(L.mean() - 4.23) < 0.15
    assert abs((L == 1).mean() - 0.641) < 0.01
    zeta = L.std() / L.mean()
    assert zeta > 5
    # distinct, ascending columns in every row
    for i in np.flatnonzero(L > 1)[:2000]:
        c = A.col[A.rpt[i]:A.rpt[i + 1]]
        assert np.all(np.diff(c) > 0)
    assert A.col.min() >= 0 and A.col.max() < A.ncols
    # about half of the entries lie within the band of width 1000
    rows = np.repeat(np.arange(A.nrows), L)
    near = np.abs(A.col.astype(np.int64) - rows) < 500
    assert 0.4 < near.mean() < 0.6


def test_powerlaw_deterministic():
    a, b = synth.powerlaw(5000, seed=9), synth.powerlaw(5000, seed=9)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val)


def test_batch_sizes_range():
    s = synth.batch_sizes(1000)
    assert s.min() >= 1000 and s.max() < 200_000
    assert abs(np.log(s).mean() - (np.log(1e3) + np.log(2e5)) / 2) < 0.15


def test_rail_like_shape():
    R = synth.rail_like(nrows=600, ncols=200_000, mean_len=800, zeta=1.6, seed=3)
    L = R.row_lengths()
    assert R.nrows == 600 and R.ncols == 200_000
    assert 0.8 < L.mean() / 800 < 1.2 and 1.0 < L.std() / L.mean() < 2.2
    for i in range(0, 600, 50):
        c = R.col[R.rpt[i]:R.rpt[i + 1]]
        assert np.all(np.diff(c) > 0) and c.min() >= 0 and c.max() < 200_000
