"""Pins of the SELL-C-sigma builder of the oracle (Sects. 3.3 and 3.4):
special cases the paper names (SELL-1-1 = CRS, SELL-N-1 = ELLPACK, global
sort = pJDS, sigma | C leaves beta unchanged, the occupancy worst case),
closed forms derived for the stencils, a statistical closed form for the
power-law matrix, and structural invariants."""
import math

import numpy as np
import pytest

import oracle
import synth


def check_invariants(A, S):
    n, C, sigma = A.nrows, S["C"], S["sigma"]
    perm, cl, cs, col, val = S["perm"], S["cl"], S["cs"], S["col"], S["val_f64"]
    lens = A.row_lengths()
    # the permutation is a bijection on [0, n) and maps each window to itself
    assert np.array_equal(np.sort(perm), np.arange(n))
    w = np.arange(n) // sigma
    assert np.array_equal(perm // sigma, w)
    # inside a window: lengths non-increasing, equal lengths in original order
    L = lens[perm]
    same_w = w[1:] == w[:-1]
    assert np.all(L[1:][same_w] <= L[:-1][same_w])
    tie = same_w & (L[1:] == L[:-1])
    assert np.all(perm[1:][tie] > perm[:-1][tie])
    # chunk widths are the chunk maxima, offsets are the prefix sums of C*cl
    nc = (n + C - 1) // C
    assert cl.size == nc and cs.size == nc + 1 and cs[0] == 0
    Lp = np.zeros(nc * C, np.int64)
    Lp[:n] = L
    assert np.array_equal(cl, Lp.reshape(nc, C).max(axis=1) if nc else cl)
    assert np.array_equal(np.diff(cs), C * cl.astype(np.int64))
    # every stored row reproduces its CRS entries in order; the rest is padding
    real = np.zeros(int(cs[-1]), bool)
    for i in range(nc):
        for r in range(C):
            p = i * C + r
            if p >= n:
                continue
            row = perm[p]
            a, b = int(A.rpt[row]), int(A.rpt[row + 1])
            idx = cs[i] + np.arange(b - a) * C + r
            assert np.array_equal(col[idx], A.col[a:b])
            assert np.array_equal(val[idx], A.val[a:b])
            real[idx] = True
    assert real.sum() == A.nnz
    assert np.all(col[~real] == 0) and np.all(val[~real] == 0.0)


CASES = [(1, 1), (4, 1), (4, 3), (4, 8), (8, 16), (32, 1), (32, 64), (64, 7), (128, 1000), (16, 10**9)]


@pytest.mark.parametrize("C,sigma", CASES)
@pytest.mark.parametrize("seed", [1, 2])
def test_invariants_random(C, sigma, seed):
    A = synth.random_crs(301, 90, seed=seed, max_len=30, empty_frac=0.3, duplicates=True, unsorted=True)
    S = oracle.sell_build(A, C, sigma)
    check_invariants(A, S)


def test_sell_1_1_is_crs():
    """SELL-1-1 stores CRS exactly: cs == rpt, same col and val arrays."""
    A = synth.random_crs(200, 70, seed=4, max_len=20, duplicates=True, unsorted=True)
    S = oracle.sell_build(A, 1, 1)
    assert np.array_equal(S["cs"], A.rpt)
    assert np.array_equal(S["col"], A.col)
    assert np.array_equal(S["val"], A.val)
    assert S["beta"] == 1.0


def test_sell_n_1_is_ellpack():
    """C >= N, sigma = 1: one chunk as wide as the longest row (ELLPACK)."""
    A = synth.random_crs(50, 40, seed=5, max_len=15)
    S = oracle.sell_build(A, 64, 1)
    L = A.row_lengths()
    assert S["nchunks"] == 1 and S["cl"][0] == L.max() and S["padded"] == 64 * L.max()
    assert np.array_equal(S["perm"], np.arange(50))


def test_global_sort_is_stable_length_sort_and_maximises_beta():
    """sigma >= N sorts all rows by descending length, ties in original order
    (pJDS); this order minimises the stored slots over all sigma."""
    A = synth.random_crs(1000, 300, seed=6, max_len=40, empty_frac=0.1)
    L = A.row_lengths()
    S = oracle.sell_build(A, 16, 5000)
    assert np.array_equal(S["perm"], np.argsort(-L, kind="stable"))
    for sigma in [1, 2, 16, 100, 256, 999]:
        assert oracle.sell_build(A, 16, sigma)["padded"] >= S["padded"]


@pytest.mark.parametrize("C", [4, 16, 32])
def test_sigma_dividing_C_keeps_beta(C):
    """Sorting scopes that divide C do not change the chunk widths' sum."""
    A = synth.powerlaw(20_000, seed=8)
    base = oracle.sell_build(A, C, 1)["padded"]
    for sigma in [d for d in [1, 2, 4, 8, 16, 32] if C % d == 0]:
        assert oracle.sell_build(A, C, sigma)["padded"] == base


@pytest.mark.parametrize("C,nchunks", [(4, 64), (8, 16), (2, 100)])
def test_worst_case_beta(C, nchunks):
    """One full row plus C-1 one-entry rows per chunk: beta = (N+C-1)/(C N)
    unsorted (Eq. (betaworst)) and beta = 1 for sigma = C^2."""
    A = synth.worst_case_beta(C, nchunks)
    N = A.nrows
    S1 = oracle.sell_build(A, C, 1)
    assert S1["padded"] * (N + C - 1) == A.nnz * C * N  # beta == (N+C-1)/(C N) exactly
    assert abs(S1["beta"] - (N + C - 1) / (C * N)) < 1e-15
    if nchunks % C == 0:
        S2 = oracle.sell_build(A, C, C * C)
        assert S2["padded"] == A.nnz and S2["beta"] == 1.0


@pytest.mark.parametrize("m,C", [(128, 32), (128, 16), (64, 64), (12, 4)])
def test_lap5_beta_closed_form(m, C):
    """5-point m x m grid, C | m, sigma = 1: every chunk of a boundary grid
    row is 4 wide, every other chunk 5 wide, so sum(cl) = (m/C)(5m-2) and
    beta = (5m-4)/(5m-2)."""
    A = synth.lap5(m)
    S = oracle.sell_build(A, C, 1)
    assert S["cl"].sum() == (m // C) * (5 * m - 2)
    assert S["padded"] * (5 * m - 4) == A.nnz * (5 * m - 2)


def test_lap5_global_sort_count():
    """m = 128, C = 32, sigma = N: the (m-2)^2 rows of length 5 come first, so
    ceil((m-2)^2 / C) chunks are 5 wide and the remaining chunks (fours, then
    the four corner rows of length 3) are 4 wide."""
    m, C = 128, 32
    A = synth.lap5(m)
    chunks5 = math.ceil((m - 2) ** 2 / C)
    want = 5 * chunks5 + 4 * (m * m // C - chunks5)
    S = oracle.sell_build(A, C, A.nrows)
    assert S["cl"].sum() == want == 2545
    assert abs(S["beta"] - A.nnz / (C * want)) < 1e-15


@pytest.mark.parametrize("m,C", [(24, 8), (40, 8), (160, 32)])
def test_stencil27_beta_closed_form(m, C):
    """27-point m^3 grid, C | m, sigma = 1: each chunk is 3*ny*nz wide, so
    sum(cl) = 3 (m/C) (3m-2)^2 and beta = (3m-2)/(3m)."""
    A = synth.stencil27(m)
    perm, cl, cs = oracle.sell_layout(A, C, 1)
    assert cl.sum() == 3 * (m // C) * (3 * m - 2) ** 2
    assert cs[-1] * (3 * m - 2) == A.nnz * 3 * m


def test_powerlaw_chunk_width_expectation():
    """Independent row lengths with tail q_l = P(L >= l): the expected width
    of a chunk of C rows is sum_l (1 - (1 - q_l)^C) (sigma = 1)."""
    n = 400_000
    lens = synth.powerlaw_lengths(n, seed=21)
    A = synth.CRS(n, n, np.concatenate([[0], np.cumsum(lens)]), np.zeros(int(lens.sum()), np.int32),
                  np.zeros(int(lens.sum())))
    k = np.arange(1, 10001, dtype=np.float64)
    p = k ** -2.1
    p /= p.sum()
    q = np.cumsum(p[::-1])[::-1]  # q[l-1] = P(L >= l)
    for C in [16, 32, 64, 128]:
        _, cl, _ = oracle.sell_layout(A, C, 1)
        expect = np.sum(1 - (1 - q) ** C)
        assert abs(cl.mean() / expect - 1) < 0.05, (C, cl.mean(), expect)


@pytest.mark.parametrize("C,sigma", [(1, 1), (4, 1), (32, 1), (32, 64), (128, 4096), (16, 10**9)])
def test_sell_spmv_equals_crs_spmv_bitwise(C, sigma):
    """The SELL product sums each row in CRS order (padding adds zeros), so
    it reproduces the CRS product bit for bit."""
    A = synth.random_crs(513, 200, seed=12, max_len=50, empty_frac=0.2, duplicates=True, unsorted=True)
    x = synth.uniform(200, 12, 1)
    S = oracle.sell_build(A, C, sigma)
    assert np.array_equal(oracle.sell_spmv(S, A.nrows, x), oracle.crs_spmv(A, x))


def test_zeta_closed_form():
    """Eq. (eq:cv): rows of lengths {1, 3} alternating have mean 2 and
    standard deviation 1, so zeta = 1/2; a constant length gives 0."""
    n = 1000
    lens = np.tile([1, 3], n // 2)
    A = synth.CRS(n, 4, np.concatenate([[0], np.cumsum(lens)]), np.zeros(int(lens.sum()), np.int32),
                  np.zeros(int(lens.sum())))
    assert abs(oracle.row_zeta(A) - 0.5) < 1e-15
    assert oracle.row_zeta(synth.stencil27(3, ones=True)) > 0
    assert oracle.row_zeta(synth.dense(10, 10)) == 0.0


@pytest.mark.parametrize("sigma", [1, 4, 100, 10**9])
def test_symmetric_permutation_identity(sigma):
    """(P A P^T)(P x) = P (A x): the permuted matrix applied to the permuted
    vector gives the permuted product, term for term in the same order."""
    A = synth.powerlaw(3000, seed=33)
    x = synth.uniform(A.ncols, 33, 1)
    perm, _, _ = oracle.sell_layout(A, 8, sigma)
    B = oracle.crs_symperm(A, perm)
    assert np.array_equal(oracle.crs_spmv(B, x[perm]), oracle.crs_spmv(A, x)[perm])
    S = oracle.sell_build(A, 8, sigma, permute_columns=True)
    D = oracle.sell_build(A, 8, sigma)
    assert np.array_equal(S["cs"], D["cs"]) and np.array_equal(S["perm"], D["perm"])
    assert np.array_equal(oracle.sell_spmv(dict(S, perm=np.arange(A.nrows, dtype=np.int32)), A.nrows, x[perm]),
                          oracle.crs_spmv(A, x)[perm])


@pytest.mark.parametrize("C", [2, 4, 8, 32])
def test_staircase_beta(C):
    """Row i holds (i mod C) + 1 entries: with sigma = 1 every chunk's
    longest row is its last, cl = C, and beta = (C + 1) / (2 C); with
    sigma = C the rows of a chunk are reversed and beta is unchanged."""
    nch = 50
    n = nch * C
    lens = np.arange(n, dtype=np.int64) % C + 1
    A = synth.CRS(n, C, np.concatenate([[0], np.cumsum(lens)]), np.concatenate([np.arange(l, dtype=np.int32) for l in lens]),
                  np.ones(int(lens.sum())))
    for sigma in (1, C):
        S = oracle.sell_build(A, C, sigma)
        assert np.all(S["cl"] == C)
        assert S["padded"] * (C + 1) == A.nnz * 2 * C
