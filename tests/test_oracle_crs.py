"""Pins of the CRS part of the oracle (Listing "CRS spMVM kernel", Sect. 3.1)
against brute force, closed forms and error bounds -- none of which reuse
the oracle's own code."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

U53 = 2.0 ** -53


def gamma(m, u=U53):
    return m * u / (1 - m * u)


def dense_exact(A, x):
    """Brute force: y_i = sum over the row's stored entries, in exact rationals."""
    y = []
    for i in range(A.nrows):
        s = Fraction(0)
        for j in range(int(A.rpt[i]), int(A.rpt[i + 1])):
            s += Fraction(float(A.val[j])) * Fraction(float(x[A.col[j]]))
        y.append(s)
    return y


def dense_matrix_int(A):
    D = [[0] * A.ncols for _ in range(A.nrows)]
    for i in range(A.nrows):
        for j in range(int(A.rpt[i]), int(A.rpt[i + 1])):
            D[i][A.col[j]] += int(A.val[j])
    return D


@pytest.mark.parametrize("shape", [(1, 1), (7, 5), (33, 40), (64, 64), (50, 17)])
@pytest.mark.parametrize("dups", [False, True])
def test_integer_matrix_equals_dense_matvec(shape, dups):
    """Integer values and x: every product and sum is exact, so the CRS sum
    must equal the dense matrix-vector product bit for bit (duplicates add)."""
    n, m = shape
    A = synth.random_crs(n, m, seed=100 + n + 7 * m + dups, max_len=min(m, 9), duplicates=dups, unsorted=dups,
                         integer_values=True)
    x = ((synth.u64(5, 1, m) % np.uint64(7)).astype(np.int64) - 3).astype(np.float64)
    D = dense_matrix_int(A)
    want = np.array([sum(D[i][c] * int(x[c]) for c in range(m)) for i in range(n)], dtype=np.float64)
    got = oracle.crs_spmv(A, x)
    assert np.array_equal(got, want)
    assert np.array_equal(oracle.crs_spmv_hi(A, x), want)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_float_matrix_within_recursive_sum_bound(seed):
    """|y_seq - y*| <= gamma_len (|A||x|)_i against the exact rational sum;
    the long double companion is within one double rounding plus
    gamma_len at 64-bit precision."""
    A = synth.random_crs(40, 30, seed=seed, max_len=25, duplicates=True, unsorted=True)
    x = synth.uniform(30, seed, 3)
    ex = dense_exact(A, x)
    y = oracle.crs_spmv(A, x)
    yh = oracle.crs_spmv_hi(A, x)
    ax = oracle.crs_absmv(A, x)
    lens = A.row_lengths()
    for i in range(A.nrows):
        e = abs(Fraction(float(y[i])) - ex[i])
        assert e <= Fraction(gamma(int(lens[i])) * ax[i] * (1 + 1e-12))
        eh = abs(Fraction(float(yh[i])) - ex[i])
        assert eh <= Fraction(gamma(int(lens[i]), 2.0 ** -64) * ax[i] * 1.01 + U53 * abs(float(ex[i])) * 1.01)


def test_empty_rows_and_empty_matrix():
    A = synth.random_crs(20, 10, seed=9, max_len=4, empty_frac=0.6)
    x = synth.uniform(10, 9, 1)
    y = oracle.crs_spmv(A, x)
    lens = A.row_lengths()
    assert np.all(y[lens == 0] == 0.0)
    Z = synth.CRS(5, 3, np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0))
    assert np.array_equal(oracle.crs_spmv(Z, np.ones(3)), np.zeros(5))


def dyadic_case(seed, n, m, max_len, vbits, xbits, vexp, xexp):
    """Random matrix (empty rows, repeated and unsorted columns, n != m) whose
    values are integers below 2^vbits times 2^vexp and x integers below
    2^xbits times 2^xexp, signs mixed. Every product is an integer times
    2^(vexp + xexp) of at most vbits + xbits bits."""
    A = synth.random_crs(n, m, seed=seed, max_len=max_len, empty_frac=0.2, duplicates=True, unsorted=True)
    iv = (synth.u64(seed, 31, A.nnz) % np.uint64(1 << vbits)).astype(np.int64)
    iv[synth.u64(seed, 32, A.nnz) % np.uint64(2) == 1] *= -1
    ix = (synth.u64(seed, 33, m) % np.uint64(1 << xbits)).astype(np.int64)
    ix[synth.u64(seed, 34, m) % np.uint64(2) == 1] *= -1
    A = synth.CRS(n, m, A.rpt, A.col, np.ldexp(iv.astype(np.float64), vexp))
    return A, np.ldexp(ix.astype(np.float64), xexp), iv, ix


@pytest.mark.parametrize("seed,vbits,xbits", [(1, 10, 10), (2, 26, 26), (3, 30, 28), (4, 31, 29)])
def test_absmv_exact_rational(seed, vbits, xbits):
    """(|A||x|)_i = sum over the row's stored entries of |a_ij| |x_col(j)|,
    computed here in exact integers and rounded once to double by Python's
    correctly rounded int -> float conversion. With at most 16 terms of at
    most 60 bits every partial sum is an integer below 2^64 times 2^-18,
    exact in the oracle's long double (64-bit significand), so
    the oracle must return exactly this rounding (the larger cases need the
    final rounding, which a mistaken sum would not reproduce)."""
    A, x, iv, ix = dyadic_case(seed, 60, 45, 16, vbits, xbits, -7, -11)
    got = oracle.crs_absmv(A, x)
    for i in range(A.nrows):
        s = sum(abs(int(iv[j])) * abs(int(ix[A.col[j]])) for j in range(int(A.rpt[i]), int(A.rpt[i + 1])))
        want = math.ldexp(float(s), -18)  # int -> float rounds to nearest even; the scaling is exact
        assert got[i] == want, (i, got[i], want)
    assert np.all(got[A.row_lengths() == 0] == 0.0)


@pytest.mark.parametrize("seed", [5, 6])
def test_absmv_two_sided_bound(seed):
    """For arbitrary doubles: S_i (1 - g) <= (|A||x|)_i <= S_i (1 + g) with
    S_i the exact rational sum, g = len_i 2^-63 + 2^-53 (long double sum,
    then one rounding). A doubled, halved, sign-cancelled or mis-indexed sum
    leaves this band."""
    A = synth.random_crs(50, 35, seed=seed, max_len=30, duplicates=True, unsorted=True)
    x = synth.uniform(35, seed, 4) * np.ldexp(1.0, (synth.u64(seed, 5, 35) % np.uint64(40)).astype(np.int64) - 20)
    got = oracle.crs_absmv(A, x)
    lens = A.row_lengths()
    for i in range(A.nrows):
        S = sum((abs(Fraction(float(A.val[j]))) * abs(Fraction(float(x[A.col[j]])))
                 for j in range(int(A.rpt[i]), int(A.rpt[i + 1]))), Fraction(0))
        g = Fraction(int(lens[i]) + 1, 2 ** 63) + Fraction(1, 2 ** 53)
        assert S * (1 - g) <= Fraction(float(got[i])) <= S * (1 + g), i


@pytest.mark.parametrize("m", [2, 5, 128])
def test_laplacian_row_sums(m):
    """5-point Laplacian (diag 4, neighbours -1) times the ones vector:
    0 inside, 1 on an edge, 2 at a corner; the sum over the grid is 4m."""
    A = synth.lap5(m)
    y = oracle.crs_spmv(A, np.ones(A.nrows))
    g = y.reshape(m, m)
    want = np.zeros((m, m))
    want[0, :] += 1
    want[-1, :] += 1
    want[:, 0] += 1
    want[:, -1] += 1
    assert np.array_equal(g, want)
    assert y.sum() == 4 * m
    assert A.nnz == 5 * m * m - 4 * m


def sin_pi_ratio(t, d):
    """sin(pi t / d) for integer arrays t, with the argument reduced exactly
    to [0, pi/2] first so that each value carries only a few ulps of error."""
    t = np.asarray(t, np.int64) % (2 * d)
    sign = np.where(t >= d, -1.0, 1.0)
    t = np.where(t >= d, t - d, t)
    t = np.where(2 * t > d, d - t, t)
    return sign * np.sin(np.pi * t / d)


@pytest.mark.parametrize("p,q", [(1, 1), (3, 7), (20, 5), (64, 64)])
def test_laplacian_eigenvectors(p, q):
    """A v = lambda v for v = sin(p pi (ix+1)/(m+1)) sin(q pi (iy+1)/(m+1)),
    lambda = 4 - 2 cos(p pi/(m+1)) - 2 cos(q pi/(m+1)) (Dirichlet grid),
    evaluated as 4 sin^2(p pi/(2(m+1))) + 4 sin^2(q pi/(2(m+1))) to avoid
    cancellation."""
    m = 128
    A = synth.lap5(m)
    ix = np.arange(m)
    vx = sin_pi_ratio(p * (ix + 1), m + 1)
    vy = sin_pi_ratio(q * (ix + 1), m + 1)
    v = np.outer(vy, vx).ravel()  # row index = ix + m*iy
    lam = 4 * math.sin(p * math.pi / (2 * (m + 1))) ** 2 + 4 * math.sin(q * math.pi / (2 * (m + 1))) ** 2
    y = oracle.crs_spmv(A, v)
    scale = oracle.crs_absmv(A, v) + abs(lam) * np.abs(v)
    assert np.all(np.abs(y - lam * v) <= 32 * U53 * scale + 1e-300)


@pytest.mark.parametrize("m", [3, 4, 40])
def test_stencil27_ones(m):
    """27-point stencil with every value 1 and x = 1: y_i is the row length,
    8 at the corners, 12 on edges, 18 on faces and 27 inside, with counts
    8, 12(m-2), 6(m-2)^2, (m-2)^3."""
    A = synth.stencil27(m, ones=True)
    y = oracle.crs_spmv(A, np.ones(A.nrows))
    vals, counts = np.unique(y, return_counts=True)
    want = {8.0: 8, 12.0: 12 * (m - 2), 18.0: 6 * (m - 2) ** 2, 27.0: (m - 2) ** 3}
    want = {k: v for k, v in want.items() if v > 0}
    assert dict(zip(vals.tolist(), counts.tolist())) == want
    assert A.nnz == (3 * m - 2) ** 3


def test_threads_do_not_change_bits():
    A = synth.powerlaw(50_000, seed=77)
    x = synth.uniform(A.ncols, 77, 2)
    y1 = oracle.crs_spmv(A, x, nthreads=1, sched=0)
    for nt, sched in [(4, 0), (8, 1), (3, 1)]:
        assert np.array_equal(y1, oracle.crs_spmv(A, x, nthreads=nt, sched=sched))


def test_powerlaw_within_bound_of_companion():
    A = synth.powerlaw(100_000, seed=5)
    x = synth.uniform(A.ncols, 5, 2)
    y = oracle.crs_spmv(A, x)
    yh = oracle.crs_spmv_hi(A, x)
    ax = oracle.crs_absmv(A, x)
    g = np.array([gamma(int(l)) for l in A.row_lengths()])
    assert np.all(np.abs(y - yh) <= (g * ax + U53 * np.abs(yh)) * 1.0001)


def test_block_form_columns_match_single_vector():
    A = synth.random_crs(60, 45, seed=3, max_len=12, duplicates=True, unsorted=True)
    X = synth.block_vector(45, 5, seed=4)
    Y, aY = oracle.crs_spmmv_hi(A, X)
    for v in range(5):
        assert np.array_equal(Y[:, v], oracle.crs_spmv_hi(A, X[:, v]))
        assert np.array_equal(aY[:, v], oracle.crs_absmv(A, X[:, v]))


@pytest.mark.parametrize("breakage,code", [("rpt0", 1), ("decr", 2), ("rptn", 3), ("colhi", 4), ("colneg", 4)])
def test_validation_codes(breakage, code):
    A = synth.random_crs(30, 20, seed=11, max_len=5, empty_frac=0.0)
    rpt, col = A.rpt.copy(), A.col.copy()
    if breakage == "rpt0":
        rpt[0] = 1
    elif breakage == "decr":
        rpt[5], rpt[6] = rpt[6], rpt[5] - 1
    elif breakage == "rptn":
        rpt[-1] += 1
    elif breakage == "colhi":
        col[3] = 20
    else:
        col[3] = -1
    B = synth.CRS(A.nrows, A.ncols, rpt, col, A.val)
    assert oracle.crs_validate(B) == code
    assert oracle.crs_validate(A) == 0
