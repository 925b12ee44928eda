"""The XCD placement of the batched launch (paper_1307_6209_amd/csrc/
batch_plan.h), compiled with g++ and checked on the host: every work unit
runs exactly once; the units of a matrix (of each piece of a large one) sit
in workgroups of one XCD (workgroup b runs on XCD b mod 8); split segments
come before whole chunks on each XCD; the estimated cost is balanced; the
persistent form deals each XCD's queue to its waves, each wave ending
within one unit's cost of the XCD's mean."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
W, X = 4, 8


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("plan") / "batch_plan_driver")
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-Werror", "-I",
                    os.path.join(ROOT, "paper_1307_6209_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "batch_plan_driver.cpp"), "-o", exe], check=True)
    return exe


def plan(driver, mat, cost, split, nmats, persistent_waves=0):
    lines = ["%d %d %d %d %d" % (len(mat), nmats, W, X, persistent_waves)]
    lines += ["%d %d %d" % t for t in zip(mat, cost, split)]
    out = subprocess.run([driver], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True).stdout
    res = {}
    for ln in out.splitlines():
        f = ln.split()
        res[f[0]] = np.array([int(v) for v in f[2:]], np.int64)
        assert len(res[f[0]]) == int(f[1])
    return res


def units_of_batch(rng, nmats, lo=1, hi=300):
    """Per matrix: some split segments (long), then whole chunks."""
    mat, cost, split = [], [], []
    for m in range(nmats):
        nseg = int(rng.integers(0, 6))
        nwhole = int(rng.integers(lo, hi)) if rng.random() < 0.9 else int(rng.integers(1000, 4000))
        for _ in range(nseg):
            mat.append(m), cost.append(68), split.append(1)
        for _ in range(nwhole):
            mat.append(m), cost.append(int(rng.integers(5, 68))), split.append(0)
    return mat, cost, split


def xcd_of_slot(i):
    return (i // W) % X


def check_common(res, mat, cost, split):
    order = res["order"]
    real = order[order >= 0]
    assert np.array_equal(np.sort(real), np.arange(len(mat)))  # each unit exactly once
    load = res["load"]
    assert load.sum() == sum(cost)
    return real


@pytest.mark.parametrize("seed,nmats", [(1, 64), (2, 8), (3, 3), (4, 1), (5, 200)])
def test_one_unit_per_wave(driver, seed, nmats):
    rng = np.random.default_rng(seed)
    mat, cost, split = units_of_batch(rng, nmats)
    mat_a, cost_a, split_a = np.array(mat), np.array(cost), np.array(split)
    res = plan(driver, mat, cost, split, nmats)
    check_common(res, mat, cost, split)
    order = res["order"]
    assert len(order) % (W * X) == 0
    xcd = np.full(len(mat), -1)
    pos = np.full(len(mat), -1)
    for i, u in enumerate(order):
        if u >= 0:
            xcd[u], pos[u] = xcd_of_slot(i), i
    # the load reported per XCD is the cost of the units placed there
    for x in range(X):
        assert res["load"][x] == cost_a[xcd == x].sum()
    # a matrix no larger than a 16th of the batch runs on one XCD
    cap = max(1, cost_a.sum() // (2 * X))
    for m in range(nmats):
        sel = mat_a == m
        if sel.any() and cost_a[sel].sum() <= cap:
            assert len(set(xcd[sel])) == 1
    # per XCD, split segments before whole chunks (in launch order)
    for x in range(X):
        sel = xcd == x
        if sel.any() and split_a[sel].any() and (~split_a[sel].astype(bool)).any():
            assert pos[sel & (split_a == 1)].max() < pos[sel & (split_a == 0)].min()
    # balance: no XCD above the mean by more than the largest piece
    mean = cost_a.sum() / X
    biggest = min(max(cost_a[mat_a == m].sum() for m in range(nmats)), cap + cost_a.max())
    assert res["load"].max() <= mean + biggest
    # no whole round of blocks is filler only
    last = order[-W * X:]
    assert (last >= 0).any()


@pytest.mark.parametrize("seed,nmats", [(6, 64), (7, 5), (8, 1)])
def test_persistent_slices(driver, seed, nmats):
    rng = np.random.default_rng(seed)
    mat, cost, split = units_of_batch(rng, nmats)
    cost_a = np.array(cost)
    nw = 256 * 8 // (W * X) * (W * X)
    res = plan(driver, mat, cost, split, nmats, persistent_waves=nw)
    real = check_common(res, mat, cost, split)
    order, sl = res["order"], res["slice"]
    assert len(real) == len(order)  # no filler in the persistent form
    assert len(sl) == nw + 1 and sl[0] == 0 and sl[-1] == len(order) and np.all(np.diff(sl) >= 0)
    xcd = np.full(len(mat), -1)
    for w in range(nw):
        for u in order[sl[w]:sl[w + 1]]:
            xcd[u] = (w // W) % X
    for x in range(X):
        assert res["load"][x] == cost_a[xcd == x].sum()
    # per XCD, the waves' estimated costs: none above the mean by more than
    # the largest unit (list scheduling); split segments first in every wave
    split_a = np.array(split)
    for x in range(X):
        waves = [w for w in range(nw) if (w // W) % X == x]
        loads = np.array([cost_a[order[sl[w]:sl[w + 1]]].sum() for w in waves])
        units = [u for w in waves for u in order[sl[w]:sl[w + 1]]]
        if units:
            assert loads.max() <= loads.mean() + cost_a[units].max()
        for w in waves:
            s = split_a[order[sl[w]:sl[w + 1]]]
            if s.size and s.any() and not s.all():
                assert np.flatnonzero(s).max() < np.flatnonzero(s == 0).min()


def test_one_oversized_matrix_is_spread(driver):
    """One matrix holding most of the work is cut into pieces over all XCDs."""
    mat = [0] * 4000 + [1] * 50 + [2] * 50
    cost = [20] * len(mat)
    split = [0] * len(mat)
    res = plan(driver, mat, cost, split, 3)
    check_common(res, mat, cost, split)
    mean = sum(cost) / X
    assert res["load"].max() <= 1.1 * mean
