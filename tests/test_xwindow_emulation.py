"""Host check of the window builder's bitmap method. Groups whose columns
span at most 32 * 8192 values mark them in a bitmap of the span: the set
bits in order are the distinct columns, a slot's position is the popcount of
the bits before its column (a per-word prefix plus a masked popcount), and
runs start and end at the edges of the set bits (a word's carry bit taken
from its neighbour). Column 0, which every padding slot holds, is kept out
of the span and put in front as a run of its own unless column 1 is present.
This emulation performs those steps on 32-bit words and must reproduce the
plain definition (sorted distinct columns, rank, runs) on the edge cases:
column 0 alone, with column 1, apart from the rest, runs across word edges,
full words, the span limit and beyond it (where the builder sorts instead)."""
import numpy as np
import pytest

import synth
from xwindow_def import group_window

SPAN_LIMIT = 32 * 8192
M32 = 0xFFFFFFFF


def popc(v):
    return bin(v & M32).count("1")


def bitmap_window(cols):
    """The bitmap method's window of one group: (positions, runs), or None
    when the group takes the sorting path (span above the limit)."""
    cols = [int(c) for c in cols]
    n = len(cols)
    nz = [c for c in cols if c != 0]
    has0 = len(nz) < n
    if not nz:
        lo = hi = 0
    else:
        lo, hi = min(nz), max(nz)
        if has0 and lo <= 1:
            lo = 0
    extra = 1 if has0 and lo > 0 else 0
    span = hi - lo + 1
    if n == 0 or span > SPAN_LIMIT:
        return None
    nw = (span + 31) // 32
    bm = [0] * nw
    for c in cols:
        if c != 0 or not extra:
            b = c - lo
            bm[b >> 5] |= 1 << (b & 31)
    wpre, acc = [], 0
    for w in range(nw):
        wpre.append(acc)
        acc += popc(bm[w])

    def starts(w):
        prev = bm[w - 1] >> 31 if w > 0 else 0
        return bm[w] & ~(((bm[w] << 1) & M32) | prev) & M32

    def ends(w):
        nxt = ((bm[w + 1] & 1) << 31) if w + 1 < nw else 0
        return bm[w] & ~((bm[w] >> 1) | nxt) & M32

    def position(c):
        if c == 0 and extra:
            return 0
        b = c - lo
        return extra + wpre[b >> 5] + popc(bm[b >> 5] & ((1 << (b & 31)) - 1))

    runs = [[0, 0, 1]] if extra else []
    start_bits = []
    for w in range(nw):
        st = starts(w)
        while st:
            b = (st & -st).bit_length() - 1
            st &= st - 1
            bit = w * 32 + b
            start_bits.append(bit)
            runs.append([lo + bit, extra + wpre[w] + popc(bm[w] & ((1 << b) - 1)), 0])
    before = 0
    for w in range(nw):
        st, en = starts(w), ends(w)
        while en:
            b = (en & -en).bit_length() - 1
            en &= en - 1
            upto = M32 if b == 31 else (2 << b) - 1
            r = before + popc(st & upto) - 1  # the run that ends here started at or before it
            runs[extra + r][2] = w * 32 + b - start_bits[r] + 1
        before += popc(st)
    return np.array([position(c) for c in cols], np.int64), np.array(runs, np.int64).reshape(-1, 3)


def cases():
    out = {
        "only_column_0": [0, 0, 0],
        "zero_and_one": [0, 1, 2, 0, 7],
        "zero_apart": [0, 2, 3, 0, 9],
        "no_zero": [5, 6, 7, 40, 41],
        "word_edge_run": [31, 32, 33, 0, 95, 96],
        "full_word": list(range(32, 64)) + [0],
        "zero_to_63": list(range(0, 64)),
        "single_bits_apart": [3, 35, 67, 99, 131],
        "duplicates": [8, 8, 9, 0, 0, 9, 70, 8],
        "span_limit": [1, SPAN_LIMIT, 1000],
        "span_limit_zero_apart": [0, 2, SPAN_LIMIT + 1, 0],
        "span_limit_with_one": [0, 1, SPAN_LIMIT - 1],
        "span_limit_plus_one": [1, SPAN_LIMIT + 1],
        "span_limit_plus_one_with_zero": [0, 1, SPAN_LIMIT],
        "wide": [0, 17, 10 ** 6],
        "last_bit_of_span": [2, 33, 34, 0],
    }
    for s in range(12):
        u = synth.u64(70 + s, 1, 600)
        base = int(synth.u64(70 + s, 2, 1)[0] % np.uint64(5000))
        c = (base + (u % np.uint64(400 + 200 * s)).astype(np.int64)).tolist()
        if s % 3 == 0:
            c += [0, 0]
        if s % 4 == 1:
            c += [1]
        out["random_%d" % s] = c
    return out


# which way the builder takes for the cases at the span limit
PATH = {"span_limit": "bitmap", "span_limit_zero_apart": "bitmap", "span_limit_with_one": "bitmap",
        "span_limit_plus_one": "sort", "span_limit_plus_one_with_zero": "sort", "wide": "sort"}


@pytest.mark.parametrize("name,cols", sorted(cases().items()))
def test_bitmap_method_equals_definition(name, cols):
    u, pos, runs = group_window(cols)
    got = bitmap_window(cols)
    nz = [c for c in cols if c != 0]
    lo = min(nz) if nz else 0
    if 0 in cols and lo <= 1:
        lo = 0
    if name in PATH:
        assert (got is None) == (PATH[name] == "sort")
    if (max(nz) if nz else 0) - lo + 1 > SPAN_LIMIT:
        assert got is None  # the sorting path builds it from the definition's sort
        return
    assert got is not None
    gpos, gruns = got
    assert np.array_equal(gpos, pos)
    assert np.array_equal(gruns, runs)
    assert runs[:, 2].sum() == u.size  # the runs cover the window exactly once
