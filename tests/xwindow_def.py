"""The x window of a group of chunks, by its plain definition: the sorted
distinct column indices that the group's slots hold, each slot's position
being the rank of its column among them, and the runs of consecutive columns
(first column, position, length). Test infrastructure: computed on the host
from a layout the oracle built."""
import numpy as np


def group_window(cols):
    """(distinct sorted columns, position of every slot, runs) of one group."""
    u = np.unique(np.asarray(cols, np.int64))
    pos = np.searchsorted(u, cols).astype(np.int64)
    if u.size == 0:
        return u, pos, np.zeros((0, 3), np.int64)
    starts = np.flatnonzero(np.r_[True, np.diff(u) != 1])
    ends = np.r_[starts[1:], u.size]
    runs = np.stack([u[starts], starts, ends - starts], axis=1)
    return u, pos, runs


def window_tables(col, cs, group_chunks, groups=None):
    """segoff, seg (runs x 3) and lcol of the given groups (all by default)
    of a layout with slot columns col and chunk offsets cs. With a subset of
    groups, segoff holds the run count of each listed group and lcol only
    the listed groups' slots (in order)."""
    nchunks = len(cs) - 1
    ngroups = (nchunks + group_chunks - 1) // group_chunks
    gl = range(ngroups) if groups is None else groups
    counts, segs, lcol = [], [], []
    for g in gl:
        sb, se = int(cs[g * group_chunks]), int(cs[min((g + 1) * group_chunks, nchunks)])
        _, pos, runs = group_window(col[sb:se])
        counts.append(len(runs))
        segs.append(runs)
        lcol.append(pos)
    segoff = np.zeros(len(counts) + 1, np.int64)
    np.cumsum(counts, out=segoff[1:])
    seg = np.concatenate(segs) if segs else np.zeros((0, 3), np.int64)
    lc = np.concatenate(lcol) if lcol else np.zeros(0, np.int64)
    return segoff, seg, lc
