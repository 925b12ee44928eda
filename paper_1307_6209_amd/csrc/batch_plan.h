// Placement of the work units of a batched launch on the XCDs (accelerator
// dies) of the device. Host code only (no HIP), so that it can be checked on
// its own.
//
// Each XCD has its own L2, and the dispatcher sends workgroup b of a launch
// to XCD b mod X. The matrices of a batch are independent and most of their
// right-hand sides are small (a matrix of 200,000 rows gathers from 1.6 MB
// of x), so a matrix whose units all run on one XCD keeps its x in that
// XCD's L2; dealt round-robin, every L2 would see the x of every matrix.
//
// Plan: matrices are the pieces of work, except that a matrix costing more
// than a 2X-th of the batch is cut into contiguous runs of its units of about
// that cost (so that no XCD is left with one oversized matrix; finer pieces,
// a 4X-th or an 8X-th, spread more matrices over two L2s and measured 2-4 %
// slower on 64 power-law matrices); pieces go to
// the least-loaded XCD, largest first (longest processing time first). Each
// XCD's queue holds its split-chunk segments first (the longest work starts
// earliest), then its whole chunks. One unit per wave: queue x fills the
// blocks x, x + X, x + 2X, ... (W waves per block), and blocks past the end
// of a shorter queue get filler slots. Persistent: each XCD's queue is dealt
// in order to its waves, each unit to the least-loaded one.
#pragma once

#include <algorithm>
#include <cstdint>
#include <numeric>
#include <utility>
#include <vector>

namespace sell {

struct XcdPlan {
  std::vector<int64_t> order;  // unit index of each slot, in launch order (-1: filler)
  std::vector<int32_t> slice;  // persistent form: waves + 1 offsets into order
  std::vector<int64_t> load;   // estimated cost placed on each XCD
};

// mat[q], cost[q], split[q]: matrix, estimated cost and split-segment flag of
// unit q, units of one matrix listed together. waves_per_block W, xcds X.
// persistent_waves: 0 for one unit per wave, else the resident waves (a
// multiple of W * X) of the persistent form.
inline XcdPlan plan_xcd(const std::vector<int32_t> &mat, const std::vector<int64_t> &cost,
                        const std::vector<uint8_t> &split, int32_t nmats, int waves_per_block, int xcds,
                        int64_t persistent_waves) {
  const int64_t n = (int64_t)mat.size();
  const int64_t W = waves_per_block, X = xcds;
  XcdPlan p;
  p.load.assign((size_t)X, 0);

  // units of each matrix, in the order given
  std::vector<std::vector<int64_t>> per(nmats > 0 ? (size_t)nmats : 0);
  int64_t total = 0;
  for (int64_t q = 0; q < n; ++q) {
    per[(size_t)mat[(size_t)q]].push_back(q);
    total += cost[(size_t)q];
  }

  // pieces: whole matrices, or runs of a matrix's units of about `cap` cost
  struct Piece {
    int32_t m;
    size_t beg, end;  // range in per[m]
    int64_t cost;
  };
  const int64_t cap = std::max<int64_t>(1, total / (2 * X));
  std::vector<Piece> pieces;
  for (int32_t m = 0; m < nmats; ++m) {
    const std::vector<int64_t> &u = per[(size_t)m];
    if (u.empty()) continue;
    int64_t mc = 0;
    for (int64_t q : u) mc += cost[(size_t)q];
    if (mc <= cap) {
      pieces.push_back({m, 0, u.size(), mc});
      continue;
    }
    size_t b = 0;
    int64_t acc = 0;
    for (size_t i = 0; i < u.size(); ++i) {
      acc += cost[(size_t)u[i]];
      if (acc >= cap || i + 1 == u.size()) {
        pieces.push_back({m, b, i + 1, acc});
        b = i + 1;
        acc = 0;
      }
    }
  }

  // longest processing time first onto the least-loaded XCD
  std::vector<size_t> byc(pieces.size());
  std::iota(byc.begin(), byc.end(), 0);
  std::stable_sort(byc.begin(), byc.end(), [&](size_t a, size_t b) { return pieces[a].cost > pieces[b].cost; });
  std::vector<std::vector<size_t>> onx((size_t)X);
  for (size_t i : byc) {
    const size_t x = (size_t)(std::min_element(p.load.begin(), p.load.end()) - p.load.begin());
    onx[x].push_back(i);
    p.load[x] += pieces[i].cost;
  }

  // per XCD: split segments first, then whole chunks
  std::vector<std::vector<int64_t>> queue((size_t)X);
  for (size_t x = 0; x < (size_t)X; ++x)
    for (int pass = 0; pass < 2; ++pass)
      for (size_t i : onx[x]) {
        const Piece &pc = pieces[i];
        const std::vector<int64_t> &u = per[(size_t)pc.m];
        for (size_t k = pc.beg; k < pc.end; ++k)
          if ((split[(size_t)u[k]] != 0) == (pass == 0)) queue[x].push_back(u[k]);
      }

  if (persistent_waves <= 0) {
    size_t nblk = 0;
    for (const auto &q : queue) nblk = std::max(nblk, (q.size() + (size_t)W - 1) / (size_t)W);
    p.order.assign(nblk * (size_t)X * (size_t)W, -1);
    for (size_t x = 0; x < (size_t)X; ++x)
      for (size_t i = 0; i < queue[x].size(); ++i) {
        const size_t blk = (i / (size_t)W) * (size_t)X + x;  // the XCD's (i/W)-th block
        p.order[blk * (size_t)W + i % (size_t)W] = queue[x][i];
      }
    return p;
  }

  // persistent: XCD x runs waves w with (w / W) mod X == x; its queue, in
  // order, is dealt to the least-loaded of them by estimated cost (list
  // scheduling: no wave ends more than one unit's cost above the XCD's mean;
  // consecutive equal-cost slices of the queue measured 2-4 % slower)
  const int64_t nw = persistent_waves, wx = nw / X;
  std::vector<std::vector<std::vector<int64_t>>> mine((size_t)X, std::vector<std::vector<int64_t>>((size_t)wx));
  for (size_t x = 0; x < (size_t)X; ++x) {
    std::vector<std::pair<int64_t, size_t>> heap;
    for (size_t li = 0; li < (size_t)wx; ++li) heap.push_back({0, li});
    auto gt = [](const std::pair<int64_t, size_t> &a, const std::pair<int64_t, size_t> &b) { return a > b; };
    for (int64_t u : queue[x]) {
      std::pop_heap(heap.begin(), heap.end(), gt);
      heap.back().first += cost[(size_t)u];
      mine[x][heap.back().second].push_back(u);
      std::push_heap(heap.begin(), heap.end(), gt);
    }
  }
  p.slice.assign((size_t)nw + 1, 0);
  for (int64_t w = 0; w < nw; ++w) {
    const size_t x = (size_t)((w / W) % X);
    const size_t li = (size_t)((w / W / X) * W + w % W);  // the XCD's li-th wave
    p.slice[(size_t)w] = (int32_t)p.order.size();
    for (int64_t u : mine[x][li]) p.order.push_back(u);
  }
  p.slice[(size_t)nw] = (int32_t)p.order.size();
  return p;
}

}  // namespace sell
