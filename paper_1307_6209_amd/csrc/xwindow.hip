// The x window of each product workgroup: the distinct column indices that
// the slots of its consecutive chunks (a group of gc) hold, sorted. The product
// kernel stages the window in LDS once per workgroup, and every slot's
// column index is stored a second time as its 16-bit position in the window,
// so the x gathers become LDS reads and the streamed index shrinks from 4 to
// 2 bytes. The window is kept as segments (runs of consecutive columns:
// start column, position in the window, length) so that staging reads x in
// contiguous runs. Padding slots hold column 0, which joins the window like
// any other column: the product is the same, bit for bit, as with the
// global column indices.
#include "sell_internal.h"

namespace sell {
namespace {

constexpr int kXwBlock = 256;

// Exclusive prefix sum over the block of one int per thread; *total gets the
// sum. tmp: kXwBlock ints of LDS.
__device__ int block_exclusive_scan(int v, int *tmp, int *total) {
  const int tid = threadIdx.x;
  tmp[tid] = v;
  __syncthreads();
  for (int off = 1; off < kXwBlock; off <<= 1) {
    const int o = tid >= off ? tmp[tid - off] : 0;
    __syncthreads();
    tmp[tid] += o;
    __syncthreads();
  }
  const int incl = tmp[tid];
  *total = tmp[kXwBlock - 1];
  __syncthreads();
  return incl - v;
}

// Compacts the positions i < n with flag(i) true, in order, into out[];
// returns their count. Each thread takes a contiguous range of positions.
template <typename F, typename W>
__device__ int block_compact(int n, F flag, W write, int *tmp) {
  const int per = (n + kXwBlock - 1) / kXwBlock;
  const int i0 = threadIdx.x * per;
  const int i1 = i0 + per < n ? i0 + per : n;
  int cnt = 0;
  for (int i = i0; i < i1; ++i) cnt += flag(i) ? 1 : 0;
  int total = 0;
  int pos = block_exclusive_scan(cnt, tmp, &total);
  for (int i = i0; i < i1; ++i)
    if (flag(i)) write(pos++, i);
  __syncthreads();
  return total;
}

// Run starts (first set bit of each run of set bits) and run ends (last set
// bit) of word w of a bitmap of nw words.
__device__ __forceinline__ uint32_t run_starts(const uint32_t *bm, int w) {
  const uint32_t x = bm[w], prev = w > 0 ? bm[w - 1] >> 31 : 0u;
  return x & ~((x << 1) | prev);
}
__device__ __forceinline__ uint32_t run_ends(const uint32_t *bm, int w, int nw) {
  const uint32_t x = bm[w], next = w + 1 < nw ? (bm[w + 1] & 1u) << 31 : 0u;
  return x & ~((x >> 1) | next);
}

// One workgroup per group of gc chunks.
// PASS 0: segment count per group into nseg[g] (and nseg[ngroups] = 0 for
//         the scan), the largest window into *maxwin and the most segments
//         of a group into *maxseg, flag bit 1 when a group holds more than
//         kXwMaxSlots slots.
// PASS 1: the segments, at 3 * segoff[g], and the window position of every
//         slot of the group.
// Groups whose columns span at most 32 * kXwMaxSlots values use a bitmap of
// the span in LDS (distinct columns in order, their ranks by popcount, runs
// from the edges of the set bits: linear in the slots and the span); the
// others sort their column indices. Column 0, which every padding slot
// holds, is kept out of the span: it becomes a window element and a run of
// its own in front, unless column 1 is present (then the span starts at 0).
// Both ways give the same window, runs and positions.
template <int PASS>
__global__ void __launch_bounds__(kXwBlock) k_xw_groups(const int32_t *__restrict__ col, const int64_t *__restrict__ cs,
                                                        int64_t nchunks, int gc, int64_t ngroups,
                                                        int64_t *__restrict__ nseg,
                                                        uint32_t *flags, int32_t *maxwin, int32_t *maxseg,
                                                        const int64_t *__restrict__ segoff, int32_t *__restrict__ seg,
                                                        uint16_t *__restrict__ lcol) {
  __shared__ int32_t keys[kXwMaxSlots];
  __shared__ int32_t uk[kXwMaxSlots];
  __shared__ int tmp[kXwBlock];
  __shared__ int32_t startb[kXwMaxSeg];
  __shared__ int red[3];
  const int64_t g = blockIdx.x;
  const int tid = threadIdx.x;
  if (PASS == 0 && g == 0 && tid == 0) nseg[ngroups] = 0;
  const int64_t c0 = g * gc;
  const int64_t c1 = c0 + gc < nchunks ? c0 + gc : nchunks;
  const int64_t sb = cs[c0], se = cs[c1];
  if (se - sb > kXwMaxSlots) {  // uniform over the block
    if (PASS == 0 && tid == 0) {
      atomicOr(flags, 1u);
      nseg[g] = 0;
    }
    return;
  }
  const int n = (int)(se - sb);

  // column range of the group, column 0 apart
  if (tid == 0) {
    red[0] = 0x7fffffff;
    red[1] = -1;
    red[2] = 0;
  }
  __syncthreads();
  {
    int lo = 0x7fffffff, hi = -1, z = 0;
    for (int i = tid; i < n; i += kXwBlock) {
      const int32_t c = col[sb + i];
      if (c == 0) z = 1;
      else {
        lo = c < lo ? c : lo;
        hi = c > hi ? c : hi;
      }
    }
    if (hi >= 0) {
      atomicMin(&red[0], lo);
      atomicMax(&red[1], hi);
    }
    if (z) atomicOr(&red[2], 1);
  }
  __syncthreads();
  int lo = red[0], hi = red[1];
  const bool has0 = red[2] != 0;
  if (hi < 0) lo = hi = 0;        // column 0 only, or no slot
  else if (has0 && lo <= 1) lo = 0;  // column 0 starts the first run
  const int extra = has0 && lo > 0 ? 1 : 0;  // column 0 in front, a run of its own
  const int64_t span = (int64_t)hi - lo + 1;
  if (n > 0 && span <= 32 * (int64_t)kXwMaxSlots) {
    uint32_t *bm = reinterpret_cast<uint32_t *>(keys);
    int32_t *wpre = uk;  // distinct columns in the words before w
    const int nw = (int)((span + 31) / 32);
    for (int w = tid; w < nw; w += kXwBlock) bm[w] = 0u;
    __syncthreads();
    for (int i = tid; i < n; i += kXwBlock) {
      const int32_t c = col[sb + i];
      if (c != 0 || !extra) {
        const int b = c - lo;
        atomicOr(&bm[b >> 5], 1u << (b & 31));
      }
    }
    __syncthreads();
    const int per = (nw + kXwBlock - 1) / kXwBlock;
    const int w0 = tid * per < nw ? tid * per : nw;
    const int w1 = w0 + per < nw ? w0 + per : nw;
    int cnt = 0, runs = 0;
    for (int w = w0; w < w1; ++w) {
      cnt += __popc(bm[w]);
      runs += __popc(run_starts(bm, w));
    }
    int tot_cnt = 0, tot_runs = 0;
    const int pc = block_exclusive_scan(cnt, tmp, &tot_cnt);
    const int pr = block_exclusive_scan(runs, tmp, &tot_runs);
    {
      int acc = pc;
      for (int w = w0; w < w1; ++w) {
        wpre[w] = acc;
        acc += __popc(bm[w]);
      }
    }
    const int nuniq = tot_cnt + extra, ns = tot_runs + extra;
    if (PASS == 0) {
      if (tid == 0) {
        nseg[g] = ns;
        atomicMax(maxwin, nuniq);
        atomicMax(maxseg, ns);
      }
      return;
    }
    if (ns > kXwMaxSeg) return;  // refused by the caller after the count pass
    __syncthreads();             // wpre complete
    int32_t *out = seg + 3 * segoff[g];
    if (extra && tid == 0) {
      out[0] = 0;
      out[1] = 0;
      out[2] = 1;
    }
    // run starts: first column and window position of each run
    int k = extra + pr;
    for (int w = w0; w < w1; ++w) {
      uint32_t st = run_starts(bm, w);
      while (st) {
        const int b = __ffs(st) - 1;
        st &= st - 1;
        const int bit = w * 32 + b;
        startb[k] = bit;
        out[3 * k] = lo + bit;
        out[3 * k + 1] = extra + wpre[w] + __popc(bm[w] & ((1u << b) - 1u));
        ++k;
      }
    }
    __syncthreads();  // startb complete
    // run ends: the run that ends at bit e is the last one started at or
    // before e
    int before = pr;
    for (int w = w0; w < w1; ++w) {
      const uint32_t st = run_starts(bm, w);
      uint32_t en = run_ends(bm, w, nw);
      while (en) {
        const int b = __ffs(en) - 1;
        en &= en - 1;
        const uint32_t upto = b == 31 ? 0xffffffffu : (2u << b) - 1u;
        const int r = extra + before + __popc(st & upto) - 1;
        out[3 * r + 2] = w * 32 + b - startb[r] + 1;
      }
      before += __popc(st);
    }
    // window position of every slot
    for (int i = tid; i < n; i += kXwBlock) {
      const int32_t c = col[sb + i];
      int p = 0;
      if (c != 0 || !extra) {
        const int b = c - lo;
        p = extra + wpre[b >> 5] + __popc(bm[b >> 5] & ((1u << (b & 31)) - 1u));
      }
      lcol[sb + i] = (uint16_t)p;
    }
    return;
  }

  int P = 1;
  while (P < n) P <<= 1;
  for (int i = tid; i < P; i += kXwBlock) keys[i] = i < n ? col[sb + i] : 0x7fffffff;
  __syncthreads();
  // bitonic sort, ascending
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = tid; t < P / 2; t += kXwBlock) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const int32_t a = keys[lo], b = keys[hi];
        if ((a > b) == asc) {
          keys[lo] = b;
          keys[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  // distinct columns, in order
  const int nuniq = block_compact(
      n, [&](int i) { return i == 0 || keys[i] != keys[i - 1]; }, [&](int p, int i) { uk[p] = keys[i]; }, tmp);
  // segment starts: positions j where the run of consecutive columns breaks
  // (their window positions go to keys[], no longer needed)
  const int ns = block_compact(
      nuniq, [&](int j) { return j == 0 || uk[j] != uk[j - 1] + 1; }, [&](int p, int j) { keys[p] = j; }, tmp);
  if (PASS == 0) {
    if (tid == 0) {
      nseg[g] = ns;
      atomicMax(maxwin, nuniq);
      atomicMax(maxseg, ns);
    }
    return;
  }
  int32_t *out = seg + 3 * segoff[g];
  for (int k = tid; k < ns; k += kXwBlock) {
    const int j = keys[k];
    const int jn = k + 1 < ns ? keys[k + 1] : nuniq;
    out[3 * k] = uk[j];
    out[3 * k + 1] = j;
    out[3 * k + 2] = jn - j;
  }
  for (int i = tid; i < n; i += kXwBlock) {
    const int32_t c = col[sb + i];
    int lo = 0, hi = nuniq - 1;  // uk[lo..hi] holds c
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (uk[mid] < c) lo = mid + 1;
      else hi = mid;
    }
    lcol[sb + i] = (uint16_t)lo;
  }
}

}  // namespace

hipError_t build_xw_count(const int32_t *col, const int64_t *cs, int64_t nchunks, int gc, int64_t *nseg,
                          uint32_t *flags, int32_t *maxwin, int32_t *maxseg, hipStream_t s) {
  if (gc <= 0) return hipErrorInvalidValue;
  const int64_t ngroups = (nchunks + gc - 1) / gc;
  if (ngroups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xw_groups<0>, dim3((unsigned)ngroups), dim3(kXwBlock), 0, s, col, cs, nchunks, gc, ngroups,
                     nseg, flags, maxwin, maxseg, nullptr, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t build_xw_fill(const int32_t *col, const int64_t *cs, int64_t nchunks, int gc, const int64_t *segoff,
                         int32_t *seg, uint16_t *lcol, hipStream_t s) {
  if (gc <= 0) return hipErrorInvalidValue;
  const int64_t ngroups = (nchunks + gc - 1) / gc;
  if (ngroups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xw_groups<1>, dim3((unsigned)ngroups), dim3(kXwBlock), 0, s, col, cs, nchunks, gc, ngroups,
                     nullptr, nullptr, nullptr, nullptr, segoff, seg, lcol);
  return hipGetLastError();
}

}  // namespace sell
