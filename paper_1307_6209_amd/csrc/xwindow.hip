// The x window of each product workgroup: the distinct column indices that
// the slots of its kXwChunks consecutive chunks hold, sorted. The product
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

// One workgroup per group of kXwChunks chunks.
// PASS 0: segment count per group into nseg[g] (and nseg[ngroups] = 0 for
//         the scan), the largest window into *maxwin and the most segments
//         of a group into *maxseg, flag bit 1 when a group holds more than
//         kXwMaxSlots slots.
// PASS 1: the segments, at 3 * segoff[g], and the window position of every
//         slot of the group.
template <int PASS>
__global__ void __launch_bounds__(kXwBlock) k_xw_groups(const int32_t *__restrict__ col, const int64_t *__restrict__ cs,
                                                        int64_t nchunks, int64_t ngroups, int64_t *__restrict__ nseg,
                                                        uint32_t *flags, int32_t *maxwin, int32_t *maxseg,
                                                        const int64_t *__restrict__ segoff, int32_t *__restrict__ seg,
                                                        uint16_t *__restrict__ lcol) {
  __shared__ int32_t keys[kXwMaxSlots];
  __shared__ int32_t uk[kXwMaxSlots];
  __shared__ int tmp[kXwBlock];
  const int64_t g = blockIdx.x;
  const int tid = threadIdx.x;
  if (PASS == 0 && g == 0 && tid == 0) nseg[ngroups] = 0;
  const int64_t c0 = g * kXwChunks;
  const int64_t c1 = c0 + kXwChunks < nchunks ? c0 + kXwChunks : nchunks;
  const int64_t sb = cs[c0], se = cs[c1];
  if (se - sb > kXwMaxSlots) {  // uniform over the block
    if (PASS == 0 && tid == 0) {
      atomicOr(flags, 1u);
      nseg[g] = 0;
    }
    return;
  }
  const int n = (int)(se - sb);
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

hipError_t build_xw_count(const int32_t *col, const int64_t *cs, int64_t nchunks, int64_t *nseg, uint32_t *flags,
                          int32_t *maxwin, int32_t *maxseg, hipStream_t s) {
  const int64_t ngroups = (nchunks + kXwChunks - 1) / kXwChunks;
  if (ngroups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xw_groups<0>, dim3((unsigned)ngroups), dim3(kXwBlock), 0, s, col, cs, nchunks, ngroups, nseg,
                     flags, maxwin, maxseg, nullptr, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t build_xw_fill(const int32_t *col, const int64_t *cs, int64_t nchunks, const int64_t *segoff, int32_t *seg,
                         uint16_t *lcol, hipStream_t s) {
  const int64_t ngroups = (nchunks + kXwChunks - 1) / kXwChunks;
  if (ngroups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xw_groups<1>, dim3((unsigned)ngroups), dim3(kXwBlock), 0, s, col, cs, nchunks, ngroups,
                     nullptr, nullptr, nullptr, nullptr, segoff, seg, lcol);
  return hipGetLastError();
}

}  // namespace sell
