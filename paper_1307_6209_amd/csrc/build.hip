// Device kernels of the SELL-C-sigma construction (Sects. 3.3 and 3.4 of
// Kreutzer et al., arXiv:1307.6209): row lengths and CRS validation, the
// sigma-window sort, chunk widths (Eq. (max)), chunk offsets (prefix sum of
// C * cl[i]) and the padded column-major fill.
#include "sell_internal.h"

#include <hip/hip_bf16.h>

namespace sell {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Validation flag bits.
constexpr uint32_t F_RPT0 = 1u, F_DECR = 2u, F_COL = 4u, F_RPTN = 8u, F_LONG = 16u;

// len[i] = rpt[i+1] - rpt[i]; flags for a malformed rpt; sum of squared
// lengths (for the coefficient of variation) and the longest row. A fixed
// grid strides over the rows and reduces per block, so the three global
// atomics are issued once per block, not once per wave.
__global__ void __launch_bounds__(kBlock) k_rowlen(const int64_t *__restrict__ rpt, int64_t n, int64_t nnz,
                                                   int32_t *__restrict__ len, uint32_t *flags,
                                                   unsigned long long *sumsq, int32_t *maxlen) {
  __shared__ unsigned long long s_sq[kBlock / 64];
  __shared__ int32_t s_mx[kBlock / 64];
  __shared__ uint32_t s_f[kBlock / 64];
  uint32_t f = 0;
  int32_t mx = 0;
  unsigned long long sq = 0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    int64_t d = rpt[i + 1] - rpt[i];
    if (d < 0) f |= F_DECR;
    if (d > 0x7fffffffLL) f |= F_LONG;
    int32_t l = (d < 0 || d > 0x7fffffffLL) ? 0 : (int32_t)d;
    len[i] = l;
    sq += (unsigned long long)l * (unsigned long long)l;
    mx = l > mx ? l : mx;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (rpt[0] != 0) f |= F_RPT0;
    if (rpt[n] != nnz) f |= F_RPTN;
  }
  sq = wave_sum_u64(sq);
  mx = wave_max(mx);
  for (int off = 32; off > 0; off >>= 1) f |= __shfl_xor(f, off);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    s_sq[w] = sq;
    s_mx[w] = mx;
    s_f[w] = f;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kBlock / 64; ++k) {
      sq += s_sq[k];
      mx = s_mx[k] > mx ? s_mx[k] : mx;
      f |= s_f[k];
    }
    if (sq) atomicAdd(sumsq, sq);
    if (mx) atomicMax(maxlen, mx);
    if (f) atomicOr(flags, f);
  }
}

__global__ void __launch_bounds__(kBlock) k_colcheck(const int32_t *__restrict__ col, int64_t nnz, int64_t ncols,
                                                     uint32_t *flags) {
  int64_t stride = (int64_t)gridDim.x * kBlock;
  bool bad = false;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < nnz; j += stride) {
    int32_t c = col[j];
    bad |= (c < 0) | ((int64_t)c >= ncols);
  }
  if (__ballot(bad) != 0ull && lane_id() == 0) atomicOr(flags, F_COL);
}

// ---------------------------------------------------------------------------
// sigma-window sort.
//
// Rows are ordered by descending length inside each window of sigma rows,
// ties by ascending row index. Each element gets a 64-bit key that is unique
// and whose ascending order is that order:
//   (window-in-tile, INT32_MAX - len, index)   when sigma <= kTile
//   (INT32_MAX - len, index in window)         when sigma >  kTile
// Step 1 sorts tiles of kTile keys in LDS (bitonic network). A tile is a run
// of whole windows (sigma <= kTile) or a kTile-aligned piece of one window.
// Step 2 (sigma > kTile only) merges sorted runs pairwise inside each
// window: with unique keys an element's place in the merged run is its
// place in its own run plus the number of smaller keys in the partner run,
// found by binary search.
// ---------------------------------------------------------------------------
constexpr int kTile = 4096;
constexpr int kSortBlock = 512;

__global__ void __launch_bounds__(kSortBlock) k_sort_tiles(const int32_t *__restrict__ len, int64_t n,
                                                           int64_t sigma, uint64_t *__restrict__ keys_out,
                                                           int32_t *__restrict__ perm_out) {
  __shared__ uint64_t sk[kTile];
  int64_t start, count;
  bool small = sigma <= kTile;
  int64_t wper = 1;
  if (small) {
    wper = kTile / sigma;  // whole windows per tile
    int64_t tile_rows = wper * sigma;
    start = (int64_t)blockIdx.x * tile_rows;
    count = n - start < tile_rows ? n - start : tile_rows;
  } else {
    int64_t tiles_per_win = (sigma + kTile - 1) / kTile;
    int64_t w = blockIdx.x / tiles_per_win, tw = blockIdx.x % tiles_per_win;
    int64_t wstart = w * sigma;
    int64_t wlen = n - wstart < sigma ? n - wstart : sigma;
    start = wstart + tw * kTile;
    int64_t end = wstart + wlen;
    count = start >= end ? 0 : (end - start < kTile ? end - start : kTile);
  }
  if (count <= 0) return;  // uniform over the block
  for (int q = threadIdx.x; q < kTile; q += kSortBlock) {
    uint64_t key = ~0ull;
    if (q < count) {
      int64_t i = start + q;
      uint64_t inv = (uint64_t)(0x7fffffff - len[i]);
      if (small) {
        uint64_t wl = (uint64_t)(q / sigma);
        key = (wl << 44) | (inv << 13) | (uint64_t)q;
      } else {
        int64_t wstart = (i / sigma) * sigma;
        key = (inv << 32) | (uint64_t)(i - wstart);
      }
    }
    sk[q] = key;
  }
  __syncthreads();
  // bitonic sort, ascending
  for (int size = 2; size <= kTile; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < kTile / 2; t += kSortBlock) {
        int lo = 2 * t - (t & (stride - 1));
        int hi = lo + stride;
        bool asc = (lo & size) == 0;
        uint64_t a = sk[lo], b = sk[hi];
        if ((a > b) == asc) {
          sk[lo] = b;
          sk[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  for (int q = threadIdx.x; q < count; q += kSortBlock) {
    uint64_t key = sk[q];
    if (small) {
      perm_out[start + q] = (int32_t)(start + (int64_t)(key & 0x1fffull));
    } else {
      keys_out[start + q] = key;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_merge_runs(const uint64_t *__restrict__ in, uint64_t *__restrict__ out,
                                                       int64_t n, int64_t sigma, int64_t R) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int64_t wstart = (i / sigma) * sigma;
  int64_t wlen = n - wstart < sigma ? n - wstart : sigma;
  int64_t q = i - wstart;
  int64_t run = q / R;
  int64_t pstart = (run ^ 1) * R;
  uint64_t key = in[i];
  if (pstart >= wlen) {
    out[i] = key;
    return;
  }
  int64_t pend = pstart + R < wlen ? pstart + R : wlen;
  // number of partner keys smaller than key (keys are unique)
  int64_t lo = pstart, hi = pend;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (in[wstart + mid] < key) lo = mid + 1;
    else hi = mid;
  }
  int64_t pos = ((run & ~(int64_t)1) * R) + (q - run * R) + (lo - pstart);
  out[wstart + pos] = key;
}

__global__ void __launch_bounds__(kBlock) k_keys_to_perm(const uint64_t *__restrict__ keys, int64_t n, int64_t sigma,
                                                         int32_t *__restrict__ perm) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int64_t wstart = (i / sigma) * sigma;
  perm[i] = (int32_t)(wstart + (int64_t)(keys[i] & 0xffffffffull));
}

// cl[i] = max length of the chunk's rows in sorted order (Eq. (max));
// csz[i] = C * cl[i] (scanned into cs afterwards); csz[nchunks] = 0.
__global__ void __launch_bounds__(kBlock) k_chunkwidth(const int32_t *__restrict__ len,
                                                       const int32_t *__restrict__ perm, int64_t n, int C,
                                                       int64_t nchunks, int32_t *__restrict__ cl,
                                                       int64_t *__restrict__ csz) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i > nchunks) return;
  if (i == nchunks) {
    csz[i] = 0;
    return;
  }
  int32_t mx = 0;
  int64_t p0 = i * C;
  for (int r = 0; r < C; ++r) {
    int64_t p = p0 + r;
    if (p < n) {
      int32_t l = len[perm ? perm[p] : p];
      mx = l > mx ? l : mx;
    }
  }
  cl[i] = mx;
  csz[i] = (int64_t)C * mx;
}

// ---------------------------------------------------------------------------
// Exclusive prefix sum of int64 values: per-block scan of kScanItems
// elements, recursive scan of the block totals, then add the block offsets.
// ---------------------------------------------------------------------------
constexpr int kScanBlock = 256;
constexpr int kScanPer = 4;
constexpr int kScanItems = kScanBlock * kScanPer;

__global__ void __launch_bounds__(kScanBlock) k_scan_block(const int64_t *__restrict__ in, int64_t *__restrict__ out,
                                                           int64_t n, int64_t *__restrict__ totals) {
  __shared__ int64_t wsum[kScanBlock / 64];
  int64_t base = (int64_t)blockIdx.x * kScanItems + (int64_t)threadIdx.x * kScanPer;
  int64_t v[kScanPer];
  int64_t run = 0;
#pragma unroll
  for (int e = 0; e < kScanPer; ++e) {
    int64_t idx = base + e;
    v[e] = idx < n ? in[idx] : 0;
    run += v[e];
  }
  // inclusive scan of the thread totals across the wave
  int lane = lane_id(), wid = threadIdx.x >> 6;
  int64_t incl = run;
  for (int off = 1; off < 64; off <<= 1) {
    int64_t o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int64_t wbase = 0;
  for (int w = 0; w < wid; ++w) wbase += wsum[w];
  int64_t excl = wbase + incl - run;
#pragma unroll
  for (int e = 0; e < kScanPer; ++e) {
    int64_t idx = base + e;
    if (idx < n) out[idx] = excl;
    excl += v[e];
  }
  if (threadIdx.x == kScanBlock - 1) {
    int64_t tot = 0;
    for (int w = 0; w < kScanBlock / 64; ++w) tot += wsum[w];
    totals[blockIdx.x] = tot;
  }
}

__global__ void __launch_bounds__(kScanBlock) k_scan_add(int64_t *__restrict__ out, int64_t n,
                                                         const int64_t *__restrict__ offs) {
  int64_t base = (int64_t)blockIdx.x * kScanItems;
  int64_t add = offs[blockIdx.x];
  for (int e = threadIdx.x; e < kScanItems; e += kScanBlock) {
    int64_t idx = base + e;
    if (idx < n) out[idx] += add;
  }
}

// ---------------------------------------------------------------------------
// Fill: slot s of the padded arrays belongs to chunk i with cs[i] <= s <
// cs[i+1]; inside it, column j = (s - cs[i]) / C and lane r = (s - cs[i]) % C
// (the layout val[cs[i] + j*C + r]). The slot receives entry j of row
// perm[i*C + r] in CRS order, or value 0 / column 0 when that row is shorter
// or does not exist.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float f64_to_f32_rne(double d) { return (float)d; }

// Nearest-even rounding of a double to bfloat16 in two steps that cannot
// double-round: round to binary32 with round-to-odd (24 >= 2*8 + 2 bits,
// Boldo and Melquiond, "Emulation of FMA and correctly rounded sums: proved
// algorithms using rounding to odd", IEEE TC 2008), then round that binary32
// to bfloat16 nearest-even on its bit pattern.
__device__ __forceinline__ uint16_t f64_to_bf16_rne(double d) {
  float f = (float)d;
  uint32_t b = __float_as_uint(f);
  double back = (double)f;
  if (back != d && !(d != d)) {
    if (fabs(back) > fabs(d)) b -= 1;  // step toward zero: the truncated value
    b |= 1u;                           // odd last bit marks the inexact result
  }
  if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) return (uint16_t)((b >> 16) | 0x40u);  // NaN
  uint32_t lsb = (b >> 16) & 1u;
  b += 0x7fffu + lsb;
  return (uint16_t)(b >> 16);
}

template <int VD>
__global__ void __launch_bounds__(kBlock) k_fill(const int64_t *__restrict__ rpt, const int32_t *__restrict__ col,
                                                 const double *__restrict__ val, int64_t n, int C,
                                                 const int32_t *__restrict__ perm, const int32_t *__restrict__ len,
                                                 const int64_t *__restrict__ cs, int64_t nchunks, int64_t padded,
                                                 const int32_t *__restrict__ cmap, int32_t *__restrict__ scol,
                                                 void *__restrict__ sval) {
  int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < padded; s += stride) {
    // largest i with cs[i] <= s
    int64_t lo = 0, hi = nchunks;  // answer in [0, nchunks)
    while (hi - lo > 1) {
      int64_t mid = (lo + hi) >> 1;
      if (cs[mid] <= s) lo = mid;
      else hi = mid;
    }
    int64_t off = s - cs[lo];
    int64_t j = off / C;
    int64_t r = off - j * C;
    int64_t p = lo * C + r;
    int32_t c = 0;
    double v = 0.0;
    if (p < n) {
      int64_t row = perm ? perm[p] : p;
      if (j < len[row]) {
        int64_t src = rpt[row] + j;
        c = cmap ? cmap[col[src]] : col[src];
        v = val[src];
      }
    }
    scol[s] = c;
    if (VD == SELL_F64) static_cast<double *>(sval)[s] = v;
    else if (VD == SELL_F32) static_cast<float *>(sval)[s] = f64_to_f32_rne(v);
    else static_cast<uint16_t *>(sval)[s] = f64_to_bf16_rne(v);
  }
}

// iperm[perm[p]] = p
__global__ void __launch_bounds__(kBlock) k_invert(const int32_t *__restrict__ perm, int64_t n,
                                                   int32_t *__restrict__ iperm) {
  int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p < n) iperm[perm[p]] = (int32_t)p;
}

// rl[p] = len[perm[p]]: the length of the row in sorted position p, 0 for
// the rows that pad the last chunk (p in [n, np))
__global__ void __launch_bounds__(kBlock) k_sorted_len(const int32_t *__restrict__ len,
                                                       const int32_t *__restrict__ perm, int64_t n, int64_t np,
                                                       int32_t *__restrict__ rl) {
  int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p < np) rl[p] = p < n ? len[perm ? (int64_t)perm[p] : p] : 0;
}

// out[p] = in[perm[p]] (gather into sorted order) or out[perm[p]] = in[p]
// (scatter back), for elements of ES bytes.
template <typename E, bool SCATTER>
__global__ void __launch_bounds__(kBlock) k_permute(const E *__restrict__ in, E *__restrict__ out,
                                                    const int32_t *__restrict__ perm, int64_t n) {
  int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  const int64_t q = perm ? (int64_t)perm[p] : p;
  if (SCATTER) out[q] = in[p];
  else out[p] = in[q];
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t build_sorted_len(const int32_t *len, const int32_t *perm, int64_t n, int64_t np, int32_t *rl,
                            hipStream_t s) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sorted_len, dim3(blocks_for(np, kBlock)), dim3(kBlock), 0, s, len, perm, n, np, rl);
  return hipGetLastError();
}

hipError_t build_invert(const int32_t *perm, int64_t n, int32_t *iperm, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_invert, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, perm, n, iperm);
  return hipGetLastError();
}

hipError_t permute_vector(const void *in, void *out, const int32_t *perm, int64_t n, int elem_bytes, bool scatter,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned nb = blocks_for(n, kBlock);
  if (elem_bytes == 8) {
    if (scatter)
      hipLaunchKernelGGL((k_permute<uint64_t, true>), dim3(nb), dim3(kBlock), 0, s, static_cast<const uint64_t *>(in),
                         static_cast<uint64_t *>(out), perm, n);
    else
      hipLaunchKernelGGL((k_permute<uint64_t, false>), dim3(nb), dim3(kBlock), 0, s,
                         static_cast<const uint64_t *>(in), static_cast<uint64_t *>(out), perm, n);
  } else {
    if (scatter)
      hipLaunchKernelGGL((k_permute<uint32_t, true>), dim3(nb), dim3(kBlock), 0, s, static_cast<const uint32_t *>(in),
                         static_cast<uint32_t *>(out), perm, n);
    else
      hipLaunchKernelGGL((k_permute<uint32_t, false>), dim3(nb), dim3(kBlock), 0, s,
                         static_cast<const uint32_t *>(in), static_cast<uint32_t *>(out), perm, n);
  }
  return hipGetLastError();
}

hipError_t build_rowlen(const int64_t *rpt, int64_t n, int64_t nnz, int32_t *len, uint32_t *flags,
                        unsigned long long *sumsq, int32_t *maxlen, hipStream_t s) {
  unsigned nb = blocks_for(n > 0 ? n : 1, kBlock);
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_rowlen, dim3(nb), dim3(kBlock), 0, s, rpt, n, nnz, len, flags, sumsq, maxlen);
  return hipGetLastError();
}

hipError_t build_colcheck(const int32_t *col, int64_t nnz, int64_t ncols, uint32_t *flags, hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  int64_t nb = blocks_for(nnz, kBlock);
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_colcheck, dim3((unsigned)nb), dim3(kBlock), 0, s, col, nnz, ncols, flags);
  return hipGetLastError();
}

hipError_t build_sort(const int32_t *len, int64_t n, int64_t sigma, uint64_t *keys_a, uint64_t *keys_b,
                      int32_t *perm, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (sigma > n) sigma = n;
  int64_t ntiles;
  if (sigma <= kTile) {
    int64_t tile_rows = (kTile / sigma) * sigma;
    ntiles = (n + tile_rows - 1) / tile_rows;
  } else {
    int64_t nwin = (n + sigma - 1) / sigma;
    ntiles = nwin * ((sigma + kTile - 1) / kTile);
  }
  hipLaunchKernelGGL(k_sort_tiles, dim3((unsigned)ntiles), dim3(kSortBlock), 0, s, len, n, sigma, keys_a, perm);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || sigma <= kTile) return e;
  uint64_t *in = keys_a, *out = keys_b;
  for (int64_t R = kTile; R < sigma; R <<= 1) {
    hipLaunchKernelGGL(k_merge_runs, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, in, out, n, sigma, R);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    uint64_t *t = in;
    in = out;
    out = t;
  }
  hipLaunchKernelGGL(k_keys_to_perm, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, in, n, sigma, perm);
  return hipGetLastError();
}

hipError_t build_chunkwidth(const int32_t *len, const int32_t *perm, int64_t n, int C, int64_t nchunks,
                            int32_t *cl, int64_t *csz, hipStream_t s) {
  hipLaunchKernelGGL(k_chunkwidth, dim3(blocks_for(nchunks + 1, kBlock)), dim3(kBlock), 0, s, len, perm, n, C,
                     nchunks, cl, csz);
  return hipGetLastError();
}

int64_t scan_tmp_elems(int64_t n) {
  int64_t total = 0;
  while (n > kScanItems) {
    int64_t nb = (n + kScanItems - 1) / kScanItems;
    total += nb;
    n = nb;
  }
  return total + 1;
}

hipError_t build_scan(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + kScanItems - 1) / kScanItems;
  hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, out, n, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nb == 1) return e;
  // scan the block totals (in place), then add them
  e = build_scan(tmp, tmp, nb, tmp + nb, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanBlock), 0, s, out, n, tmp);
  return hipGetLastError();
}

hipError_t build_fill(const int64_t *rpt, const int32_t *col, const double *val, int64_t n, int C,
                      const int32_t *perm, const int32_t *len, const int64_t *cs, int64_t nchunks, int64_t padded,
                      const int32_t *cmap, int32_t *scol, void *sval, int val_dtype, hipStream_t s) {
  if (padded <= 0) return hipSuccess;
  int64_t nb = blocks_for(padded, kBlock);
  if (nb > 262144) nb = 262144;
  if (val_dtype == SELL_F64)
    hipLaunchKernelGGL(k_fill<SELL_F64>, dim3((unsigned)nb), dim3(kBlock), 0, s, rpt, col, val, n, C, perm, len, cs,
                       nchunks, padded, cmap, scol, sval);
  else if (val_dtype == SELL_F32)
    hipLaunchKernelGGL(k_fill<SELL_F32>, dim3((unsigned)nb), dim3(kBlock), 0, s, rpt, col, val, n, C, perm, len, cs,
                       nchunks, padded, cmap, scol, sval);
  else
    hipLaunchKernelGGL(k_fill<SELL_BF16>, dim3((unsigned)nb), dim3(kBlock), 0, s, rpt, col, val, n, C, perm, len,
                       cs, nchunks, padded, cmap, scol, sval);
  return hipGetLastError();
}

}  // namespace sell
