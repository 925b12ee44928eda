// Bandwidth microbenchmarks that set the roofline bandwidth b of the
// performance model (Sect. 2.1 of Kreutzer et al., arXiv:1307.6209): a
// read-only sum over an array (the paper's "reduction" benchmark) and an
// array copy, both with 16-byte non-temporal accesses; a random-gather
// rate (8-byte loads at hashed positions of an array), the ceiling of
// products whose right-hand-side accesses have no locality; and a random-row
// rate (whole rows of 128, 256 or 512 bytes at hashed row positions), the
// same ceiling for the block form, whose k right-hand sides make each
// access one row of 8k bytes; a write-only stream, the rate of the
// result's stores; and random rows read with rows written in order, four
// to one, the block form's mix of both.
#include "sell_internal.h"

namespace sell {
namespace {

constexpr int kBlock = 256;
typedef double d2 __attribute__((ext_vector_type(2)));  // one 16-byte access

// Each wave streams one contiguous slab of the array, eight 16-byte
// non-temporal loads per lane in flight (measured the fastest read pattern
// on this device: contiguous per-wave streams beat a grid-stride sweep).
__global__ void __launch_bounds__(kBlock) k_read(const d2 *__restrict__ a, int64_t n2, int64_t per_wave,
                                                 double *sink) {
  constexpr int U = 8;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t b0 = wave * per_wave;
  const int64_t b1 = b0 + per_wave < n2 ? b0 + per_wave : n2;
  double s0 = 0.0, s1 = 0.0;
  int64_t i = b0 + lane;
  for (; i + (U - 1) * 64 < b1; i += U * 64) {
    d2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(a + i + u * 64);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      s0 += v[u].x;
      s1 += v[u].y;
    }
  }
  for (; i < b1; i += 64) {
    d2 v = __builtin_nontemporal_load(a + i);
    s0 += v.x;
    s1 += v.y;
  }
  // keep the sum observable without a global reduction: one store per
  // block, from thread 0 or from a lane that sees a NaN sum (never for
  // zeroed input)
  double s = s0 + s1;
  if (threadIdx.x == 0 || s != s) sink[blockIdx.x] = s;
}

// Write-only stream: each wave fills one contiguous slab of the array with
// eight 16-byte non-temporal stores per lane in flight (the store kind of
// the products' y and Y).
__global__ void __launch_bounds__(kBlock) k_write(d2 *__restrict__ a, int64_t n2, int64_t per_wave, double v) {
  constexpr int U = 8;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t b0 = wave * per_wave;
  const int64_t b1 = b0 + per_wave < n2 ? b0 + per_wave : n2;
  d2 w;
  w.x = v;
  w.y = v;
  int64_t i = b0 + lane;
  for (; i + (U - 1) * 64 < b1; i += U * 64) {
#pragma unroll
    for (int u = 0; u < U; ++u) __builtin_nontemporal_store(w, a + i + u * 64);
  }
  for (; i < b1; i += 64) __builtin_nontemporal_store(w, a + i);
}

__global__ void __launch_bounds__(kBlock) k_copy(const d2 *__restrict__ a, d2 *__restrict__ b, int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

// 32-bit integer hash "lowbias32" (C. Wellons, hash-prospector): position
// generator of the gather probe, so no index array is streamed.
__device__ __forceinline__ uint32_t lowbias32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// Each lane loads per_lane doubles at hashed positions of a (n = mask + 1
// elements, a power of two), eight loads in flight; plain (cached) loads,
// as the x gathers of the product.
__global__ void __launch_bounds__(kBlock) k_gather(const double *__restrict__ a, uint32_t mask, int32_t per_lane,
                                                   double *sink) {
  const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
  double s = 0.0;
  for (int32_t i = 0; i < per_lane; i += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = a[lowbias32(t * (uint32_t)per_lane + (uint32_t)(i + u)) & mask];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  if (threadIdx.x == 0 || s != s) sink[blockIdx.x] = s;
}

// Random rows of R = 16*LPR bytes: LPR lanes read one row (16 bytes each),
// a wave 64/LPR rows per access; every lane keeps eight accesses in flight.
// Row positions are hashed, so no index array is streamed. Plain (cached)
// loads, as the block form's reads of X.
template <int LPR>
__global__ void __launch_bounds__(kBlock) k_rows(const d2 *__restrict__ a, uint32_t row_mask, int32_t per_lane,
                                                 double *sink) {
  constexpr int RPA = 64 / LPR;  // rows per access of a wave
  const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const uint32_t g = (uint32_t)(lane / LPR), q = (uint32_t)(lane % LPR);
  double s = 0.0;
  for (int32_t i = 0; i < per_lane; i += 8) {
    d2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t r = lowbias32((wave * (uint32_t)per_lane + (uint32_t)(i + u)) * RPA + g) & row_mask;
      v[u] = a[(size_t)r * LPR + q];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u].x + v[u].y;
  }
  if (threadIdx.x == 0 || s != s) sink[blockIdx.x] = s;
}

// Random rows in, rows out: output row o (rows of 16*LPR bytes, in order)
// is the sum of four input rows at hashed positions -- the block form's
// access pattern (a few random rows of X read per row of Y written) without
// the matrix. Each lane keeps eight row reads in flight (two output rows of
// its group); consecutive waves write consecutive output rows.
template <int LPR>
__global__ void __launch_bounds__(kBlock) k_rows_write(const d2 *__restrict__ a, uint32_t row_mask,
                                                       d2 *__restrict__ out, int64_t ngroups) {
  constexpr int RPA = 64 / LPR;  // output rows per access of a wave
  const int64_t nw = (int64_t)gridDim.x * (kBlock / 64);
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int g = lane / LPR, q = lane % LPR;
  for (int64_t gi = wave; gi < ngroups; gi += 2 * nw) {
    d2 v[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t gg = gi + h * nw;
      const uint32_t o = (uint32_t)(gg * RPA + g);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t r = lowbias32(o * 4u + (uint32_t)j) & row_mask;
        v[h][j] = (d2){0.0, 0.0};
        if (gg < ngroups) v[h][j] = a[(size_t)r * LPR + q];
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t gg = gi + h * nw;
      if (gg < ngroups)
        __builtin_nontemporal_store(v[h][0] + v[h][1] + v[h][2] + v[h][3],
                                    out + (size_t)(gg * RPA + g) * LPR + q);
    }
  }
}

}  // namespace

constexpr int kProbeBlocks = 256 * 16;

hipError_t probe_read(const void *a, size_t bytes, double *sink, hipStream_t s) {
  const int64_t n2 = (int64_t)(bytes / sizeof(d2));
  const int64_t waves = (int64_t)kProbeBlocks * (kBlock / 64) / 2;  // 8192 slabs
  const int64_t per_wave = (n2 + waves - 1) / waves;
  hipLaunchKernelGGL(k_read, dim3((unsigned)(waves * 64 / kBlock)), dim3(kBlock), 0, s, static_cast<const d2 *>(a), n2,
                     per_wave, sink);
  return hipGetLastError();
}

int64_t probe_gather(const void *a, size_t bytes, double *sink, hipStream_t s, hipError_t *err) {
  uint32_t mask = 1;
  while ((uint64_t)(mask + 1) * 2 * sizeof(double) <= bytes && mask < 0x7fffffffu) mask = mask * 2 + 1;
  constexpr int32_t kPerLane = 256;
  constexpr int kBlocks = 2048;  // 524,288 lanes x 256 loads = 2^27 gathers
  hipLaunchKernelGGL(k_gather, dim3(kBlocks), dim3(kBlock), 0, s, static_cast<const double *>(a), mask, kPerLane,
                     sink);
  *err = hipGetLastError();
  return (int64_t)kBlocks * kBlock * kPerLane;
}

int64_t probe_rows(const void *a, size_t bytes, int row_bytes, double *sink, hipStream_t s, hipError_t *err) {
  const int lpr = row_bytes / (int)sizeof(d2);
  uint32_t mask = 1;
  while ((uint64_t)(mask + 1) * 2 * (uint64_t)row_bytes <= bytes && mask < 0x7fffffffu) mask = mask * 2 + 1;
  constexpr int32_t kPerLane = 64;
  constexpr int kBlocks = 2048;  // 8,192 waves x 64 accesses x 64/LPR rows
  const dim3 grid(kBlocks), block(kBlock);
  const d2 *p = static_cast<const d2 *>(a);
  if (lpr == 8) hipLaunchKernelGGL(k_rows<8>, grid, block, 0, s, p, mask, kPerLane, sink);
  else if (lpr == 16) hipLaunchKernelGGL(k_rows<16>, grid, block, 0, s, p, mask, kPerLane, sink);
  else if (lpr == 32) hipLaunchKernelGGL(k_rows<32>, grid, block, 0, s, p, mask, kPerLane, sink);
  else {
    *err = hipErrorInvalidValue;
    return 0;
  }
  *err = hipGetLastError();
  return (int64_t)kBlocks * (kBlock / 64) * kPerLane * (64 / lpr);
}

hipError_t probe_write(void *a, size_t bytes, hipStream_t s) {
  const int64_t n2 = (int64_t)(bytes / sizeof(d2));
  const int64_t waves = (int64_t)kProbeBlocks * (kBlock / 64) / 2;  // 8192 slabs
  const int64_t per_wave = (n2 + waves - 1) / waves;
  hipLaunchKernelGGL(k_write, dim3((unsigned)(waves * 64 / kBlock)), dim3(kBlock), 0, s, static_cast<d2 *>(a), n2,
                     per_wave, 0.0);
  return hipGetLastError();
}

int64_t probe_rows_write(const void *a, void *out, size_t bytes, int row_bytes, hipStream_t s, hipError_t *err) {
  const int lpr = row_bytes / (int)sizeof(d2);
  uint32_t mask = 1;
  while ((uint64_t)(mask + 1) * 2 * (uint64_t)row_bytes <= bytes && mask < 0x7fffffffu) mask = mask * 2 + 1;
  const int64_t rows = (int64_t)mask + 1;  // output rows, as many as input rows
  const int64_t ngroups = rows / (64 / lpr);
  const dim3 grid(2048), block(kBlock);
  const d2 *p = static_cast<const d2 *>(a);
  d2 *o = static_cast<d2 *>(out);
  if (lpr == 8) hipLaunchKernelGGL(k_rows_write<8>, grid, block, 0, s, p, mask, o, ngroups);
  else if (lpr == 16) hipLaunchKernelGGL(k_rows_write<16>, grid, block, 0, s, p, mask, o, ngroups);
  else if (lpr == 32) hipLaunchKernelGGL(k_rows_write<32>, grid, block, 0, s, p, mask, o, ngroups);
  else {
    *err = hipErrorInvalidValue;
    return 0;
  }
  *err = hipGetLastError();
  return rows * 5;  // four rows read and one written per output row
}

hipError_t probe_copy(const void *a, void *b, size_t bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(kProbeBlocks), dim3(kBlock), 0, s, static_cast<const d2 *>(a),
                     static_cast<d2 *>(b), (int64_t)(bytes / sizeof(d2)));
  return hipGetLastError();
}

}  // namespace sell
