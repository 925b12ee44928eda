// Bandwidth microbenchmarks that set the roofline bandwidth b of the
// performance model (Sect. 2.1 of Kreutzer et al., arXiv:1307.6209): a
// read-only sum over an array (the paper's "reduction" benchmark) and an
// array copy, both with 16-byte non-temporal accesses.
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

__global__ void __launch_bounds__(kBlock) k_copy(const d2 *__restrict__ a, d2 *__restrict__ b, int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
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

hipError_t probe_copy(const void *a, void *b, size_t bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(kProbeBlocks), dim3(kBlock), 0, s, static_cast<const d2 *>(a),
                     static_cast<d2 *>(b), (int64_t)(bytes / sizeof(d2)));
  return hipGetLastError();
}

}  // namespace sell
