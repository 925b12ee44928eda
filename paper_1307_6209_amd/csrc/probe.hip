// Bandwidth microbenchmarks that set the roofline bandwidth b of the
// performance model (Sect. 2.1 of Kreutzer et al., arXiv:1307.6209): a
// read-only sum over an array (the paper's "reduction" benchmark) and an
// array copy. Both stream 16-byte vectors with a grid-stride loop.
#include "sell_internal.h"

namespace sell {
namespace {

constexpr int kBlock = 256;
typedef double d2 __attribute__((ext_vector_type(2)));  // one 16-byte access

__global__ void __launch_bounds__(kBlock) k_read(const d2 *__restrict__ a, int64_t n4, double *sink) {
  double s0 = 0.0, s1 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  for (; i + 3 * stride < n4; i += 4 * stride) {
    d2 v0 = __builtin_nontemporal_load(a + i);
    d2 v1 = __builtin_nontemporal_load(a + i + stride);
    d2 v2 = __builtin_nontemporal_load(a + i + 2 * stride);
    d2 v3 = __builtin_nontemporal_load(a + i + 3 * stride);
    s0 += v0.x + v1.x + v2.x + v3.x;
    s1 += v0.y + v1.y + v2.y + v3.y;
  }
  for (; i < n4; i += stride) {
    d2 v = __builtin_nontemporal_load(a + i);
    s0 += v.x;
    s1 += v.y;
  }
  // keep the sum observable without a global reduction: one store per
  // block, from the lane that happens to see a NaN sum (never for zeroed
  // input) or from thread 0
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
  hipLaunchKernelGGL(k_read, dim3(kProbeBlocks), dim3(kBlock), 0, s, static_cast<const d2 *>(a),
                     (int64_t)(bytes / sizeof(d2)), sink);
  return hipGetLastError();
}

hipError_t probe_copy(const void *a, void *b, size_t bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(kProbeBlocks), dim3(kBlock), 0, s, static_cast<const d2 *>(a),
                     static_cast<d2 *>(b), (int64_t)(bytes / sizeof(d2)));
  return hipGetLastError();
}

}  // namespace sell
