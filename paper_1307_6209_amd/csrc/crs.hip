// CRS spMVM kernels (Sect. 3.1, Listing "CRS spMVM kernel", y zeroed first)
// on the same device, for the comparison the paper draws between CRS and
// SELL-C-sigma (Sects. 3.2 and 5.1). L lanes of a wavefront share one row:
// L = 1 is the scalar row-per-thread kernel (rows side by side, uncoalesced
// matrix loads), L > 1 walks a row with L lanes (coalesced for long rows) and
// adds the L partial sums with cross-lane shuffles -- the reduction overhead
// the paper names as the weakness of CRS on wide SIMD units.
#include "sell_internal.h"

namespace sell {
namespace {

constexpr int kBlock = 256;

template <int L>
__global__ void __launch_bounds__(kBlock) k_crs(const int64_t *__restrict__ rpt, const int32_t *__restrict__ col,
                                                const double *__restrict__ val, const double *__restrict__ x,
                                                double *__restrict__ y, int64_t n) {
  const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / L;
  const int lane = threadIdx.x % L;
  if (row >= n) return;  // all L lanes of a row leave together
  const int64_t a = rpt[row], b = rpt[row + 1];
  double s = 0.0;
  for (int64_t j = a + lane; j < b; j += L) s = __builtin_fma(__builtin_nontemporal_load(val + j),
                                                           x[__builtin_nontemporal_load(col + j)], s);
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, L);
  if (lane == 0) y[row] = s;
}

}  // namespace

hipError_t launch_crs(const int64_t *rpt, const int32_t *col, const double *val, const double *x, double *y,
                      int64_t n, int L, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t threads = n * L;
  const unsigned nb = (unsigned)((threads + kBlock - 1) / kBlock);
  switch (L) {
#define SELL_L(LL) \
  case LL: hipLaunchKernelGGL(k_crs<LL>, dim3(nb), dim3(kBlock), 0, s, rpt, col, val, x, y, n); break;
    SELL_L(1) SELL_L(2) SELL_L(4) SELL_L(8) SELL_L(16) SELL_L(32) SELL_L(64)
#undef SELL_L
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sell
