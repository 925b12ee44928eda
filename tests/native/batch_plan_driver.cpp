// Host driver of the batch XCD placement (batch_plan.h) for the CPU tests:
// reads  nunits nmats waves_per_block xcds persistent_waves  and then one
// "mat cost split" line per unit on stdin; prints the plan as
//   order <n> <slot unit indices...>
//   slice <n> <offsets...>
//   load <n> <per-XCD costs...>
#include <cstdio>
#include <vector>

#include "batch_plan.h"

int main() {
  long long n, nmats, W, X, pw;
  if (std::scanf("%lld %lld %lld %lld %lld", &n, &nmats, &W, &X, &pw) != 5) return 2;
  std::vector<int32_t> mat((size_t)n);
  std::vector<int64_t> cost((size_t)n);
  std::vector<uint8_t> split((size_t)n);
  for (long long q = 0; q < n; ++q) {
    long long m, c, s;
    if (std::scanf("%lld %lld %lld", &m, &c, &s) != 3) return 2;
    mat[(size_t)q] = (int32_t)m;
    cost[(size_t)q] = c;
    split[(size_t)q] = (uint8_t)s;
  }
  const sell::XcdPlan p = sell::plan_xcd(mat, cost, split, (int32_t)nmats, (int)W, (int)X, pw);
  std::printf("order %zu", p.order.size());
  for (long long v : p.order) std::printf(" %lld", v);
  std::printf("\nslice %zu", p.slice.size());
  for (int v : p.slice) std::printf(" %d", v);
  std::printf("\nload %zu", p.load.size());
  for (long long v : p.load) std::printf(" %lld", v);
  std::printf("\n");
  return 0;
}
