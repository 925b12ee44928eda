// Instantiation of the spMVM kernels for one dtype combination (values, x,
// accumulation). The build compiles this file once per combination, with
// SELL_COMBO set to the combination's DtypeCombo enumerator and SELL_LC to
// the suffix of its launcher names (f64_f64, f32_f32, f32_f64, bf16_f32,
// bf16_f64), so that the five sets of kernels compile in parallel.
#include "spmv_impl.h"

#if !defined(SELL_COMBO) || !defined(SELL_LC)
#error "compile with -DSELL_COMBO=<DtypeCombo enumerator> -DSELL_LC=<launcher suffix>"
#endif

#define SELL_NAME2(base, lc) base##lc
#define SELL_NAME(base, lc) SELL_NAME2(base, lc)

namespace sell {
hipError_t SELL_NAME(launch_spmv_, SELL_LC)(int C, int U, int V, bool skip_zero, const SpmvArgs &a,
                                            hipStream_t s) {
  return dev::launch_spmv_t<SELL_COMBO>(C, U, V, skip_zero, a, s);
}
hipError_t SELL_NAME(launch_spmv_xw_, SELL_LC)(int C, int V, int U, const SpmvArgs &a, const XwArgs &w,
                                               size_t lds, hipStream_t s) {
  return dev::launch_spmv_xw_t<SELL_COMBO>(C, V, U, a, w, lds, s);
}
hipError_t SELL_NAME(launch_batch_, SELL_LC)(int C, int U, const BatchArgs &a, hipStream_t s) {
  return dev::launch_batch_t<SELL_COMBO>(C, U, a, s);
}
int SELL_NAME(batch_waves_per_cu_, SELL_LC)(int C, int U) { return dev::batch_waves_per_cu_t<SELL_COMBO>(C, U); }
}  // namespace sell
