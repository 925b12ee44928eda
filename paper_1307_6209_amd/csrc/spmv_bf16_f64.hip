// Instantiation of the spMVM kernels for one dtype combination (values, x,
// accumulation) = COMBO_BF16_F64.
#include "spmv_impl.h"

namespace sell {
hipError_t launch_spmv_bf16_f64(int C, int U, int V, bool skip_zero, const SpmvArgs &a, hipStream_t s) {
  return dev::launch_spmv_t<COMBO_BF16_F64>(C, U, V, skip_zero, a, s);
}
hipError_t launch_spmv_xw_bf16_f64(int C, int V, int U, const SpmvArgs &a, const XwArgs &w, size_t lds,
                               hipStream_t s) {
  return dev::launch_spmv_xw_t<COMBO_BF16_F64>(C, V, U, a, w, lds, s);
}
hipError_t launch_batch_bf16_f64(int C, int U, const BatchArgs &a, hipStream_t s) {
  return dev::launch_batch_t<COMBO_BF16_F64>(C, U, a, s);
}
int batch_waves_per_cu_bf16_f64(int C, int U) { return dev::batch_waves_per_cu_t<COMBO_BF16_F64>(C, U); }
}  // namespace sell
