// Dispatch of the kernel launchers by dtype combination and chunk height.
#include "spmv_impl.h"

namespace sell {

#define SELL_DECL(lc)                                                                 \
  hipError_t launch_spmv_##lc(int C, int U, int V, bool sz, const SpmvArgs &a, hipStream_t s);      \
  hipError_t launch_spmv_xw_##lc(int C, int V, int U, const SpmvArgs &a, const XwArgs &w, size_t lds, hipStream_t s); \
  hipError_t launch_batch_##lc(int C, int U, const BatchArgs &a, hipStream_t s); \
  int batch_waves_per_cu_##lc(int C, int U);
SELL_DECL(f64_f64)
SELL_DECL(f32_f32)
SELL_DECL(f32_f64)
SELL_DECL(bf16_f32)
SELL_DECL(bf16_f64)
#undef SELL_DECL

hipError_t launch_spmv(int combo, int C, int U, int V, bool sz, const SpmvArgs &a, hipStream_t s) {
  switch (combo) {
    case COMBO_F64_F64: return launch_spmv_f64_f64(C, U, V, sz, a, s);
    case COMBO_F32_F32: return launch_spmv_f32_f32(C, U, V, sz, a, s);
    case COMBO_F32_F64: return launch_spmv_f32_f64(C, U, V, sz, a, s);
    case COMBO_BF16_F32: return launch_spmv_bf16_f32(C, U, V, sz, a, s);
    case COMBO_BF16_F64: return launch_spmv_bf16_f64(C, U, V, sz, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_spmv_xw(int combo, int C, int V, int U, const SpmvArgs &a, const XwArgs &w, size_t lds,
                          hipStream_t s) {
  switch (combo) {
    case COMBO_F64_F64: return launch_spmv_xw_f64_f64(C, V, U, a, w, lds, s);
    case COMBO_F32_F32: return launch_spmv_xw_f32_f32(C, V, U, a, w, lds, s);
    case COMBO_F32_F64: return launch_spmv_xw_f32_f64(C, V, U, a, w, lds, s);
    case COMBO_BF16_F32: return launch_spmv_xw_bf16_f32(C, V, U, a, w, lds, s);
    case COMBO_BF16_F64: return launch_spmv_xw_bf16_f64(C, V, U, a, w, lds, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch(int combo, int C, int U, const BatchArgs &a, hipStream_t s) {
  switch (combo) {
    case COMBO_F64_F64: return launch_batch_f64_f64(C, U, a, s);
    case COMBO_F32_F32: return launch_batch_f32_f32(C, U, a, s);
    case COMBO_F32_F64: return launch_batch_f32_f64(C, U, a, s);
    case COMBO_BF16_F32: return launch_batch_bf16_f32(C, U, a, s);
    case COMBO_BF16_F64: return launch_batch_bf16_f64(C, U, a, s);
  }
  return hipErrorInvalidValue;
}

int batch_waves_per_cu(int combo, int C, int U) {
  switch (combo) {
    case COMBO_F64_F64: return batch_waves_per_cu_f64_f64(C, U);
    case COMBO_F32_F32: return batch_waves_per_cu_f32_f32(C, U);
    case COMBO_F32_F64: return batch_waves_per_cu_f32_f64(C, U);
    case COMBO_BF16_F32: return batch_waves_per_cu_bf16_f32(C, U);
    case COMBO_BF16_F64: return batch_waves_per_cu_bf16_f64(C, U);
  }
  return 4;
}

// Block form (FP64 only): C in {8, ..., 128}, KV in {1, 2, 4, 8}.
hipError_t launch_spmmv(int C, int KV, const SpmvArgs &a, hipStream_t s) {
  if (a.nwork <= 0 || a.k <= 0) return hipSuccess;
  const int G = 64 / (C < 64 ? C : 64);
  const int KT = G * KV;
  const unsigned nb = (unsigned)((a.nwork + kWavesPerBlock - 1) / kWavesPerBlock);
  const unsigned nt = (unsigned)((a.k + KT - 1) / KT);
#define SELL_L(CC, KK)                                                                                       \
  if (C == CC && KV == KK) {                                                                                \
    hipLaunchKernelGGL((dev::k_spmmv<CC, KK>), dim3(nb, nt), dim3(64 * kWavesPerBlock), 0, s, a);     \
    hipError_t e_ = hipGetLastError();                                                                      \
    if (e_ != hipSuccess || a.nsplit == 0) return e_;                                                       \
    hipLaunchKernelGGL((dev::k_combine_mm<CC>), dim3((unsigned)a.nsplit, nt), dim3(64 * KK), 0, s, a);     \
    return hipGetLastError();                                                                               \
  }
  SELL_L(8, 1) SELL_L(8, 2) SELL_L(8, 4) SELL_L(8, 8)
  SELL_L(16, 1) SELL_L(16, 2) SELL_L(16, 4) SELL_L(16, 8)
  SELL_L(32, 1) SELL_L(32, 2) SELL_L(32, 4) SELL_L(32, 8)
  SELL_L(64, 1) SELL_L(64, 2) SELL_L(64, 4) SELL_L(64, 8)
  SELL_L(128, 1) SELL_L(128, 2) SELL_L(128, 4) SELL_L(128, 8)
#undef SELL_L
  return hipErrorInvalidValue;
}

hipError_t launch_spmmv_rows(int C, int LPR, const SpmvArgs &a, hipStream_t s) {
  if (a.nwork <= 0 || a.k <= 0) return hipSuccess;
  const int rpw = C < 64 ? C : 64;
  const int64_t waves = a.nwork * (rpw / 16);  // 16 rows per wave
  const unsigned nb = (unsigned)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
  // threads per block of a combined slice, and blocks per slice: one
  // thread per (row, right-hand side)
  const unsigned ncomb = (unsigned)std::min(512, rpw * a.k);
  const unsigned nzc = (unsigned)((rpw * a.k + (int)ncomb - 1) / (int)ncomb);
  const int KV = a.k / LPR;
#define SELL_L(CC, LL, KK)                                                                                   \
  if (C == CC && LPR == LL && KV == KK) {                                                                   \
    hipLaunchKernelGGL((dev::k_spmmv_rows<CC, LL, KK>), dim3(nb), dim3(64 * kWavesPerBlock), 0, s, a); \
    hipError_t e_ = hipGetLastError();                                                                      \
    if (e_ != hipSuccess || a.nsplit == 0) return e_;                                                       \
    hipLaunchKernelGGL((dev::k_combine_mm<CC>), dim3((unsigned)a.nsplit, 1, nzc), dim3(ncomb), 0, s, a);  \
    return hipGetLastError();                                                                               \
  }
#define SELL_LC(LL, KK) SELL_L(16, LL, KK) SELL_L(32, LL, KK) SELL_L(64, LL, KK) SELL_L(128, LL, KK)
  SELL_LC(4, 4) SELL_LC(8, 4) SELL_LC(8, 8)
#undef SELL_LC
#undef SELL_L
  return hipErrorInvalidValue;
}

}  // namespace sell
