// Fused FIR + FFT kernels over complex FP16 or int8 input (the reduced-
// precision input of the precision form): the same engine as the FP32
// kernels, with each sample widened exactly to FP32 as it is loaded, so
// HBM carries 4 or 2 bytes per input sample instead of 8 and the FIR and
// FFT run in FP32 as before.

#include "ppf_engine.h"

namespace ppf {

template <int N, int IT>
static FusedFn widened_for_taps(int TP) {
  switch (TP) {
    case 1: return &fused_launch<N, 1, false, false, IT>;
    case 2: if constexpr (fused_ok(N, 2)) return &fused_launch<N, 2, false, false, IT>; else return nullptr;
    case 4: if constexpr (fused_ok(N, 4)) return &fused_launch<N, 4, false, false, IT>; else return nullptr;
    case 8: if constexpr (fused_ok(N, 8)) return &fused_launch<N, 8, false, false, IT>; else return nullptr;
    case 16: if constexpr (fused_ok(N, 16)) return &fused_launch<N, 16, false, false, IT>; else return nullptr;
    default: return nullptr;
  }
}

template <int IT>
static FusedFn widened_fn(int N, int TP) {
  switch (N) {
    case 16: return widened_for_taps<16, IT>(TP);
    case 32: return widened_for_taps<32, IT>(TP);
    case 64: return widened_for_taps<64, IT>(TP);
    case 128: return widened_for_taps<128, IT>(TP);
    case 256: return widened_for_taps<256, IT>(TP);
    case 512: return widened_for_taps<512, IT>(TP);
    case 1024: return widened_for_taps<1024, IT>(TP);
    case 2048: return widened_for_taps<2048, IT>(TP);
    case 4096: return widened_for_taps<4096, IT>(TP);
    case 8192: return widened_for_taps<8192, IT>(TP);
    case 16384: return widened_for_taps<16384, IT>(TP);
    default: return nullptr;
  }
}

FusedFn fused_fn_widened(int N, int TP, int IT) {
  return IT == 1 ? widened_fn<1>(N, TP) : (IT == 2 ? widened_fn<2>(N, TP) : nullptr);
}

}  // namespace ppf
