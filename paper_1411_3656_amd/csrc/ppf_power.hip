// Detection after the filter bank: the power |X[m][k]|^2 of every bin summed
// over K consecutive spectra, in the epilogue of the fused FP32 kernel (or
// of the FFT pass of the two-pass form), so the spectra never reach HBM.
// Each thread owns the same bins of every spectrum it transforms, so the
// sum stays in registers; tiles start at multiples of K.

#include "ppf_engine.h"

namespace ppf {

typedef hipError_t (*PowerFn)(const PlanDev&, const BatchArgs&, const float*, int, hipStream_t, float*, int);

template <int N>
static PowerFn power_for_taps(int TP) {
  switch (TP) {
    case 1: return &fused_launch<N, 1, false, true>;
    case 2: if constexpr (fused_ok(N, 2)) return &fused_launch<N, 2, false, true>; else return nullptr;
    case 4: if constexpr (fused_ok(N, 4)) return &fused_launch<N, 4, false, true>; else return nullptr;
    case 8: if constexpr (fused_ok(N, 8)) return &fused_launch<N, 8, false, true>; else return nullptr;
    case 16: if constexpr (fused_ok(N, 16)) return &fused_launch<N, 16, false, true>; else return nullptr;
    default: return nullptr;
  }
}

static PowerFn power_fn(int N, int TP) {
  switch (N) {
    case 16: return power_for_taps<16>(TP);
    case 32: return power_for_taps<32>(TP);
    case 64: return power_for_taps<64>(TP);
    case 128: return power_for_taps<128>(TP);
    case 256: return power_for_taps<256>(TP);
    case 512: return power_for_taps<512>(TP);
    case 1024: return power_for_taps<1024>(TP);
    case 2048: return power_for_taps<2048>(TP);
    case 4096: return power_for_taps<4096>(TP);
    case 8192: return power_for_taps<8192>(TP);
    case 16384: return power_for_taps<16384>(TP);
    default: return nullptr;
  }
}

static PowerFn fft_power_fn(int N) {
  switch (N) {
    case 16: return &fused_launch<16, 1, true, true>;
    case 32: return &fused_launch<32, 1, true, true>;
    case 64: return &fused_launch<64, 1, true, true>;
    case 128: return &fused_launch<128, 1, true, true>;
    case 256: return &fused_launch<256, 1, true, true>;
    case 512: return &fused_launch<512, 1, true, true>;
    case 1024: return &fused_launch<1024, 1, true, true>;
    case 2048: return &fused_launch<2048, 1, true, true>;
    case 4096: return &fused_launch<4096, 1, true, true>;
    case 8192: return &fused_launch<8192, 1, true, true>;
    case 16384: return &fused_launch<16384, 1, true, true>;
    default: return nullptr;
  }
}

hipError_t launch_fused_power(const PlanDev& pd, const BatchArgs& a, float* pout, int K, hipStream_t st) {
  PowerFn f = power_fn(pd.N, pd.TP);
  if (!f) return hipErrorInvalidValue;
  return f(pd, a, pd.coef, pd.T, st, pout, K);
}

hipError_t launch_fft_power(const PlanDev& pd, const void* in, float* pout, long long M, int K, hipStream_t st) {
  PowerFn f = fft_power_fn(pd.N);
  if (!f) return hipErrorInvalidValue;
  BatchArgs a{in, in, 0, nullptr, M};
  return f(pd, a, pd.ones, 1, st, pout, K);
}

}  // namespace ppf
