// C-ABI layer of libppf.so: argument validation, plan objects, streams.
//
// Every entry point validates its arguments before the first HIP call,
// catches every C++ exception, and records failures in a thread-local
// status and message (ppf_last_error / ppf_last_error_message).

#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/ppf.h"
#include "ppf_internal.h"

namespace {

thread_local int g_status = PPF_OK;
thread_local char g_message[512] = "";

int fail(int status, const char* fmt, ...) {
  g_status = status;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_message, sizeof g_message, fmt, ap);
  va_end(ap);
  return status;
}

int fail_hip(hipError_t e, const char* what) {
  const int st = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? PPF_ERR_NOMEM : PPF_ERR_HIP;
  return fail(st, "%s: %s", what, hipGetErrorString(e));
}

bool is_pow2(long long v) { return v > 0 && (v & (v - 1)) == 0; }

int sample_bytes(int dtype) {
  switch (dtype) {
    case PPF_C32: return 8;
    case PPF_C16: return 4;
    case PPF_CI8: return 2;
    default: return 0;
  }
}

bool overlaps(uintptr_t a, size_t na, uintptr_t b, size_t nb) { return a < b + nb && b < a + na; }

// IEEE binary16 -> binary32 (exact)
float half_to_float(uint16_t h) {
  const uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
  uint32_t exp = (h >> 10) & 0x1Fu;
  uint32_t man = h & 0x3FFu;
  uint32_t bits;
  if (exp == 0) {
    if (man == 0) {
      bits = sign;
    } else {                       // subnormal: normalise
      int e = -1;
      do { man <<= 1; ++e; } while (!(man & 0x400u));
      bits = sign | ((uint32_t)(127 - 15 - e) << 23) | ((man & 0x3FFu) << 13);
    }
  } else if (exp == 31) {
    bits = sign | 0x7F800000u | (man << 13);
  } else {
    bits = sign | ((exp - 15 + 127) << 23) | (man << 13);
  }
  float f;
  std::memcpy(&f, &bits, 4);
  return f;
}

// The fused kernels read complex FP32 input; other input types take the
// two-pass path, whose FIR pass widens them as it loads.
bool fused_ok_for(int N, int TP, int in_type) {
  (void)in_type;   // FP16 and int8 input are widened in the fused kernels' loads
  return ppf::fused_available(N, TP) || TP == 1;
}

// Largest FIR workspace of the two-pass path, in bytes: chunks of 128 MiB
// (enough spectra per launch to fill the GPU at N <= 4096; larger chunks
// gained nothing there), and 512 MiB for N >= 8192, where longer chunks
// (fewer launches, longer tiles and so fewer tap-window re-reads) measured
// faster:
// N=16384 at 2^28 samples, T = 4, 8, 16: 1.85, 1.92, 2.07 ms with 128 MiB,
// 1.72, 1.76, 1.84 with 512 MiB (32 and 64 MiB were slower still). Build-time
// overrides for tuning.
#ifndef PPF_WORKSPACE_MIB
#define PPF_WORKSPACE_MIB 128
#endif
#ifndef PPF_WORKSPACE_LARGE_N_MIB
#define PPF_WORKSPACE_LARGE_N_MIB 512
#endif
constexpr size_t workspace_bytes(int N) {
  return (size_t)(N >= 8192 ? PPF_WORKSPACE_LARGE_N_MIB : PPF_WORKSPACE_MIB) << 20;
}

// Single mode: staging pairs in the copy-in / transform / copy-out pipeline
// and the default input bytes per chunk (build-time tuning).
#ifndef PPF_HOST_STAGES
#define PPF_HOST_STAGES 3
#endif
#ifndef PPF_HOST_CHUNK_MIB
#define PPF_HOST_CHUNK_MIB 192
#endif
constexpr int kHostStages = PPF_HOST_STAGES;

// Detection: a fused launch integrates whole groups of K spectra of at most
// 2^28 spectra; the two-pass form passes whole groups through its
// workspace (2^24 samples).
constexpr int kMaxPowerK = 1 << 28;
constexpr long long kMaxPowerKN = 1ll << 24;

// Every plan has a process-unique id; a host thread's stream binding for a
// plan is kept under that id (ppf_set_stream), so a plan object is never
// written by ppf_set_stream and threads may share it.
std::atomic<unsigned long long> g_next_plan_id{1};
struct StreamBinding {
  unsigned long long plan_id;
  hipStream_t stream;
};
thread_local std::vector<StreamBinding> t_bindings;

}  // namespace

struct ppf_plan_s {
  int N = 0, T = 0, TP = 0;
  int in_type = PPF_C32, coeff_type = PPF_R32, coeff_shift = 0, fft_mode = PPF_FFT_F32;
  int path = PPF_PATH_FUSED;
  float* d_coef = nullptr;
  float* d_ones = nullptr;
  void* d_tw = nullptr;
  void* d_coef16 = nullptr;    // matrix-core mode: FP16 coefficients in lane order
  void* d_w256 = nullptr;      // matrix-core mode: FP16 values exp(-2 pi i k/256)
  void* d_tw1 = nullptr;       // four-step two-pass form: N1- and N2-point FP32 twiddles
  void* d_tw2 = nullptr;
  int mfma_e1 = 0;             // matrix-core mode: samples are scaled by 2^-e1
  unsigned long long id = 0;
  // Two-pass workspaces, one per HIP stream the plan has run on, so calls
  // on different streams never share one; guarded by mu.
  struct Workspace {
    hipStream_t stream;
    void* ptr;
    size_t bytes;
    long long spectra;
  };
  std::mutex mu;
  std::vector<Workspace> ws;
  std::vector<hipStream_t> used_streams;   // streams to wait for in ppf_destroy
  // single mode (host-resident data): staging buffers, copy streams, events
  void* h_in[kHostStages] = {};
  void* h_out[kHostStages] = {};
  size_t h_in_cap = 0, h_out_cap = 0;
  hipStream_t h2d = nullptr, d2h = nullptr;
  hipEvent_t ev_in[kHostStages] = {}, ev_comp[kHostStages] = {}, ev_out[kHostStages] = {};
  hipEvent_t ev_start = nullptr;

  // the calling thread's stream for this plan (ppf_set_stream), also
  // remembered for ppf_destroy
  hipStream_t stream() {
    for (const StreamBinding& b : t_bindings)
      if (b.plan_id == id) return b.stream;
    return nullptr;
  }
  void note_stream(hipStream_t st) {
    std::lock_guard<std::mutex> lk(mu);
    for (hipStream_t u : used_streams)
      if (u == st) return;
    used_streams.push_back(st);
  }

  ppf::PlanDev dev() const {
    ppf::PlanDev p;
    p.N = N;
    p.T = T;
    p.TP = TP;
    p.coef = d_coef;
    p.ones = d_ones;
    p.tw = d_tw;
    p.in_type = in_type == PPF_C32 ? 0 : (in_type == PPF_C16 ? 1 : 2);
    return p;
  }
  ppf::MfmaDev mfma() const {
    ppf::MfmaDev m;
    m.N = N;
    m.tq = ppf::mfma_tap_slots(N, T);
    m.coef16 = d_coef16;
    m.tw = d_tw;
    m.w256 = d_w256;
    m.d = m.tq - T;
    m.in_type = in_type == PPF_C16 ? 1 : 2;
    m.in_scale = std::ldexp(1.0f, -mfma_e1);
    m.out_scale = std::ldexp(1.0f, mfma_e1 - coeff_shift);
    return m;
  }
  ~ppf_plan_s() {
    if (d_coef) (void)hipFree(d_coef);
    if (d_ones) (void)hipFree(d_ones);
    if (d_tw) (void)hipFree(d_tw);
    for (const Workspace& w : ws) (void)hipFree(w.ptr);
    for (int i = 0; i < kHostStages; ++i) {
      if (h_in[i]) (void)hipFree(h_in[i]);
      if (h_out[i]) (void)hipFree(h_out[i]);
      if (ev_in[i]) (void)hipEventDestroy(ev_in[i]);
      if (ev_comp[i]) (void)hipEventDestroy(ev_comp[i]);
      if (ev_out[i]) (void)hipEventDestroy(ev_out[i]);
    }
    if (ev_start) (void)hipEventDestroy(ev_start);
    if (h2d) (void)hipStreamDestroy(h2d);
    if (d2h) (void)hipStreamDestroy(d2h);
    if (d_coef16) (void)hipFree(d_coef16);
    if (d_w256) (void)hipFree(d_w256);
    if (d_tw1) (void)hipFree(d_tw1);
    if (d_tw2) (void)hipFree(d_tw2);
  }
};

ppf_stream_s::~ppf_stream_s() {
  if (hist[0]) (void)hipFree(hist[0]);
  if (hist[1]) (void)hipFree(hist[1]);
}

namespace {

// The two-pass workspace of HIP stream `st` (at least min_spectra spectra),
// allocated on the stream's first two-pass call. Work on one stream runs in
// order, so calls on that stream may reuse it; other streams have their own.
int ensure_workspace(ppf_plan_t p, hipStream_t st, long long min_spectra, void** ptr, long long* spectra) {
  std::lock_guard<std::mutex> lk(p->mu);
  ppf_plan_s::Workspace* w = nullptr;
  for (ppf_plan_s::Workspace& x : p->ws)
    if (x.stream == st) w = &x;
  if (w && w->spectra >= min_spectra) {
    *ptr = w->ptr;
    *spectra = w->spectra;
    return PPF_OK;
  }
  if (w) {   // grow: earlier work on this stream may still read it
    const hipError_t es = hipStreamSynchronize(st);
    if (es != hipSuccess) return fail_hip(es, "workspace synchronize");
    (void)hipFree(w->ptr);
    w->ptr = nullptr;
  }
  long long k = (long long)(workspace_bytes(p->N) / (8ull * p->N));
  if (k < min_spectra) k = min_spectra;
  if (k < 1) k = 1;
  void* d = nullptr;
  const size_t bytes = (size_t)k * p->N * 8;
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) {
    if (w) {
      *w = p->ws.back();
      p->ws.pop_back();
    }
    return fail_hip(e, "workspace allocation");
  }
  if (!w) {
    p->ws.push_back(ppf_plan_s::Workspace{st, nullptr, 0, 0});
    w = &p->ws.back();
  }
  w->ptr = d;
  w->bytes = bytes;
  w->spectra = k;
  *ptr = d;
  *spectra = k;
  return PPF_OK;
}

// FIR + FFT over M spectra of the concatenation x0 (h0 blocks) ++ x1.
// ext_ws: a caller-provided workspace of ext_spectra spectra for the
// two-pass path (nothing is allocated then), or NULL for the stream's own.
int run_batch(ppf_plan_t p, hipStream_t stream, const void* x0, long long h0, const void* x1, void* out,
              long long M, void* ext_ws = nullptr, long long ext_spectra = 0) {
  const ppf::PlanDev pd = p->dev();
  const size_t sb = (size_t)sample_bytes(p->in_type);
  if (p->fft_mode == PPF_FFT_MFMA_F16) {
    ppf::BatchArgs a{x0, x1, h0, out, M};
    hipError_t e = ppf::launch_mfma(p->mfma(), a, stream);
    if (e != hipSuccess) return fail_hip(e, "matrix-core kernel launch");
    return PPF_OK;
  }
  if (p->path == PPF_PATH_FUSED) {
    ppf::BatchArgs a{x0, x1, h0, out, M};
    hipError_t e = ppf::launch_fused(pd, a, stream);
    if (e != hipSuccess) return fail_hip(e, "fused kernel launch");
    return PPF_OK;
  }
  void* ws = nullptr;
  long long chunk = 0;
  if (ext_ws) {
    ws = ext_ws;
    chunk = ext_spectra;
  } else {
    int st = ensure_workspace(p, stream, 1, &ws, &chunk);
    if (st != PPF_OK) return st;
  }
  for (long long c0 = 0; c0 < M; c0 += chunk) {
    const long long k = (M - c0 < chunk) ? (M - c0) : chunk;
    // blocks c0 .. of the concatenation: split between x0 and x1
    ppf::BatchArgs a;
    if (c0 < h0) {
      a.x0 = (const char*)x0 + (size_t)c0 * pd.N * sb;
      a.h0 = h0 - c0;
      a.x1 = x1;
    } else {
      a.x0 = x1;
      a.h0 = 0;
      a.x1 = (const char*)x1 + (size_t)(c0 - h0) * pd.N * sb;
    }
    a.out = ws;
    a.M = k;
    if (p->d_tw1 && p->in_type == PPF_C32) {
      // four-step form (N = N1 * N2): FIR + N1-point transforms, then N2-point
      hipError_t e = ppf::launch_fourstep_a(pd, a, p->d_tw1, stream);
      if (e != hipSuccess) return fail_hip(e, "four-step pass A launch");
      e = ppf::launch_fourstep_b(pd, ws, (char*)out + (size_t)c0 * pd.N * 8, k, p->d_tw2, stream);
      if (e != hipSuccess) return fail_hip(e, "four-step pass B launch");
      continue;
    }
    hipError_t e = ppf::launch_fir(pd, a, stream);
    if (e != hipSuccess) return fail_hip(e, "FIR kernel launch");
    e = ppf::launch_fft(pd, ws, (char*)out + (size_t)c0 * pd.N * 8, k, stream);
    if (e != hipSuccess) return fail_hip(e, "FFT kernel launch");
  }
  return PPF_OK;
}

// Detection: |X|^2 summed over K spectra, M a multiple of K.
int run_power(ppf_plan_t p, hipStream_t stream, const void* in, float* pout, long long M, int K) {
  const ppf::PlanDev pd = p->dev();
  const size_t sb = (size_t)sample_bytes(p->in_type);
  if (p->fft_mode == PPF_FFT_MFMA_F16) {
    ppf::BatchArgs a{in, in, 0, nullptr, M};
    hipError_t e = ppf::launch_mfma_power(p->mfma(), a, pout, K, stream);
    if (e != hipSuccess) return fail_hip(e, "matrix-core power kernel launch");
    return PPF_OK;
  }
  if (p->path == PPF_PATH_FUSED && p->in_type == PPF_C32) {
    ppf::BatchArgs a{in, in, 0, nullptr, M};
    hipError_t e = ppf::launch_fused_power(pd, a, pout, K, stream);
    if (e != hipSuccess) return fail_hip(e, "fused power kernel launch");
    return PPF_OK;
  }
  // two-pass: chunks of whole groups of K spectra
  void* ws = nullptr;
  long long wsk = 0;
  int st = ensure_workspace(p, stream, K, &ws, &wsk);
  if (st != PPF_OK) return st;
  const long long chunk = wsk / K * K;
  for (long long c0 = 0; c0 < M; c0 += chunk) {
    const long long k = (M - c0 < chunk) ? (M - c0) : chunk;
    ppf::BatchArgs a{(const char*)in + (size_t)c0 * pd.N * sb, (const char*)in + (size_t)c0 * pd.N * sb, 0,
                     ws, k};
    hipError_t e = ppf::launch_fir(pd, a, stream);
    if (e != hipSuccess) return fail_hip(e, "FIR kernel launch");
    e = ppf::launch_fft_power(pd, ws, pout + (size_t)(c0 / K) * pd.N, k, K, stream);
    if (e != hipSuccess) return fail_hip(e, "FFT power kernel launch");
  }
  return PPF_OK;
}

// Single mode: staging buffers for chunks of `chunk` spectra (grown on demand).
int ensure_host_pipe(ppf_plan_t p, hipStream_t stream, long long chunk) {
  const size_t sb = (size_t)sample_bytes(p->in_type);
  const size_t in_need = (size_t)(chunk + p->T - 1) * p->N * sb;
  const size_t out_need = (size_t)chunk * p->N * 8;
  hipError_t e = hipSuccess;
  if (!p->h2d) {
    e = hipStreamCreateWithFlags(&p->h2d, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->d2h, hipStreamNonBlocking);
    for (int i = 0; i < kHostStages && e == hipSuccess; ++i) {
      e = hipEventCreateWithFlags(&p->ev_in[i], hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_comp[i], hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_out[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_start, hipEventDisableTiming);
    if (e != hipSuccess) return fail_hip(e, "single-mode streams");
  }
  if (p->h_in_cap < in_need || p->h_out_cap < out_need) {
    // earlier work on the staging buffers must be finished before they go
    for (hipStream_t st : {stream, p->h2d, p->d2h}) {
      e = hipStreamSynchronize(st);
      if (e != hipSuccess) return fail_hip(e, "single-mode synchronize");
    }
    for (int i = 0; i < kHostStages; ++i) {
      if (p->h_in[i]) (void)hipFree(p->h_in[i]);
      if (p->h_out[i]) (void)hipFree(p->h_out[i]);
      p->h_in[i] = p->h_out[i] = nullptr;
    }
    p->h_in_cap = p->h_out_cap = 0;
    for (int i = 0; i < kHostStages && e == hipSuccess; ++i) {
      e = hipMalloc(&p->h_in[i], in_need);
      if (e == hipSuccess) e = hipMalloc(&p->h_out[i], out_need);
    }
    if (e != hipSuccess) {
      for (int i = 0; i < kHostStages; ++i) {
        if (p->h_in[i]) (void)hipFree(p->h_in[i]);
        if (p->h_out[i]) (void)hipFree(p->h_out[i]);
        p->h_in[i] = p->h_out[i] = nullptr;
      }
      return fail_hip(e, "single-mode staging buffers");
    }
    p->h_in_cap = in_need;
    p->h_out_cap = out_need;
  }
  return PPF_OK;
}

ppf_plan_t make_plan(int N, int taps, const void* coeffs, int coeff_type, int coeff_shift, int in_type,
                     int fft_mode) {
  if (!coeffs) { fail(PPF_ERR_INVALID, "coeffs is NULL"); return nullptr; }
  if (N < 1 || taps < 1) { fail(PPF_ERR_INVALID, "N=%d and taps=%d must be >= 1", N, taps); return nullptr; }
  if (!is_pow2(N) || N < 16 || N > 16384) {
    fail(PPF_ERR_UNSUPPORTED, "N=%d: supported N is a power of two in [16, 16384]", N);
    return nullptr;
  }
  const int TP = ppf::taps_template(taps);
  if (TP == 0) { fail(PPF_ERR_UNSUPPORTED, "taps=%d: supported taps are 1..64", taps); return nullptr; }
  if (coeff_type != PPF_R32 && coeff_type != PPF_R16) {
    fail(PPF_ERR_INVALID, "coeff_type=%d is not a real coefficient type", coeff_type);
    return nullptr;
  }
  if (sample_bytes(in_type) == 0) { fail(PPF_ERR_INVALID, "in_type=%d is not a complex input type", in_type); return nullptr; }
  if (fft_mode != PPF_FFT_F32 && fft_mode != PPF_FFT_MFMA_F16) {
    fail(PPF_ERR_INVALID, "fft_mode=%d unknown", fft_mode);
    return nullptr;
  }
  if (coeff_type == PPF_R32 && coeff_shift != 0) {
    fail(PPF_ERR_INVALID, "coeff_shift must be 0 for float32 coefficients");
    return nullptr;
  }
  if (coeff_shift < 0 || coeff_shift > 30) { fail(PPF_ERR_INVALID, "coeff_shift=%d outside 0..30", coeff_shift); return nullptr; }
  if (fft_mode == PPF_FFT_MFMA_F16) {
    if (!ppf::mfma_available(N, taps) || (in_type != PPF_CI8 && in_type != PPF_C16) || coeff_type != PPF_R16) {
      fail(PPF_ERR_UNSUPPORTED,
           "fft_mode=MFMA_F16 takes N=256, 1024 or 4096, taps <= 16, complex int8 or FP16 input and FP16 coefficients "
           "(got N=%d taps=%d in_type=%d coeff_type=%d)", N, taps, in_type, coeff_type);
      return nullptr;
    }
  }
  if (!ppf::fft_available(N) || !ppf::fir_available(TP)) {
    fail(PPF_ERR_UNSUPPORTED, "no kernel for N=%d taps=%d", N, taps);
    return nullptr;
  }

  ppf_plan_s* p = new (std::nothrow) ppf_plan_s;
  if (!p) { fail(PPF_ERR_NOMEM, "host allocation"); return nullptr; }
  p->N = N;
  p->T = taps;
  p->TP = TP;
  p->in_type = in_type;
  p->coeff_type = coeff_type;
  p->coeff_shift = coeff_shift;
  p->fft_mode = fft_mode;
  p->path = (fft_mode == PPF_FFT_MFMA_F16 || fused_ok_for(N, TP, in_type)) ? PPF_PATH_FUSED : PPF_PATH_TWO_PASS;
  p->id = g_next_plan_id.fetch_add(1);

  // coefficients padded at the front with TP-T zero segments; FP16
  // coefficients are widened exactly and the 2^-shift is applied (exact)
  std::vector<float> hpad((size_t)TP * N, 0.0f);
  if (coeff_type == PPF_R32) {
    std::memcpy(hpad.data() + (size_t)(TP - taps) * N, coeffs, (size_t)taps * N * sizeof(float));
  } else {
    const uint16_t* h16 = (const uint16_t*)coeffs;
    const float scale = std::ldexp(1.0f, -coeff_shift);
    for (size_t i = 0; i < (size_t)taps * N; ++i) hpad[(size_t)(TP - taps) * N + i] = half_to_float(h16[i]) * scale;
  }
  std::vector<float> ones((size_t)N, 1.0f);

  hipError_t e;
  if ((e = hipMalloc(&p->d_coef, hpad.size() * sizeof(float))) != hipSuccess) { p->d_coef = nullptr; goto hip_fail; }
  if ((e = hipMalloc(&p->d_ones, ones.size() * sizeof(float))) != hipSuccess) { p->d_ones = nullptr; goto hip_fail; }
  if ((e = hipMalloc(&p->d_tw, (size_t)N * 8)) != hipSuccess) { p->d_tw = nullptr; goto hip_fail; }
  if ((e = hipMemcpy(p->d_coef, hpad.data(), hpad.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) goto hip_fail;
  if ((e = hipMemcpy(p->d_ones, ones.data(), ones.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) goto hip_fail;
  if ((e = ppf::launch_twiddles(p->d_tw, N, nullptr)) != hipSuccess) goto hip_fail;
  if (ppf::fourstep_available(N, TP)) {
    const int n1 = ppf::fourstep_n1(N), n2 = ppf::fourstep_n2(N);
    if ((e = hipMalloc(&p->d_tw1, (size_t)n1 * 8)) != hipSuccess) { p->d_tw1 = nullptr; goto hip_fail; }
    if ((e = hipMalloc(&p->d_tw2, (size_t)n2 * 8)) != hipSuccess) { p->d_tw2 = nullptr; goto hip_fail; }
    if ((e = ppf::launch_twiddles(p->d_tw1, n1, nullptr)) != hipSuccess) goto hip_fail;
    if ((e = ppf::launch_twiddles(p->d_tw2, n2, nullptr)) != hipSuccess) goto hip_fail;
  }
  if (fft_mode == PPF_FFT_MFMA_F16) {
    // FP16 coefficients in the kernel's lane order, and the sample scale:
    // the largest FP16 stage input is at most X * g * S * 2^-e1 with
    // S = max over channels of sum_t |h16[t][c]|, X the largest input
    // magnitude (128 for int8, 65504 for FP16: any finite FP16 input) and
    // g the growth before the last FP16 stage input: 256 at N = 4096 (two
    // radix-16 stages), 64 at N = 1024 (radix 4, then 16), 16 at N = 256;
    // e1 keeps it below 60000.
    const uint16_t* h16 = (const uint16_t*)coeffs;
    const int tq = ppf::mfma_tap_slots(N, taps);
    std::vector<uint16_t> lane(ppf::mfma_coef_bytes(N, tq) / 2);
    ppf::mfma_coef_layout(N, tq, h16, taps, lane.data());
    const double growth = N == 4096 ? 256.0 : (N == 1024 ? 64.0 : 16.0);
    double smax = 0.0;
    for (int c = 0; c < N; ++c) {
      double sc = 0.0;
      for (int t = 0; t < taps; ++t) sc += std::fabs((double)half_to_float(h16[(size_t)t * N + c]));
      smax = sc > smax ? sc : smax;
    }
    // Bounds on e1: for int8, >= -8 keeps 128 * 2^-e1 in FP16 range and
    // <= 24 keeps every sample times 2^-e1 exact (FP16 samples are not
    // scaled themselves: the FIR's FP32 sums are); the output scale 2^(e1-s)
    // is folded into the FP16 stage-3 DFT matrix, exact for e1 - s in
    // [-12, 15]. Among the admissible values the smallest (the most FP16
    // headroom used) is taken.
    const double xmax = in_type == PPF_CI8 ? 128.0 : 65504.0;
    const int e1_range = smax > 0.0 ? (int)std::ceil(std::log2(xmax * growth * smax / 60000.0)) : -8;
    int e1 = e1_range;
    if (e1 < -8) e1 = -8;
    if (e1 < coeff_shift - 12) e1 = coeff_shift - 12;
    int e1_hi = coeff_shift + 15;
    if (in_type == PPF_CI8 && e1_hi > 24) e1_hi = 24;
    if (e1 > e1_hi) {
      delete p;
      fail(PPF_ERR_UNSUPPORTED,
           "fft_mode=MFMA_F16: FP16 coefficients with sum_t |h16| up to %.6g need a sample scale beyond "
           "2^-%d; raise coeff_shift or scale the coefficients down", smax, e1_hi);
      return nullptr;
    }
    p->mfma_e1 = e1;
    if ((e = hipMalloc(&p->d_coef16, lane.size() * 2)) != hipSuccess) { p->d_coef16 = nullptr; goto hip_fail; }
    if ((e = hipMalloc(&p->d_w256, 256 * 4)) != hipSuccess) { p->d_w256 = nullptr; goto hip_fail; }
    if ((e = hipMemcpy(p->d_coef16, lane.data(), lane.size() * 2, hipMemcpyHostToDevice)) != hipSuccess) goto hip_fail;
    if ((e = ppf::launch_w256(p->d_w256, nullptr)) != hipSuccess) goto hip_fail;
  }
  if ((e = hipStreamSynchronize(nullptr)) != hipSuccess) goto hip_fail;
  g_status = PPF_OK;
  return p;

hip_fail:
  fail_hip(e, "plan creation");
  delete p;
  return nullptr;
}

}  // namespace

ppf::PlanDev ppf_internal_plan_dev(const ppf_plan_s* plan) { return plan->dev(); }

int ppf_internal_execute_in(ppf_plan_s* plan, const void* in, void* out, long long nspectra, void* ws,
                            size_t ws_bytes) {
  try {
    if (!plan) return fail(PPF_ERR_INVALID, "plan is NULL");
    if (nspectra < 0) return fail(PPF_ERR_INVALID, "nspectra=%lld is negative", nspectra);
    if (nspectra == 0) { g_status = PPF_OK; return PPF_OK; }
    if (!in || !out) return fail(PPF_ERR_INVALID, "in or out is NULL");
    if (((uintptr_t)in & 15) || ((uintptr_t)out & 15)) return fail(PPF_ERR_ALIGN, "in and out must be 16-byte aligned");
    const size_t sb = (size_t)sample_bytes(plan->in_type);
    const size_t in_bytes = (size_t)(nspectra + plan->T - 1) * plan->N * sb;
    const size_t out_bytes = (size_t)nspectra * plan->N * 8;
    if (overlaps((uintptr_t)in, in_bytes, (uintptr_t)out, out_bytes)) return fail(PPF_ERR_INVALID, "in and out overlap");
    const bool two_pass = plan->fft_mode != PPF_FFT_MFMA_F16 && plan->path == PPF_PATH_TWO_PASS;
    if (two_pass && out_bytes > ws_bytes)
      return fail(PPF_ERR_UNSUPPORTED,
                  "%lld spectra of N=%d need %zu bytes of workspace, above the %zu-byte static workspace: "
                  "split the batch", nspectra, plan->N, out_bytes, ws_bytes);
    const hipStream_t stream = plan->stream();
    plan->note_stream(stream);   // host bookkeeping for ppf_destroy; no device memory
    const int st = run_batch(plan, stream, in, 0, in, out, nspectra, ws, nspectra);
    if (st == PPF_OK) g_status = PPF_OK;
    return st;
  } catch (...) {
    return fail(PPF_ERR_HIP, "unexpected exception in ppf_execute_noalloc");
  }
}

void ppf_internal_set_error(int status, const char* message) {
  g_status = status;
  snprintf(g_message, sizeof g_message, "%s", message);
}

extern "C" {

ppf_plan_t ppf_plan(int n_channels, int taps, const float* coeffs) {
  try {
    return make_plan(n_channels, taps, coeffs, PPF_R32, 0, PPF_C32, PPF_FFT_F32);
  } catch (...) {
    fail(PPF_ERR_NOMEM, "unexpected exception in ppf_plan");
    return nullptr;
  }
}

ppf_plan_t ppf_plan_ex(int n_channels, int taps, const void* coeffs, int coeff_type, int coeff_shift,
                       int in_type, int fft_mode) {
  try {
    return make_plan(n_channels, taps, coeffs, coeff_type, coeff_shift, in_type, fft_mode);
  } catch (...) {
    fail(PPF_ERR_NOMEM, "unexpected exception in ppf_plan_ex");
    return nullptr;
  }
}

int ppf_set_stream(ppf_plan_t plan, void* hip_stream) {
  if (!plan) return fail(PPF_ERR_INVALID, "plan is NULL");
  try {
    for (StreamBinding& b : t_bindings)
      if (b.plan_id == plan->id) {
        b.stream = (hipStream_t)hip_stream;
        return PPF_OK;
      }
    // bindings of destroyed plans are dropped now and then
    if (t_bindings.size() >= 64) t_bindings.erase(t_bindings.begin());
    t_bindings.push_back(StreamBinding{plan->id, (hipStream_t)hip_stream});
  } catch (...) {
    return fail(PPF_ERR_NOMEM, "host allocation");
  }
  return PPF_OK;
}

int ppf_plan_set_path(ppf_plan_t plan, int path) {
  if (!plan) return fail(PPF_ERR_INVALID, "plan is NULL");
  switch (path) {
    case PPF_PATH_AUTO:
      plan->path = (plan->fft_mode == PPF_FFT_MFMA_F16 || fused_ok_for(plan->N, plan->TP, plan->in_type))
                       ? PPF_PATH_FUSED : PPF_PATH_TWO_PASS;
      return PPF_OK;
    case PPF_PATH_FUSED:
      if (plan->fft_mode != PPF_FFT_MFMA_F16 && !fused_ok_for(plan->N, plan->TP, plan->in_type))
        return fail(PPF_ERR_UNSUPPORTED, "no fused kernel for N=%d taps=%d", plan->N, plan->T);
      plan->path = PPF_PATH_FUSED;
      return PPF_OK;
    case PPF_PATH_TWO_PASS:
      if (plan->fft_mode == PPF_FFT_MFMA_F16)
        return fail(PPF_ERR_UNSUPPORTED, "the matrix-core mode has only the fused path");
      plan->path = PPF_PATH_TWO_PASS;
      return PPF_OK;
    default:
      return fail(PPF_ERR_INVALID, "path=%d unknown", path);
  }
}

int ppf_plan_query(ppf_plan_t plan, int key, long long* value) {
  if (!plan) return fail(PPF_ERR_INVALID, "plan is NULL");
  if (!value) return fail(PPF_ERR_INVALID, "value is NULL");
  switch (key) {
    case PPF_Q_N: *value = plan->N; return PPF_OK;
    case PPF_Q_TAPS: *value = plan->T; return PPF_OK;
    case PPF_Q_PATH: *value = plan->path; return PPF_OK;
    case PPF_Q_WORKSPACE_BYTES: {
      std::lock_guard<std::mutex> lk(plan->mu);
      long long total = 0;
      for (const ppf_plan_s::Workspace& w : plan->ws) total += (long long)w.bytes;
      *value = total;
      return PPF_OK;
    }
    case PPF_Q_IN_TYPE: *value = plan->in_type; return PPF_OK;
    case PPF_Q_FFT_MODE: *value = plan->fft_mode; return PPF_OK;
    case PPF_Q_COEFF_SHIFT: *value = plan->coeff_shift; return PPF_OK;
    case PPF_Q_FUSED_AVAILABLE:
      *value = (plan->fft_mode == PPF_FFT_MFMA_F16 || fused_ok_for(plan->N, plan->TP, plan->in_type)) ? 1 : 0;
      return PPF_OK;
    default: return fail(PPF_ERR_INVALID, "query key %d unknown", key);
  }
}

int ppf_execute(ppf_plan_t plan, const void* in, void* out, long long nspectra) {
  try {
    if (!plan) return fail(PPF_ERR_INVALID, "plan is NULL");
    if (nspectra < 0) return fail(PPF_ERR_INVALID, "nspectra=%lld is negative", nspectra);
    if (nspectra == 0) { g_status = PPF_OK; return PPF_OK; }
    if (!in || !out) return fail(PPF_ERR_INVALID, "in or out is NULL");
    if (((uintptr_t)in & 15) || ((uintptr_t)out & 15)) return fail(PPF_ERR_ALIGN, "in and out must be 16-byte aligned");
    const size_t sb = (size_t)sample_bytes(plan->in_type);
    const size_t in_bytes = (size_t)(nspectra + plan->T - 1) * plan->N * sb;
    const size_t out_bytes = (size_t)nspectra * plan->N * 8;
    if (overlaps((uintptr_t)in, in_bytes, (uintptr_t)out, out_bytes)) return fail(PPF_ERR_INVALID, "in and out overlap");
    const hipStream_t stream = plan->stream();
    plan->note_stream(stream);
    const int st = run_batch(plan, stream, in, 0, in, out, nspectra);
    if (st == PPF_OK) g_status = PPF_OK;
    return st;
  } catch (...) {
    return fail(PPF_ERR_HIP, "unexpected exception in ppf_execute");
  }
}

int ppf_execute_power(ppf_plan_t plan, const void* in, float* out_power, long long nspectra, int K) {
  try {
    if (!plan) return fail(PPF_ERR_INVALID, "plan is NULL");
    if (K < 1) return fail(PPF_ERR_INVALID, "K=%d must be >= 1", K);
    if (K > kMaxPowerK) return fail(PPF_ERR_UNSUPPORTED, "K=%d exceeds 2^28", K);
    if (plan->path == PPF_PATH_TWO_PASS && (long long)K * plan->N > kMaxPowerKN)
      return fail(PPF_ERR_UNSUPPORTED, "two-pass detection takes K*N <= 2^24 (K=%d, N=%d)", K, plan->N);
    if (nspectra < 0) return fail(PPF_ERR_INVALID, "nspectra=%lld is negative", nspectra);
    if (nspectra % K) return fail(PPF_ERR_INVALID, "nspectra=%lld is not a multiple of K=%d", nspectra, K);
    if (nspectra == 0) { g_status = PPF_OK; return PPF_OK; }
    if (!in || !out_power) return fail(PPF_ERR_INVALID, "in or out_power is NULL");
    if (((uintptr_t)in & 15) || ((uintptr_t)out_power & 15))
      return fail(PPF_ERR_ALIGN, "in and out_power must be 16-byte aligned");
    const size_t sb = (size_t)sample_bytes(plan->in_type);
    const size_t in_bytes = (size_t)(nspectra + plan->T - 1) * plan->N * sb;
    const size_t out_bytes = (size_t)(nspectra / K) * plan->N * 4;
    if (overlaps((uintptr_t)in, in_bytes, (uintptr_t)out_power, out_bytes))
      return fail(PPF_ERR_INVALID, "in and out_power overlap");
    const hipStream_t stream = plan->stream();
    plan->note_stream(stream);
    const int st = run_power(plan, stream, in, out_power, nspectra, K);
    if (st == PPF_OK) g_status = PPF_OK;
    return st;
  } catch (...) {
    return fail(PPF_ERR_NOMEM, "unexpected exception in ppf_execute_power");
  }
}

int ppf_execute_host(ppf_plan_t plan, const void* host_in, void* host_out, long long nspectra,
                     long long chunk_spectra) {
  try {
    if (!plan) return fail(PPF_ERR_INVALID, "plan is NULL");
    if (nspectra < 0) return fail(PPF_ERR_INVALID, "nspectra=%lld is negative", nspectra);
    if (chunk_spectra < 0) return fail(PPF_ERR_INVALID, "chunk_spectra=%lld is negative", chunk_spectra);
    if (nspectra == 0) { g_status = PPF_OK; return PPF_OK; }
    if (!host_in || !host_out) return fail(PPF_ERR_INVALID, "host_in or host_out is NULL");
    const size_t sb = (size_t)sample_bytes(plan->in_type);
    const long long N = plan->N;
    const size_t in_bytes = (size_t)(nspectra + plan->T - 1) * N * sb;
    const size_t out_bytes = (size_t)nspectra * N * 8;
    if (overlaps((uintptr_t)host_in, in_bytes, (uintptr_t)host_out, out_bytes))
      return fail(PPF_ERR_INVALID, "host_in and host_out overlap");
    long long chunk = chunk_spectra > 0 ? chunk_spectra : (long long)(((size_t)PPF_HOST_CHUNK_MIB << 20) / ((size_t)N * sb));
    if (chunk < 1) chunk = 1;
    if (chunk > nspectra) chunk = nspectra;
    const hipStream_t stream = plan->stream();
    plan->note_stream(stream);
    int st = ensure_host_pipe(plan, stream, chunk);
    if (st != PPF_OK) return st;
    // the copy streams start after what the plan's stream already holds
    hipError_t e = hipEventRecord(plan->ev_start, stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(plan->h2d, plan->ev_start, 0);
    if (e == hipSuccess) e = hipStreamWaitEvent(plan->d2h, plan->ev_start, 0);
    const long long nch = (nspectra + chunk - 1) / chunk;
    for (long long i = 0; i < nch && e == hipSuccess; ++i) {
      const int b = (int)(i % kHostStages);
      const long long m0 = i * chunk;
      const long long k = nspectra - m0 < chunk ? nspectra - m0 : chunk;
      const size_t kin = (size_t)(k + plan->T - 1) * N * sb;
      // buffer b is free once chunk i-kHostStages was transformed (input)
      // and copied back (output)
      if (i >= kHostStages) e = hipStreamWaitEvent(plan->h2d, plan->ev_comp[b], 0);
      if (e == hipSuccess)
        e = hipMemcpyAsync(plan->h_in[b], (const char*)host_in + (size_t)m0 * N * sb, kin, hipMemcpyHostToDevice,
                           plan->h2d);
      if (e == hipSuccess) e = hipEventRecord(plan->ev_in[b], plan->h2d);
      if (e == hipSuccess) e = hipStreamWaitEvent(stream, plan->ev_in[b], 0);
      if (e == hipSuccess && i >= kHostStages) e = hipStreamWaitEvent(stream, plan->ev_out[b], 0);
      if (e != hipSuccess) break;
      st = run_batch(plan, stream, plan->h_in[b], 0, plan->h_in[b], plan->h_out[b], k);
      if (st != PPF_OK) return st;
      e = hipEventRecord(plan->ev_comp[b], stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(plan->d2h, plan->ev_comp[b], 0);
      if (e == hipSuccess)
        e = hipMemcpyAsync((char*)host_out + (size_t)m0 * N * 8, plan->h_out[b], (size_t)k * N * 8,
                           hipMemcpyDeviceToHost, plan->d2h);
      if (e == hipSuccess) e = hipEventRecord(plan->ev_out[b], plan->d2h);
    }
    // the plan's stream completes after the last copy back
    if (e == hipSuccess) e = hipStreamWaitEvent(stream, plan->ev_out[(nch - 1) % kHostStages], 0);
    if (e != hipSuccess) return fail_hip(e, "single-mode pipeline");
    g_status = PPF_OK;
    return PPF_OK;
  } catch (...) {
    return fail(PPF_ERR_NOMEM, "unexpected exception in ppf_execute_host");
  }
}

int ppf_design_coeffs(int n_channels, int taps, int window, double beta, const double* user_window,
                      float* coeffs) {
  if (n_channels < 1 || taps < 1) return fail(PPF_ERR_INVALID, "n_channels and taps must be >= 1");
  const long long L = (long long)n_channels * taps;
  if (L > (1ll << 20)) return fail(PPF_ERR_UNSUPPORTED, "prototype of %lld points exceeds 2^20", L);
  if (window < PPF_WIN_RECT || window > PPF_WIN_USER) return fail(PPF_ERR_INVALID, "unknown window %d", window);
  if (window == PPF_WIN_KAISER && !(beta >= 0.0 && beta <= 60.0))
    return fail(PPF_ERR_INVALID, "Kaiser beta must be in [0, 60]");
  if (window == PPF_WIN_USER && user_window == nullptr) return fail(PPF_ERR_INVALID, "user window is NULL");
  if (coeffs == nullptr) return fail(PPF_ERR_INVALID, "coeffs is NULL");

  // one device buffer: v (L doubles), user window (L doubles), h (L floats), sum
  const size_t vb = (size_t)L * sizeof(double);
  const size_t bytes = 2 * vb + (size_t)L * sizeof(float) + sizeof(double);
  char* d = nullptr;
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) return fail_hip(e, "hipMalloc (design)");
  double* v = (double*)d;
  double* user = (double*)(d + vb);
  float* h = (float*)(d + 2 * vb);
  double* sum = (double*)(d + 2 * vb + (size_t)L * sizeof(float));
  double total = 0.0;
  int st = PPF_OK;
  if (window == PPF_WIN_USER && (e = hipMemcpy(user, user_window, vb, hipMemcpyHostToDevice)) != hipSuccess) {
    st = fail_hip(e, "hipMemcpy (user window)");
  } else if ((e = ppf::launch_design((int)L, n_channels, window, beta, user, v, h, sum, nullptr)) != hipSuccess) {
    st = fail_hip(e, "design kernels");
  } else if ((e = hipMemcpy(&total, sum, sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess) {
    st = fail_hip(e, "hipMemcpy (design sum)");
  } else if (!std::isfinite(total) || total == 0.0) {
    st = fail(PPF_ERR_INVALID, "the windowed sinc sums to %g", total);
  } else if ((e = hipMemcpy(coeffs, h, (size_t)L * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess) {
    st = fail_hip(e, "hipMemcpy (coefficients)");
  }
  const hipError_t ef = hipFree(d);
  if (st == PPF_OK && ef != hipSuccess) st = fail_hip(ef, "hipFree (design)");
  return st;
}

int ppf_kaiser_beta(double atten_db, double* beta) {
  if (beta == nullptr || std::isnan(atten_db)) return fail(PPF_ERR_INVALID, "atten_db is NaN or beta is NULL");
  const double a = atten_db;
  if (a > 50.0) *beta = 0.1102 * (a - 8.7);
  else if (a >= 21.0) *beta = 0.5842 * std::pow(a - 21.0, 0.4) + 0.07886 * (a - 21.0);
  else *beta = 0.0;
  return PPF_OK;
}

int ppf_destroy(ppf_plan_t plan) {
  if (!plan) return PPF_OK;
  if (plan->h2d) (void)hipStreamSynchronize(plan->h2d);
  if (plan->d2h) (void)hipStreamSynchronize(plan->d2h);
  // every stream the plan has run on, and the caller's
  hipError_t e = hipStreamSynchronize(plan->stream());
  for (hipStream_t st : plan->used_streams) {
    const hipError_t es = hipStreamSynchronize(st);
    if (e == hipSuccess) e = es;
  }
  delete plan;
  if (e != hipSuccess) return fail_hip(e, "ppf_destroy synchronize");
  return PPF_OK;
}

ppf_stream_t ppf_stream_create(ppf_plan_t plan) {
  try {
    if (!plan) { fail(PPF_ERR_INVALID, "plan is NULL"); return nullptr; }
    ppf_stream_s* s = new (std::nothrow) ppf_stream_s;
    if (!s) { fail(PPF_ERR_NOMEM, "host allocation"); return nullptr; }
    s->plan = plan;
    s->hist_samples = (long long)(plan->T - 1) * plan->N;
    const size_t bytes = (size_t)s->hist_samples * sample_bytes(plan->in_type);
    if (bytes > 0) {
      for (int i = 0; i < 2; ++i) {
        hipError_t e = hipMalloc(&s->hist[i], bytes);
        if (e != hipSuccess) { s->hist[i] = nullptr; fail_hip(e, "stream history allocation"); delete s; return nullptr; }
        e = hipMemset(s->hist[i], 0, bytes);
        if (e != hipSuccess) { fail_hip(e, "stream history clear"); delete s; return nullptr; }
      }
    }
    g_status = PPF_OK;
    return s;
  } catch (...) {
    fail(PPF_ERR_NOMEM, "unexpected exception in ppf_stream_create");
    return nullptr;
  }
}

int ppf_stream_push(ppf_stream_t stream, const ppf_chunk* chunk) {
  try {
    if (!stream || !chunk) return fail(PPF_ERR_INVALID, "stream or chunk is NULL");
    if (stream->server_stream) return ppf_internal_server_push(stream, chunk, -1);
    ppf_plan_t plan = stream->plan;
    const long long S = chunk->nspectra;
    if (S < 0) return fail(PPF_ERR_INVALID, "nspectra=%lld is negative", S);
    if (S == 0) { g_status = PPF_OK; return PPF_OK; }
    if (!chunk->in || !chunk->out) return fail(PPF_ERR_INVALID, "chunk in or out is NULL");
    if (((uintptr_t)chunk->in & 15) || ((uintptr_t)chunk->out & 15))
      return fail(PPF_ERR_ALIGN, "chunk in and out must be 16-byte aligned");
    const size_t sb = (size_t)sample_bytes(plan->in_type);
    if (overlaps((uintptr_t)chunk->in, (size_t)S * plan->N * sb, (uintptr_t)chunk->out, (size_t)S * plan->N * 8))
      return fail(PPF_ERR_INVALID, "chunk in and out overlap");
    const long long h0 = plan->T - 1;
    const hipStream_t hs = plan->stream();
    if (stream->last_stream != hs && stream->pushed_spectra > 0) {
      // the previous push ran on another HIP stream: keep the pushes ordered
      const hipError_t es = hipStreamSynchronize(stream->last_stream);
      if (es != hipSuccess) return fail_hip(es, "stream synchronize");
    }
    plan->note_stream(hs);
    stream->last_stream = hs;
    void* cur = stream->hist[stream->cur];
    int st = run_batch(plan, hs, cur, h0, chunk->in, chunk->out, S);
    if (st != PPF_OK) return st;
    if (h0 > 0) {
      void* nxt = stream->hist[1 - stream->cur];
      hipError_t e = ppf::launch_history(cur, chunk->in, nxt, stream->hist_samples, S * plan->N, (int)sb, hs);
      if (e != hipSuccess) return fail_hip(e, "history kernel launch");
      stream->cur = 1 - stream->cur;
    }
    stream->pushed_spectra += S;
    g_status = PPF_OK;
    return PPF_OK;
  } catch (...) {
    return fail(PPF_ERR_HIP, "unexpected exception in ppf_stream_push");
  }
}

int ppf_stream_get_history(ppf_stream_t stream, void* host_dst) {
  if (!stream) return fail(PPF_ERR_INVALID, "stream is NULL");
  if (stream->server_stream) return fail(PPF_ERR_UNSUPPORTED, "a server stream's history stays with the server");
  const size_t bytes = (size_t)stream->hist_samples * sample_bytes(stream->plan->in_type);
  if (bytes == 0) return PPF_OK;
  if (!host_dst) return fail(PPF_ERR_INVALID, "host_dst is NULL");
  hipError_t e = hipStreamSynchronize(stream->last_stream);
  if (e != hipSuccess) return fail_hip(e, "history synchronize");
  e = hipMemcpy(host_dst, stream->hist[stream->cur], bytes, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail_hip(e, "history copy");
  g_status = PPF_OK;
  return PPF_OK;
}

int ppf_stream_set_history(ppf_stream_t stream, const void* host_src) {
  if (!stream) return fail(PPF_ERR_INVALID, "stream is NULL");
  if (stream->server_stream) return fail(PPF_ERR_UNSUPPORTED, "a server stream's history stays with the server");
  const size_t bytes = (size_t)stream->hist_samples * sample_bytes(stream->plan->in_type);
  if (bytes == 0) return PPF_OK;
  if (!host_src) return fail(PPF_ERR_INVALID, "host_src is NULL");
  hipError_t e = hipStreamSynchronize(stream->last_stream);
  if (e != hipSuccess) return fail_hip(e, "history synchronize");
  e = hipMemcpy(stream->hist[stream->cur], host_src, bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail_hip(e, "history copy");
  g_status = PPF_OK;
  return PPF_OK;
}

long long ppf_stream_position(ppf_stream_t stream) {
  if (!stream) { fail(PPF_ERR_INVALID, "stream is NULL"); return -1; }
  return stream->pushed_spectra;
}

int ppf_stream_destroy(ppf_stream_t stream) {
  if (!stream) return PPF_OK;
  if (stream->server_stream) return ppf_internal_server_stream_destroy(stream);
  hipError_t e = hipStreamSynchronize(stream->last_stream);
  delete stream;
  if (e != hipSuccess) return fail_hip(e, "ppf_stream_destroy synchronize");
  return PPF_OK;
}

int ppf_last_error(void) { return g_status; }

const char* ppf_last_error_message(void) { return g_message; }

const char* ppf_status_str(int status) {
  switch (status) {
    case PPF_OK: return "PPF_OK";
    case PPF_ERR_INVALID: return "PPF_ERR_INVALID";
    case PPF_ERR_UNSUPPORTED: return "PPF_ERR_UNSUPPORTED";
    case PPF_ERR_ALIGN: return "PPF_ERR_ALIGN";
    case PPF_ERR_NOMEM: return "PPF_ERR_NOMEM";
    case PPF_ERR_BUDGET: return "PPF_ERR_BUDGET";
    case PPF_ERR_HIP: return "PPF_ERR_HIP";
    case PPF_ERR_BUSY: return "PPF_ERR_BUSY";
    default: return "PPF_ERR_UNKNOWN";
  }
}

}  // extern "C"
