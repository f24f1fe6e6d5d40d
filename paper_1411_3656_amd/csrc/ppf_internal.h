// Internal interface between the C-ABI layer (ppf_api.cpp) and the HIP
// kernels (ppf_kernels.hip, ppf_mfma.hip). Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>

namespace ppf {

// Launch description for one batch of spectra. The input is read as the
// concatenation of two segments: x0 holds h0 blocks (a stream's history,
// h0 = 0 for the plain batch form) and x1 the rest. Block b of the
// concatenation is b*N samples in. The output of spectrum m (0 <= m < M)
// goes to out + m*N.
struct BatchArgs {
  const void* x0;
  const void* x1;
  long long h0;        // blocks in x0
  void* out;           // complex FP32 output (or the FIR workspace)
  long long M;         // spectra to produce
};

// Plan-owned device constants used by the kernels.
struct PlanDev {
  int N;
  int T;               // taps as given
  int TP;              // taps rounded up to the kernel's template tap count
  const float* coef;   // TP*N, zero-padded at the front (TP-T leading zero segments)
  const float* ones;   // N ones: identity coefficients for the FFT-only pass
  const void* tw;      // N complex FP32 twiddles exp(-2 pi i k/N)
  int in_type;         // 0 complex FP32, 1 complex FP16, 2 complex int8
};

// Descriptor tables of the serving form (device memory, filled by the host).
// A tile is a run of spectra whose input is x0 (h0 blocks) ++ x1 (h1
// blocks) ++ x2 and whose spectrum m goes to out + m*N.
struct TileDesc {
  const void* x0;
  const void* x1;
  const void* x2;
  void* out;
  int h0;
  int h1;
  int count;
  int pad_;
};
// The tiles of one kernel class are tiles[first .. first+ntiles).
struct DescClass {
  int first;
  int ntiles;
};
// History update: dst = last hs samples of (a0 ++ a1 ++ b); a0 holds n0 and
// a1 hs - n0 samples (together the hs samples before b), b holds cs samples
// (complex FP32).
struct HistDesc {
  const void* a0;
  const void* a1;
  const void* b;
  void* dst;
  int n0;
  int hs;
  int cs;
  int pad_;
};

int taps_template(int T);                       // smallest supported TP >= T, 0 if none
bool fused_available(int N, int TP);
bool fft_available(int N);
bool fir_available(int TP);

// One fused kernel over args.M spectra.
hipError_t launch_fused(const PlanDev& pd, const BatchArgs& a, hipStream_t st);
// FIR presum only: writes u (complex FP32, M*N) to a.out.
hipError_t launch_fir(const PlanDev& pd, const BatchArgs& a, hipStream_t st);
// Batched N-point FFT of M contiguous blocks (in x1) to a.out.
hipError_t launch_fft(const PlanDev& pd, const void* in, void* out, long long M, hipStream_t st);
// Four-step two-pass form for N = N1 * N2 (N = 8192, 16384; FP32 input):
// pass A = FIR + N1-point transforms + W_N twiddles into the workspace,
// pass B = N2-point transforms of the workspace's columns to the spectra.
bool fourstep_available(int N, int TP);
int fourstep_n1(int N);
int fourstep_n2(int N);
hipError_t launch_fourstep_a(const PlanDev& pd, const BatchArgs& a, const void* tw_n1, hipStream_t st);
hipError_t launch_fourstep_b(const PlanDev& pd, const void* ws, void* out, long long M, const void* tw_n2,
                             hipStream_t st);
// Descriptor launches with persistent grids sized for at most max_tiles
// tiles (max_entries history entries); the counts are read on the device.
hipError_t launch_fused_desc(const PlanDev& pd, const DescClass* cls, const TileDesc* tiles, int max_tiles,
                             hipStream_t st);
hipError_t launch_fft_desc(const PlanDev& pd, const DescClass* cls, const TileDesc* tiles, int max_tiles,
                           hipStream_t st);
hipError_t launch_fir_desc(const PlanDev& pd, const DescClass* cls, const TileDesc* tiles, int max_tiles,
                           hipStream_t st);
hipError_t launch_history_desc(const int* count, const HistDesc* h, int max_entries, long long max_samples,
                               hipStream_t st);
// One-time set-up of a plan's descriptor launchers, to run before capture.
hipError_t prepare_desc(const PlanDev& pd, bool fused);
// FP64 twiddle generation: tw[k] = exp(-2 pi i k/N) rounded to FP32.
hipError_t launch_twiddles(void* tw, int N, hipStream_t st);
// Stream history update: new = last `hist_samples` samples of (old ++ chunk).
hipError_t launch_history(const void* old_hist, const void* chunk, void* new_hist,
                          long long hist_samples, long long chunk_samples, int sample_bytes,
                          hipStream_t st);

// Detection: |X|^2 summed over K consecutive spectra (M a multiple of K),
// written to pout as (M / K) x N floats instead of the spectra.
hipError_t launch_fused_power(const PlanDev& pd, const BatchArgs& a, float* pout, int K, hipStream_t st);
hipError_t launch_fft_power(const PlanDev& pd, const void* in, float* pout, long long M, int K, hipStream_t st);

// Reduced-precision fused kernel with matrix-core DFT stages (N = 4096,
// complex int8 or FP16 input, FP16 coefficients).
struct MfmaDev {
  int N;               // 4096, 1024 or 256
  int tq;              // tap slots of the kernel (16; 8 or 16 below N = 4096)
  const void* coef16;  // tq tap slots x N FP16 coefficients in lane order
  const void* tw;      // N complex FP32 twiddles
  const void* w256;    // 256 complex FP16 values exp(-2 pi i k/256)
  int d;               // leading zero tap slots (tq - T)
  int in_type;         // 2 complex int8, 1 complex FP16
  float in_scale;      // 2^-e1: on the int8 samples (exact in FP16), or on the FIR's FP32 sums
  float out_scale;     // 2^(e1 - coeff_shift), folded exactly into the FP16 stage-3 matrix
};
bool mfma_available(int N, int TP);
int mfma_tap_slots(int N, int T);
size_t mfma_coef_bytes(int N, int TQ);
void mfma_coef_layout(int N, int TQ, const uint16_t* h16, int T, uint16_t* dst);
hipError_t launch_w256(void* table, hipStream_t st);

// Prototype-filter design (plan time): v (L doubles) and h (L floats) and
// sum (1 double) are device buffers; user holds L doubles for PPF_WIN_USER.
hipError_t launch_design(int L, int N, int window, double beta, const double* user, double* v, float* h,
                         double* sum, hipStream_t st);
hipError_t launch_mfma(const MfmaDev& md, const BatchArgs& a, hipStream_t st);
// Detection with the matrix-core transform: |X|^2 summed over K spectra.
hipError_t launch_mfma_power(const MfmaDev& md, const BatchArgs& a, float* pout, int K, hipStream_t st);

}  // namespace ppf

// Plan internals for the server (implemented beside the plan object).
struct ppf_plan_s;
struct ppf_server_s;
struct ppf_chunk;
ppf::PlanDev ppf_internal_plan_dev(const ppf_plan_s* plan);
// Record a failure as the calling thread's last error.
void ppf_internal_set_error(int status, const char* message);
// ppf_execute with the two-pass workspace given by the caller (ws_bytes
// bytes of device memory): allocates nothing; batches whose presums exceed
// ws_bytes are rejected (ppf_noalloc.hip).
int ppf_internal_execute_in(ppf_plan_s* plan, const void* in, void* out, long long nspectra, void* ws,
                            size_t ws_bytes);

namespace ppf {
struct SrvStream;   // a server's per-stream state (ppf_server.cpp)
}

// A stream handle. A plain stream owns its history and runs its chunks on
// the plan's HIP stream; a server stream (server_stream true) hands its
// chunks to the server, which owns the history.
struct ppf_stream_s {
  ppf_plan_s* plan = nullptr;
  void* hist[2] = {nullptr, nullptr};   // ping-pong history buffers, (T-1)*N samples each
  int cur = 0;
  long long hist_samples = 0;
  long long pushed_spectra = 0;
  hipStream_t last_stream = nullptr;    // HIP stream of the latest push (plain streams)
  bool server_stream = false;
  ppf_server_s* server = nullptr;       // NULL once the server is destroyed
  std::shared_ptr<ppf::SrvStream> srv;
  ~ppf_stream_s();
};

// Server streams (ppf_server.cpp): a push queues the chunk at the server;
// destroy closes the stream, waits for its chunks and frees the handle.
int ppf_internal_server_push(ppf_stream_s* stream, const ppf_chunk* chunk, long long arrival_ns);
int ppf_internal_server_stream_destroy(ppf_stream_s* stream);
