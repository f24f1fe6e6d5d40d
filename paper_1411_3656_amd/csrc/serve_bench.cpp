// Load generator for the serving form of libppf.so.
//
// Streams draw N from {256, 1024, 4096} and T from {8, 16} with their own
// seeds; one plan per (N, T) with sinc x Hamming coefficients. Chunks arrive
// as one Poisson process whose rate makes the offered input rate
// `load` x 6.5 GB/s (the single-SKA-channel rate of the paper's real-time
// multiple); each arrival picks a stream uniformly and S uniform in 1..64
// spectra. Payloads are complex Gaussian (sigma 1) staged in device memory
// beforehand, so the measurement excludes host transfers. The producer
// submits each chunk at its scheduled arrival time and latency is measured
// from that time, so a late producer counts against the server. Prints one
// JSON line of throughput and latency.

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ppf.h"

namespace {

#define CK(x)                                                                              \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) {                                                                \
      fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); \
      exit(2);                                                                             \
    }                                                                                      \
  } while (0)

#define PK(x)                                                                                    \
  do {                                                                                           \
    int s_ = (x);                                                                                \
    if (s_ != PPF_OK) {                                                                          \
      fprintf(stderr, "ppf error %s: %s at line %d\n", ppf_status_str(s_), ppf_last_error_message(), \
              __LINE__);                                                                         \
      exit(3);                                                                                   \
    }                                                                                            \
  } while (0)

struct Rng {  // splitmix64
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed) {}
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (next() >> 11) * (1.0 / 9007199254740992.0); }
  int range(int lo, int hi) { return lo + (int)(next() % (uint64_t)(hi - lo + 1)); }
};

// complex Gaussian payload: counter-based hash -> two uniforms -> Box-Muller
__global__ void fill_gaussian(float2* x, long long n, unsigned long long seed) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const double u1 = ((z >> 11) + 1) * (1.0 / 9007199254740993.0);
  const double u2 = ((z & 0x7FFull) + 0.5) * (1.0 / 2048.0);
  const double r = sqrt(-2.0 * log(u1));
  x[i] = make_float2((float)(r * cos(6.283185307179586 * u2)), (float)(r * sin(6.283185307179586 * u2)));
}

std::vector<float> sinc_hamming(int N, int T) {
  const int L = N * T;
  std::vector<double> h(L);
  double sum = 0;
  for (int j = 0; j < L; ++j) {
    const double w = L > 1 ? 0.54 - 0.46 * cos(2.0 * M_PI * j / (L - 1)) : 1.0;
    const double u = (j - (L - 1) / 2.0) / N;
    const double s = u == 0.0 ? 1.0 : sin(M_PI * u) / (M_PI * u);
    h[j] = w * s;
    sum += h[j];
  }
  std::vector<float> out(L);
  for (int j = 0; j < L; ++j) out[j] = (float)(h[j] / sum);
  return out;
}

struct Stream {
  int id = -1;
  int N = 0, T = 0;
  float2* in = nullptr;
  float2* out = nullptr;
  long long ring_spectra = 0;
  long long in_pos = 0, out_pos = 0;   // spectra
};

double arg_d(int argc, char** argv, const char* name, double def) {
  for (int i = 1; i + 1 < argc; ++i)
    if (!strcmp(argv[i], name)) return atof(argv[i + 1]);
  return def;
}

}  // namespace

int main(int argc, char** argv) {
  const double load = arg_d(argc, argv, "--load", 50.0);
  const double seconds = arg_d(argc, argv, "--seconds", 10.0);
  const double warmup = arg_d(argc, argv, "--warmup", 1.0);
  const int nstreams = (int)arg_d(argc, argv, "--streams", 64);
  const uint64_t seed = (uint64_t)arg_d(argc, argv, "--seed", 14113660);
  const double budget = arg_d(argc, argv, "--budget", 32e9);
  const int inflight = (int)arg_d(argc, argv, "--inflight", 2);
  const int max_s = (int)arg_d(argc, argv, "--max-spectra", 64);
  const long long ring_spectra = 512;   // per stream, input and output rings
  // restrict the (N, T) mix: --only-n 1024 --only-t 8 (diagnostics)
  const int only_n = (int)arg_d(argc, argv, "--only-n", 0);
  const int only_t = (int)arg_d(argc, argv, "--only-t", 0);

  CK(hipSetDevice(0));
  int Ns[3] = {256, 1024, 4096};
  int Ts[2] = {8, 16};
  if (only_n) Ns[0] = Ns[1] = Ns[2] = only_n;
  if (only_t) Ts[0] = Ts[1] = only_t;
  std::map<std::pair<int, int>, ppf_plan_t> plans;
  std::vector<Stream> streams(nstreams);
  double mean_n = 0;
  for (int i = 0; i < nstreams; ++i) {
    Rng r(seed + 1000ull * (uint64_t)i);
    streams[i].N = Ns[r.range(0, 2)];
    streams[i].T = Ts[r.range(0, 1)];
    mean_n += streams[i].N;
    auto key = std::make_pair(streams[i].N, streams[i].T);
    if (!plans.count(key)) {
      std::vector<float> h = sinc_hamming(key.first, key.second);
      ppf_plan_t p = ppf_plan(key.first, key.second, h.data());
      if (!p) PK(ppf_last_error());
      plans[key] = p;
    }
  }
  mean_n /= nstreams;

  ppf_server_t srv = ppf_server_create((size_t)budget, inflight);
  if (!srv) PK(ppf_last_error());
  for (int i = 0; i < nstreams; ++i) {
    Stream& st = streams[i];
    st.ring_spectra = ring_spectra;
    const long long n = ring_spectra * st.N;
    CK(hipMalloc(&st.in, n * sizeof(float2)));
    CK(hipMalloc(&st.out, n * sizeof(float2)));
    hipLaunchKernelGGL(fill_gaussian, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, st.in, n,
                       (unsigned long long)(seed * 7919ull + i));
    CK(hipGetLastError());
    PK(ppf_server_open_stream(srv, plans[std::make_pair(st.N, st.T)], 0, &st.id));
  }
  CK(hipDeviceSynchronize());

  // offered rate: load x 6.5 GB/s of complex FP32 input, mean chunk 32.5 spectra
  const double mean_s = (1 + max_s) / 2.0;
  const double lambda = load * 6.5e9 / (8.0 * mean_s * mean_n);   // chunks per second
  std::atomic<bool> stop_poll{false};
  std::thread poller([&] {
    std::vector<unsigned long long> tags(65536);
    while (!stop_poll.load(std::memory_order_relaxed)) {
      int n = ppf_server_poll(srv, tags.data(), (int)tags.size());
      if (n <= 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
  });

  Rng arr(seed ^ 0xA5A5A5A5ull);
  long long submitted = 0, late = 0;
  const long long t0 = ppf_clock_ns() + 1000000;        // start 1 ms from now
  const long long t_meas = t0 + (long long)(warmup * 1e9);
  const long long t_end = t_meas + (long long)(seconds * 1e9);
  bool reset_done = false;
  double t_next = (double)t0;
  while (true) {
    t_next += -log(1.0 - arr.uniform()) / lambda * 1e9;
    const long long ta = (long long)t_next;
    if (ta >= t_end) break;
    if (!reset_done && ta >= t_meas) {
      PK(ppf_server_reset_stats(srv));
      reset_done = true;
    }
    Stream& st = streams[arr.range(0, nstreams - 1)];
    const int S = arr.range(1, max_s);
    if (st.in_pos + S > st.ring_spectra) st.in_pos = 0;
    if (st.out_pos + S > st.ring_spectra) st.out_pos = 0;
    ppf_chunk c;
    c.in = st.in + st.in_pos * st.N;
    c.out = st.out + st.out_pos * st.N;
    c.nspectra = S;
    c.tag = (unsigned long long)submitted;
    st.in_pos += S;
    st.out_pos += S;
    long long now = ppf_clock_ns();
    while (now < ta) now = ppf_clock_ns();
    if (now - ta > 20000) late++;
    PK(ppf_server_submit(srv, st.id, &c, ta));
    submitted++;
  }
  const int drain_status = ppf_server_drain(srv, 60.0);
  stop_poll = true;
  poller.join();
  ppf_server_stats s;
  PK(ppf_server_get_stats(srv, &s));
  const double offered = load * 6.5;
  printf("{\"workload\": \"serve_%dstreams_load%g\", \"load_multiple\": %g, \"offered_gbps\": %.2f, "
         "\"sustained_gbps\": %.2f, \"realtime_multiple\": %.2f, \"p50_us\": %.1f, \"p99_us\": %.1f, "
         "\"max_us\": %.1f, \"mean_us\": %.1f, \"chunks\": %lld, \"batches\": %lld, \"mean_batch_chunks\": %.1f, "
         "\"chunk_rate_per_s\": %.0f, \"streams\": %d, \"mean_n\": %.1f, \"seconds\": %g, \"late_submits\": %lld, "
         "\"drain_status\": %d, \"state_bytes_used\": %lld, \"mean_batch_gpu_us\": %.1f, \"mean_form_us\": %.1f, "
         "\"mean_launch_us\": %.1f}\n",
         nstreams, load, load, offered, s.input_gbps, s.input_gbps / 6.5, s.p50_us, s.p99_us, s.max_us,
         s.mean_us, s.chunks_done, s.batches, s.mean_batch_chunks, s.elapsed_s > 0 ? s.chunks_done / s.elapsed_s : 0.0,
         nstreams, mean_n, seconds, late, drain_status, s.state_bytes_used, s.mean_batch_gpu_us, s.mean_form_us,
         s.mean_launch_us);
  fflush(stdout);
  for (auto& st : streams) PK(ppf_server_close_stream(srv, st.id));
  PK(ppf_server_destroy(srv));
  for (auto& st : streams) {
    CK(hipFree(st.in));
    CK(hipFree(st.out));
  }
  for (auto& kv : plans) ppf_destroy(kv.second);
  return drain_status == PPF_OK ? 0 : 4;
}
