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
// from that time, so a late producer counts against the server. Several
// producer threads (--producers, default 4) share the streams, so that the
// offered rate is not capped by one thread's submission rate. Prints one
// JSON line of throughput and latency.
//
// Checked mode (--check-dir D): the coefficients of every plan come from
// D/coef_<N>_<T>.f32, and the streams listed in D/manifest.txt (lines
// "index N T samples") take their N and T from there and read their first
// `samples` input samples from D/in_<index>.c64 instead of the ring: their
// chunks move forward through that input and through an output buffer of
// the same length (nothing reused) until it is used up, after which they
// fall back to the ring. After the run the filled output prefix of each
// such stream is written to D/out_<index>.c64 and its spectrum count to
// D/out_<index>.txt, for a comparison against a reference outside.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
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
  ppf_stream_t h = nullptr;
  int N = 0, T = 0;
  float2* in = nullptr;
  float2* out = nullptr;
  long long ring_spectra = 0;
  long long in_pos = 0, out_pos = 0;   // spectra
  // checked mode: a forward-only input and output of chk_spectra spectra
  float2* chk_in = nullptr;
  float2* chk_out = nullptr;
  long long chk_spectra = 0, chk_pos = 0;
  bool chk_done = false;
};

double arg_d(int argc, char** argv, const char* name, double def) {
  for (int i = 1; i + 1 < argc; ++i)
    if (!strcmp(argv[i], name)) return atof(argv[i + 1]);
  return def;
}

std::string arg_s(int argc, char** argv, const char* name) {
  for (int i = 1; i + 1 < argc; ++i)
    if (!strcmp(argv[i], name)) return argv[i + 1];
  return "";
}

bool read_file(const std::string& path, void* dst, size_t bytes) {
  FILE* f = fopen(path.c_str(), "rb");
  if (!f) return false;
  const size_t got = fread(dst, 1, bytes, f);
  fclose(f);
  return got == bytes;
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
  // submitting threads (one thread tops out near 2M submissions per second)
  const int producers = std::max(1, std::min(16, (int)arg_d(argc, argv, "--producers", 4)));
  const std::string check_dir = arg_s(argc, argv, "--check-dir");
  // checked streams: index -> (N, T, samples)
  std::map<int, std::vector<long long>> checked;
  if (!check_dir.empty()) {
    std::ifstream mf(check_dir + "/manifest.txt");
    if (!mf) {
      fprintf(stderr, "cannot read %s/manifest.txt\n", check_dir.c_str());
      return 5;
    }
    long long idx, n, t, samples;
    while (mf >> idx >> n >> t >> samples) {
      if (idx < 0 || idx >= nstreams || n <= 0 || t <= 0 || samples <= 0 || samples % n) {
        fprintf(stderr, "bad manifest line %lld %lld %lld %lld\n", idx, n, t, samples);
        return 5;
      }
      checked[(int)idx] = {n, t, samples};
    }
  }

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
    if (checked.count(i)) {
      streams[i].N = (int)checked[i][0];
      streams[i].T = (int)checked[i][1];
    }
    mean_n += streams[i].N;
    auto key = std::make_pair(streams[i].N, streams[i].T);
    if (!plans.count(key)) {
      std::vector<float> h = sinc_hamming(key.first, key.second);
      if (!check_dir.empty()) {
        const std::string cf = check_dir + "/coef_" + std::to_string(key.first) + "_" + std::to_string(key.second) +
                               ".f32";
        if (!read_file(cf, h.data(), h.size() * sizeof(float))) {
          fprintf(stderr, "cannot read %s\n", cf.c_str());
          return 5;
        }
      }
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
    if (checked.count(i)) {
      st.chk_spectra = checked[i][2] / st.N;
      const size_t bytes = (size_t)checked[i][2] * sizeof(float2);
      std::vector<float2> host((size_t)checked[i][2]);
      const std::string inf = check_dir + "/in_" + std::to_string(i) + ".c64";
      if (!read_file(inf, host.data(), bytes)) {
        fprintf(stderr, "cannot read %s\n", inf.c_str());
        return 5;
      }
      CK(hipMalloc(&st.chk_in, bytes));
      CK(hipMalloc(&st.chk_out, bytes));
      CK(hipMemcpy(st.chk_in, host.data(), bytes, hipMemcpyHostToDevice));
      CK(hipMemset(st.chk_out, 0xFF, bytes));   // NaN until written
    }
    PK(ppf_server_open_stream_ex(srv, plans[std::make_pair(st.N, st.T)], PPF_OPEN_NOWAIT, &st.h));
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

  // P producer threads, producer q owning the streams i with i % P == q
  // and offering 1/P of the load as its own Poisson process (together one
  // Poisson process of rate lambda over uniformly chosen streams); each
  // stream's chunks therefore come from one thread, in order.
  std::atomic<long long> submitted{0}, late{0};
  const long long t0 = ppf_clock_ns() + 1000000;        // start 1 ms from now
  const long long t_meas = t0 + (long long)(warmup * 1e9);
  const long long t_end = t_meas + (long long)(seconds * 1e9);
  auto produce = [&](int q) {
    Rng arr(seed ^ 0xA5A5A5A5ull ^ (0x9E3779B97F4A7C15ull * (uint64_t)q));
    std::vector<int> mine;
    for (int i = q; i < nstreams; i += producers) mine.push_back(i);
    if (mine.empty()) return;
    const double lam = lambda * (double)mine.size() / nstreams;
    bool reset_done = q != 0;
    double t_next = (double)t0;
    long long count = 0, nlate = 0;
    while (true) {
      t_next += -log(1.0 - arr.uniform()) / lam * 1e9;
      const long long ta = (long long)t_next;
      if (ta >= t_end) break;
      if (!reset_done && ta >= t_meas) {
        PK(ppf_server_reset_stats(srv));
        reset_done = true;
      }
      Stream& st = streams[mine[arr.range(0, (int)mine.size() - 1)]];
      const int S = arr.range(1, max_s);
      ppf_chunk c;
      c.nspectra = S;
      c.tag = ((unsigned long long)q << 48) | (unsigned long long)count;
      if (st.chk_in && !st.chk_done && st.chk_pos + S <= st.chk_spectra) {
        c.in = st.chk_in + st.chk_pos * st.N;
        c.out = st.chk_out + st.chk_pos * st.N;
        st.chk_pos += S;
      } else {
        // a checked stream whose input is used up stays on the ring from here
        st.chk_done = true;
        if (st.in_pos + S > st.ring_spectra) st.in_pos = 0;
        if (st.out_pos + S > st.ring_spectra) st.out_pos = 0;
        c.in = st.in + st.in_pos * st.N;
        c.out = st.out + st.out_pos * st.N;
        st.in_pos += S;
        st.out_pos += S;
      }
      long long now = ppf_clock_ns();
      while (now < ta) now = ppf_clock_ns();
      if (now - ta > 20000) nlate++;
      PK(ppf_server_submit(st.h, &c, ta));
      count++;
    }
    submitted += count;
    late += nlate;
  };
  std::vector<std::thread> prod;
  for (int q = 0; q < producers; ++q) prod.emplace_back(produce, q);
  for (auto& t : prod) t.join();
  const int drain_status = ppf_server_drain(srv, 60.0);
  stop_poll = true;
  poller.join();
  ppf_server_stats_t s;
  PK(ppf_server_get_stats(srv, &s));
  long long checked_chunks_spectra = 0;
  for (auto& kv : checked) {
    Stream& st = streams[kv.first];
    const size_t bytes = (size_t)st.chk_pos * st.N * sizeof(float2);
    std::vector<float2> host((size_t)st.chk_pos * st.N);
    if (bytes) CK(hipMemcpy(host.data(), st.chk_out, bytes, hipMemcpyDeviceToHost));
    const std::string of = check_dir + "/out_" + std::to_string(kv.first) + ".c64";
    FILE* f = fopen(of.c_str(), "wb");
    if (!f || fwrite(host.data(), 1, bytes, f) != bytes) {
      fprintf(stderr, "cannot write %s\n", of.c_str());
      return 5;
    }
    fclose(f);
    std::ofstream(check_dir + "/out_" + std::to_string(kv.first) + ".txt") << st.chk_pos << "\n";
    checked_chunks_spectra += st.chk_pos;
  }
  const double offered = load * 6.5;
  printf("{\"workload\": \"serve_%dstreams_load%g\", \"load_multiple\": %g, \"offered_gbps\": %.2f, "
         "\"sustained_gbps\": %.2f, \"realtime_multiple\": %.2f, \"p50_us\": %.1f, \"p99_us\": %.1f, "
         "\"max_us\": %.1f, \"mean_us\": %.1f, \"chunks\": %lld, \"batches\": %lld, \"mean_batch_chunks\": %.1f, "
         "\"chunk_rate_per_s\": %.0f, \"streams\": %d, \"mean_n\": %.1f, \"seconds\": %g, \"late_submits\": %lld, "
         "\"drain_status\": %d, \"producers\": %d, \"state_bytes_used\": %lld, \"mean_batch_gpu_us\": %.1f, \"mean_form_us\": %.1f, "
         "\"mean_launch_us\": %.1f, \"checked_spectra\": %lld, \"tags_dropped\": %lld}\n",
         nstreams, load, load, offered, s.input_gbps, s.input_gbps / 6.5, s.p50_us, s.p99_us, s.max_us,
         s.mean_us, s.chunks_done, s.batches, s.mean_batch_chunks, s.elapsed_s > 0 ? s.chunks_done / s.elapsed_s : 0.0,
         nstreams, mean_n, seconds, late.load(), drain_status, producers, s.state_bytes_used, s.mean_batch_gpu_us, s.mean_form_us,
         s.mean_launch_us, checked_chunks_spectra, s.tags_dropped);
  fflush(stdout);
  for (auto& st : streams) PK(ppf_stream_destroy(st.h));
  PK(ppf_server_destroy(srv));
  for (auto& st : streams) {
    CK(hipFree(st.in));
    CK(hipFree(st.out));
    if (st.chk_in) CK(hipFree(st.chk_in));
    if (st.chk_out) CK(hipFree(st.chk_out));
  }
  for (auto& kv : plans) ppf_destroy(kv.second);
  return drain_status == PPF_OK ? 0 : 4;
}
