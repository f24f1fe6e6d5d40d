// HIP kernels of the polyphase filter bank for CDNA4 (gfx950).
//
// The PPF computes, for every output spectrum m,
//   u[m][c] = sum_t h[t*N + c] * x[(m+t)*N + c]        (section 2, Eq. 1 per channel)
//   X[m][k] = sum_c u[m][c] * exp(-2 pi i c k / N)      (the DFT after the FIR, section 3)
//
// Fused kernel (one pass over HBM): a group of W = N/R threads owns one
// contiguous tile of spectra. Thread j of the group owns the R channels
// j + e*W (e < R). That is at once
//   - a coalesced layout for the input blocks (W consecutive lanes read W
//     consecutive samples),
//   - the column layout in which a Stockham FFT with radix <= R reads its
//     first stage and writes its last stage, so FIR output feeds the FFT
//     without an exchange and the spectrum leaves in natural order with
//     coalesced stores.
// Each thread keeps a ring of TP+PF input blocks of its channels in
// registers: TP blocks form the tap window of the current spectrum and PF
// blocks are loads already in flight for later spectra. The ring index of a
// block is static because the spectrum loop is unrolled by the ring size.
// Between Stockham stages the group exchanges data through LDS (split
// re/im planes, swizzled or padded to spread banks, double-buffered
// when it fits so that one barrier per exchange suffices). Twiddles per
// thread are constant across spectra and are loaded into registers once.
//
// Two-pass form (taps windows too large for registers): a FIR-only kernel
// with a per-thread register ring writes u to a workspace, then the same
// fused kernel with one identity tap performs the FFTs.

#include "ppf_engine.h"

namespace ppf {

// --------------------------------------------------------------------------
// FIR-only kernel (two-pass form): one channel per thread, register ring
// --------------------------------------------------------------------------

struct FirParams {
  const void* x0;
  const void* x1;
  v2f* out;            // u, M*N
  const float* coef;   // TP*N
  int h0;
  int M;
  int N;
  int S;
  int d;
};

template <int TP, int PF, int IT>
__global__ void __launch_bounds__(256) ppf_fir_kernel(FirParams p) {
  constexpr int Q = TP + PF;
  const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
  const int c = (int)(g & (p.N - 1));
  const long long tile = g / p.N;
  if (tile * p.S >= p.M) return;
  const int m0 = (int)tile * p.S;
  const int rem = p.M - m0;
  const int ng = rem < p.S ? rem : p.S;
  const int vb_lo = m0 > p.d ? m0 : p.d;
  const int vb_hi = m0 + ng + TP - 1;

  float hreg[TP];
#pragma unroll
  for (int t = 0; t < TP; ++t) hreg[t] = p.coef[(long long)t * p.N + c];

  v2f ring[Q];
#pragma unroll
  for (int s = 0; s < Q; ++s) { ring[s].x = 0.f; ring[s].y = 0.f; }
  auto load = [&](v2f& dst, int vb) {
    if (vb >= vb_lo && vb < vb_hi) {
      const int rb = vb - p.d;
      dst = rb < p.h0 ? load_sample<IT>(p.x0, (long long)rb * p.N + c)
                      : load_sample<IT>(p.x1, (long long)(rb - p.h0) * p.N + c);
    }
  };
#pragma unroll
  for (int s = 0; s < Q - 1; ++s) load(ring[s], m0 + s);

  v2f* outg = p.out + (long long)m0 * p.N + c;
  for (int base = 0; base < ng; base += Q) {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int it = base + k;
      if (it >= ng) break;
      load(ring[(k + Q - 1) % Q], m0 + it + Q - 1);
      v2f a;
      a.x = hreg[0] * ring[k % Q].x;
      a.y = hreg[0] * ring[k % Q].y;
#pragma unroll
      for (int t = 1; t < TP; ++t) {
        a.x = fmaf(hreg[t], ring[(k + t) % Q].x, a.x);
        a.y = fmaf(hreg[t], ring[(k + t) % Q].y, a.y);
      }
      outg[(long long)it * p.N] = a;
    }
  }
}

// Descriptor form of the FIR pass (serving): work item w of the persistent
// grid is channel w % N of tile w / N; the tile's out is its workspace.
template <int TP, int PF>
__global__ void __launch_bounds__(256)
ppf_fir_desc_kernel(const DescClass* cls, const TileDesc* tiles, const float* coef, int N, int d) {
  constexpr int Q = TP + PF;
  const int first = cls->first;
  const long long items = (long long)cls->ntiles * N;
  for (long long w = (long long)blockIdx.x * 256 + threadIdx.x; w < items; w += (long long)gridDim.x * 256) {
    const int t = (int)(w / N);
    const int c = (int)(w - (long long)t * N);
    const TileDesc& td = tiles[first + t];
    const int ng = td.count;
    const int vb_lo = d;
    const int vb_hi = ng + TP - 1;
    float hreg[TP];
#pragma unroll
    for (int k = 0; k < TP; ++k) hreg[k] = coef[(long long)k * N + c];
    v2f ring[Q];
#pragma unroll
    for (int s = 0; s < Q; ++s) { ring[s].x = 0.f; ring[s].y = 0.f; }
    auto load = [&](v2f& dst, int vb) {
      if (vb >= vb_lo && vb < vb_hi) {
        const int rb = vb - d;
        const int h01 = td.h0 + td.h1;
        dst = rb < td.h0 ? ((const v2f*)td.x0)[(long long)rb * N + c]
                         : (rb < h01 ? ((const v2f*)td.x1)[(long long)(rb - td.h0) * N + c]
                                     : ((const v2f*)td.x2)[(long long)(rb - h01) * N + c]);
      }
    };
#pragma unroll
    for (int s = 0; s < Q - 1; ++s) load(ring[s], s);
    v2f* outg = (v2f*)td.out + c;
    for (int base = 0; base < ng; base += Q) {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const int it = base + k;
        if (it >= ng) break;
        load(ring[(k + Q - 1) % Q], it + Q - 1);
        v2f acc;
        acc.x = hreg[0] * ring[k % Q].x;
        acc.y = hreg[0] * ring[k % Q].y;
#pragma unroll
        for (int tt = 1; tt < TP; ++tt) {
          acc.x = fmaf(hreg[tt], ring[(k + tt) % Q].x, acc.x);
          acc.y = fmaf(hreg[tt], ring[(k + tt) % Q].y, acc.y);
        }
        outg[(long long)it * N] = acc;
      }
    }
  }
}

// --------------------------------------------------------------------------
// FP64 twiddles, history tail
// --------------------------------------------------------------------------

__global__ void ppf_twiddle_kernel(v2f* tw, int N) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) {
    double s, c;
    sincospi(-2.0 * (double)k / (double)N, &s, &c);   // angle -2 pi k/N, k/N exact
    v2f w;
    w.x = (float)c;
    w.y = (float)s;
    tw[k] = w;
  }
}

template <typename E>
__global__ void ppf_history_kernel(const E* old_h, const E* chunk, E* new_h, long long hs, long long cs) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < hs) new_h[i] = (i + cs < hs) ? old_h[i + cs] : chunk[i + cs - hs];
}

// Descriptor form: entry e writes the last hs samples of (a0 ++ a1 ++ b) to
// dst, a0 and a1 holding the hs samples before b and b holding cs samples.
// Block (x, y) copies piece x (kHistPiece samples) of entries y, y + gridDim.y, ...
constexpr int kHistPiece = 1024;
__global__ void __launch_bounds__(256) ppf_history_desc_kernel(const int* count, const HistDesc* h) {
  const int n = *count;
  for (int e = blockIdx.y; e < n; e += gridDim.y) {
    const HistDesc hd = h[e];
    const int i0 = blockIdx.x * kHistPiece;
    if (i0 >= hd.hs) continue;
    const v2f* a0 = (const v2f*)hd.a0;
    const v2f* a1 = (const v2f*)hd.a1;
    const v2f* b = (const v2f*)hd.b;
    v2f* dst = (v2f*)hd.dst;
    const int i1 = i0 + kHistPiece < hd.hs ? i0 + kHistPiece : hd.hs;
#pragma unroll 4
    for (int i = i0 + threadIdx.x; i < i1; i += 256) {
      const long long k = (long long)i + hd.cs;
      dst[i] = k < hd.n0 ? a0[k] : (k < hd.hs ? a1[k - hd.n0] : b[k - hd.hs]);
    }
  }
}


template <int N>
static FusedFn fused_for_taps(int TP) {
  switch (TP) {
    case 1: return &fused_launch<N, 1>;
    case 2: if constexpr (fused_ok(N, 2)) return &fused_launch<N, 2>; else return nullptr;
    case 4: if constexpr (fused_ok(N, 4)) return &fused_launch<N, 4>; else return nullptr;
    case 8: if constexpr (fused_ok(N, 8)) return &fused_launch<N, 8>; else return nullptr;
    case 16: if constexpr (fused_ok(N, 16)) return &fused_launch<N, 16>; else return nullptr;
    default: return nullptr;
  }
}

static FusedFn fused_fn(int N, int TP) {
  switch (N) {
    case 16: return fused_for_taps<16>(TP);
    case 32: return fused_for_taps<32>(TP);
    case 64: return fused_for_taps<64>(TP);
    case 128: return fused_for_taps<128>(TP);
    case 256: return fused_for_taps<256>(TP);
    case 512: return fused_for_taps<512>(TP);
    case 1024: return fused_for_taps<1024>(TP);
    case 2048: return fused_for_taps<2048>(TP);
    case 4096: return fused_for_taps<4096>(TP);
    case 8192: return fused_for_taps<8192>(TP);
    case 16384: return fused_for_taps<16384>(TP);
    default: return nullptr;
  }
}

int taps_template(int T) {
  if (T < 1 || T > 64) return 0;
  int tp = 1;
  while (tp < T) tp <<= 1;
  return tp;
}

bool fused_available(int N, int TP) { return TP > 1 && fused_fn(N, TP) != nullptr; }
bool fft_available(int N) { return fused_fn(N, 1) != nullptr; }

hipError_t launch_fused(const PlanDev& pd, const BatchArgs& a, hipStream_t st) {
  FusedFn f = pd.in_type == 0 ? fused_fn(pd.N, pd.TP) : fused_fn_widened(pd.N, pd.TP, pd.in_type);
  if (!f) return hipErrorInvalidValue;
  return f(pd, a, pd.coef, pd.T, st, nullptr, 1);
}

static FusedFn fft_fn(int N) {
  switch (N) {
    case 16: return &fused_launch<16, 1, true>;
    case 32: return &fused_launch<32, 1, true>;
    case 64: return &fused_launch<64, 1, true>;
    case 128: return &fused_launch<128, 1, true>;
    case 256: return &fused_launch<256, 1, true>;
    case 512: return &fused_launch<512, 1, true>;
    case 1024: return &fused_launch<1024, 1, true>;
    case 2048: return &fused_launch<2048, 1, true>;
    case 4096: return &fused_launch<4096, 1, true>;
    case 8192: return &fused_launch<8192, 1, true>;
    case 16384: return &fused_launch<16384, 1, true>;
    default: return nullptr;
  }
}

hipError_t launch_fft(const PlanDev& pd, const void* in, void* out, long long M, hipStream_t st) {
  FusedFn f = fft_fn(pd.N);
  if (!f) return hipErrorInvalidValue;
  BatchArgs a{in, in, 0, out, M};
  return f(pd, a, pd.ones, 1, st, nullptr, 1);
}

template <int TP, int IT>
static hipError_t fir_launch(const PlanDev& pd, const BatchArgs& a, hipStream_t st) {
  constexpr int PF = TP >= 32 ? 2 : 4;
  static const int occ = [] {
    KernelInfo ki{(const void*)&ppf_fir_kernel<TP, PF, IT>, 256, 1, 0};
    return occupancy(ki);
  }();
  const long long resident = (long long)device_cus() * occ * 256;   // threads
  const long long chans = pd.N;
  // tiles per channel so that all resident threads are busy once
  long long tiles = resident / chans;
  if (tiles < 1) tiles = 1;
  long long S = (a.M + tiles - 1) / tiles;
  if (S < 2 * TP) S = 2 * TP;
  if (S > (1 << 30)) S = 1 << 30;
  const long long ntiles = (a.M + S - 1) / S;
  const long long threads = ntiles * chans;
  const long long nblocks = (threads + 255) / 256;
  if (nblocks <= 0) return hipSuccess;
  if (nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (a.M > kMaxLaunchSpectra || a.h0 > kMaxLaunchSpectra) return hipErrorInvalidValue;
  FirParams p;
  p.x0 = a.x0;
  p.x1 = a.x1;
  p.out = (v2f*)a.out;
  p.coef = pd.coef;
  p.h0 = (int)a.h0;
  p.M = (int)a.M;
  p.N = pd.N;
  p.S = (int)S;
  p.d = TP - pd.T;
  hipLaunchKernelGGL((ppf_fir_kernel<TP, PF, IT>), dim3((unsigned)nblocks), dim3(256), 0, st, p);
  return hipGetLastError();
}

bool fir_available(int TP) {
  return TP == 1 || TP == 2 || TP == 4 || TP == 8 || TP == 16 || TP == 32 || TP == 64;
}

template <int IT>
static hipError_t fir_launch_taps(const PlanDev& pd, const BatchArgs& a, hipStream_t st) {
  switch (pd.TP) {
    case 1: return fir_launch<1, IT>(pd, a, st);
    case 2: return fir_launch<2, IT>(pd, a, st);
    case 4: return fir_launch<4, IT>(pd, a, st);
    case 8: return fir_launch<8, IT>(pd, a, st);
    case 16: return fir_launch<16, IT>(pd, a, st);
    case 32: return fir_launch<32, IT>(pd, a, st);
    case 64: return fir_launch<64, IT>(pd, a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fir(const PlanDev& pd, const BatchArgs& a, hipStream_t st) {
  switch (pd.in_type) {
    case 0: return fir_launch_taps<0>(pd, a, st);
    case 1: return fir_launch_taps<1>(pd, a, st);
    case 2: return fir_launch_taps<2>(pd, a, st);
    default: return hipErrorInvalidValue;
  }
}

// ---- descriptor launchers (persistent grids, fixed across graph replays)

template <int N, int TP, bool UNIT = false>
static hipError_t fused_desc_launch(const PlanDev& pd, const DescClass* cls, const TileDesc* tiles, int max_tiles,
                                    const float* coef, int T, hipStream_t st) {
  constexpr int R = cfg_R(N, TP), RX = cfg_RX(N, TP), G = cfg_G(N, TP), PF = cfg_PF(N, TP), B = cfg_B(N, TP);
  constexpr bool DB = cfg_DB(N, B, TP), TWG = cfg_TWG(N);
  using Eng = FusedEngine<N, R, RX, G, B, TP, PF, DB, TWG, UNIT>;
  auto kern = &ppf_fused_desc_kernel<N, R, RX, G, B, TP, PF, DB, TWG, UNIT>;
  static const int occ = [&] {
    KernelInfo ki{(const void*)kern, (N / R) * G, G, Eng::lds_bytes()};
    return occupancy(ki);
  }();
  if (!cls) return hipSuccess;                 // warm-up call: occupancy only
  long long grid = (long long)device_cus() * occ;
  const long long need = (max_tiles + G - 1) / G;
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3((N / R) * G), Eng::lds_bytes(), st, cls, tiles, coef,
                     (const v2f*)pd.tw, TP - T);
  return hipGetLastError();
}

typedef hipError_t (*FusedDescFn)(const PlanDev&, const DescClass*, const TileDesc*, int, const float*, int,
                                  hipStream_t);

template <int N>
static FusedDescFn fused_desc_for_taps(int TP) {
  switch (TP) {
    case 1: return &fused_desc_launch<N, 1>;
    case 2: if constexpr (fused_ok(N, 2)) return &fused_desc_launch<N, 2>; else return nullptr;
    case 4: if constexpr (fused_ok(N, 4)) return &fused_desc_launch<N, 4>; else return nullptr;
    case 8: if constexpr (fused_ok(N, 8)) return &fused_desc_launch<N, 8>; else return nullptr;
    case 16: if constexpr (fused_ok(N, 16)) return &fused_desc_launch<N, 16>; else return nullptr;
    default: return nullptr;
  }
}

static FusedDescFn fused_desc_fn(int N, int TP) {
  switch (N) {
    case 16: return fused_desc_for_taps<16>(TP);
    case 32: return fused_desc_for_taps<32>(TP);
    case 64: return fused_desc_for_taps<64>(TP);
    case 128: return fused_desc_for_taps<128>(TP);
    case 256: return fused_desc_for_taps<256>(TP);
    case 512: return fused_desc_for_taps<512>(TP);
    case 1024: return fused_desc_for_taps<1024>(TP);
    case 2048: return fused_desc_for_taps<2048>(TP);
    case 4096: return fused_desc_for_taps<4096>(TP);
    case 8192: return fused_desc_for_taps<8192>(TP);
    case 16384: return fused_desc_for_taps<16384>(TP);
    default: return nullptr;
  }
}

hipError_t launch_fused_desc(const PlanDev& pd, const DescClass* cls, const TileDesc* tiles, int max_tiles,
                             hipStream_t st) {
  FusedDescFn f = fused_desc_fn(pd.N, pd.TP);
  if (!f) return hipErrorInvalidValue;
  return f(pd, cls, tiles, max_tiles, pd.coef, pd.T, st);
}

static FusedDescFn fft_desc_fn(int N) {
  switch (N) {
    case 16: return &fused_desc_launch<16, 1, true>;
    case 32: return &fused_desc_launch<32, 1, true>;
    case 64: return &fused_desc_launch<64, 1, true>;
    case 128: return &fused_desc_launch<128, 1, true>;
    case 256: return &fused_desc_launch<256, 1, true>;
    case 512: return &fused_desc_launch<512, 1, true>;
    case 1024: return &fused_desc_launch<1024, 1, true>;
    case 2048: return &fused_desc_launch<2048, 1, true>;
    case 4096: return &fused_desc_launch<4096, 1, true>;
    case 8192: return &fused_desc_launch<8192, 1, true>;
    case 16384: return &fused_desc_launch<16384, 1, true>;
    default: return nullptr;
  }
}

hipError_t launch_fft_desc(const PlanDev& pd, const DescClass* cls, const TileDesc* tiles, int max_tiles,
                           hipStream_t st) {
  FusedDescFn f = fft_desc_fn(pd.N);
  if (!f) return hipErrorInvalidValue;
  return f(pd, cls, tiles, max_tiles, pd.ones, 1, st);
}

template <int TP>
static hipError_t fir_desc_launch(const PlanDev& pd, const DescClass* cls, const TileDesc* tiles, int max_tiles,
                                  hipStream_t st) {
  // serving tiles are short and few: more loads in flight per thread
  constexpr int PF = TP >= 32 ? 2 : 8;
  auto kern = &ppf_fir_desc_kernel<TP, PF>;
  static const int occ = [&] {
    KernelInfo ki{(const void*)kern, 256, 1, 0};
    return occupancy(ki);
  }();
  if (!cls) return hipSuccess;                 // warm-up call: occupancy only
  long long grid = (long long)device_cus() * occ;
  const long long need = ((long long)max_tiles * pd.N + 255) / 256;
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), 0, st, cls, tiles, pd.coef, pd.N, TP - pd.T);
  return hipGetLastError();
}

hipError_t launch_fir_desc(const PlanDev& pd, const DescClass* cls, const TileDesc* tiles, int max_tiles,
                           hipStream_t st) {
  switch (pd.TP) {
    case 1: return fir_desc_launch<1>(pd, cls, tiles, max_tiles, st);
    case 2: return fir_desc_launch<2>(pd, cls, tiles, max_tiles, st);
    case 4: return fir_desc_launch<4>(pd, cls, tiles, max_tiles, st);
    case 8: return fir_desc_launch<8>(pd, cls, tiles, max_tiles, st);
    case 16: return fir_desc_launch<16>(pd, cls, tiles, max_tiles, st);
    case 32: return fir_desc_launch<32>(pd, cls, tiles, max_tiles, st);
    case 64: return fir_desc_launch<64>(pd, cls, tiles, max_tiles, st);
    default: return hipErrorInvalidValue;
  }
}

// First-use work of the descriptor launchers (occupancy queries, LDS
// limits) done ahead of a graph capture.
hipError_t prepare_desc(const PlanDev& pd, bool fused) {
  hipError_t e = hipSuccess;
  device_cus();
  if (fused) {
    e = launch_fused_desc(pd, nullptr, nullptr, 0, nullptr);
  } else {
    e = launch_fir_desc(pd, nullptr, nullptr, 0, nullptr);
    if (e == hipSuccess) e = launch_fft_desc(pd, nullptr, nullptr, 0, nullptr);
  }
  return e;
}

hipError_t launch_history_desc(const int* count, const HistDesc* h, int max_entries, long long max_samples,
                               hipStream_t st) {
  const long long px = (max_samples + kHistPiece - 1) / kHistPiece;
  const int gx = (int)(px < 1 ? 1 : px);
  // entries are strided over gridDim.y; about 4096 blocks in all
  long long gy = 4096 / gx;
  if (gy > max_entries) gy = max_entries;
  if (gy < 1) gy = 1;
  hipLaunchKernelGGL(ppf_history_desc_kernel, dim3(gx, (unsigned)gy), dim3(256), 0, st, count, h);
  return hipGetLastError();
}

hipError_t launch_twiddles(void* tw, int N, hipStream_t st) {
  const int block = 256;
  const int grid = (N + block - 1) / block;
  hipLaunchKernelGGL(ppf_twiddle_kernel, dim3(grid), dim3(block), 0, st, (v2f*)tw, N);
  return hipGetLastError();
}

hipError_t launch_history(const void* old_hist, const void* chunk, void* new_hist, long long hist_samples,
                          long long chunk_samples, int sample_bytes, hipStream_t st) {
  if (hist_samples <= 0) return hipSuccess;
  const int block = 256;
  const long long grid = (hist_samples + block - 1) / block;
  if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
  switch (sample_bytes) {
    case 8:
      hipLaunchKernelGGL(ppf_history_kernel<uint64_t>, dim3((unsigned)grid), dim3(block), 0, st,
                         (const uint64_t*)old_hist, (const uint64_t*)chunk, (uint64_t*)new_hist, hist_samples,
                         chunk_samples);
      break;
    case 4:
      hipLaunchKernelGGL(ppf_history_kernel<uint32_t>, dim3((unsigned)grid), dim3(block), 0, st,
                         (const uint32_t*)old_hist, (const uint32_t*)chunk, (uint32_t*)new_hist, hist_samples,
                         chunk_samples);
      break;
    case 2:
      hipLaunchKernelGGL(ppf_history_kernel<uint16_t>, dim3((unsigned)grid), dim3(block), 0, st,
                         (const uint16_t*)old_hist, (const uint16_t*)chunk, (uint16_t*)new_hist, hist_samples,
                         chunk_samples);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ppf
