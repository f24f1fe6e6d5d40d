// Two-pass form for large N as a four-step transform (N = N1 * N2).
//
// With c = n2 + N2 n1 and k = k1 + N1 k2 the DFT of the presum splits into
//   X[k1 + N1 k2] = sum_n2 W_N2^(n2 k2) [ W_N^(n2 k1) sum_n1 W_N1^(n1 k1) u[n2 + N2 n1] ]:
// pass A applies the FIR (section 2, Eq. 1) to the N1 channels n2 + N2 n1 of
// a column n2, takes their N1-point DFT over n1, multiplies by W_N^(n2 k1)
// and writes the column as row n2 of a workspace Z[n2][k1]; pass B takes,
// for each k1, the N2-point DFT over n2 of Z[.][k1] and writes X[k1 + N1 k2].
// Each workgroup handles 16 neighbouring columns over a tile of spectra,
// so both passes read and write 128-byte runs, hold 16 small transforms in
// LDS (tens of KiB instead of the whole spectrum) and keep several
// workgroups per CU in flight. Traffic is that of the two-pass form: the
// presums make one round trip through the workspace.
//
// Lane (grp, j) of a workgroup (grp = tid % G, j = tid / G, G = 16) owns
// column col = col0 + grp and elements j + W e (e < 4, W = ND / 4) of its
// ND-point transform, which is the layout of the group FFT (grp selects
// its plane). A group's lanes are spread over every wavefront of the
// workgroup, so its exchanges take block barriers.
// Pass A, like the fused kernels, keeps a ring of TP + PF input blocks and
// the TP coefficients of its 4 channels in registers.

#include "ppf_engine.h"

namespace ppf {

struct FsParams {
  const v2f* x0;      // pass A: input segments x0 (h0 blocks) ++ x1; pass B: the workspace Z
  const v2f* x1;
  v2f* out;           // pass A: Z; pass B: spectra
  const float* coef;  // pass A: TP * N coefficients, zero-padded at the front
  const v2f* twd;     // ND twiddles exp(-2 pi i k / ND) of the pass's transform
  const v2f* twn;     // pass A: N twiddles exp(-2 pi i k / N)
  int h0;
  int M;              // spectra of this launch
  int S;              // spectra per tile
  int d;              // leading zero tap segments (TP - T)
};

constexpr int kFsR = 4;       // elements per lane
// columns per workgroup: 16, so that every access is a run of 128 bytes
// (whole cache lines; 8 columns, 64-byte runs, measured 1.6x slower; 32
// columns in pass B, 1024-thread workgroups, 11% slower)
#ifndef PPF_FS_COLS
#define PPF_FS_COLS 16
#endif
#ifndef PPF_FS_COLS_B
#define PPF_FS_COLS_B 16
#endif
constexpr int kFsG = PPF_FS_COLS;
constexpr int kFsGB = PPF_FS_COLS_B;

// A = pass A (ND = N1, other factor NO = N2); otherwise pass B (ND = N2,
// NO = N1). Both read element (col, j + W e) of spectrum m at
// m N + col + NO (j + W e).
template <int N, int ND, int TP, int PF, bool A>
struct FsEngine {
  static constexpr int R = kFsR, G = A ? kFsG : kFsGB, W = ND / R, NO = N / ND;
  static constexpr int Q = TP + PF;
  static constexpr bool DB = 2ull * 2 * G * plane_floats(ND, W) * sizeof(float) <= 64 * 1024;
  using Fft = GroupFft<ND, R, R, G, 1, DB, false, false>;
  // pass A hands its output rows over through LDS (row stride ND + 1
  // elements: the lanes of one write are 16 different rows)
  static constexpr size_t xpose_bytes() { return A ? (size_t)G * (ND + 1) * sizeof(v2f) : 0; }
  static constexpr size_t lds_bytes() { return Fft::lds_bytes() > xpose_bytes() ? Fft::lds_bytes() : xpose_bytes(); }
  static_assert(A || TP == 1, "pass B has no FIR");
  static_assert(!A || W == 32, "pass A's row hand-over assumes 32 lanes per row");

  Fft fft;
  v2f* xl;                     // pass A: the hand-over rows (aliases the FFT planes)
  int grp, j, col, col0_;
  float hreg[A ? TP : 1][R];
  v2f twc[A ? R : 1];          // pass A: W_N^(col k1), k1 = j + W e
  uint32_t loff;               // lane byte offset of element 0 in a block
  uint32_t soff;               // lane byte offset of element 0 in an output block

  __device__ __forceinline__ void init(float* smem, const FsParams& p, int col0) {
    const int tid = threadIdx.x;
    grp = tid % G;
    j = tid / G;
    col = col0 + grp;
    col0_ = col0;
    xl = (v2f*)smem;
    fft.init(smem, grp, j, p.twd);
    loff = (uint32_t)(col + NO * j) * 8u;
    // pass A stores whole rows: lane tid writes row col0 + tid / 32,
    // elements tid % 32 + 32 e
    soff = A ? (uint32_t)((col0 + tid / 32) * ND + tid % 32) * 8u : (uint32_t)(col + NO * j) * 8u;
    if constexpr (A) {
#pragma unroll
      for (int t = 0; t < TP; ++t)
#pragma unroll
        for (int e = 0; e < R; ++e) hreg[t][e] = p.coef[(long long)t * N + col + NO * (j + W * e)];
#pragma unroll
      for (int e = 0; e < R; ++e) twc[e] = p.twn[(col * (j + W * e)) & (N - 1)];
    }
  }

  __device__ __forceinline__ const v2f* block_ptr(const FsParams& p, int rb) const {
    return rb < p.h0 ? p.x0 + (long long)rb * N : p.x1 + (long long)(rb - p.h0) * N;
  }

  // spectra m0 .. m0+ng-1 (the whole workgroup works on the same spectra)
  __device__ __forceinline__ void run(const FsParams& p, int m0, int ng) {
    const int vb_lo = m0 > p.d ? m0 : p.d;
    const int vb_hi = m0 + ng + TP - 1;
    v2f ring[Q][R];
#pragma unroll
    for (int s = 0; s < Q; ++s)
#pragma unroll
      for (int e = 0; e < R; ++e) { ring[s][e].x = 0.f; ring[s][e].y = 0.f; }
    // a block outside [vb_lo, vb_hi) gets an empty range and reads zeros
    auto load = [&](v2f (&dst)[R], int vb) {
      const bool ok = vb >= vb_lo && vb < vb_hi;
      const __amdgpu_buffer_rsrc_t rs = block_rsrc(block_ptr(p, ok ? vb - p.d : 0), ok ? N * 8 : 0);
#pragma unroll
      for (int e = 0; e < R; ++e)
        dst[e] = buf_load<kNtLoads ? kAuxNt : 0>(rs, loff, (uint32_t)(e * W * NO * 8));
    };
#pragma unroll
    for (int s = 0; s < Q - 1; ++s) load(ring[s], m0 + s);
    for (int base = 0; base < ng; base += Q) {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const int it = base + k;
        if (it >= ng) break;
        load(ring[(k + Q - 1) % Q], m0 + it + Q - 1);
        v2f v[1][R];
#pragma unroll
        for (int e = 0; e < R; ++e) {
          if constexpr (A) {
            v2f acc;
            acc.x = hreg[0][e] * ring[k % Q][e].x;
            acc.y = hreg[0][e] * ring[k % Q][e].y;
#pragma unroll
            for (int t = 1; t < TP; ++t) {
              acc.x = fmaf(hreg[t][e], ring[(k + t) % Q][e].x, acc.x);
              acc.y = fmaf(hreg[t][e], ring[(k + t) % Q][e].y, acc.y);
            }
            v[0][e] = acc;
          } else {
            v[0][e] = ring[k % Q][e];
          }
        }
        fft.run(v);
        const __amdgpu_buffer_rsrc_t rs = block_rsrc(p.out + (long long)(m0 + it) * N, N * 8);
        if constexpr (A) {
          __syncthreads();                       // the planes are free
#pragma unroll
          for (int e = 0; e < R; ++e) xl[grp * (ND + 1) + j + W * e] = cmul(v[0][e], twc[e]);
          __syncthreads();
          const int r = threadIdx.x / 32, kk = threadIdx.x % 32;
#pragma unroll
          for (int e = 0; e < R; ++e)
            buf_store<kAuxNt>(xl[r * (ND + 1) + kk + 32 * e], rs, soff, (uint32_t)(e * 32 * 8));
          __syncthreads();                       // before the next transform's writes
        } else {
#pragma unroll
          for (int e = 0; e < R; ++e) buf_store<kAuxNt>(v[0][e], rs, soff, (uint32_t)(e * W * NO * 8));
        }
      }
    }
  }
};

template <int N, int ND, int TP, int PF, bool A>
__global__ void __launch_bounds__((A ? kFsG : kFsGB) * ND / kFsR) ppf_fs_kernel(FsParams p) {
  extern __shared__ float smem[];
  constexpr int NO = N / ND;
  const int col0 = (int)blockIdx.x * (A ? kFsG : kFsGB);
  const int m0 = (int)blockIdx.y * p.S;
  if (m0 >= p.M || col0 >= NO) return;
  const int rem = p.M - m0;
  const int ng = rem < p.S ? rem : p.S;
  FsEngine<N, ND, TP, PF, A> eng;
  eng.init(smem, p, col0);
  eng.run(p, m0, ng);
}

namespace {

// N1 (pass A's transform over n1) and N2 (pass B's over n2)
constexpr int fs_n1(int N) { return 128; }
constexpr int fs_n2(int N) { return N / 128; }

template <int N, int ND, int TP, int PF, bool A>
hipError_t fs_launch(const FsParams& p0, long long M, hipStream_t st) {
  using Eng = FsEngine<N, ND, TP, PF, A>;
  auto kern = &ppf_fs_kernel<N, ND, TP, PF, A>;
  constexpr int threads = Eng::G * ND / kFsR;
  constexpr int cols = (N / ND) / Eng::G;     // workgroups across the columns
  static const int occ = [&] {
    KernelInfo ki{(const void*)kern, threads, 1, Eng::lds_bytes()};
    return occupancy(ki);
  }();
  if (M <= 0) return hipSuccess;
  // tiles: enough workgroups to fill every CU's resident slots, none
  // shorter than the tap count
  const long long resident = (long long)device_cus() * occ;
  long long tiles = (resident + cols - 1) / cols;
  long long S = (M + tiles - 1) / tiles;
  if (S < TP) S = TP;
  tiles = (M + S - 1) / S;
  FsParams p = p0;
  p.M = (int)M;
  p.S = (int)S;
  hipLaunchKernelGGL(kern, dim3((unsigned)cols, (unsigned)tiles), dim3(threads), Eng::lds_bytes(), st, p);
  return hipGetLastError();
}

// prefetch depths of the two passes (build-time tuning)
#ifndef PPF_FS_PFA
#define PPF_FS_PFA 2
#endif
#ifndef PPF_FS_PFB
#define PPF_FS_PFB 6
#endif

template <int N>
hipError_t fs_pass_a(const FsParams& p, int TP, long long M, hipStream_t st) {
  constexpr int N1 = fs_n1(N);
  switch (TP) {
    case 1: return fs_launch<N, N1, 1, PPF_FS_PFA, true>(p, M, st);
    case 2: return fs_launch<N, N1, 2, PPF_FS_PFA, true>(p, M, st);
    case 4: return fs_launch<N, N1, 4, PPF_FS_PFA, true>(p, M, st);
    case 8: return fs_launch<N, N1, 8, PPF_FS_PFA, true>(p, M, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// Build-time switch (tuning): 0 keeps N = 8192 and 16384 on the FIR-pass /
// whole-spectrum FFT-pass form.
#ifndef PPF_FOURSTEP
#define PPF_FOURSTEP 1
#endif
bool fourstep_available(int N, int TP) { return PPF_FOURSTEP && (N == 8192 || N == 16384) && TP <= 8; }
int fourstep_n1(int N) { return fs_n1(N); }
int fourstep_n2(int N) { return fs_n2(N); }

hipError_t launch_fourstep_a(const PlanDev& pd, const BatchArgs& a, const void* tw_n1, hipStream_t st) {
  FsParams p{};
  p.x0 = (const v2f*)a.x0;
  p.x1 = (const v2f*)a.x1;
  p.h0 = (int)a.h0;
  p.out = (v2f*)a.out;
  p.coef = pd.coef;
  p.twd = (const v2f*)tw_n1;
  p.twn = (const v2f*)pd.tw;
  p.d = pd.TP - pd.T;
  switch (pd.N) {
    case 8192: return fs_pass_a<8192>(p, pd.TP, a.M, st);
    case 16384: return fs_pass_a<16384>(p, pd.TP, a.M, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fourstep_b(const PlanDev& pd, const void* ws, void* out, long long M, const void* tw_n2,
                             hipStream_t st) {
  FsParams p{};
  p.x0 = (const v2f*)ws;
  p.x1 = (const v2f*)ws;
  p.h0 = 0;
  p.out = (v2f*)out;
  p.twd = (const v2f*)tw_n2;
  p.d = 0;
  switch (pd.N) {
    case 8192: return fs_launch<8192, fs_n2(8192), 1, PPF_FS_PFB, false>(p, M, st);
    case 16384: return fs_launch<16384, fs_n2(16384), 1, PPF_FS_PFB, false>(p, M, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ppf
