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
// re/im planes, padded one word per 32 to spread banks, double-buffered
// when it fits so that one barrier per exchange suffices). Twiddles per
// thread are constant across spectra and are loaded into registers once.
//
// Two-pass form (taps windows too large for registers): a FIR-only kernel
// with a per-thread register ring writes u to a workspace, then the same
// fused kernel with one identity tap performs the FFTs.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ppf_internal.h"

namespace ppf {

typedef float v2f __attribute__((ext_vector_type(2)));

// --------------------------------------------------------------------------
// complex helpers
// --------------------------------------------------------------------------

__device__ __forceinline__ v2f cadd(v2f a, v2f b) { v2f r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
__device__ __forceinline__ v2f csub(v2f a, v2f b) { v2f r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
// a * w (complex)
__device__ __forceinline__ v2f cmul(v2f a, v2f w) {
  v2f r;
  r.x = fmaf(a.x, w.x, -(a.y * w.y));
  r.y = fmaf(a.x, w.y, a.y * w.x);
  return r;
}
// a * (-i)
__device__ __forceinline__ v2f mul_mi(v2f a) { v2f r; r.x = a.y; r.y = -a.x; return r; }
// a * (c - i s) for a compile-time root of unity
__device__ __forceinline__ v2f mul_cs(v2f a, float c, float s) {
  v2f r;
  r.x = fmaf(a.x, c, a.y * s);
  r.y = fmaf(a.y, c, -(a.x * s));
  return r;
}

// exp(-2 pi i p/16) * a for compile-time p (0 <= p < 16)
template <int P>
__device__ __forceinline__ v2f w16(v2f a) {
  constexpr int p = P & 15;
  constexpr float C1 = 0.92387953251128674f;  // cos(pi/8)
  constexpr float S1 = 0.38268343236508978f;  // sin(pi/8)
  constexpr float H = 0.70710678118654752f;   // sqrt(2)/2
  if constexpr (p == 0) return a;
  else if constexpr (p == 4) return mul_mi(a);
  else if constexpr (p == 8) { v2f r; r.x = -a.x; r.y = -a.y; return r; }
  else if constexpr (p == 12) { v2f r; r.x = -a.y; r.y = a.x; return r; }
  else if constexpr (p == 2) { v2f r; r.x = (a.x + a.y) * H; r.y = (a.y - a.x) * H; return r; }
  else if constexpr (p == 6) { v2f r; r.x = (a.y - a.x) * H; r.y = -(a.x + a.y) * H; return r; }
  else if constexpr (p == 10) { v2f r; r.x = -(a.x + a.y) * H; r.y = (a.x - a.y) * H; return r; }
  else if constexpr (p == 14) { v2f r; r.x = (a.x - a.y) * H; r.y = (a.x + a.y) * H; return r; }
  else if constexpr (p == 1) return mul_cs(a, C1, S1);
  else if constexpr (p == 3) return mul_cs(a, S1, C1);
  else if constexpr (p == 5) return mul_cs(a, -S1, C1);
  else if constexpr (p == 7) return mul_cs(a, -C1, S1);
  else if constexpr (p == 9) return mul_cs(a, -C1, -S1);
  else if constexpr (p == 11) return mul_cs(a, -S1, -C1);
  else if constexpr (p == 13) return mul_cs(a, S1, -C1);
  else return mul_cs(a, C1, -S1);  // p == 15
}

// --------------------------------------------------------------------------
// small forward DFTs on registers: a[k] <- sum_n a[n] exp(-2 pi i nk/r)
// --------------------------------------------------------------------------

__device__ __forceinline__ void dft2(v2f& a0, v2f& a1) {
  v2f t = a0;
  a0 = cadd(t, a1);
  a1 = csub(t, a1);
}

__device__ __forceinline__ void dft4(v2f& a0, v2f& a1, v2f& a2, v2f& a3) {
  v2f t0 = cadd(a0, a2), t1 = csub(a0, a2);
  v2f t2 = cadd(a1, a3), t3 = mul_mi(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <int r>
__device__ __forceinline__ void dft(v2f (&a)[r]) {
  if constexpr (r == 1) {
  } else if constexpr (r == 2) {
    dft2(a[0], a[1]);
  } else if constexpr (r == 4) {
    dft4(a[0], a[1], a[2], a[3]);
  } else if constexpr (r == 8) {
    // even/odd split: X[k] = E[k] + W8^k O[k], X[k+4] = E[k] - W8^k O[k]
    dft4(a[0], a[2], a[4], a[6]);
    dft4(a[1], a[3], a[5], a[7]);
    v2f o1 = w16<2>(a[3]), o2 = w16<4>(a[5]), o3 = w16<6>(a[7]);
    v2f e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
    a[0] = cadd(e0, a[1]); a[4] = csub(e0, a[1]);
    a[1] = cadd(e1, o1);   a[5] = csub(e1, o1);
    a[2] = cadd(e2, o2);   a[6] = csub(e2, o2);
    a[3] = cadd(e3, o3);   a[7] = csub(e3, o3);
  } else if constexpr (r == 16) {
    // 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
    v2f y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      v2f b0 = a[n2], b1 = a[4 + n2], b2 = a[8 + n2], b3 = a[12 + n2];
      dft4(b0, b1, b2, b3);
      y[n2][0] = b0; y[n2][1] = b1; y[n2][2] = b2; y[n2][3] = b3;
    }
    y[1][1] = w16<1>(y[1][1]); y[1][2] = w16<2>(y[1][2]); y[1][3] = w16<3>(y[1][3]);
    y[2][1] = w16<2>(y[2][1]); y[2][2] = w16<4>(y[2][2]); y[2][3] = w16<6>(y[2][3]);
    y[3][1] = w16<3>(y[3][1]); y[3][2] = w16<6>(y[3][2]); y[3][3] = w16<9>(y[3][3]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      v2f b0 = y[0][k1], b1 = y[1][k1], b2 = y[2][k1], b3 = y[3][k1];
      dft4(b0, b1, b2, b3);
      a[k1] = b0; a[k1 + 4] = b1; a[k1 + 8] = b2; a[k1 + 12] = b3;
    }
  } else {
    static_assert(r == 1 || r == 2 || r == 4 || r == 8 || r == 16, "unsupported radix");
  }
}

// --------------------------------------------------------------------------
// Stockham stage plan (compile time). Stage s has radix r_s (R while R
// points remain, then the power-of-two remainder) and span Ns = prod r_<s.
// Butterfly b (0 <= b < N/r) reads elements b + q*N/r and writes
// (b/Ns)*Ns*r + b%Ns + q*Ns after the twiddle exp(-2 pi i (b%Ns) q/(Ns r)).
// --------------------------------------------------------------------------

// RX is the largest radix used (a divisor of R); a thread holding R
// elements performs R/r butterflies of radix r per stage.
constexpr int radix_at(int N, int RX, int s) {
  int n = 1;
  for (int i = 0; i < s; ++i) n *= (N / n >= RX ? RX : N / n);
  return N / n >= RX ? RX : N / n;
}
constexpr int ns_at(int N, int RX, int s) {
  int n = 1;
  for (int i = 0; i < s; ++i) n *= radix_at(N, RX, i);
  return n;
}
constexpr int num_stages(int N, int RX) {
  int n = 1, s = 0;
  while (n < N) { n *= (N / n >= RX ? RX : N / n); ++s; }
  return s;
}
// twiddles a thread keeps for stage s: butterflies j + i*W share b % Ns
// when Ns <= W, so one set serves all of them
constexpr int tw_count(int N, int R, int RX, int s) {
  if (s == 0) return 0;
  const int r = radix_at(N, RX, s), Ns = ns_at(N, RX, s), W = N / R;
  return (Ns <= W ? 1 : R / r) * (r - 1);
}
constexpr int tw_offset(int N, int R, int RX, int s) {
  int o = 0;
  for (int i = 0; i < s; ++i) o += tw_count(N, R, RX, i);
  return o;
}
constexpr int tw_total(int N, int R, int RX) { return tw_offset(N, R, RX, num_stages(N, RX)); }

// LDS plane: N floats padded one word per 32, rounded so that groups that
// share a wave start on distinct bank offsets.
__device__ __forceinline__ int pad32(int i) { return i + (i >> 5); }
constexpr int plane_floats(int N, int W) {
  const int p = N + N / 32;
  return W < 32 ? ((p + 31) / 32) * 32 + W : p;
}

// --------------------------------------------------------------------------
// Per-group FFT through LDS
// --------------------------------------------------------------------------

template <int N, int R, int RX, int G, bool DB, bool TWG>
struct GroupFft {
  static constexpr int W = N / R;
  static constexpr int L = num_stages(N, RX);
  static constexpr int PL = plane_floats(N, W);      // floats per plane
  static constexpr int NBUF = DB ? 2 : 1;
  static constexpr int NTW = TWG ? 1 : (tw_total(N, R, RX) > 0 ? tw_total(N, R, RX) : 1);
  static constexpr size_t lds_bytes() { return size_t(NBUF) * 2 * G * PL * sizeof(float); }

  float* lds;      // shared memory base of the block
  int grp, j;
  int par;         // buffer of the next exchange (double-buffered mode)
  const v2f* tw;   // twiddle table (global)
  v2f twr[NTW];

  __device__ __forceinline__ float* plane(int buf, int reim) const {
    return lds + ((buf * 2 + reim) * G + grp) * PL;
  }

  template <int S>
  __device__ __forceinline__ void load_stage_tw() {
    if constexpr (S < L) {
      if constexpr (S > 0) {
        constexpr int r = radix_at(N, RX, S), Ns = ns_at(N, RX, S);
        constexpr int nset = (Ns <= W) ? 1 : R / r;
        constexpr int off = tw_offset(N, R, RX, S);
        constexpr int step = N / (Ns * r);
#pragma unroll
        for (int ib = 0; ib < nset; ++ib) {
          const int k = (j + ib * W) % Ns;
#pragma unroll
          for (int q = 1; q < r; ++q) twr[off + ib * (r - 1) + q - 1] = tw[k * q * step];
        }
      }
      load_stage_tw<S + 1>();
    }
  }

  __device__ __forceinline__ void init(float* smem, int grp_, int j_, const v2f* tw_) {
    lds = smem; grp = grp_; j = j_; par = 0; tw = tw_;
    if constexpr (!TWG) load_stage_tw<1>();
  }

  template <int S>
  __device__ __forceinline__ v2f twiddle(int i, int q) const {
    constexpr int r = radix_at(N, RX, S), Ns = ns_at(N, RX, S);
    if constexpr (TWG) {
      const int k = (j + i * W) % Ns;
      return tw[k * q * (N / (Ns * r))];
    } else {
      const int ib = (Ns <= W) ? 0 : i;
      return twr[tw_offset(N, R, RX, S) + ib * (r - 1) + q - 1];
    }
  }

  template <int S>
  __device__ __forceinline__ void stage(v2f (&v)[R]) {
    constexpr int r = radix_at(N, RX, S), Ns = ns_at(N, RX, S);
    constexpr int nb = R / r;
    if constexpr (S > 0) {
      const int b = DB ? par : 0;
      const float* re = plane(b, 0);
      const float* im = plane(b, 1);
#pragma unroll
      for (int e = 0; e < R; ++e) {
        const int idx = pad32(j + e * W);
        v[e].x = re[idx];
        v[e].y = im[idx];
      }
      if constexpr (DB) par ^= 1;
#pragma unroll
      for (int i = 0; i < nb; ++i)
#pragma unroll
        for (int q = 1; q < r; ++q) v[i + q * nb] = cmul(v[i + q * nb], twiddle<S>(i, q));
    }
    if constexpr (S == L - 1) {
#pragma unroll
      for (int i = 0; i < nb; ++i) {
        v2f t[r];
#pragma unroll
        for (int q = 0; q < r; ++q) t[q] = v[i + q * nb];
        dft<r>(t);
#pragma unroll
        for (int q = 0; q < r; ++q) v[i + q * nb] = t[q];
      }
    } else {
      if constexpr (!DB) __syncthreads();   // earlier reads of the single buffer are done
      const int b = DB ? par : 0;
      float* re = plane(b, 0);
      float* im = plane(b, 1);
#pragma unroll
      for (int i = 0; i < nb; ++i) {
        v2f t[r];
#pragma unroll
        for (int q = 0; q < r; ++q) t[q] = v[i + q * nb];
        dft<r>(t);
        const int bf = j + i * W;
        const int base = (bf / Ns) * Ns * r + (bf % Ns);
#pragma unroll
        for (int q = 0; q < r; ++q) {
          const int idx = pad32(base + q * Ns);
          re[idx] = t[q].x;
          im[idx] = t[q].y;
        }
      }
      __syncthreads();
    }
  }

  template <int S>
  __device__ __forceinline__ void run_from(v2f (&v)[R]) {
    if constexpr (S < L) {
      stage<S>(v);
      run_from<S + 1>(v);
    }
  }

  // in: v[e] = u[j + e*W]; out: v[e] = X[j + e*W]
  __device__ __forceinline__ void run(v2f (&v)[R]) { run_from<0>(v); }
};

// --------------------------------------------------------------------------
// block index -> tile: hardware hands consecutive workgroups to the 8 XCDs
// in turn; give each XCD a contiguous range of tiles so neighbouring tiles,
// which share tap-window blocks, meet in the same L2.
// --------------------------------------------------------------------------

__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int q = nblocks >> 3, rem = nblocks & 7;
  const int xcd = bid & 7, k = bid >> 3;
  return xcd * q + (xcd < rem ? xcd : rem) + k;
}

// --------------------------------------------------------------------------
// fused FIR + FFT kernel
// --------------------------------------------------------------------------

struct FusedParams {
  const v2f* x0;       // first input segment (h0 blocks)
  const v2f* x1;       // second input segment
  long long h0;
  v2f* out;
  const float* coef;   // TP*N
  const v2f* tw;       // N twiddles
  long long M;         // spectra
  int S;               // spectra per group tile
  int d;               // leading zero tap segments (TP - T)
  int nblocks;
};

template <int N>
__device__ __forceinline__ const v2f* block_ptr(const FusedParams& p, long long rb) {
  return rb < p.h0 ? p.x0 + rb * N : p.x1 + (rb - p.h0) * N;
}

template <int N, int R, int RX, int G, int TP, int PF, bool DB, bool TWG>
__global__ void __launch_bounds__((N / R) * G)
ppf_fused_kernel(FusedParams p) {
  constexpr int W = N / R;
  constexpr int Q = TP + PF;
  using Fft = GroupFft<N, R, RX, G, DB, TWG>;
  extern __shared__ float smem[];

  const int tid = threadIdx.x;
  const int grp = (G == 1) ? 0 : tid / W;
  const int j = (G == 1) ? tid : tid % W;
  const int lb = xcd_remap(blockIdx.x, p.nblocks);
  const long long blk_m0 = (long long)lb * G * p.S;
  if (blk_m0 >= p.M) return;                                   // whole block idle
  const long long m0 = blk_m0 + (long long)grp * p.S;
  const long long rem = p.M - m0;
  const int ng = rem <= 0 ? 0 : (rem < p.S ? (int)rem : p.S);  // this group's spectra
  const long long brem = p.M - blk_m0;
  const int niter = brem < p.S ? (int)brem : p.S;              // uniform over the block
  // virtual blocks this group reads: [m0, vb_end); none for an idle group
  const long long vb_end = ng > 0 ? m0 + ng + TP - 1 : m0;

  Fft fft;
  fft.init(smem, grp, j, p.tw);

  float hreg[TP][R];
#pragma unroll
  for (int t = 0; t < TP; ++t)
#pragma unroll
    for (int e = 0; e < R; ++e) hreg[t][e] = p.coef[t * N + j + e * W];

  v2f ring[Q][R];
  auto load = [&](v2f (&dst)[R], long long vb) {
    const long long rb = vb - p.d;
    if (vb < vb_end && rb >= 0) {
      const v2f* src = block_ptr<N>(p, rb) + j;
#pragma unroll
      for (int e = 0; e < R; ++e) dst[e] = src[e * W];
    } else {
#pragma unroll
      for (int e = 0; e < R; ++e) { dst[e].x = 0.f; dst[e].y = 0.f; }
    }
  };

#pragma unroll
  for (int s = 0; s < Q - 1; ++s) load(ring[s], m0 + s);

  v2f* outg = p.out + m0 * N + j;
  for (int base = 0; base < niter; base += Q) {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int it = base + k;
      if (it >= niter) break;
      load(ring[(k + Q - 1) % Q], m0 + it + Q - 1);
      v2f v[R];
#pragma unroll
      for (int e = 0; e < R; ++e) {
        v2f a;
        a.x = hreg[0][e] * ring[k % Q][e].x;
        a.y = hreg[0][e] * ring[k % Q][e].y;
#pragma unroll
        for (int t = 1; t < TP; ++t) {
          a.x = fmaf(hreg[t][e], ring[(k + t) % Q][e].x, a.x);
          a.y = fmaf(hreg[t][e], ring[(k + t) % Q][e].y, a.y);
        }
        v[e] = a;
      }
      fft.run(v);
      if (it < ng) {
        v2f* dst = outg + (long long)it * N;
#pragma unroll
        for (int e = 0; e < R; ++e) __builtin_nontemporal_store(v[e], dst + e * W);
      }
    }
  }
}

// --------------------------------------------------------------------------
// FIR-only kernel (two-pass form): one channel per thread, register ring
// --------------------------------------------------------------------------

struct FirParams {
  const v2f* x0;
  const v2f* x1;
  long long h0;
  v2f* out;            // u, M*N
  const float* coef;   // TP*N
  long long M;
  int N;
  int S;
  int d;
  int pad_;
};

template <int TP, int PF>
__global__ void __launch_bounds__(256) ppf_fir_kernel(FirParams p) {
  constexpr int Q = TP + PF;
  const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
  const int c = (int)(g & (p.N - 1));
  const long long m0 = (g / p.N) * p.S;
  if (m0 >= p.M) return;
  const long long rem = p.M - m0;
  const int ng = rem < p.S ? (int)rem : p.S;
  const long long vb_end = m0 + ng + TP - 1;

  float hreg[TP];
#pragma unroll
  for (int t = 0; t < TP; ++t) hreg[t] = p.coef[(long long)t * p.N + c];

  v2f ring[Q];
  auto load = [&](v2f& dst, long long vb) {
    const long long rb = vb - p.d;
    if (vb < vb_end && rb >= 0) {
      dst = rb < p.h0 ? p.x0[rb * p.N + c] : p.x1[(rb - p.h0) * p.N + c];
    } else {
      dst.x = 0.f; dst.y = 0.f;
    }
  };
#pragma unroll
  for (int s = 0; s < Q - 1; ++s) load(ring[s], m0 + s);

  v2f* outg = p.out + m0 * p.N + c;
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

// --------------------------------------------------------------------------
// configurations and dispatch
// --------------------------------------------------------------------------

// elements per thread R and groups per block G for the FFT of N points
constexpr int cfg_R(int N) { return N <= 1024 ? 4 : (N == 2048 ? 8 : (N <= 8192 ? 16 : 32)); }
constexpr int cfg_RX(int N) { return cfg_R(N) < 16 ? cfg_R(N) : 16; }
constexpr int cfg_W(int N) { return N / cfg_R(N); }
constexpr int cfg_G(int N) { return cfg_W(N) >= 256 ? 1 : 256 / cfg_W(N); }
constexpr int cfg_PF(int N, int TP) {
  return TP == 1 ? (N >= 16384 ? 0 : (N >= 4096 ? 1 : (N >= 2048 ? 2 : 3))) : (N >= 2048 ? 2 : 4);
}
constexpr bool cfg_TWG(int N) { return N >= 16384; }
constexpr bool cfg_DB(int N) {
  return 2ull * 2 * cfg_G(N) * plane_floats(N, cfg_W(N)) * sizeof(float) <= 80 * 1024;
}

struct KernelInfo {
  const void* fn;
  int block;
  int G;
  size_t lds;
};

static int device_cus() {
  static const int cus = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    return n;
  }();
  return cus;
}

static int occupancy(const KernelInfo& ki) {
  int occ = 0;
  if (ki.lds > 64 * 1024) hipFuncSetAttribute(ki.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ki.lds);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, ki.fn, ki.block, ki.lds) != hipSuccess || occ <= 0) occ = 1;
  return occ;
}

template <int N, int TP>
static const KernelInfo& fused_info() {
  constexpr int R = cfg_R(N), RX = cfg_RX(N), G = cfg_G(N), PF = cfg_PF(N, TP);
  constexpr bool DB = cfg_DB(N), TWG = cfg_TWG(N);
  using Fft = GroupFft<N, R, RX, G, DB, TWG>;
  static const KernelInfo ki{(const void*)&ppf_fused_kernel<N, R, RX, G, TP, PF, DB, TWG>,
                             (N / R) * G, G, Fft::lds_bytes()};
  return ki;
}

template <int N, int TP>
static hipError_t fused_launch(const PlanDev& pd, const BatchArgs& a, const float* coef, int T, hipStream_t st) {
  const KernelInfo& ki = fused_info<N, TP>();
  static const int occ = occupancy(ki);
  const long long resident_groups = (long long)device_cus() * occ * ki.G;
  long long S = (a.M + resident_groups - 1) / resident_groups;
  if (S < 2 * TP) S = 2 * TP;                                  // bound the tap-window re-reads
  if (S > (1 << 30)) S = 1 << 30;
  const long long groups = (a.M + S - 1) / S;
  const long long nblocks = (groups + ki.G - 1) / ki.G;
  if (nblocks <= 0) return hipSuccess;
  if (nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
  FusedParams p;
  p.x0 = (const v2f*)a.x0;
  p.x1 = (const v2f*)a.x1;
  p.h0 = a.h0;
  p.out = (v2f*)a.out;
  p.coef = coef;
  p.tw = (const v2f*)pd.tw;
  p.M = a.M;
  p.S = (int)S;
  p.d = TP - T;
  p.nblocks = (int)nblocks;
  constexpr int R = cfg_R(N), RX = cfg_RX(N), G = cfg_G(N), PF = cfg_PF(N, TP);
  constexpr bool DB = cfg_DB(N), TWG = cfg_TWG(N);
  hipLaunchKernelGGL((ppf_fused_kernel<N, R, RX, G, TP, PF, DB, TWG>), dim3((unsigned)nblocks), dim3(ki.block),
                     ki.lds, st, p);
  return hipGetLastError();
}

typedef hipError_t (*FusedFn)(const PlanDev&, const BatchArgs&, const float*, int, hipStream_t);

// The fused path exists where the tap window of a thread (R channels x TP
// taps, plus coefficients) fits the register file at useful occupancy.
constexpr bool fused_ok(int N, int TP) {
  return TP == 1 || (N <= 1024 && TP <= 16) || (N == 2048 && TP <= 8);
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
  FusedFn f = fused_fn(pd.N, pd.TP);
  if (!f) return hipErrorInvalidValue;
  return f(pd, a, pd.coef, pd.T, st);
}

hipError_t launch_fft(const PlanDev& pd, const void* in, void* out, long long M, hipStream_t st) {
  FusedFn f = fused_fn(pd.N, 1);
  if (!f) return hipErrorInvalidValue;
  BatchArgs a{in, in, 0, out, M};
  return f(pd, a, pd.ones, 1, st);
}

template <int TP>
static hipError_t fir_launch(const PlanDev& pd, const BatchArgs& a, hipStream_t st) {
  constexpr int PF = TP >= 32 ? 2 : 4;
  static const int occ = [] {
    KernelInfo ki{(const void*)&ppf_fir_kernel<TP, PF>, 256, 1, 0};
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
  FirParams p;
  p.x0 = (const v2f*)a.x0;
  p.x1 = (const v2f*)a.x1;
  p.h0 = a.h0;
  p.out = (v2f*)a.out;
  p.coef = pd.coef;
  p.M = a.M;
  p.N = pd.N;
  p.S = (int)S;
  p.d = TP - pd.T;
  p.pad_ = 0;
  hipLaunchKernelGGL((ppf_fir_kernel<TP, PF>), dim3((unsigned)nblocks), dim3(256), 0, st, p);
  return hipGetLastError();
}

bool fir_available(int TP) {
  return TP == 1 || TP == 2 || TP == 4 || TP == 8 || TP == 16 || TP == 32 || TP == 64;
}

hipError_t launch_fir(const PlanDev& pd, const BatchArgs& a, hipStream_t st) {
  switch (pd.TP) {
    case 1: return fir_launch<1>(pd, a, st);
    case 2: return fir_launch<2>(pd, a, st);
    case 4: return fir_launch<4>(pd, a, st);
    case 8: return fir_launch<8>(pd, a, st);
    case 16: return fir_launch<16>(pd, a, st);
    case 32: return fir_launch<32>(pd, a, st);
    case 64: return fir_launch<64>(pd, a, st);
    default: return hipErrorInvalidValue;
  }
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
