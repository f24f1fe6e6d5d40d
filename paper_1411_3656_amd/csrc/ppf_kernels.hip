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

// LDS word address of element i of a plane. gfx950 LDS has 64 four-byte
// banks serving a whole wave per access. For N >= 256 (one group per wave)
// element i goes to i XOR a mask of its 64-word row that spreads the row
// index over bits 0-5 (row ^ row<<2 ^ row<<4): contiguous reads stay one
// row, and the strided Stockham writes, whose lanes fall in rows with
// different low row bits but fixed low offset bits, land in distinct banks.
// Smaller N (several groups per wave) pad one word per 32 and shift group
// planes by W words.
template <int N>
__device__ __forceinline__ int lds_index(int i) {
  if constexpr (N >= 8192) {
    // plain layout: every stage's addresses are one per-thread base plus
    // immediates, which keeps 16 elements per thread within the registers
    return i;
  } else if constexpr (N >= 256) {
    const int row = i >> 6;
    return i ^ ((row ^ (row << 2) ^ (row << 4)) & 63);
  } else {
    return i + (i >> 5);
  }
}
constexpr int plane_floats(int N, int W) {
  if (N >= 8192) return N;
  if (N >= 256) return N;
  const int p = N + N / 32;
  return W < 32 ? ((p + 31) / 32) * 32 + W : p;
}

// --------------------------------------------------------------------------
// Per-group FFT through LDS
// --------------------------------------------------------------------------

// B spectra go through the stages together: they share every barrier and
// twiddle, and give each wave independent work between barriers.
template <int N, int R, int RX, int G, int B, bool DB, bool TWG>
struct GroupFft {
  static constexpr int W = N / R;
  static constexpr int L = num_stages(N, RX);
  static constexpr int PL = plane_floats(N, W);      // floats per plane
  static constexpr int NBUF = DB ? 2 : 1;
  static constexpr int NTW = TWG ? 1 : (tw_total(N, R, RX) > 0 ? tw_total(N, R, RX) : 1);
  static constexpr size_t lds_bytes() { return size_t(NBUF) * B * 2 * G * PL * sizeof(float); }

  float* lds;      // shared memory base of the block
  int grp, j;
  int par;         // buffer of the next exchange (double-buffered mode)
  const v2f* tw;   // twiddle table (global)
  v2f twr[NTW];

  __device__ __forceinline__ float* plane(int buf, int b, int reim) const {
    return lds + (((buf * B + b) * 2 + reim) * G + grp) * PL;
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
      // read at the point of use: the address is loop-invariant, and a
      // hoisted load would keep every stage's twiddles live in registers;
      // an opaque zero ties the load to this stage
      int z;
      asm volatile("s_mov_b32 %0, 0" : "=s"(z));
      const int k = (j + i * W) % Ns;
      return tw[k * q * (N / (Ns * r)) + z];
    } else {
      const int ib = (Ns <= W) ? 0 : i;
      return twr[tw_offset(N, R, RX, S) + ib * (r - 1) + q - 1];
    }
  }

  template <int S>
  __device__ __forceinline__ void stage(v2f (&v)[B][R]) {
    constexpr int r = radix_at(N, RX, S), Ns = ns_at(N, RX, S);
    constexpr int nb = R / r;
    if constexpr (S > 0) {
      const int buf = DB ? par : 0;
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const float* re = plane(buf, b, 0);
        const float* im = plane(buf, b, 1);
#pragma unroll
        for (int e = 0; e < R; ++e) {
          const int idx = lds_index<N>(j + e * W);
          v[b][e].x = re[idx];
          v[b][e].y = im[idx];
        }
      }
      if constexpr (DB) par ^= 1;
#pragma unroll
      for (int i = 0; i < nb; ++i)
#pragma unroll
        for (int q = 1; q < r; ++q) {
          const v2f w = twiddle<S>(i, q);
#pragma unroll
          for (int b = 0; b < B; ++b) v[b][i + q * nb] = cmul(v[b][i + q * nb], w);
        }
    }
    if constexpr (S == L - 1) {
#pragma unroll
      for (int b = 0; b < B; ++b)
#pragma unroll
        for (int i = 0; i < nb; ++i) {
          v2f t[r];
#pragma unroll
          for (int q = 0; q < r; ++q) t[q] = v[b][i + q * nb];
          dft<r>(t);
#pragma unroll
          for (int q = 0; q < r; ++q) v[b][i + q * nb] = t[q];
        }
    } else {
      if constexpr (!DB) __syncthreads();   // earlier reads of the single buffer are done
      const int buf = DB ? par : 0;
#pragma unroll
      for (int b = 0; b < B; ++b) {
        float* re = plane(buf, b, 0);
        float* im = plane(buf, b, 1);
#pragma unroll
        for (int i = 0; i < nb; ++i) {
          v2f t[r];
#pragma unroll
          for (int q = 0; q < r; ++q) t[q] = v[b][i + q * nb];
          dft<r>(t);
          const int bf = j + i * W;
          const int base = (bf / Ns) * Ns * r + (bf % Ns);
#pragma unroll
          for (int q = 0; q < r; ++q) {
            const int idx = lds_index<N>(base + q * Ns);
            re[idx] = t[q].x;
            im[idx] = t[q].y;
          }
        }
      }
      __syncthreads();
    }
  }

  template <int S>
  __device__ __forceinline__ void run_from(v2f (&v)[B][R]) {
    if constexpr (S < L) {
      stage<S>(v);
      run_from<S + 1>(v);
    }
  }

  // in: v[b][e] = u_b[j + e*W]; out: v[b][e] = X_b[j + e*W]
  __device__ __forceinline__ void run(v2f (&v)[B][R]) { run_from<0>(v); }
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

// Input blocks are streamed with non-temporal loads unless disabled at
// build time (measured faster on MI355X for the one-pass batch).
#ifndef PPF_NT_LOADS
#define PPF_NT_LOADS 1
#endif
constexpr bool kNtLoads = PPF_NT_LOADS != 0;

// Raw buffer access (gfx9 descriptor): a scalar resource per block of N
// samples, a 32-bit per-thread offset, and each element's extra offset as
// a scalar constant. Reads outside the block's range return zero.
constexpr int kBufDword3 = 0x00020000;
constexpr int kAuxNt = 2;   // non-temporal cache policy bit of buffer instructions
__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, bytes, kBufDword3);
}
template <int AUX>
__device__ __forceinline__ v2f buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(v2f, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
}
template <int AUX>
__device__ __forceinline__ void buf_store(v2f v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v),
                                        r, voff, soff, AUX);
}

// Block and spectrum indices of one launch fit in 32 bits (the host splits
// larger batches), so their arithmetic and compares stay on the scalar unit.
struct FusedParams {
  const v2f* x0;       // first input segment (h0 blocks)
  const v2f* x1;       // second input segment
  v2f* out;
  const float* coef;   // TP*N
  const v2f* tw;       // N twiddles
  int h0;
  int M;               // spectra
  int S;               // spectra per group tile
  int d;               // leading zero tap segments (TP - T)
  int nblocks;
};

// One tile of spectra: the input is the concatenation x0 (h0 blocks) ++ x1
// (h01 - h0 blocks) ++ x2, spectrum m of the tile reads blocks m .. m+T-1
// of it and is written to out + m*N.
struct TileArgs {
  const v2f* x0;
  const v2f* x1;
  const v2f* x2;
  v2f* out;
  int h0;
  int h01;
};

template <int N>
__device__ __forceinline__ const v2f* block_ptr(const TileArgs& a, int rb) {
  return rb < a.h0 ? a.x0 + (long long)rb * N
                   : (rb < a.h01 ? a.x1 + (long long)(rb - a.h0) * N : a.x2 + (long long)(rb - a.h01) * N);
}

// Per-block engine of the fused kernel: coefficients, twiddles and lane
// offsets are loaded once and reused by every tile the block processes.
//
// Ring of Q = TP + PF blocks; slot s always holds a block whose index is
// s modulo Q (counted from the tile start). B spectra are computed per
// step; the B blocks loaded at a step replace the B oldest, which no later
// spectrum needs, so any Q >= TP + B - 1 is hazard-free and PF - B + 1
// blocks of each step are loads running ahead.
// UNIT: all coefficients are one (the FFT pass of the two-pass form), so the
// presum is the loaded block itself and no coefficients are held.
template <int N, int R, int RX, int G, int B, int TP, int PF, bool DB, bool TWG, bool UNIT>
struct FusedEngine {
  static constexpr int W = N / R;
  static constexpr int Q = TP + PF;
  static_assert(Q % B == 0 && Q >= TP + B - 1, "ring size");
  static_assert(!UNIT || TP == 1, "unit coefficients are a single tap");
  using Fft = GroupFft<N, R, RX, G, B, DB, TWG>;

  Fft fft;
  int j;
  int d;
  float hreg[UNIT ? 1 : TP][R];
  uint32_t loff;       // byte offset of channel j inside a block; element e adds e*W*8

  __device__ __forceinline__ void init(float* smem, int grp, int j_, const float* coef, const v2f* tw, int d_) {
    j = j_;
    d = d_;
    fft.init(smem, grp, j, tw);
    if constexpr (!UNIT) {
#pragma unroll
      for (int t = 0; t < TP; ++t)
#pragma unroll
        for (int e = 0; e < R; ++e) hreg[t][e] = coef[t * N + j + e * W];
    }
    loff = (uint32_t)j * (uint32_t)sizeof(v2f);
  }

  // Spectra m0 .. m0+ng-1 of the tile; niter >= ng is the same for every
  // group of the block (barriers), extra steps compute but store nothing.
  __device__ __forceinline__ void run(const TileArgs& a, int m0, int ng, int niter) {
    // virtual blocks this group reads: [vb_lo, vb_hi). Below vb_lo the taps
    // are the zero padding; at or above vb_hi only spectra beyond the tile
    // would use them. Those slots are not loaded.
    const int vb_lo = m0 > d ? m0 : d;
    const int vb_hi = ng > 0 ? m0 + ng + TP - 1 : m0;

    // zero start: a slot that is never loaded holds a finite value, so a
    // zero padding tap times it is exactly zero
    v2f ring[Q][R];
#pragma unroll
    for (int s = 0; s < Q; ++s)
#pragma unroll
      for (int e = 0; e < R; ++e) { ring[s][e].x = 0.f; ring[s][e].y = 0.f; }
    auto load = [&](v2f (&dst)[R], int vb) {
      if (vb >= vb_lo && vb < vb_hi) {
        if constexpr (G == 1) {
          const __amdgpu_buffer_rsrc_t rs = block_rsrc(block_ptr<N>(a, vb - d), N * (int)sizeof(v2f));
#pragma unroll
          for (int e = 0; e < R; ++e)
            dst[e] = buf_load<kNtLoads ? kAuxNt : 0>(rs, loff, (uint32_t)(e * W * (int)sizeof(v2f)));
        } else {
          const v2f* src = block_ptr<N>(a, vb - d) + j;
#pragma unroll
          for (int e = 0; e < R; ++e) dst[e] = src[e * W];
        }
      }
    };

#pragma unroll
    for (int s = 0; s < Q - B; ++s) load(ring[s], m0 + s);

    for (int base = 0; base < niter; base += Q) {
#pragma unroll
      for (int k = 0; k < Q; k += B) {
        const int it = base + k;
        if (it >= niter) break;
#pragma unroll
        for (int b = 0; b < B; ++b) load(ring[(k + Q - B + b) % Q], m0 + it + Q - B + b);
        v2f v[B][R];
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
          for (int e = 0; e < R; ++e) {
            if constexpr (UNIT) {
              v[b][e] = ring[(k + b) % Q][e];
            } else {
              v2f acc;
              acc.x = hreg[0][e] * ring[(k + b) % Q][e].x;
              acc.y = hreg[0][e] * ring[(k + b) % Q][e].y;
#pragma unroll
              for (int t = 1; t < TP; ++t) {
                acc.x = fmaf(hreg[t][e], ring[(k + b + t) % Q][e].x, acc.x);
                acc.y = fmaf(hreg[t][e], ring[(k + b + t) % Q][e].y, acc.y);
              }
              v[b][e] = acc;
            }
          }
        fft.run(v);
#pragma unroll
        for (int b = 0; b < B; ++b) {
          if (it + b < ng) {
            if constexpr (G == 1) {
              const __amdgpu_buffer_rsrc_t rs =
                  block_rsrc(a.out + (long long)(m0 + it + b) * N, N * (int)sizeof(v2f));
#pragma unroll
              for (int e = 0; e < R; ++e) buf_store<kAuxNt>(v[b][e], rs, loff, (uint32_t)(e * W * (int)sizeof(v2f)));
            } else {
              v2f* dst = a.out + (long long)(m0 + it + b) * N + j;
#pragma unroll
              for (int e = 0; e < R; ++e) __builtin_nontemporal_store(v[b][e], dst + e * W);
            }
          }
        }
      }
    }
  }
};

// Batch form: a wave of tiles of S consecutive spectra covers the batch;
// group g of block lb owns the tile (lb*G + g).
template <int N, int R, int RX, int G, int B, int TP, int PF, bool DB, bool TWG, bool UNIT>
__global__ void __launch_bounds__((N / R) * G)
ppf_fused_kernel(FusedParams p) {
  constexpr int W = N / R;
  extern __shared__ float smem[];
  const int tid = threadIdx.x;
  const int grp = (G == 1) ? 0 : tid / W;
  const int j = (G == 1) ? tid : tid % W;
  const int lb = xcd_remap(blockIdx.x, p.nblocks);
  const int blk_m0 = lb * G * p.S;
  if (blk_m0 >= p.M) return;                                   // whole block idle
  const int m0 = blk_m0 + grp * p.S;
  const int rem = p.M - m0;
  const int ng = rem <= 0 ? 0 : (rem < p.S ? rem : p.S);       // this group's spectra
  const int brem = p.M - blk_m0;
  const int niter = brem < p.S ? brem : p.S;                   // uniform over the block

  FusedEngine<N, R, RX, G, B, TP, PF, DB, TWG, UNIT> eng;
  eng.init(smem, grp, j, p.coef, p.tw, p.d);
  TileArgs a{p.x0, p.x1, p.x1, p.out, p.h0, p.h0};
  eng.run(a, m0, ng, niter);
}

// Descriptor form (serving): the tiles are listed in device memory; a
// persistent grid walks them, G tiles per block at a time. Every wave of a
// block exits at the same tile index, after the same number of barriers.

template <int N, int R, int RX, int G, int B, int TP, int PF, bool DB, bool TWG, bool UNIT>
__global__ void __launch_bounds__((N / R) * G)
ppf_fused_desc_kernel(const DescClass* cls, const TileDesc* tiles, const float* coef, const v2f* tw, int d) {
  constexpr int W = N / R;
  extern __shared__ float smem[];
  __shared__ int s_count[G];
  const int tid = threadIdx.x;
  const int grp = (G == 1) ? 0 : tid / W;
  const int j = (G == 1) ? tid : tid % W;
  const int first = cls->first;
  const int ntiles = cls->ntiles;
  if ((int)blockIdx.x * G >= ntiles) return;                  // whole block idle
  FusedEngine<N, R, RX, G, B, TP, PF, DB, TWG, UNIT> eng;
  eng.init(smem, grp, j, coef, tw, d);
  for (int t0 = blockIdx.x * G; t0 < ntiles; t0 += gridDim.x * G) {
    const int t = t0 + grp;
    TileArgs a{nullptr, nullptr, nullptr, nullptr, 0, 0};
    int count = 0;
    if (t < ntiles) {
      const TileDesc& td = tiles[first + t];
      a = TileArgs{(const v2f*)td.x0, (const v2f*)td.x1, (const v2f*)td.x2, (v2f*)td.out, td.h0, td.h0 + td.h1};
      count = td.count;
    }
    int niter = count;
    if constexpr (G > 1) {
      if (j == 0) s_count[grp] = count;
      __syncthreads();
      niter = 0;
#pragma unroll
      for (int g = 0; g < G; ++g) niter = s_count[g] > niter ? s_count[g] : niter;
      __syncthreads();
    }
    eng.run(a, 0, count, niter);
  }
}

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

// Stored complex input types, widened to FP32 as they are loaded:
// 0 = complex FP32, 1 = complex FP16, 2 = complex int8 (exact conversions).
template <int IT>
__device__ __forceinline__ v2f load_sample(const void* base, long long i) {
  if constexpr (IT == 0) {
    return ((const v2f*)base)[i];
  } else if constexpr (IT == 1) {
    const uint32_t w = ((const uint32_t*)base)[i];
    _Float16 re, im;
    const uint16_t lo = (uint16_t)(w & 0xFFFFu), hi = (uint16_t)(w >> 16);
    __builtin_memcpy(&re, &lo, 2);
    __builtin_memcpy(&im, &hi, 2);
    v2f r;
    r.x = (float)re;
    r.y = (float)im;
    return r;
  } else {
    const uint16_t w = ((const uint16_t*)base)[i];
    v2f r;
    r.x = (float)(int)(int8_t)(w & 0xFFu);
    r.y = (float)(int)(int8_t)(w >> 8);
    return r;
  }
}

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

// --------------------------------------------------------------------------
// configurations and dispatch
// --------------------------------------------------------------------------

// Build-time override of the prefetch depth of the fused kernels (tuning).
#ifndef PPF_PF_FUSED_OVERRIDE
#define PPF_PF_FUSED_OVERRIDE 0
#endif

// elements per thread R and groups per block G for the FFT of N points
constexpr int cfg_R(int N) { return N <= 1024 ? 4 : (N == 2048 ? 8 : 16); }
constexpr int cfg_RX(int N) { return cfg_R(N) < 16 ? cfg_R(N) : 16; }
constexpr int cfg_W(int N) { return N / cfg_R(N); }
constexpr int cfg_G(int N) { return cfg_W(N) >= 256 ? 1 : 256 / cfg_W(N); }
constexpr int cfg_PF(int N, int TP) {
  return TP == 1 ? (N >= 16384 ? 0 : (N >= 4096 ? 1 : (N >= 2048 ? 2 : 3)))
                 : (N >= 2048 ? 2 : (PPF_PF_FUSED_OVERRIDE > 0 ? PPF_PF_FUSED_OVERRIDE : 4));
}
constexpr bool cfg_TWG(int N) { return N >= 16384; }
// spectra per FFT pass (build-time tuning; 4 measured best at N=1024, T=8)
#ifndef PPF_BATCH_OVERRIDE
#define PPF_BATCH_OVERRIDE 4
#endif
constexpr bool batch_fits(int N, int TP, int B) {
  return (TP + cfg_PF(N, TP)) % B == 0 && TP + cfg_PF(N, TP) >= TP + B - 1;
}
constexpr int cfg_B(int N, int TP) {
  // with 16 taps the ring already fills the register file
  return PPF_BATCH_OVERRIDE > 1 && TP <= 8 && batch_fits(N, TP, PPF_BATCH_OVERRIDE) ? PPF_BATCH_OVERRIDE : 1;
}
constexpr bool cfg_DB(int N, int B) {
  return 2ull * B * 2 * cfg_G(N) * plane_floats(N, cfg_W(N)) * sizeof(float) <= 80 * 1024;
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

template <int N, int TP, bool UNIT>
static const KernelInfo& fused_info() {
  constexpr int R = cfg_R(N), RX = cfg_RX(N), G = cfg_G(N), PF = cfg_PF(N, TP), B = cfg_B(N, TP);
  constexpr bool DB = cfg_DB(N, B), TWG = cfg_TWG(N);
  using Fft = GroupFft<N, R, RX, G, B, DB, TWG>;
  static const KernelInfo ki{(const void*)&ppf_fused_kernel<N, R, RX, G, B, TP, PF, DB, TWG, UNIT>,
                             (N / R) * G, G, Fft::lds_bytes()};
  return ki;
}

// Largest number of spectra in one launch: block and spectrum indices stay
// below 2^31 inside the kernels.
constexpr long long kMaxLaunchSpectra = 1ll << 28;

// Part [s0, s0+k) of a batch: the concatenated input starts at block s0.
static BatchArgs sub_batch(const BatchArgs& a, int N, size_t sample_bytes, long long s0, long long k) {
  BatchArgs o;
  if (s0 < a.h0) {
    o.x0 = (const char*)a.x0 + (size_t)s0 * N * sample_bytes;
    o.h0 = a.h0 - s0;
    o.x1 = a.x1;
  } else {
    o.x0 = a.x1;
    o.h0 = 0;
    o.x1 = (const char*)a.x1 + (size_t)(s0 - a.h0) * N * sample_bytes;
  }
  o.out = (char*)a.out + (size_t)s0 * N * 8;
  o.M = k;
  return o;
}

template <int N, int TP, bool UNIT>
static hipError_t fused_launch_one(const PlanDev& pd, const BatchArgs& a, const float* coef, int T,
                                   hipStream_t st) {
  const KernelInfo& ki = fused_info<N, TP, UNIT>();
  static const int occ = occupancy(ki);
  const long long resident_groups = (long long)device_cus() * occ * ki.G;
  long long S = (a.M + resident_groups - 1) / resident_groups;
  if (S < 2 * TP) S = 2 * TP;                                  // bound the tap-window re-reads
  const long long groups = (a.M + S - 1) / S;
  const long long nblocks = (groups + ki.G - 1) / ki.G;
  if (nblocks <= 0) return hipSuccess;
  FusedParams p;
  p.x0 = (const v2f*)a.x0;
  p.x1 = (const v2f*)a.x1;
  p.out = (v2f*)a.out;
  p.coef = coef;
  p.tw = (const v2f*)pd.tw;
  p.h0 = (int)a.h0;
  p.M = (int)a.M;
  p.S = (int)S;
  p.d = TP - T;
  p.nblocks = (int)nblocks;
  constexpr int R = cfg_R(N), RX = cfg_RX(N), G = cfg_G(N), PF = cfg_PF(N, TP), B = cfg_B(N, TP);
  constexpr bool DB = cfg_DB(N, B), TWG = cfg_TWG(N);
  hipLaunchKernelGGL((ppf_fused_kernel<N, R, RX, G, B, TP, PF, DB, TWG, UNIT>), dim3((unsigned)nblocks), dim3(ki.block),
                     ki.lds, st, p);
  return hipGetLastError();
}

template <int N, int TP, bool UNIT = false>
static hipError_t fused_launch(const PlanDev& pd, const BatchArgs& a, const float* coef, int T, hipStream_t st) {
  for (long long s0 = 0; s0 < a.M; s0 += kMaxLaunchSpectra) {
    const long long k = a.M - s0 < kMaxLaunchSpectra ? a.M - s0 : kMaxLaunchSpectra;
    const hipError_t e = fused_launch_one<N, TP, UNIT>(pd, sub_batch(a, N, 8, s0, k), coef, T, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
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
  return f(pd, a, pd.ones, 1, st);
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
  constexpr int R = cfg_R(N), RX = cfg_RX(N), G = cfg_G(N), PF = cfg_PF(N, TP), B = cfg_B(N, TP);
  constexpr bool DB = cfg_DB(N, B), TWG = cfg_TWG(N);
  using Fft = GroupFft<N, R, RX, G, B, DB, TWG>;
  auto kern = &ppf_fused_desc_kernel<N, R, RX, G, B, TP, PF, DB, TWG, UNIT>;
  static const int occ = [&] {
    KernelInfo ki{(const void*)kern, (N / R) * G, G, Fft::lds_bytes()};
    return occupancy(ki);
  }();
  if (!cls) return hipSuccess;                 // warm-up call: occupancy only
  long long grid = (long long)device_cus() * occ;
  const long long need = (max_tiles + G - 1) / G;
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3((N / R) * G), Fft::lds_bytes(), st, cls, tiles, coef,
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
