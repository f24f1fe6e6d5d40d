// Shared engine of the FP32 PPF kernels for CDNA4 (gfx950): complex
// helpers, the per-group Stockham FFT through LDS, the fused FIR + FFT
// engine and its batch and descriptor kernels, and the launch
// configuration. Included by the translation units that instantiate
// them (spectra out; detected power out).
#pragma once

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
// Table-twiddle mode (TWG) with TWR: stages whose butterflies share one set
// (Ns <= W) keep it in registers; the others read theirs from the table per
// stage.
constexpr int tw_count_twg(int N, int R, int RX, int s) {
  if (s == 0) return 0;
  return ns_at(N, RX, s) <= N / R ? radix_at(N, RX, s) - 1 : 0;
}
constexpr int tw_offset_twg(int N, int R, int RX, int s) {
  int o = 0;
  for (int i = 0; i < s; ++i) o += tw_count_twg(N, R, RX, i);
  return o;
}

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
// Interleaved exchange layout (N in 256..PPF_LDS_B64_MAX_N): each element
// is one (re, im) pair, so an exchange moves 8 bytes per lane and
// instruction (ds_write_b64 / ds_read_b64, measured 1.35x / 1.7x the bytes
// per clock of 4-byte accesses on gfx950). Element i is stored at
// i ^ f(i >> 5), f linear over GF(2) on the four low bits of the 32-element
// row; the masks were found by enumerating every stage's reads and writes
// of every configuration with N >= 256 (radix 4, 8 and 16 Stockham stages,
// 1..4 groups per block): within each half-wave of 32 lanes the 8-byte
// slots are then distinct modulo 32, i.e. no bank conflicts.
#ifndef PPF_LDS_B64
#define PPF_LDS_B64 1
#endif
#ifndef PPF_LDS_B64_MAX_N
#define PPF_LDS_B64_MAX_N 16384
#endif
constexpr bool lds_b64(int N) { return PPF_LDS_B64 && N >= 256 && N <= PPF_LDS_B64_MAX_N; }
__device__ __forceinline__ int swz64(int i) {
  const int r = i >> 5;
  return i ^ ((r & 1 ? 22 : 0) ^ (r & 2 ? 29 : 0) ^ (r & 4 ? 12 : 0) ^ (r & 8 ? 18 : 0));
}

// Groups of at most 64 lanes run their exchanges wave-synchronously
// (build-time switch).
#ifndef PPF_WAVE_SYNC
#define PPF_WAVE_SYNC 1
#endif
constexpr bool wave_sync(int W) { return PPF_WAVE_SYNC && W <= 64; }

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
// WS: each group lies within one wavefront (W divides 64) and owns its
// planes, so an exchange needs no block barrier: a wavefront's LDS
// instructions execute in issue order, and wavefront-scope fences keep the
// compiler from moving its LDS accesses across the exchange.
template <int N, int R, int RX, int G, int B, bool DB, bool TWG, bool TWR = false, bool WS = false>
struct GroupFft {
  static constexpr int W = N / R;
  static constexpr int L = num_stages(N, RX);
  static constexpr int PL = plane_floats(N, W);      // floats per plane
  static constexpr int NBUF = DB ? 2 : 1;
  // TWR (with TWG): stages with one shared set keep it in registers
  static constexpr int NTW_ = TWG ? (TWR ? tw_offset_twg(N, R, RX, L) : 0) : tw_total(N, R, RX);
  static constexpr int NTW = NTW_ > 0 ? NTW_ : 1;
  // offset of stage S's register twiddles
  static constexpr int tw_off(int S) { return TWG ? tw_offset_twg(N, R, RX, S) : tw_offset(N, R, RX, S); }
  // stage S reads its twiddles from the table when it starts
  static constexpr bool tw_fetched(int S) { return TWG && S > 0 && (!TWR || ns_at(N, RX, S) > W); }
  static constexpr size_t lds_bytes() { return size_t(NBUF) * B * 2 * G * PL * sizeof(float); }
  static constexpr bool IL = lds_b64(N);             // interleaved (re, im) elements
  // XL (N >= 4096 with a multiple of 512 threads per group: 16 or 32
  // elements per thread at N >= 8192, 4 over 1024 threads in the fused
  // N = 4096 kernel, where every e*W is a multiple of 512): swz64 is linear, changes
  // only bits 0-4 and depends only on bits 5-8, and a Stockham stage's
  // element index is the thread's base with the q digit (and the
  // butterfly's offset) in bits of their own; so an element's address is
  // one base per stage XORed with swz64 of its offset, which is a plain
  // add for offsets that are multiples of 512. One base register per stage
  // instead of one per element keeps the register file for the elements.
  static constexpr bool XL = IL && N >= 4096 && W % 512 == 0;

  float* lds;      // shared memory base of the block
  int grp, j;
  int par;         // buffer of the next exchange (double-buffered mode)
  const v2f* tw;   // twiddle table (global)
  v2f twr[NTW];
  int rb;          // XL: swizzled element j (the reads of every stage add e*W)
  int wb[L];       // XL: swizzled first write element of each stage

  static_assert(!WS || (N / R <= 64 && 64 % (N / R) == 0), "a wave-synchronous group lies within one wavefront");
  __device__ __forceinline__ static void sync() {
    if constexpr (WS) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
  }

  __device__ __forceinline__ float* plane(int buf, int b, int reim) const {
    return lds + (((buf * B + b) * 2 + reim) * G + grp) * PL;
  }
  // IL: the plane of (re, im) elements of spectrum b
  __device__ __forceinline__ v2f* cplane(int buf, int b) const {
    return (v2f*)lds + ((buf * B + b) * G + grp) * PL;
  }

  template <int S>
  __device__ __forceinline__ void load_stage_tw() {
    if constexpr (S < L) {
      if constexpr (S > 0 && !tw_fetched(S)) {
        constexpr int r = radix_at(N, RX, S), Ns = ns_at(N, RX, S);
        constexpr int nset = (Ns <= W) ? 1 : R / r;
        constexpr int off = tw_off(S);
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
    if constexpr (XL) {
      rb = swz64(j);
#pragma unroll
      for (int s = 0; s < L; ++s) {
        const int ns = ns_at(N, RX, s), r = radix_at(N, RX, s);
        wb[s] = swz64((j / ns) * ns * r + j % ns);
      }
    }
    load_stage_tw<1>();
  }

  // twiddle sets of stage S: butterflies j + i*W share b % Ns when Ns <= W
  template <int S>
  static constexpr int stage_sets() {
    return ns_at(N, RX, S) <= W ? 1 : R / radix_at(N, RX, S);
  }

  // TWG: stage S's twiddles are read from the global table when the stage
  // starts, all in one batch. The addresses are loop-invariant, so a
  // hoisted load would keep every stage's twiddles live in registers; one
  // opaque zero per stage ties the batch to its stage, and the loads are
  // in flight together (one wait) while the stage reads its LDS inputs.
  template <int S>
  __device__ __forceinline__ void fetch_stage_tw(v2f* tl) const {
    constexpr int r = radix_at(N, RX, S), Ns = ns_at(N, RX, S);
    int z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
#pragma unroll
    for (int ib = 0; ib < stage_sets<S>(); ++ib) {
      const int k = (j + ib * W) % Ns;
#pragma unroll
      for (int q = 1; q < r; ++q) tl[ib * (r - 1) + q - 1] = tw[k * q * (N / (Ns * r)) + z];
    }
  }

  template <int S>
  __device__ __forceinline__ v2f twiddle(const v2f* tl, int i, int q) const {
    constexpr int r = radix_at(N, RX, S), Ns = ns_at(N, RX, S);
    const int ib = (Ns <= W) ? 0 : i;
    if constexpr (tw_fetched(S)) {
      return tl[ib * (r - 1) + q - 1];
    } else {
      return twr[tw_off(S) + ib * (r - 1) + q - 1];
    }
  }

  template <int S>
  __device__ __forceinline__ void stage(v2f (&v)[B][R]) {
    constexpr int r = radix_at(N, RX, S), Ns = ns_at(N, RX, S);
    constexpr int nb = R / r;
    v2f tl[tw_fetched(S) ? stage_sets<S>() * (r - 1) : 1];
    if constexpr (tw_fetched(S)) fetch_stage_tw<S>(tl);
    if constexpr (S > 0) {
      const int buf = DB ? par : 0;
#pragma unroll
      for (int b = 0; b < B; ++b) {
        if constexpr (XL) {
          // e*W is a multiple of 512: above the swizzle
          const v2f* pl = cplane(buf, b);
#pragma unroll
          for (int e = 0; e < R; ++e) v[b][e] = pl[rb + e * W];
        } else if constexpr (IL && WS) {
          // swz64 is linear over GF(2) and j (< W, a power of two) shares no
          // bit with e*W: one lane base XORed with a constant per element
          const v2f* pl = cplane(buf, b);
          const int rb0 = swz64(j);
#pragma unroll
          for (int e = 0; e < R; ++e) v[b][e] = pl[rb0 ^ swz64(e * W)];
        } else if constexpr (IL) {
          const v2f* pl = cplane(buf, b);
#pragma unroll
          for (int e = 0; e < R; ++e) v[b][e] = pl[swz64(j + e * W)];
        } else {
          const float* re = plane(buf, b, 0);
          const float* im = plane(buf, b, 1);
#pragma unroll
          for (int e = 0; e < R; ++e) {
            const int idx = lds_index<N>(j + e * W);
            v[b][e].x = re[idx];
            v[b][e].y = im[idx];
          }
        }
      }
      if constexpr (DB) par ^= 1;
#pragma unroll
      for (int i = 0; i < nb; ++i)
#pragma unroll
        for (int q = 1; q < r; ++q) {
          const v2f w = twiddle<S>(tl, i, q);
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
      if constexpr (!DB) sync();   // earlier reads of the single buffer are done
      const int buf = DB ? par : 0;
      // XL: this stage's base, opaque so that the per-element addresses are
      // formed here rather than held in registers across the spectrum loop
      int wbs = 0;
      if constexpr (XL) {
        wbs = wb[S];
        asm volatile("" : "+v"(wbs));
      }
      // WS: the write index of butterfly j + i*W is a bit insertion of it,
      // so (with swz64 linear) one lane base XORed with a constant per write
      const int wl = swz64((j / Ns) * Ns * r + j % Ns);
#pragma unroll
      for (int b = 0; b < B; ++b) {
        float* re = plane(buf, b, 0);
        float* im = plane(buf, b, 1);
        v2f* pl = cplane(buf, b);
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
            if constexpr (XL) {
              // butterfly i sits i*W*r (Ns <= W) or i*W (Ns > W) above
              // butterfly 0, a multiple of 512 in both cases
              const int di = (Ns <= W) ? i * W * r : i * W;
              const int qo = q * Ns;
              const int idx = ((qo & 511) == 0 ? wbs + qo : (wbs ^ swz64(qo))) + di;
              pl[idx] = t[q];
            } else if constexpr (IL && WS) {
              pl[wl ^ swz64(((i * W) / Ns) * Ns * r + (i * W) % Ns + q * Ns)] = t[q];
            } else if constexpr (IL) {
              pl[swz64(base + q * Ns)] = t[q];
            } else {
              const int idx = lds_index<N>(base + q * Ns);
              re[idx] = t[q].x;
              im[idx] = t[q].y;
            }
          }
        }
      }
      sync();
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
// 16-tap kernels for N <= 256: prefetch 2 and two waves per SIMD (tuning).
#ifndef PPF_SMALL16
#define PPF_SMALL16 1
#endif

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
  float* pout;         // detected power out (power kernels): (M / K) x N
  int K;               // spectra integrated per power spectrum (power kernels)
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
  float* pout = nullptr;   // power kernels: |X|^2 summed over K spectra, spectrum m to pout + (m/K)*N
  int K = 1;
};

template <int N>
__device__ __forceinline__ const v2f* block_ptr(const TileArgs& a, int rb) {
  return rb < a.h0 ? a.x0 + (long long)rb * N
                   : (rb < a.h01 ? a.x1 + (long long)(rb - a.h0) * N : a.x2 + (long long)(rb - a.h01) * N);
}

// Stored complex input types, widened to FP32 as they are loaded:
// 0 = complex FP32, 1 = complex FP16, 2 = complex int8 (exact conversions).
constexpr int in_bytes(int IT) { return IT == 0 ? 8 : (IT == 1 ? 4 : 2); }

// block rb of the tile's input, for samples of SB bytes
template <int N, int SB>
__device__ __forceinline__ const char* block_addr(const TileArgs& a, int rb) {
  const char* x0 = (const char*)a.x0;
  const char* x1 = (const char*)a.x1;
  const char* x2 = (const char*)a.x2;
  return rb < a.h0 ? x0 + (long long)rb * N * SB
                   : (rb < a.h01 ? x1 + (long long)(rb - a.h0) * N * SB : x2 + (long long)(rb - a.h01) * N * SB);
}

__device__ __forceinline__ v2f widen_c16(uint32_t w) {
  _Float16 re, im;
  const uint16_t lo = (uint16_t)(w & 0xFFFFu), hi = (uint16_t)(w >> 16);
  __builtin_memcpy(&re, &lo, 2);
  __builtin_memcpy(&im, &hi, 2);
  v2f r;
  r.x = (float)re;
  r.y = (float)im;
  return r;
}
__device__ __forceinline__ v2f widen_ci8(uint32_t w) {
  v2f r;
  r.x = (float)(int)(int8_t)(w & 0xFFu);
  r.y = (float)(int)(int8_t)((w >> 8) & 0xFFu);
  return r;
}

template <int IT>
__device__ __forceinline__ v2f load_sample(const void* base, long long i) {
  if constexpr (IT == 0) {
    return ((const v2f*)base)[i];
  } else if constexpr (IT == 1) {
    return widen_c16(((const uint32_t*)base)[i]);
  } else {
    return widen_ci8(((const uint16_t*)base)[i]);
  }
}

// Fused FIR + FFT at N = 4096 with up to 8 taps: four channels per lane
// over a 1024-thread block, so that a lane's tap window (8 taps x 4
// channels) is the same size as at N = 1024. Build-time switch (tuning).
#ifndef PPF_FUSED_4096
#define PPF_FUSED_4096 1
#endif
constexpr bool fused4096(int N, int TP) { return PPF_FUSED_4096 && N == 4096 && TP > 1 && TP <= 8; }
// With 5..8 taps a ring of 8 + 2 blocks, the coefficients (8 x 4 per
// lane) and the twiddles exceed the 128 registers of a lane at 4 waves per
// SIMD: the coefficients go to LDS (128 KiB beside one 32 KiB exchange
// buffer, so the exchanges are single-buffered) and the ring prefetches
// one block.
constexpr bool fused4096_cl(int N, int TP) { return fused4096(N, TP) && TP == 8; }

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
template <int N, int R, int RX, int G, int B, int TP, int PF, bool DB, bool TWG, bool UNIT, bool POW = false,
          int IT = 0>
struct FusedEngine {
  static constexpr int W = N / R;
  static constexpr int SB = in_bytes(IT);   // bytes per stored input sample
  static_assert(!UNIT || IT == 0, "the FFT pass reads FP32 presums");
  static constexpr int Q = TP + PF;
  static_assert(Q % B == 0 && Q >= TP + B - 1, "ring size");
  static_assert(!UNIT || TP == 1, "unit coefficients are a single tap");
  // the FFT pass keeps shared twiddle sets; groups within one wavefront
  // exchange without block barriers
  using Fft = GroupFft<N, R, RX, G, B, DB, TWG, UNIT && !POW, wave_sync(N / R)>;

  // Long tap windows keep their coefficients in LDS (TP x N floats after
  // the FFT planes, shared by the groups of the block) instead of TP x R
  // registers per thread, which would leave one wave per SIMD.
  static constexpr bool CL = !UNIT && (TP >= 16 || fused4096_cl(N, TP));
  static constexpr size_t coef_lds_bytes() { return CL ? (size_t)TP * N * sizeof(float) : 0; }

  static constexpr size_t lds_bytes() { return Fft::lds_bytes() + coef_lds_bytes(); }

  Fft fft;
  int j;
  int d;
  float hreg[(UNIT || CL) ? 1 : TP][R];
  uint32_t hl;         // CL: LDS byte address of this thread's coefficient column
  uint32_t loff;       // byte offset of channel j inside a block; element e adds e*W*8

  __device__ __forceinline__ void init(float* smem, int grp, int j_, const float* coef, const v2f* tw, int d_) {
    j = j_;
    d = d_;
    fft.init(smem, grp, j, tw);
    if constexpr (CL) {
      float* cl = (float*)((char*)smem + Fft::lds_bytes());
      for (int i = threadIdx.x; i < TP * N; i += blockDim.x) cl[i] = coef[i];
      __syncthreads();
      hl = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) float*)(cl + j);
    } else if constexpr (!UNIT) {
#pragma unroll
      for (int t = 0; t < TP; ++t)
#pragma unroll
        for (int e = 0; e < R; ++e) hreg[t][e] = coef[t * N + j + e * W];
    }
    loff = (uint32_t)j * (uint32_t)sizeof(v2f);
  }

  // coefficient of tap t, element e; CL reads LDS through a base the caller
  // refreshes every step (so the reads are not hoisted into registers)
  __device__ __forceinline__ float hcoef(uint32_t base, int t, int e) const {
    if constexpr (CL) {
      return *(const __attribute__((address_space(3))) float*)(uintptr_t)(base + (uint32_t)((t * N + e * W) *
                                                                                           (int)sizeof(float)));
    } else {
      return hreg[t][e];
    }
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
    float pw[POW ? R : 1];
#pragma unroll
    for (int e = 0; e < (POW ? R : 1); ++e) pw[e] = 0.f;
    v2f ring[Q][R];
#pragma unroll
    for (int s = 0; s < Q; ++s)
#pragma unroll
      for (int e = 0; e < R; ++e) { ring[s][e].x = 0.f; ring[s][e].y = 0.f; }
    auto load = [&](v2f (&dst)[R], int vb) {
      if constexpr (G == 1 && IT != 0) {
        // widened input: no branch around the load (a merge of the loaded
        // bits with the slot's old value would wait for the load here); a
        // block outside [vb_lo, vb_hi) gets an empty range and reads zeros
        const bool ok = vb >= vb_lo && vb < vb_hi;
        const __amdgpu_buffer_rsrc_t rs = block_rsrc(block_addr<N, SB>(a, ok ? vb - d : 0), ok ? N * SB : 0);
        constexpr int aux = kNtLoads ? kAuxNt : 0;
#pragma unroll
        for (int e = 0; e < R; ++e) {
          const uint32_t so = (uint32_t)(e * W * SB);
          if constexpr (IT == 1) {
            dst[e].x = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, loff / 2, so, aux));
          } else {
            dst[e].x = __builtin_bit_cast(float, (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rs, loff / 4, so, aux));
          }
        }
      } else if (vb >= vb_lo && vb < vb_hi) {
        if constexpr (G == 1) {
          const __amdgpu_buffer_rsrc_t rs = block_rsrc(block_addr<N, SB>(a, vb - d), N * SB);
          constexpr int aux = kNtLoads ? kAuxNt : 0;
#pragma unroll
          for (int e = 0; e < R; ++e) {
            const uint32_t so = (uint32_t)(e * W * SB);
            if constexpr (IT == 0) {
              dst[e] = buf_load<aux>(rs, loff, so);
            } else if constexpr (IT == 1) {
              dst[e].x = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, loff / 2, so, aux));
            } else {
              dst[e].x = __builtin_bit_cast(float, (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rs, loff / 4, so, aux));
            }
          }
        } else {
          const char* src = block_addr<N, SB>(a, vb - d);
#pragma unroll
          for (int e = 0; e < R; ++e) {
            if constexpr (IT == 0) {
              dst[e] = ((const v2f*)src)[j + e * W];
            } else if constexpr (IT == 1) {
              dst[e].x = __builtin_bit_cast(float, ((const uint32_t*)src)[j + e * W]);
            } else {
              dst[e].x = __builtin_bit_cast(float, (uint32_t)((const uint16_t*)src)[j + e * W]);
            }
          }
        }
      }
    };

    // FP16 / int8 input: a slot first holds the stored bits in .x and is
    // widened in place at the start of the step that first reads it, so the
    // wait for its load falls there, PF steps after the load was issued
    auto widen = [&](v2f (&slot)[R]) {
      if constexpr (IT != 0) {
#pragma unroll
        for (int e = 0; e < R; ++e) {
          const uint32_t w = __builtin_bit_cast(uint32_t, slot[e].x);
          slot[e] = IT == 1 ? widen_c16(w) : widen_ci8(w);
        }
      }
    };

#pragma unroll
    for (int s = 0; s < Q - B; ++s) load(ring[s], m0 + s);
#pragma unroll
    for (int s = 0; s < TP - 1; ++s) widen(ring[s]);

    for (int base = 0; base < niter; base += Q) {
#pragma unroll
      for (int k = 0; k < Q; k += B) {
        const int it = base + k;
        if (it >= niter) break;
#pragma unroll
        for (int b = 0; b < B; ++b) load(ring[(k + Q - B + b) % Q], m0 + it + Q - B + b);
#pragma unroll
        for (int b = 0; b < B; ++b) widen(ring[(k + TP - 1 + b) % Q]);
        v2f v[B][R];
        uint32_t hb = hl;
        if constexpr (CL) asm volatile("" : "+v"(hb));
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
          for (int e = 0; e < R; ++e) {
            if constexpr (UNIT) {
              v[b][e] = ring[(k + b) % Q][e];
            } else {
              v2f acc;
              const float h0 = hcoef(hb, 0, e);
              acc.x = h0 * ring[(k + b) % Q][e].x;
              acc.y = h0 * ring[(k + b) % Q][e].y;
#pragma unroll
              for (int t = 1; t < TP; ++t) {
                const float ht = hcoef(hb, t, e);
                acc.x = fmaf(ht, ring[(k + b + t) % Q][e].x, acc.x);
                acc.y = fmaf(ht, ring[(k + b + t) % Q][e].y, acc.y);
              }
              v[b][e] = acc;
            }
          }
        fft.run(v);
#pragma unroll
        for (int b = 0; b < B; ++b) {
          if (it + b < ng) {
            if constexpr (POW) {
              // detection: |X|^2 of this thread's bins, summed over K spectra
              // (tiles start at multiples of K)
#pragma unroll
              for (int e = 0; e < R; ++e) pw[e] += fmaf(v[b][e].x, v[b][e].x, v[b][e].y * v[b][e].y);
              if ((it + b + 1) % a.K == 0) {
                const long long q = (long long)(m0 + it + b) / a.K;
                if constexpr (G == 1) {
                  const __amdgpu_buffer_rsrc_t rs = block_rsrc(a.pout + q * N, N * (int)sizeof(float));
#pragma unroll
                  for (int e = 0; e < R; ++e)
                    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, pw[e]), rs, loff / 2,
                                                          (uint32_t)(e * W * (int)sizeof(float)), kAuxNt);
                } else {
                  float* dst = a.pout + q * N + j;
#pragma unroll
                  for (int e = 0; e < R; ++e) __builtin_nontemporal_store(pw[e], dst + e * W);
                }
#pragma unroll
                for (int e = 0; e < R; ++e) pw[e] = 0.f;
              }
            } else if constexpr (G == 1) {
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
template <int N, int R, int RX, int G, int B, int TP, int PF, bool DB, bool TWG, bool UNIT, bool POW = false,
          int IT = 0>
__global__ void __launch_bounds__((N / R) * G) __attribute__((amdgpu_waves_per_eu(PPF_SMALL16 && TP >= 16 && N <= 256 ? 2 : 1)))
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

  FusedEngine<N, R, RX, G, B, TP, PF, DB, TWG, UNIT, POW, IT> eng;
  eng.init(smem, grp, j, p.coef, p.tw, p.d);
  TileArgs a{p.x0, p.x1, p.x1, p.out, p.h0, p.h0, p.pout, p.K};
  eng.run(a, m0, ng, niter);
}

// Descriptor form (serving): the tiles are listed in device memory; a
// persistent grid walks them, G tiles per block at a time. Every wave of a
// block exits at the same tile index, after the same number of barriers.
// (Claiming tiles from a per-class atomic counter instead measured slower:
// 64x against 100x real time sustained at an offered 100x.)

template <int N, int R, int RX, int G, int B, int TP, int PF, bool DB, bool TWG, bool UNIT>
__global__ void __launch_bounds__((N / R) * G) __attribute__((amdgpu_waves_per_eu(PPF_SMALL16 && TP >= 16 && N <= 256 ? 2 : 1)))
ppf_fused_desc_kernel(const DescClass* cls, const TileDesc* tiles, const float* coef, const v2f* tw, int d) {
  constexpr int W = N / R;
  extern __shared__ float smem[];
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
      __shared__ int s_count[G];     // only where G > 1: the G = 1 kernels may use all of LDS
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
// configurations and dispatch
// --------------------------------------------------------------------------

// Build-time override of the prefetch depth of the fused kernels (tuning).
#ifndef PPF_PF_FUSED_OVERRIDE
#define PPF_PF_FUSED_OVERRIDE 0
#endif


// elements per thread R and groups per block G for the FFT of N points
// (TP = 1: the FFT pass of the two-pass form)
constexpr int cfg_R(int N, int TP = 1) {
  return fused4096(N, TP) ? 4 : (N <= 1024 ? 4 : (N == 2048 ? 8 : (N >= 16384 ? 32 : 16)));
}
constexpr int cfg_RX(int N, int TP = 1) { return cfg_R(N, TP) < 16 ? cfg_R(N, TP) : 16; }
constexpr int cfg_W(int N, int TP = 1) { return N / cfg_R(N, TP); }
constexpr int cfg_G(int N, int TP = 1) { return cfg_W(N, TP) >= 256 ? 1 : 256 / cfg_W(N, TP); }
#ifndef PPF_PF_16K
#define PPF_PF_16K 0
#endif
constexpr int cfg_PF(int N, int TP) {
  if (fused4096_cl(N, TP)) return 1;
  return TP == 1 ? (N >= 16384 ? PPF_PF_16K : (N >= 4096 ? 1 : (N >= 2048 ? 2 : 3)))
                 : (N >= 2048 || (PPF_SMALL16 && TP >= 16 && N <= 256) ? 2
                                  : (PPF_PF_FUSED_OVERRIDE > 0 ? PPF_PF_FUSED_OVERRIDE : 4));
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
constexpr bool cfg_DB(int N, int B, int TP = 1) {
  return !fused4096_cl(N, TP) && 2ull * B * 2 * cfg_G(N, TP) * plane_floats(N, cfg_W(N, TP)) * sizeof(float) <= 80 * 1024;
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
  if (ki.lds > 64 * 1024) (void)hipFuncSetAttribute(ki.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ki.lds);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, ki.fn, ki.block, ki.lds) != hipSuccess || occ <= 0) occ = 1;
  return occ;
}

template <int N, int TP, bool UNIT, bool POW = false, int IT = 0>
static const KernelInfo& fused_info() {
  constexpr int R = cfg_R(N, TP), RX = cfg_RX(N, TP), G = cfg_G(N, TP), PF = cfg_PF(N, TP), B = cfg_B(N, TP);
  constexpr bool DB = cfg_DB(N, B, TP), TWG = cfg_TWG(N);
  static const KernelInfo ki{(const void*)&ppf_fused_kernel<N, R, RX, G, B, TP, PF, DB, TWG, UNIT, POW, IT>,
                             (N / R) * G, G, FusedEngine<N, R, RX, G, B, TP, PF, DB, TWG, UNIT, POW, IT>::lds_bytes()};
  return ki;
}

// Shortest tile of a batch launch, in units of the tap count (build-time
// tuning): a tile of S spectra reads S + TP - 1 input blocks.
#ifndef PPF_MIN_TILE
#define PPF_MIN_TILE 1
#endif
// Tiles per resident group slot of a batch launch. One tile per slot
// streams each group's own region; for N <= 256 the groups' runs are short
// (N*8 bytes per spectrum) and more, shorter tiles, dispatched in order so
// that the tiles running at once on an XCD are neighbours, measured faster
// (same box, in one process, 2^28 samples, best of 5):
//   N=16 all T 32 (1.13 -> 0.91 ms at T=4); N=32, T <= 8: 4 (0.88 -> 0.78);
//   N=64 all T 8 (0.87 -> 0.75 at T=8); N=128, T <= 4: 8 (0.86 -> 0.71);
//   N=256, T <= 8: 32 (0.87 -> 0.79 at T=8).
// Elsewhere, and for N >= 512, one tile per slot was as fast or faster.
// PPF_TILE_SPLIT > 0 overrides the table at build time (tuning).
#ifndef PPF_TILE_SPLIT
#define PPF_TILE_SPLIT 0
#endif
constexpr int tile_split(int N, int TP) {
  if (PPF_TILE_SPLIT > 0) return PPF_TILE_SPLIT;
  if (N == 16) return 32;
  if (N == 32) return TP <= 8 ? 4 : 1;
  if (N == 64) return TP <= 16 ? 8 : 1;
  if (N == 128) return TP <= 4 ? 8 : 1;
  if (N == 256) return TP <= 8 ? 32 : 1;
  return 1;
}
// Longest tile at N = 512 and 1024 with up to 8 taps: 2 MiB of input.
// N=1024, T=8 at 2^28 samples measured 0.868 ms with 512-spectrum (4 MiB)
// tiles, 0.806 with 256 and 0.824 with 128; N=512 was fastest at its
// 512-spectrum (2 MiB) tiles.
constexpr long long tile_max_spectra(int N, int TP) {
  return (PPF_TILE_SPLIT == 0 && (N == 512 || N == 1024) && TP <= 8) ? (2ll << 20) / (8ll * N) : 0;
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

// POW: the kernel writes |X|^2 summed over K consecutive spectra to pout
// instead of the spectra (a.M a multiple of K; tiles start at multiples of K).
template <int N, int TP, bool UNIT, bool POW = false, int IT = 0>
static hipError_t fused_launch_one(const PlanDev& pd, const BatchArgs& a, const float* coef, int T,
                                   hipStream_t st, float* pout = nullptr, int K = 1) {
  const KernelInfo& ki = fused_info<N, TP, UNIT, POW, IT>();
  static const int occ = occupancy(ki);
  const long long resident_groups = (long long)device_cus() * occ * ki.G * tile_split(N, TP);
  long long S = (a.M + resident_groups - 1) / resident_groups;
  if (tile_max_spectra(N, TP) > 0 && S > tile_max_spectra(N, TP)) S = tile_max_spectra(N, TP);
  if (S < PPF_MIN_TILE * TP) S = PPF_MIN_TILE * TP;            // bound the tap-window re-reads
  if (POW) S = (S + K - 1) / K * K;
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
  p.pout = pout;
  p.K = K;
  constexpr int R = cfg_R(N, TP), RX = cfg_RX(N, TP), G = cfg_G(N, TP), PF = cfg_PF(N, TP), B = cfg_B(N, TP);
  constexpr bool DB = cfg_DB(N, B, TP), TWG = cfg_TWG(N);
  hipLaunchKernelGGL((ppf_fused_kernel<N, R, RX, G, B, TP, PF, DB, TWG, UNIT, POW, IT>), dim3((unsigned)nblocks),
                     dim3(ki.block), ki.lds, st, p);
  return hipGetLastError();
}

// IT: stored input type (widened to FP32 as it is loaded)
template <int N, int TP, bool UNIT = false, bool POW = false, int IT = 0>
static hipError_t fused_launch(const PlanDev& pd, const BatchArgs& a, const float* coef, int T, hipStream_t st,
                               float* pout, int K) {
  const long long step = POW ? kMaxLaunchSpectra / K * K : kMaxLaunchSpectra;
  for (long long s0 = 0; s0 < a.M; s0 += step) {
    const long long k = a.M - s0 < step ? a.M - s0 : step;
    const hipError_t e = fused_launch_one<N, TP, UNIT, POW, IT>(pd, sub_batch(a, N, in_bytes(IT), s0, k), coef, T,
                                                                st, POW ? pout + (s0 / K) * N : nullptr, K);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

typedef hipError_t (*FusedFn)(const PlanDev&, const BatchArgs&, const float*, int, hipStream_t, float*, int);


// The fused path exists where the tap window of a thread (R channels x TP
// taps, plus coefficients) fits the register file at useful occupancy.
constexpr bool fused_ok(int N, int TP) {
  return TP == 1 || (N <= 1024 && TP <= 16) || (N == 2048 && TP <= 8) || fused4096(N, TP);
}

// Fused kernels reading complex FP16 (IT = 1) or int8 (IT = 2) input,
// built in a translation unit of their own.
FusedFn fused_fn_widened(int N, int TP, int IT);

}  // namespace ppf
