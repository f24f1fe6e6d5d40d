// Fused reduced-precision PPF kernel for N = 4096 = 16^3 channels and up to
// 16 taps on CDNA4 (gfx950): complex int8 input, FP16 coefficients, FP32
// FIR accumulation, and the 4096-point DFT as three radix-16 stages whose
// 16-point DFTs run on the matrix cores (v_mfma_f32_16x16x32_f16: FP16
// operands, FP32 accumulation) with FP32 twiddle multiplies in between.
//
// What is computed (section 2, Eq. 1 per channel, then the DFT of section 3):
//   u[m][c] = sum_t h[t][c] x[m+t][c],   X[m][k] = sum_c u[m][c] W^(c k),
// W = exp(-2 pi i / 4096). With c = c0 + 256 p (c0 = a + 16 b) and
// k = k1 + 16 k2 + 256 k3 the exponent c k splits (mod 4096) so that
//   X = sum_a W16^(a k3) W^(a (k1 + 16 k2)) sum_b W256^(b (16 k2 + k1)) sum_p W16^(p k1) u[a + 16 b + 256 p]:
// stage 1 is a plain 16-point DFT over p, stage 2 a 16-point transform over
// b whose matrix W256^(b (16 k2 + k1)) also carries the usual inter-stage
// twiddle W256^(b k1) (k1 is the same for all vectors of a wave there), one
// FP32 twiddle W^(a (k1 + 16 k2)) follows stage 2, and stage 3 is a plain
// 16-point DFT over a.
//
// One workgroup of 1024 threads (16 waves) owns a tile of consecutive
// spectra. A 16-point complex DFT of 16 vectors is two MFMAs: the DFT
// matrix as the 16x32 real A operand ([Re F, -Im F] and [Im F, Re F] rows
// over interleaved (re, im) inputs) and the 16 vectors as the 32x16 B
// operand. Lane l of wave w supplies points 4h..4h+3 (h = l / 16) of
// vector l % 16 and receives outputs 4h..4h+3 of that vector.
//
// The FIR lane layout is the stage-1 operand layout: lane (w, j, h) owns
// channels c0 + 256 (4h + e), c0 = 16 w + j, e < 4, so its presums are
// exactly its B operand and need no exchange. Each lane keeps a ring of
// the last 16 input blocks of its 4 channels as packed FP16 (re, im) in
// registers (int8 values, pre-scaled by a power of two, are exact in FP16);
// the coefficients of all taps live in LDS in lane order. The spectrum loop
// is unrolled by the ring size so ring slots are static registers.
// Stage outputs are exchanged through two swizzled LDS buffers of FP16
// complex values; two barriers per spectrum.
//
// Scaling: the ring holds x * 2^-e1 and the FIR uses the FP16 coefficients
// h16 = h * 2^s as given, so stage inputs are 2^(s-e1) times the true
// values; e1 is chosen on the host so that no FP16 stage input can
// overflow for any int8 input, and the output is multiplied by 2^(e1-s).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ppf_internal.h"

namespace ppf {
namespace {

typedef float v2f __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef uint32_t u2 __attribute__((ext_vector_type(2)));

constexpr int kN = 4096;
constexpr int kTaps = 16;                       // ring size and coefficient slots
constexpr int kThreads = 1024;
constexpr int kCoefBytes = kTaps * kN * 2;      // FP16 coefficients in LDS
constexpr int kXchgBytes = kN * 4;              // one FP16 complex exchange buffer
constexpr int kLdsBytes = kCoefBytes + 2 * kXchgBytes;
#ifndef PPF_MFMA_COEF_GROUP
#define PPF_MFMA_COEF_GROUP 0
#endif
constexpr int kCoefGroup = PPF_MFMA_COEF_GROUP;   // taps per batch of coefficient reads (0: free)

constexpr int kBufDword3 = 0x00020000;
constexpr int kAuxNt = 2;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, bytes, kBufDword3);
}

// Exchange-buffer swizzle in 4-byte element units: XOR element bits 2-3
// with bits 6-7 and bits 4-5 with bits 10-11. Bits 0-1 are kept, so the
// four points a lane reads stay one aligned 16-byte group.
__device__ __forceinline__ constexpr int swz(int e) {
  return e ^ (((e >> 6) & 3) << 2) ^ (((e >> 10) & 3) << 4);
}

__device__ __forceinline__ uint32_t pack_h2(float re, float im) {
  h2 v;
  v.x = (_Float16)re;
  v.y = (_Float16)im;
  return __builtin_bit_cast(uint32_t, v);
}

// One complex int8 sample (bytes re, im in the low half of raw) to a packed
// FP16 (re, im) pair scaled by sc = 2^-e1, exactly: with the sign bit
// flipped, byte b becomes the FP16 number 1024 + b + 128 when 0x64 is placed
// above it, and sc * (that - 1152) = sc * x is representable.
__device__ __forceinline__ uint32_t widen1(uint32_t raw, h2 sc, h2 bias) {
  const uint32_t t = __builtin_amdgcn_perm(0x64646464u, raw ^ 0x8080u, 0x04010400u);
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_fma(__builtin_bit_cast(h2, t), sc, bias));
}

}  // namespace

struct MfmaParams {
  const void* x0;            // complex int8 or FP16, first segment (h0 blocks)
  const void* x1;            // second segment
  v2f* out;                  // complex FP32 spectra
  float* pout;               // detection: |X|^2 summed over K spectra, (M / K) x N
  int K;
  const uint4* coef;         // [16][4096] FP16 coefficients in lane order
  const v2f* tw;             // 4096 FP32 twiddles exp(-2 pi i k / 4096)
  const uint32_t* w256;      // 256 FP16 complex exp(-2 pi i k / 256), (re, im) packed
  int h0;
  int M;                     // spectra
  int S;                     // spectra per tile
  int d;                     // leading zero tap slots (16 - T)
  int nblocks;
  float in_scale;            // 2^-e1
  float out_scale;           // 2^(e1 - s), exact on the FP16 stage-3 matrix
};

// Input types of the matrix-core kernel: complex int8 (2 bytes per sample,
// scaled by 2^-e1 as it is widened, exactly) and complex FP16 (4 bytes, used
// as stored; the FIR's FP32 sums are scaled by 2^-e1 instead, exactly).
constexpr int kInI8 = 2;
constexpr int kInF16 = 1;

namespace {

__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
  const int q = nblocks >> 3, rem = nblocks & 7;
  const int xcd = bid & 7, k = bid >> 3;
  return xcd * q + (xcd < rem ? xcd : rem) + k;
}

template <int PF, int AUX, int IT, bool POW>
struct MfmaEngine {
  static constexpr int SB = IT == kInI8 ? 2 : 4;   // bytes per input sample
  static_assert(kTaps % PF == 0, "prefetch depth divides the ring");
  const MfmaParams& p;
  uint8_t* lds;
  int w, j, h, tid;
  int m0, ng;
  int vb_lo, vb_hi;
  uint32_t in_off;           // lane byte offset in an input block (channel 16w+j+1024h)
  uint32_t out_off;          // lane byte offset in an output spectrum
  uint32_t wr1, wr2, rd;     // swizzled exchange byte offsets (r = 0 terms)
  h8 a1, a2, a3;             // A operands (real-part rows) of stages 1, 2, 3
  v2f tw2[4];                // FP32 twiddles after stage 2 of this lane's outputs
  h2 sc, bias;

  __device__ __forceinline__ MfmaEngine(const MfmaParams& p_, uint8_t* lds_) : p(p_), lds(lds_) {}

  __device__ __forceinline__ const uint8_t* block_ptr(int rb) const {
    return rb < p.h0 ? (const uint8_t*)p.x0 + (size_t)rb * kN * SB
                     : (const uint8_t*)p.x1 + (size_t)(rb - p.h0) * kN * SB;
  }

  // raw int8 pairs of this lane's 4 channels of virtual block vb, one per
  // register (zero-extended 16-bit loads; combining them here would make the
  // step wait for its own prefetch). A block outside [vb_lo, vb_hi) (zero
  // padding, or beyond what the tile uses) gets an empty buffer range, so
  // its loads return zero without touching memory; no branch either.
  __device__ __forceinline__ void load(uint32_t (&dst)[4], int vb) const {
    const bool in = vb >= vb_lo && vb < vb_hi;
    const __amdgpu_buffer_rsrc_t rs = rsrc(in ? block_ptr(vb - p.d) : p.x1, in ? kN * SB : 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if constexpr (IT == kInI8) dst[e] = __builtin_amdgcn_raw_buffer_load_b16(rs, in_off, 256 * SB * e, AUX);
      else dst[e] = __builtin_amdgcn_raw_buffer_load_b32(rs, in_off, 256 * SB * e, AUX);
    }
  }

  __device__ __forceinline__ void widen(const uint32_t (&raw)[4], uint32_t (&slot)[4]) const {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if constexpr (IT == kInI8) slot[e] = widen1(raw[e], sc, bias);
      else slot[e] = raw[e];   // packed FP16 (re, im) as stored
    }
  }

  __device__ __forceinline__ void init(int lb) {
    tid = threadIdx.x;
    w = tid >> 6;
    j = tid & 15;
    h = (tid >> 4) & 3;
    m0 = lb * p.S;
    const int rem = p.M - m0;
    ng = rem < p.S ? rem : p.S;
    vb_lo = m0 > p.d ? m0 : p.d;
    vb_hi = m0 + ng + kTaps - 1;
    in_off = (uint32_t)(16 * w + j + 1024 * h) * (uint32_t)SB;
    out_off = (uint32_t)(j + 16 * w + 1024 * h) * 8u;
    wr1 = kCoefBytes + swz(1024 * h + 16 * j + w) * 4;                 // in X
    wr2 = kCoefBytes + kXchgBytes + swz(1024 * h + 16 * w + j) * 4;    // in Y
    rd = swz(256 * w + 16 * j + 4 * h) * 4;
    const _Float16 s16 = (_Float16)p.in_scale;
    sc = h2{s16, s16};
    const _Float16 b16 = (_Float16)(-1152.0f * p.in_scale);
    bias = h2{b16, b16};

    // coefficients into LDS (lane order: tap t, lane tid -> 8 bytes)
#pragma unroll
    for (int i = 0; i < kCoefBytes / 16 / kThreads; ++i)
      ((uint4*)lds)[tid + i * kThreads] = p.coef[tid + i * kThreads];

    // A operands, real-part row j, inputs (point 4h+e, re/im): (wr, -wi) of
    // stage 1: W16^(p j); stage 2 (wave w holds k1 = w): W256^(b (16 j + w));
    // stage 3: W16^(a j) times the output scale (a power of two, exact)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int q = 4 * h + e;
      const h2 w1 = __builtin_bit_cast(h2, p.w256[(16 * q * j) & 255]);
      const h2 w2 = __builtin_bit_cast(h2, p.w256[(q * (16 * j + w)) & 255]);
      a1[2 * e] = w1.x;
      a1[2 * e + 1] = -w1.y;
      a2[2 * e] = w2.x;
      a2[2 * e + 1] = -w2.y;
      a3[2 * e] = (_Float16)((float)w1.x * p.out_scale);
      a3[2 * e + 1] = (_Float16)(-(float)w1.y * p.out_scale);
    }
    // stage-2 outputs of this lane: vector (a = j, k1 = w), k2 = 4h + r
#pragma unroll
    for (int r = 0; r < 4; ++r) tw2[r] = p.tw[(j * (w + 16 * (4 * h + r))) & (kN - 1)];
  }

  // Re X = A_re . (xr, xi) and Im X = A_re . (xi, -xr): the -i rotation of
  // the inputs replaces a second matrix (one packed multiply per register)
  __device__ __forceinline__ void dft16(const h8& a, const h8& b, f4& dre, f4& dim) const {
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    dre = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, z, 0, 0, 0);
    // (re, im) -> (im, -re) per register: one packed multiply by (1, -1)
    // with the halves of the first operand swapped by op_sel
    const uint4 bu = __builtin_bit_cast(uint4, b);
    uint4 bq;
    const uint32_t one_neg = 0xBC003C00u;   // FP16 (1.0, -1.0)
    asm("v_pk_mul_f16 %0, %1, %2 op_sel:[1,0] op_sel_hi:[0,1]" : "=v"(bq.x) : "v"(bu.x), "s"(one_neg));
    asm("v_pk_mul_f16 %0, %1, %2 op_sel:[1,0] op_sel_hi:[0,1]" : "=v"(bq.y) : "v"(bu.y), "s"(one_neg));
    asm("v_pk_mul_f16 %0, %1, %2 op_sel:[1,0] op_sel_hi:[0,1]" : "=v"(bq.z) : "v"(bu.z), "s"(one_neg));
    asm("v_pk_mul_f16 %0, %1, %2 op_sel:[1,0] op_sel_hi:[0,1]" : "=v"(bq.w) : "v"(bu.w), "s"(one_neg));
    const h8 bi = __builtin_bit_cast(h8, bq);
    dim = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, bi, z, 0, 0, 0);
  }

  // twiddle in FP32, round to FP16, scatter to the next stage's layout
  __device__ __forceinline__ void twiddle_store(const f4& dre, const f4& dim, const v2f (&tw)[4], uint32_t base) const {
    // a fresh base per use: the four stores then take immediate offsets
    // instead of four loop-invariant address registers
    asm volatile("" : "+v"(base));
    uint32_t* dst = (uint32_t*)(lds + base);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float yr = fmaf(dre[r], tw[r].x, -dim[r] * tw[r].y);
      const float yi = fmaf(dre[r], tw[r].y, dim[r] * tw[r].x);
      dst[256 * r] = pack_h2(yr, yi);
    }
  }

  // stage-1 outputs need no twiddle: round to FP16 and scatter
  __device__ __forceinline__ void plain_store(const f4& dre, const f4& dim, uint32_t base) const {
    asm volatile("" : "+v"(base));
    uint32_t* dst = (uint32_t*)(lds + base);
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[256 * r] = pack_h2(dre[r], dim[r]);
  }

  __device__ __forceinline__ h8 read_vec(int buf) const {
    return __builtin_bit_cast(h8, *(const uint4*)(lds + buf + rd));
  }

  float pw[4] = {0.f, 0.f, 0.f, 0.f};   // detection sums

  __device__ __forceinline__ void run() {
    constexpr int X = kCoefBytes, Y = kCoefBytes + kXchgBytes;

    uint32_t ring[kTaps][4];
    uint32_t stage[PF][4];
#pragma unroll
    for (int s = 0; s < kTaps; ++s)
#pragma unroll
      for (int e = 0; e < 4; ++e) ring[s][e] = 0u;
#pragma unroll
    for (int s = 0; s < PF; ++s)
#pragma unroll
      for (int e = 0; e < 4; ++e) stage[s][e] = 0u;

    // blocks 0 .. 14 into ring slots 0 .. 14; loads of 15 .. 14+PF in flight
#pragma unroll
    for (int s = 0; s < kTaps - 1; ++s) {
      uint32_t raw[4];
      load(raw, m0 + s);   // zero (which widens to 0.0) outside the read range
      widen(raw, ring[s]);
    }
#pragma unroll
    for (int s = 0; s < PF; ++s) load(stage[s], m0 + kTaps - 1 + s);
    __syncthreads();   // coefficients in LDS

    // Tiles hold a multiple of 16 spectra except the last; its extra steps
    // run on zero input and their stores get an empty range (discarded), so
    // the 16 unrolled steps have no branches and the scheduler can overlap
    // one spectrum's last DFT stage with the next spectrum's FIR.
    for (int base = 0; base < ng; base += kTaps) {
#pragma unroll
      for (int k = 0; k < kTaps; ++k) {
        const int it = base + k;
        // block it+15 into the slot of block it-1; refill its staging slot
        widen(stage[k % PF], ring[(k + kTaps - 1) % kTaps]);
        load(stage[k % PF], m0 + it + kTaps - 1 + PF);

        // each step widens the ring values itself (in the FMA) instead of
        // keeping FP32 copies alive across steps
#pragma unroll
        for (int s = 0; s < kTaps; ++s)
#pragma unroll
          for (int e = 0; e < 4; ++e) asm volatile("" : "+v"(ring[s][e]));
        // FIR: taps t = 0 .. 15 over ring slots (k + t) % 16, FP32 sums
        float ar[4] = {0.f, 0.f, 0.f, 0.f}, ai[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < kTaps; ++t) {
          // coefficient reads issued a few taps ahead, not all at once
          if (kCoefGroup > 0 && t % kCoefGroup == 0) __builtin_amdgcn_sched_barrier(0);
          const h4 hv = *(const h4*)(lds + t * (kN * 2) + tid * 8);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const h2 xv = __builtin_bit_cast(h2, ring[(k + t) % kTaps][e]);
            ar[e] = fmaf((float)hv[e], (float)xv.x, ar[e]);
            ai[e] = fmaf((float)hv[e], (float)xv.y, ai[e]);
          }
        }
        if (kCoefGroup > 0) __builtin_amdgcn_sched_barrier(0);
        h8 b;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if constexpr (IT == kInF16) {
            // FP16 samples enter unscaled: scale the FP32 sums (exact)
            ar[e] *= p.in_scale;
            ai[e] *= p.in_scale;
          }
          b[2 * e] = (_Float16)ar[e];
          b[2 * e + 1] = (_Float16)ai[e];
        }

        f4 dre, dim;
        dft16(a1, b, dre, dim);                   // stage 1 over p
        plain_store(dre, dim, wr1);               // to the stage-2 layout (X)
        __syncthreads();
        dft16(a2, read_vec(X), dre, dim);         // stage 2 over b (with W256^(b k1))
        twiddle_store(dre, dim, tw2, wr2);        // W^(a (k1 + 16 k2)), to the stage-3 layout (Y)
        __syncthreads();
        dft16(a3, read_vec(Y), dre, dim);         // stage 3 over a, output scale folded in

        if constexpr (POW) {
          // detection: this lane's four bins summed over K spectra (tiles
          // start at multiples of K); steps past the tile add nothing
          if (it < ng) {
#pragma unroll
            for (int r = 0; r < 4; ++r) pw[r] += fmaf(dre[r], dre[r], dim[r] * dim[r]);
            if ((m0 + it + 1) % p.K == 0) {
              const long long q = (long long)(m0 + it) / p.K;
              const __amdgpu_buffer_rsrc_t rs = rsrc(p.pout + q * kN, kN * 4);
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, pw[r]), rs, out_off / 2,
                                                      (uint32_t)(1024 * r), kAuxNt);
                pw[r] = 0.f;
              }
            }
          }
        } else {
          const __amdgpu_buffer_rsrc_t rs = rsrc(p.out + (size_t)(m0 + it) * kN, it < ng ? kN * 8 : 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            v2f o;
            o.x = dre[r];
            o.y = dim[r];
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, o),
                                                  rs, out_off, (uint32_t)(2048 * r), kAuxNt);
          }
        }
      }
    }
  }
};

template <int PF, int AUX, int IT, bool POW>
__global__ void __launch_bounds__(kThreads) ppf_mfma_kernel(MfmaParams p) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds_mfma[];
  const int lb = xcd_tile(blockIdx.x, p.nblocks);
  if (lb * p.S >= p.M) return;    // whole block idle
  MfmaEngine<PF, AUX, IT, POW> eng(p, lds_mfma);
  eng.init(lb);
  eng.run();
}

// ---------------------------------------------------------------------------
// N = 256 = 16^2 and N = 1024 = 16^2 * 4
//
// With c = a + 16 b + 256 p (p < 4 at N = 1024, absent at N = 256) and
// k = k1 + 4 k2 + 64 k3 at N = 1024 the exponent c k splits so that
//   X = sum_a W16^(a k3) W1024^(a (k1 + 4 k2)) sum_b W64^(b (k1 + 4 k2)) sum_p W4^(p k1) u[c]:
// a radix-4 DFT over p in FP32 registers (the four channels a lane holds),
// a 16-point transform over b whose matrix W64^(b (4 k2 + k1)) carries the
// inter-stage twiddle (k1 is fixed per wave), one FP32 twiddle, and a
// plain 16-point DFT over a; the last two on the matrix cores. At N = 256
// (c = a + 16 b, k = k1 + 16 k2): a 16-point DFT over b, the FP32 twiddle
// W256^(a k1), a 16-point DFT over a.
//
// A spectrum takes N / 256 waves; a 1024-thread workgroup holds 16 / (N /
// 256) groups, each with its own tile of spectra (all groups of a block
// step together). Lane (w, j, h) of a group owns channels
//   N = 1024: j + 16 h + 64 w + 256 e  (a = j, b = h + 4 w, p = e),
//   N = 256:  j + 64 h + 16 e          (a = j, b = 4 h + e),
// e < 4, so the FIR output is the stage-1 input without an exchange. The
// ring has TQ slots (8 or 16 taps). Stage outputs go through swizzled LDS
// buffers (per group) with every half-wave's 4-byte writes on distinct
// banks and 16-byte reads of whole groups.
// ---------------------------------------------------------------------------

template <int N, int TQ, int PF, int AUX, int IT, bool POW>
struct MfmaSmall {
  static constexpr int GW = N / 256;           // waves per spectrum
  static constexpr int GL = 64 * GW;           // lanes per group
#ifndef PPF_MFMA_SMALL_G
#define PPF_MFMA_SMALL_G 1
#endif
  // groups per workgroup (each its own tile); one group per workgroup lets
  // the workgroups on a CU pass their barriers independently
  static constexpr int G = PPF_MFMA_SMALL_G > kThreads / GL ? kThreads / GL : PPF_MFMA_SMALL_G;
  static constexpr int BT = G * GL;            // threads per workgroup
  static constexpr int SB = IT == kInI8 ? 2 : 4;
  static constexpr int CoefBytes = TQ * N * 2;
  static constexpr int XB = N * 4;             // one FP16 complex exchange buffer
  static constexpr int NX = N == 1024 ? 2 : 1;
  static constexpr int LdsBytes = CoefBytes + G * NX * XB;
  static constexpr int ESTRIDE = N == 1024 ? 256 : 16;   // channel step of element e
  static_assert(N == 256 || N == 1024, "built for N = 256 and 1024");
  static_assert(TQ % PF == 0, "prefetch depth divides the ring");

  const MfmaParams& p;
  uint8_t* lds;
  int tid, grp, lg, w, j, h;
  int m0, ng, niter;
  int vb_lo, vb_hi;
  uint32_t in_off, out_off, cf;
  uint32_t xw, xr, yw, yr;   // exchange byte offsets (r = 0 writes, reads)
  h8 a2, a3;                 // A operands of the matrix-core stages
  v2f twv[4];                // FP32 twiddles of this lane's stage outputs
  h2 sc, bias;
  float pw[4] = {0.f, 0.f, 0.f, 0.f};

  __device__ __forceinline__ MfmaSmall(const MfmaParams& p_, uint8_t* lds_) : p(p_), lds(lds_) {}

  // X (N = 1024, stage 1 -> 2): word 256 k1 + 16 a + b, bits 2-3 ^= bits 6-7
  static __device__ __forceinline__ constexpr int swx(int x) { return x ^ (((x >> 6) & 3) << 2); }
  // Y: N = 1024 word 16 kappa + a (kappa = k1 + 4 k2), bits 4-5 ^= bits 8-9;
  //    N = 256 word 16 k1 + a, bits 4-5 ^= bits 6-7
  static __device__ __forceinline__ constexpr int swy(int x) {
    return N == 1024 ? x ^ (((x >> 8) & 3) << 4) : x ^ (((x >> 6) & 3) << 4);
  }

  __device__ __forceinline__ const uint8_t* block_ptr(int rb) const {
    return rb < p.h0 ? (const uint8_t*)p.x0 + (size_t)rb * N * SB
                     : (const uint8_t*)p.x1 + (size_t)(rb - p.h0) * N * SB;
  }
  __device__ __forceinline__ void load(uint32_t (&dst)[4], int vb) const {
    const bool in = vb >= vb_lo && vb < vb_hi;
    const __amdgpu_buffer_rsrc_t rs = rsrc(in ? block_ptr(vb - p.d) : p.x1, in ? N * SB : 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if constexpr (IT == kInI8) dst[e] = __builtin_amdgcn_raw_buffer_load_b16(rs, in_off, ESTRIDE * SB * e, AUX);
      else dst[e] = __builtin_amdgcn_raw_buffer_load_b32(rs, in_off, ESTRIDE * SB * e, AUX);
    }
  }
  __device__ __forceinline__ void widen(const uint32_t (&raw)[4], uint32_t (&slot)[4]) const {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if constexpr (IT == kInI8) {
        slot[e] = widen1(raw[e], sc, bias);
      } else {
        // FP16 as stored; an explicit move gives the slot a definition of
        // its own at this step (letting the load's register be the slot
        // measured 70+ VGPRs of spills)
        asm volatile("v_mov_b32 %0, %1" : "=v"(slot[e]) : "v"(raw[e]));
      }
    }
  }

  __device__ __forceinline__ void init(int lb) {
    tid = threadIdx.x;
    grp = tid / GL;
    lg = tid % GL;
    w = lg >> 6;
    j = tid & 15;
    h = (tid >> 4) & 3;
    const int blk_m0 = lb * G * p.S;
    const int brem = p.M - blk_m0;
    niter = brem < p.S ? brem : p.S;          // the block's first group has the most
    m0 = blk_m0 + grp * p.S;
    const int rem = p.M - m0;
    ng = rem <= 0 ? 0 : (rem < p.S ? rem : p.S);
    vb_lo = m0 > p.d ? m0 : p.d;
    vb_hi = ng > 0 ? m0 + ng + TQ - 1 : m0;
    const int c0 = N == 1024 ? j + 16 * h + 64 * w : j + 64 * h;
    in_off = (uint32_t)c0 * (uint32_t)SB;
    cf = (uint32_t)lg * 8u;
    const uint32_t xg = CoefBytes + grp * NX * XB;
    if constexpr (N == 1024) {
      out_off = (uint32_t)(16 * w + j + 256 * h) * 8u;
      xw = xg + swx(16 * j + 4 * w + h) * 4;                  // + 1024 r (k1 = r: above the swizzle)
      xr = xg + swx(256 * w + 16 * j + 4 * h) * 4;            // k1 = w, a = j, b = 4h..4h+3
      yw = xg + XB + swy(16 * w + 256 * h + j) * 4;           // + 256 r bytes (bits 6-7: not swizzled)
      yr = xg + XB + swy(256 * w + 16 * j + 4 * h) * 4;       // kappa = 16 w + j, a = 4h..4h+3
    } else {
      out_off = (uint32_t)(j + 64 * h) * 8u;
      yw = xg + (64 * h + j) * 4;                             // word 64 h + 16 (r ^ h) + j
      yr = xg + swy(16 * j + 4 * h) * 4;                      // k1 = j, a = 4h..4h+3
    }
    const _Float16 s16 = (_Float16)p.in_scale;
    sc = h2{s16, s16};
    const _Float16 b16 = (_Float16)(-1152.0f * p.in_scale);
    bias = h2{b16, b16};

    for (int i = tid; i < CoefBytes / 16; i += BT) ((uint4*)lds)[i] = p.coef[i];

    // A operands (real-part row j; inputs point 4h+e, re/im interleaved)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int q = 4 * h + e;
      const h2 wa = __builtin_bit_cast(h2, p.w256[N == 1024 ? (4 * q * (4 * j + w)) & 255 : (16 * q * j) & 255]);
      const h2 w3 = __builtin_bit_cast(h2, p.w256[(16 * q * j) & 255]);
      a2[2 * e] = wa.x;                       // N = 1024: W64^(b (4 k2 + k1)); N = 256: W16^(b k1)
      a2[2 * e + 1] = -wa.y;
      a3[2 * e] = (_Float16)((float)w3.x * p.out_scale);
      a3[2 * e + 1] = (_Float16)(-(float)w3.y * p.out_scale);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
      twv[r] = N == 1024 ? p.tw[(j * (w + 4 * (4 * h + r))) & (N - 1)] : p.tw[(j * (4 * h + r)) & (N - 1)];
  }

  __device__ __forceinline__ void dft16(const h8& a, const h8& b, f4& dre, f4& dim) const {
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    dre = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, z, 0, 0, 0);
    const uint4 bu = __builtin_bit_cast(uint4, b);
    uint4 bq;
    const uint32_t one_neg = 0xBC003C00u;   // FP16 (1.0, -1.0)
    asm("v_pk_mul_f16 %0, %1, %2 op_sel:[1,0] op_sel_hi:[0,1]" : "=v"(bq.x) : "v"(bu.x), "s"(one_neg));
    asm("v_pk_mul_f16 %0, %1, %2 op_sel:[1,0] op_sel_hi:[0,1]" : "=v"(bq.y) : "v"(bu.y), "s"(one_neg));
    asm("v_pk_mul_f16 %0, %1, %2 op_sel:[1,0] op_sel_hi:[0,1]" : "=v"(bq.z) : "v"(bu.z), "s"(one_neg));
    asm("v_pk_mul_f16 %0, %1, %2 op_sel:[1,0] op_sel_hi:[0,1]" : "=v"(bq.w) : "v"(bu.w), "s"(one_neg));
    dim = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, __builtin_bit_cast(h8, bq), z, 0, 0, 0);
  }

  // exchange within a wave (N = 256): LDS operations of one wave complete
  // in order; the fences keep the compiler from moving them across
  __device__ __forceinline__ static void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }

  __device__ __forceinline__ void run() {
    uint32_t ring[TQ][4];
    uint32_t stage[PF][4];
#pragma unroll
    for (int s = 0; s < TQ; ++s)
#pragma unroll
      for (int e = 0; e < 4; ++e) ring[s][e] = 0u;
#pragma unroll
    for (int s = 0; s < PF; ++s)
#pragma unroll
      for (int e = 0; e < 4; ++e) stage[s][e] = 0u;
#pragma unroll
    for (int s = 0; s < TQ - 1; ++s) {
      uint32_t raw[4];
      load(raw, m0 + s);
      widen(raw, ring[s]);
    }
#pragma unroll
    for (int s = 0; s < PF; ++s) load(stage[s], m0 + TQ - 1 + s);
    __syncthreads();   // coefficients in LDS

    // every group runs the block's step count (barriers); steps past its
    // own spectra run on zero input and store into an empty range
    for (int base = 0; base < niter; base += TQ) {
#pragma unroll
      for (int k = 0; k < TQ; ++k) {
        const int it = base + k;
        widen(stage[k % PF], ring[(k + TQ - 1) % TQ]);
        load(stage[k % PF], m0 + it + TQ - 1 + PF);
#pragma unroll
        for (int s = 0; s < TQ; ++s)
#pragma unroll
          for (int e = 0; e < 4; ++e) asm volatile("" : "+v"(ring[s][e]));
        float ar[4] = {0.f, 0.f, 0.f, 0.f}, ai[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < TQ; ++t) {
          const h4 hv = *(const h4*)(lds + t * (GL * 8) + cf);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const h2 xv = __builtin_bit_cast(h2, ring[(k + t) % TQ][e]);
            ar[e] = fmaf((float)hv[e], (float)xv.x, ar[e]);
            ai[e] = fmaf((float)hv[e], (float)xv.y, ai[e]);
          }
        }
        if constexpr (IT == kInF16) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            ar[e] *= p.in_scale;
            ai[e] *= p.in_scale;
          }
        }
        f4 dre, dim;
        if constexpr (N == 1024) {
          // stage 1: radix-4 over p = e in FP32 (y_k1 = sum_p (-i)^(p k1) u_p)
          const float t0r = ar[0] + ar[2], t0i = ai[0] + ai[2];
          const float t1r = ar[0] - ar[2], t1i = ai[0] - ai[2];
          const float t2r = ar[1] + ar[3], t2i = ai[1] + ai[3];
          const float t3r = ar[1] - ar[3], t3i = ai[1] - ai[3];
          uint32_t* dx = (uint32_t*)(lds + xw);
          asm volatile("" : "+v"(dx));
          dx[0] = pack_h2(t0r + t2r, t0i + t2i);         // k1 = 0
          dx[256] = pack_h2(t1r + t3i, t1i - t3r);       // k1 = 1: t1 - i t3
          dx[512] = pack_h2(t0r - t2r, t0i - t2i);       // k1 = 2
          dx[768] = pack_h2(t1r - t3i, t1i + t3r);       // k1 = 3: t1 + i t3
          __syncthreads();
          dft16(a2, __builtin_bit_cast(h8, *(const uint4*)(lds + xr)), dre, dim);   // over b
          // W1024^(a (k1 + 4 k2)) in FP32, to the stage-3 layout
          uint32_t* dy = (uint32_t*)(lds + yw);
          asm volatile("" : "+v"(dy));
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float yr_ = fmaf(dre[r], twv[r].x, -dim[r] * twv[r].y);
            const float yi_ = fmaf(dre[r], twv[r].y, dim[r] * twv[r].x);
            dy[64 * r] = pack_h2(yr_, yi_);
          }
          __syncthreads();
          dft16(a3, __builtin_bit_cast(h8, *(const uint4*)(lds + yr)), dre, dim);   // over a
        } else {
          h8 b;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            b[2 * e] = (_Float16)ar[e];
            b[2 * e + 1] = (_Float16)ai[e];
          }
          dft16(a2, b, dre, dim);                                  // over b
          uint32_t yb = yw;
          int hh = h;
          asm volatile("" : "+v"(yb), "+v"(hh));
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float yr_ = fmaf(dre[r], twv[r].x, -dim[r] * twv[r].y);
            const float yi_ = fmaf(dre[r], twv[r].y, dim[r] * twv[r].x);
            *(uint32_t*)(lds + yb + ((r ^ hh) << 6)) = pack_h2(yr_, yi_);   // 16 (r ^ h) words
          }
          wave_sync();
          dft16(a3, __builtin_bit_cast(h8, *(const uint4*)(lds + yr)), dre, dim);   // over a
          wave_sync();                                             // reads done before the next writes
        }
        // bins: N = 1024 k = 16 w + j + 256 h + 64 r; N = 256 k = j + 64 h + 16 r
        constexpr uint32_t RSTEP = N == 1024 ? 64u : 16u;
        if constexpr (POW) {
          if (it < ng) {
#pragma unroll
            for (int r = 0; r < 4; ++r) pw[r] += fmaf(dre[r], dre[r], dim[r] * dim[r]);
            if ((m0 + it + 1) % p.K == 0) {
              const long long q = (long long)(m0 + it) / p.K;
              const __amdgpu_buffer_rsrc_t rs = rsrc(p.pout + q * N, N * 4);
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, pw[r]), rs, out_off / 2,
                                                      RSTEP * 4u * r, kAuxNt);
                pw[r] = 0.f;
              }
            }
          }
        } else {
          const __amdgpu_buffer_rsrc_t rs = rsrc(p.out + (size_t)(m0 + it) * N, it < ng ? N * 8 : 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            v2f o;
            o.x = dre[r];
            o.y = dim[r];
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, o), rs, out_off, RSTEP * 8u * r, kAuxNt);
          }
        }
      }
    }
  }
};

// 4 waves per SIMD (128 VGPRs) whatever the workgroup size
template <int N, int TQ, int PF, int AUX, int IT, bool POW>
__global__ void __launch_bounds__((MfmaSmall<N, TQ, PF, AUX, IT, POW>::BT)) __attribute__((amdgpu_waves_per_eu(4)))
ppf_mfma_small_kernel(MfmaParams p) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds_small[];
  using E = MfmaSmall<N, TQ, PF, AUX, IT, POW>;
  const int lb = xcd_tile(blockIdx.x, p.nblocks);
  if (lb * E::G * p.S >= p.M) return;    // whole block idle
  E eng(p, lds_small);
  eng.init(lb);
  eng.run();
}

__global__ void ppf_w256_kernel(uint32_t* t) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < 256) {
    double s, c;
    sincospi(-2.0 * (double)k / 256.0, &s, &c);   // exact angle, rounded once to FP16
    h2 v;
    v.x = (_Float16)c;
    v.y = (_Float16)s;
    t[k] = __builtin_bit_cast(uint32_t, v);
  }
}

#ifndef PPF_MFMA_PF
#define PPF_MFMA_PF 1
#endif
#ifndef PPF_MFMA_NT
#define PPF_MFMA_NT 0
#endif
using MfmaKernel = void (*)(MfmaParams);
template <int IT, bool POW>
constexpr MfmaKernel mfma_kernel() { return ppf_mfma_kernel<PPF_MFMA_PF, PPF_MFMA_NT ? kAuxNt : 0, IT, POW>; }
template <int N, int TQ, int IT, bool POW>
constexpr MfmaKernel mfma_small_kernel() {
  return ppf_mfma_small_kernel<N, TQ, PPF_MFMA_PF, PPF_MFMA_NT ? kAuxNt : 0, IT, POW>;
}

int cu_count() {
  static int n = 0;
  if (!n) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
      n = 256;
  }
  return n;
}

}  // namespace

bool mfma_available(int N, int TP) { return (N == kN || N == 1024 || N == 256) && TP <= kTaps; }

int mfma_tap_slots(int N, int T) { return N == kN ? kTaps : (T <= 8 ? 8 : 16); }

size_t mfma_coef_bytes(int N, int TQ) { return (size_t)TQ * N * 2; }

// FP16 coefficients h16[t*N + c] (T taps) -> lane-order table of TQ slots,
// the first TQ-T zero: slot t, lane l (of a group of N/4), element e holds
// the coefficient of the channel that lane loads:
//   N = 4096: 16*(l/64) + l%16 + 1024*((l/16)%4) + 256*e
//   N = 1024: l%16 + 16*((l/16)%4) + 64*(l/64) + 256*e
//   N = 256:  l%16 + 64*((l/16)%4) + 16*e
void mfma_coef_layout(int N, int TQ, const uint16_t* h16, int T, uint16_t* dst) {
  const int d = TQ - T;
  for (int t = 0; t < TQ; ++t)
    for (int l = 0; l < N / 4; ++l)
      for (int e = 0; e < 4; ++e) {
        const int j = l & 15, h = (l >> 4) & 3, w = l >> 6;
        const int c = N == kN ? 16 * w + j + 1024 * h + 256 * e
                              : (N == 1024 ? j + 16 * h + 64 * w + 256 * e : j + 64 * h + 16 * e);
        dst[(size_t)t * N + l * 4 + e] = t < d ? (uint16_t)0 : h16[(size_t)(t - d) * N + c];
      }
}

hipError_t launch_w256(void* table, hipStream_t st) {
  hipLaunchKernelGGL(ppf_w256_kernel, dim3(1), dim3(256), 0, st, (uint32_t*)table);
  return hipGetLastError();
}

namespace {

// Tiles per resident workgroup slot: two at N = 1024 (the C2 shape at 2^27
// samples: FP16 input 0.364 -> 0.343 ms, int8 0.296 -> 0.288 ms, same box),
// one at N = 4096 (two measured 3% slower) and N = 256.
// PPF_MFMA_TILE_SPLIT > 0 overrides it at build time (tuning).
#ifndef PPF_MFMA_TILE_SPLIT
#define PPF_MFMA_TILE_SPLIT 0
#endif
constexpr int mfma_tile_split(int n) { return PPF_MFMA_TILE_SPLIT > 0 ? PPF_MFMA_TILE_SPLIT : (n == 1024 ? 2 : 1); }

// NN = 4096 (three matrix-core stages) or 1024 / 256 (MfmaSmall, TQ tap
// slots); G spectra tiles per workgroup
template <int NN, int TQ, int IT, bool POW>
hipError_t mfma_launch(const MfmaDev& md, const BatchArgs& a, float* pout, int K, hipStream_t st) {
  if (a.M <= 0) return hipSuccess;
  constexpr bool big = NN == kN;
  constexpr MfmaKernel kern = big ? mfma_kernel<IT, POW>() : mfma_small_kernel<big ? 256 : NN, TQ, IT, POW>();
  constexpr int kN = NN;
  constexpr int G = big ? 1 : MfmaSmall<big ? 256 : NN, TQ, 1, 0, IT, POW>::G;
  constexpr int kLdsBytes = big ? ppf::kLdsBytes : MfmaSmall<big ? 256 : NN, TQ, 1, 0, IT, POW>::LdsBytes;
  constexpr int kStep = big ? kTaps : TQ;     // unrolled steps per tile round
  constexpr int kBlock = big ? kThreads : MfmaSmall<big ? 256 : NN, TQ, 1, 0, IT, POW>::BT;
  constexpr int kPerCu = kThreads / kBlock;     // workgroups resident per CU (1024 threads)
  constexpr int SB = IT == kInI8 ? 2 : 4;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (e != hipSuccess) return e;
    attr = true;
  }
  // one workgroup per CU (the LDS holds a single one); split larger
  // batches into launches whose spectrum indices fit in 32 bits (whole
  // groups of K spectra when detecting)
  const long long kMaxLaunch = POW ? (1ll << 28) / K * K : (1ll << 28);
  for (long long s0 = 0; s0 < a.M; s0 += kMaxLaunch) {
    const long long k = a.M - s0 < kMaxLaunch ? a.M - s0 : kMaxLaunch;
    MfmaParams p;
    if (s0 < a.h0) {
      p.x0 = (const uint8_t*)a.x0 + (size_t)s0 * kN * SB;
      p.h0 = (int)(a.h0 - s0);
      p.x1 = a.x1;
    } else {
      p.x0 = a.x1;
      p.h0 = 0;
      p.x1 = (const uint8_t*)a.x1 + (size_t)(s0 - a.h0) * kN * SB;
    }
    p.out = POW ? nullptr : (v2f*)a.out + (size_t)s0 * kN;
    p.pout = POW ? pout + (size_t)(s0 / K) * kN : nullptr;
    p.K = K;
    p.coef = (const uint4*)md.coef16;
    p.tw = (const v2f*)md.tw;
    p.w256 = (const uint32_t*)md.w256;
    p.M = (int)k;
    // tiles of a multiple of the unrolled step count, and of K when
    // detecting, about one workgroup (G tiles) per CU
    const int cus = cu_count();
    const long long slots = (long long)cus * kPerCu * G * mfma_tile_split(NN);
    long long S = (k + slots - 1) / slots;
    S = (S + kStep - 1) / kStep * kStep;
    if (POW) {
      long long unit = kStep;
      while (unit % K) unit += kStep;   // lcm(step, K)
      S = (S + unit - 1) / unit * unit;
    }
    p.S = (int)S;
    p.nblocks = (int)((k + S * G - 1) / (S * G));
    p.d = md.d;
    p.in_scale = md.in_scale;
    p.out_scale = md.out_scale;
    hipLaunchKernelGGL(kern, dim3(p.nblocks), dim3(kBlock), kLdsBytes, st, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <bool POW>
hipError_t mfma_dispatch(const MfmaDev& md, const BatchArgs& a, float* pout, int K, hipStream_t st) {
  const bool f16 = md.in_type == kInF16;
  switch (md.N) {
    case kN:
      return f16 ? mfma_launch<kN, 16, kInF16, POW>(md, a, pout, K, st) : mfma_launch<kN, 16, kInI8, POW>(md, a, pout, K, st);
    case 1024:
      if (md.tq == 8)
        return f16 ? mfma_launch<1024, 8, kInF16, POW>(md, a, pout, K, st) : mfma_launch<1024, 8, kInI8, POW>(md, a, pout, K, st);
      return f16 ? mfma_launch<1024, 16, kInF16, POW>(md, a, pout, K, st) : mfma_launch<1024, 16, kInI8, POW>(md, a, pout, K, st);
    case 256:
      if (md.tq == 8)
        return f16 ? mfma_launch<256, 8, kInF16, POW>(md, a, pout, K, st) : mfma_launch<256, 8, kInI8, POW>(md, a, pout, K, st);
      return f16 ? mfma_launch<256, 16, kInF16, POW>(md, a, pout, K, st) : mfma_launch<256, 16, kInI8, POW>(md, a, pout, K, st);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_mfma(const MfmaDev& md, const BatchArgs& a, hipStream_t st) {
  return mfma_dispatch<false>(md, a, nullptr, 1, st);
}

hipError_t launch_mfma_power(const MfmaDev& md, const BatchArgs& a, float* pout, int K, hipStream_t st) {
  return mfma_dispatch<true>(md, a, pout, K, st);
}

}  // namespace ppf
