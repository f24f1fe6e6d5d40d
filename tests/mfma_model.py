"""Rounding-point model of the matrix-core precision form, for its error bar.

Test infrastructure: it derives the SNR that the FP16 matrix-core DFT
stages can reach, so that the GPU test's bar rests on a computation rather
than on a guess. It is not a reference for parity (the FP64 oracle is) and
shares nothing with the HIP library.

The N = 4096 = 16^3 transform is taken as three 16-point stages, with
c = a + 16 b + 256 p and k = k1 + 16 k2 + 256 k3:

    X[k] = sum_a W16^(a k3) W4096^(a (k1 + 16 k2))
             sum_b W256^(b (16 k2 + k1)) sum_p W16^(p k1) u[c]

and values are rounded where the kernel rounds them:
  * samples x * 2^-e1 and coefficients h16 are exact FP16 values; the FIR
    products are exact and each tap's sum is rounded to FP32, taps in
    order;
  * the presum, the stage-1 output and the twiddled stage-2 output are
    rounded to FP16 (round to nearest even) before the next stage;
  * every DFT matrix entry is exp(-2 pi i k/256) rounded once to FP16, and
    the stage-3 matrix also carries the exact factor 2^(e1 - s);
  * each stage's 16-term sum of exact FP16 x FP16 products, and the
    twiddle multiply with exp(-2 pi i k/4096) rounded to FP32, are rounded
    to FP32.
The sample scale e1 follows the plan's rule: the smallest power that keeps
every FP16 stage input below 60000 for any input (|x| <= 128 for int8,
65504 for FP16; growth <= 16 per stage), at least -8, at least s - 12, and
at most s + 15 (and 24 for int8). int8 samples are scaled as they are
widened, FP16 samples enter as stored and the FP32 sums are scaled; both
scalings are exact powers of two, so the model scales the samples.

N = 1024 = 16^2 * 4 (c = a + 16 b + 256 p, k = k1 + 4 k2 + 64 k3):
  X[k] = sum_a W16^(a k3) W1024^(a (k1 + 4 k2)) sum_b W64^(b (k1 + 4 k2)) sum_p W4^(p k1) u[c]
with the radix-4 DFT over p in FP32 (t0 = u0 + u2, t1 = u0 - u2, t2 = u1 + u3,
t3 = u1 - u3; y0 = t0 + t2, y2 = t0 - t2, y1 = t1 - i t3, y3 = t1 + i t3,
every addition rounded to FP32), its outputs rounded to FP16, the stage-2
matrix entries W64^(b (4 k2 + k1)) = W256^(4 b (4 k2 + k1)) rounded to
FP16, then the FP32 twiddle, FP16 rounding and the stage-3 DFT-16 as at
N = 4096. N = 256 (c = a + 16 b, k = k1 + 16 k2): FIR output to FP16, a
DFT-16 over b, the FP32 twiddle W256^(a k1), FP16, a DFT-16 over a.
The growth before the last FP16 stage input is 256, 64 and 16 for N =
4096, 1024 and 256.
"""

from __future__ import annotations

import math

import numpy as np

N = 4096


GROWTH = {4096: 256.0, 1024: 64.0, 256: 16.0}


def sample_exponent(h16: np.ndarray, shift: int, taps: int, fp16_input: bool = False) -> int:
    n = h16.size // taps
    h = np.abs(h16.astype(np.float64)).reshape(taps, n)
    smax = float(h.sum(axis=0).max())
    xmax = 65504.0 if fp16_input else 128.0
    e1 = math.ceil(math.log2(xmax * GROWTH[n] * smax / 60000.0)) if smax > 0 else -8
    e1 = max(e1, -8, shift - 12)
    if e1 > (shift + 15 if fp16_input else min(shift + 15, 24)):
        raise ValueError("coefficients outside the matrix-core scaling window")
    return e1


_EXACT = False   # set by model(..., exact=True): no rounding anywhere (checks the factorisation)


def _f16c(z):
    """Round a complex array's parts to FP16 (nearest even)."""
    if _EXACT:
        return z
    return z.real.astype(np.float16).astype(np.float64) + 1j * z.imag.astype(np.float16).astype(np.float64)


def _f32c(z):
    if _EXACT:
        return z
    return z.real.astype(np.float32).astype(np.float64) + 1j * z.imag.astype(np.float32).astype(np.float64)


def w256_fp16() -> np.ndarray:
    k = np.arange(256)
    return _f16c(np.exp(-2j * np.pi * k / 256.0))


def model(x_int8: np.ndarray, h16: np.ndarray, shift: int, taps: int, spectra, exact: bool = False) -> np.ndarray:
    """The modelled matrix-core output for the listed spectra (complex128).

    x_int8: (L, 2) int8 or float16 (re, im) pairs; h16: FP16 coefficients
    h[t*N + c] scaled by 2^shift. exact=True drops every rounding (the factorisation
    alone, which must reproduce the plain DFT).
    """
    global _EXACT
    _EXACT = exact
    try:
        return _model(x_int8, h16, shift, taps, spectra)
    finally:
        _EXACT = False


def _fir(x_int8, h16, shift, taps, spectra, n):
    """FP32 FIR sums of the scaled samples (taps in order) and e1."""
    e1 = sample_exponent(h16, shift, taps, fp16_input=x_int8.dtype == np.float16)
    m_idx = np.asarray(list(spectra), dtype=np.int64)
    xs = (x_int8[:, 0].astype(np.float64) + 1j * x_int8[:, 1].astype(np.float64)) * 2.0 ** -e1
    blocks = xs.reshape(-1, n)
    hf = h16.astype(np.float64).reshape(taps, n)
    acc_t = np.float64 if _EXACT else np.float32
    acc_r = np.zeros((m_idx.size, n), acc_t)
    acc_i = np.zeros((m_idx.size, n), acc_t)
    for t in range(taps):
        b = blocks[m_idx + t]
        acc_r = (acc_r.astype(np.float64) + hf[t] * b.real).astype(acc_t)
        acc_i = (acc_i.astype(np.float64) + hf[t] * b.imag).astype(acc_t)
    return acc_r.astype(np.float64), acc_i.astype(np.float64), e1


def _r32(v):
    return v if _EXACT else v.astype(np.float32).astype(np.float64)


def _model_1024(x_int8, h16, shift, taps, spectra):
    n = 1024
    ur, ui, e1 = _fir(x_int8, h16, shift, taps, spectra, n)
    # c = a + 16 b + 256 p -> [m, p, b, a]
    ur = ur.reshape(-1, 4, 16, 16)
    ui = ui.reshape(-1, 4, 16, 16)
    t0r, t0i = _r32(ur[:, 0] + ur[:, 2]), _r32(ui[:, 0] + ui[:, 2])
    t1r, t1i = _r32(ur[:, 0] - ur[:, 2]), _r32(ui[:, 0] - ui[:, 2])
    t2r, t2i = _r32(ur[:, 1] + ur[:, 3]), _r32(ui[:, 1] + ui[:, 3])
    t3r, t3i = _r32(ur[:, 1] - ur[:, 3]), _r32(ui[:, 1] - ui[:, 3])
    y = np.stack([_r32(t0r + t2r) + 1j * _r32(t0i + t2i),
                  _r32(t1r + t3i) + 1j * _r32(t1i - t3r),
                  _r32(t0r - t2r) + 1j * _r32(t0i - t2i),
                  _r32(t1r - t3i) + 1j * _r32(t1i + t3r)], axis=1)        # [m, k1, b, a]
    Y1 = _f16c(y)
    w = w256_fp16()
    r16, r4 = np.arange(16), np.arange(4)
    # stage 2 matrix [k1, k2, b] = W64^(b (4 k2 + k1)) = W256^(4 b (4 k2 + k1))
    M2 = w[(4 * r16[None, None, :] * (4 * r16[None, :, None] + r4[:, None, None])) & 255]
    D = _f32c(np.einsum("jkb,mjba->mjka", M2, Y1))                           # [m, k1, k2, a]
    kk = r4[:, None] + 4 * r16[None, :]                                      # [k1, k2]
    tw = _f32c(np.exp(-2j * np.pi * ((r16[None, None, :] * kk[:, :, None]) % n) / n))   # [k1, k2, a]
    Y3 = _f16c(_f32c(D * tw[None]))
    H = w[(16 * np.outer(r16, r16)) & 255] * 2.0 ** (e1 - shift)              # [k3, a]
    X = _f32c(np.einsum("ta,mjka->mtkj", H, Y3))                              # [m, k3, k2, k1]
    return X.reshape(-1, n)


def _model_256(x_int8, h16, shift, taps, spectra):
    n = 256
    ur, ui, e1 = _fir(x_int8, h16, shift, taps, spectra, n)
    U = _f16c(ur + 1j * ui).reshape(-1, 16, 16)                               # [m, b, a]
    w = w256_fp16()
    r16 = np.arange(16)
    F1 = w[(16 * np.outer(r16, r16)) & 255]                                   # [k1, b]
    D = _f32c(np.einsum("kb,mba->mka", F1, U))                                # [m, k1, a]
    tw = _f32c(np.exp(-2j * np.pi * ((np.outer(r16, r16)) % n) / n))          # [k1, a]
    Y = _f16c(_f32c(D * tw[None]))
    H = w[(16 * np.outer(r16, r16)) & 255] * 2.0 ** (e1 - shift)              # [k2, a]
    X = _f32c(np.einsum("ta,mka->mtk", H, Y))                                 # [m, k2, k1]
    return X.reshape(-1, n)


def _model(x_int8, h16, shift, taps, spectra):
    n = h16.size // taps
    if n == 1024:
        return _model_1024(x_int8, h16, shift, taps, spectra)
    if n == 256:
        return _model_256(x_int8, h16, shift, taps, spectra)
    e1 = sample_exponent(h16, shift, taps, fp16_input=x_int8.dtype == np.float16)
    m_idx = np.asarray(list(spectra), dtype=np.int64)
    xs = (x_int8[:, 0].astype(np.float64) + 1j * x_int8[:, 1].astype(np.float64)) * 2.0 ** -e1
    blocks = xs.reshape(-1, N)
    hf = h16.astype(np.float64).reshape(taps, N)
    # FIR: FP32 sums of exact products, taps in order
    acc_r = np.zeros((m_idx.size, N), np.float32)
    acc_i = np.zeros((m_idx.size, N), np.float32)
    acc_t = np.float64 if _EXACT else np.float32
    acc_r = acc_r.astype(acc_t)
    acc_i = acc_i.astype(acc_t)
    for t in range(taps):
        b = blocks[m_idx + t]
        acc_r = (acc_r.astype(np.float64) + hf[t] * b.real).astype(acc_t)
        acc_i = (acc_i.astype(np.float64) + hf[t] * b.imag).astype(acc_t)
    u = _f16c(acc_r.astype(np.float64) + 1j * acc_i.astype(np.float64))
    # u[m, c] with c = a + 16 b + 256 p  ->  U[m, p, b, a]
    U = u.reshape(-1, 16, 16, 16)
    w = w256_fp16()
    r16 = np.arange(16)
    F1 = w[(16 * np.outer(r16, r16)) & 255]                                   # [k1, p]
    Y1 = _f16c(_f32c(np.einsum("kp,mpba->mkba", F1, U)))                      # [m, k1, b, a]
    G = w[(r16[None, None, :] * (16 * r16[None, :, None] + r16[:, None, None])) & 255]   # [k1, k2, b]
    Y2 = _f32c(np.einsum("jkb,mjba->mjka", G, Y1))                             # [m, k1, k2, a]
    kk = (r16[:, None] + 16 * r16[None, :])                                   # [k1, k2]
    tw = np.exp(-2j * np.pi * ((r16[None, None, :] * kk[:, :, None]) % N) / N)  # [k1, k2, a]
    tw = _f32c(tw)
    Y3 = _f16c(_f32c(Y2 * tw[None]))
    H = w[(16 * np.outer(r16, r16)) & 255] * 2.0 ** (e1 - shift)              # [k3, a]
    X = _f32c(np.einsum("ta,mjka->mtkj", H, Y3))                               # [m, k3, k2, k1]
    return X.reshape(-1, N)
