"""Seeded synthetic inputs for the polyphase filter bank (PPF).

This module only *makes inputs*: prototype filter coefficients, complex
voltage streams and their storage encodings. It holds none of the PPF's own
arithmetic (no FIR presum, no DFT), so both the HIP path and the FP64 oracle
can be fed from it without sharing any of the method's code.

Coefficients (paper section 2, the paragraphs after Eq. 1): the ideal
frequency-domain rectangle becomes a sampled sinc in time, its tails are cut
at a finite length and a window tapers the cut. Here the length is T*N (one
segment of N per tap), the cutoff is one channel width (1/N cycles/sample),
the window is applied symmetrically over the whole length and the result is
normalised to unit DC gain (sum of h = 1).

Signals: the paper models its input as complex sampled voltages (section 2,
after Eq. 1) arriving at the single-SKA-LFAA-channel rate (section 1). The
synthetic stand-ins are complex Gaussian noise, optionally with unit tones,
generated on the host with numpy's PCG64 from fixed seeds.
"""

from __future__ import annotations

import numpy as np

#: Base seed for the standard workloads; config i uses SEED_BASE + i.
SEED_BASE = 14113656

#: One second of the single-SKA-LFAA-channel stream is 6.5 GB (section 1 and
#: the definition of the real-time multiple in section 3, Eq. 2).
REALTIME_BYTES_PER_S = 6.5e9


# ---------------------------------------------------------------------------
# prototype filter
# ---------------------------------------------------------------------------

def window(length: int, kind: str = "hamming", beta: float = 8.0) -> np.ndarray:
    """Symmetric window of ``length`` points in FP64.

    ``hamming``: 0.54 - 0.46 cos(2 pi j/(L-1)); ``hann``: 0.5 - 0.5 cos(...);
    ``rect``: all ones; ``kaiser``: I0(beta sqrt(1-(2j/(L-1)-1)^2))/I0(beta),
    the window the paper names (section 2, last paragraph) with its beta left
    to the caller because the paper does not state it.
    """
    if length < 1:
        raise ValueError("window length must be >= 1")
    if length == 1 or kind == "rect":
        return np.ones(length, dtype=np.float64)
    j = np.arange(length, dtype=np.float64)
    phase = 2.0 * np.pi * j / (length - 1)
    if kind == "hamming":
        return 0.54 - 0.46 * np.cos(phase)
    if kind == "hann":
        return 0.5 - 0.5 * np.cos(phase)
    if kind == "kaiser":
        return np.kaiser(length, beta).astype(np.float64)
    raise ValueError(f"unknown window {kind!r}")


def design_coeffs(n_channels: int, taps: int, kind: str = "hamming",
                  beta: float = 8.0) -> np.ndarray:
    """Prototype coefficients h[0 .. taps*n_channels-1] in FP64.

    h[j] = w[j] * sinc((j - (L-1)/2) / N) with sinc(u) = sin(pi u)/(pi u),
    L = taps*N, then scaled so that sum(h) = 1. Segment t of the prototype,
    h[t*N : (t+1)*N], weights input block m+t of output spectrum m.
    """
    n, t = int(n_channels), int(taps)
    if n < 1 or t < 1:
        raise ValueError("n_channels and taps must be >= 1")
    length = n * t
    j = np.arange(length, dtype=np.float64)
    h = window(length, kind, beta) * np.sinc((j - (length - 1) / 2.0) / n)
    return h / h.sum()


def coeffs_fp16(h: np.ndarray, shift: int | None = None) -> tuple[np.ndarray, int]:
    """Stored FP16 form of FP64 coefficients for the reduced-precision plan.

    Coefficients near 2^-12 and below would lose bits to FP16's subnormal
    range, so they are stored as h * 2^shift (an exact power-of-two scale)
    and the FP32 accumulation is multiplied by 2^-shift afterwards. The
    default shift is the largest that keeps max|h| * 2^shift below 2^14.
    Returns (float16 array, shift).
    """
    h = np.asarray(h, dtype=np.float64)
    if shift is None:
        peak = float(np.max(np.abs(h))) if h.size else 1.0
        shift = int(np.floor(14 - np.log2(peak))) if peak > 0 else 0
        shift = max(0, min(shift, 24))
    return (h * (2.0 ** shift)).astype(np.float16), int(shift)


# ---------------------------------------------------------------------------
# signals
# ---------------------------------------------------------------------------

def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def complex_gaussian(n_samples: int, sigma: float, seed: int,
                     dtype=np.complex64) -> np.ndarray:
    """Complex noise: real and imaginary parts independent N(0, sigma^2)."""
    rng = rng_for(seed)
    parts = np.dtype(dtype).type(0).real.dtype
    out = np.empty(int(n_samples), dtype=dtype)
    view = out.view(parts).reshape(-1, 2)
    view[:, 0] = rng.standard_normal(int(n_samples), dtype=np.float64 if parts == np.float64 else np.float32)
    view[:, 1] = rng.standard_normal(int(n_samples), dtype=np.float64 if parts == np.float64 else np.float32)
    if sigma != 1.0:
        view *= parts.type(sigma)
    return out


def tone_plan(n_channels: int, seed: int, count: int = 3, spacing: int = 4):
    """Seed-placed tones: (numerator, denominator, phase) per tone.

    Frequency = numerator/denominator cycles/sample. The first count-1 tones
    sit at bin centres k/N, the last one half a bin above a centre,
    (2k+1)/(2N). Bins are distinct, at least ``spacing`` apart and inside
    [N/8, 7N/8); phases are uniform on [0, 2 pi).
    """
    n = int(n_channels)
    rng = rng_for(seed + 7)
    lo, hi = n // 8, (7 * n) // 8
    if hi - lo < count * spacing:
        raise ValueError("too few channels for the requested tones")
    bins: list[int] = []
    while len(bins) < count:
        k = int(rng.integers(lo, hi))
        if all(abs(k - b) >= spacing for b in bins):
            bins.append(k)
    phases = rng.uniform(0.0, 2.0 * np.pi, size=count)
    tones = [(k, n, float(p)) for k, p in zip(bins[:-1], phases[:-1])]
    tones.append((2 * bins[-1] + 1, 2 * n, float(phases[-1])))
    return tones


def tones(n_samples: int, plan, amplitude: float = 1.0,
          dtype=np.complex128) -> np.ndarray:
    """Sum of amplitude*exp(i(2 pi f n + phi)) with f = num/den.

    The phase is reduced with integers, (n*num mod den)/den, so it stays
    exact for long streams.
    """
    n = np.arange(int(n_samples), dtype=np.int64)
    acc = np.zeros(int(n_samples), dtype=np.complex128)
    for num, den, phi in plan:
        frac = ((n * int(num)) % int(den)).astype(np.float64) / float(den)
        acc += amplitude * np.exp(1j * (2.0 * np.pi * frac + phi))
    return acc.astype(dtype)


def quantize_int8(x: np.ndarray) -> np.ndarray:
    """Complex int8 storage: round half to even, clip to [-127, 127].

    Returns an int8 array of shape (len(x), 2) holding (re, im) pairs, the
    interleaved layout the library reads.
    """
    x = np.asarray(x)
    out = np.empty((x.shape[0], 2), dtype=np.int8)
    out[:, 0] = np.clip(np.rint(x.real), -127, 127)
    out[:, 1] = np.clip(np.rint(x.imag), -127, 127)
    return out


def to_complex_fp16(x: np.ndarray) -> np.ndarray:
    """Complex FP16 storage: float16 (re, im) pairs, shape (len(x), 2)."""
    x = np.asarray(x)
    out = np.empty((x.shape[0], 2), dtype=np.float16)
    out[:, 0] = x.real
    out[:, 1] = x.imag
    return out


# ---------------------------------------------------------------------------
# standard workloads
# ---------------------------------------------------------------------------

def plain_input(n_channels: int, n_samples: int, seed: int, sigma: float = 1.0,
                with_tones: bool = True) -> np.ndarray:
    """Complex FP32 noise (sigma per component) plus three unit tones."""
    x = complex_gaussian(n_samples, sigma, seed, dtype=np.complex64)
    if with_tones:
        x += tones(n_samples, tone_plan(n_channels, seed)).astype(np.complex64)
    return x


def int8_input(n_samples: int, seed: int, sigma: float = 16.0) -> np.ndarray:
    """Complex int8 noise (Gaussian sigma per component, rounded, clipped)."""
    return quantize_int8(complex_gaussian(n_samples, sigma, seed, dtype=np.complex64))
