"""FP64 oracle of the prototype-filter design (plan time): test infrastructure only.

Nothing on the product path imports, calls or links this module. It shares
no code with the HIP library or with the seeded input generators.

The coefficients of the PPF come from a constant response function: the
ideal rectangular pass band in frequency is a sinc in time. The sinc is
sampled and its tails are cut off, and the cut is tapered by a window. The
paper uses the Kaiser window (section 2, the paragraphs after Eq. 1).

Readings of the paper, which states neither the cutoff, the window
parameter nor the scaling:

* Prototype of L = T*N points, sampled about its centre with a pass band of
  one channel (cutoff half a bin on each side):

      h[j] = w[j] * sinc((j - (L-1)/2) / N),   sinc(u) = sin(pi u) / (pi u),
      sinc(0) = 1,

  then scaled so that sum_j h[j] = 1 (unit gain at DC).
* Windows (symmetric, L points; L = 1 gives the single value 1):
  rectangular 1; Hamming 0.54 - 0.46 cos(2 pi j/(L-1)); Hann
  0.5 - 0.5 cos(2 pi j/(L-1)); Kaiser I0(beta sqrt(1 - r^2)) / I0(beta)
  with r = 2j/(L-1) - 1; or a window the caller gives.
* beta is the caller's. ``kaiser_beta`` gives Kaiser's published empirical
  rule from the wanted stop-band attenuation A in dB: 0.1102 (A - 8.7) above
  50 dB, 0.5842 (A - 21)^0.4 + 0.07886 (A - 21) from 21 to 50 dB, 0 below.

I0 is the modified Bessel function of the first kind, order zero, summed
from its power series sum_k ((x/2)^k / k!)^2 until the terms no longer
change the sum.
"""

from __future__ import annotations

import numpy as np


def bessel_i0(x) -> np.ndarray:
    """I0(x) from its power series, elementwise, in FP64."""
    x = np.asarray(x, dtype=np.float64)
    q = 0.25 * x * x
    term = np.ones_like(x)
    total = np.ones_like(x)
    k = 0
    while True:
        k += 1
        term = term * q / (k * k)
        total = total + term
        if np.all(term <= total * 1e-17) or k > 1000:
            return total


def window(length: int, kind: str, beta: float | None = None, user=None) -> np.ndarray:
    """Symmetric window of ``length`` points in FP64 (the readings above)."""
    if length < 1:
        raise ValueError("window length must be >= 1")
    if kind == "user":
        w = np.asarray(user, dtype=np.float64).reshape(-1)
        if w.size != length:
            raise ValueError("user window has the wrong length")
        return w.copy()
    if length == 1:
        return np.ones(1)
    j = np.arange(length, dtype=np.float64)
    if kind == "rect":
        return np.ones(length)
    if kind == "hamming":
        return 0.54 - 0.46 * np.cos(2.0 * np.pi * j / (length - 1))
    if kind == "hann":
        return 0.5 - 0.5 * np.cos(2.0 * np.pi * j / (length - 1))
    if kind == "kaiser":
        if beta is None or beta < 0:
            raise ValueError("the Kaiser window needs beta >= 0")
        r = 2.0 * j / (length - 1) - 1.0
        return bessel_i0(beta * np.sqrt(np.maximum(0.0, 1.0 - r * r))) / bessel_i0(beta)
    raise ValueError(f"unknown window {kind!r}")


def sinc(u) -> np.ndarray:
    """sin(pi u) / (pi u), with the value 1 at u = 0."""
    u = np.asarray(u, dtype=np.float64)
    out = np.ones_like(u)
    nz = u != 0
    out[nz] = np.sin(np.pi * u[nz]) / (np.pi * u[nz])
    return out


def prototype(n_channels: int, taps: int, kind: str, beta: float | None = None, user=None) -> np.ndarray:
    """h[0 .. T*N-1] in FP64: windowed sinc of one channel's width, sum 1."""
    n, t = int(n_channels), int(taps)
    if n < 1 or t < 1:
        raise ValueError("n_channels and taps must be >= 1")
    length = n * t
    j = np.arange(length, dtype=np.float64)
    h = window(length, kind, beta, user) * sinc((j - (length - 1) / 2.0) / n)
    s = h.sum()
    if not np.isfinite(s) or s == 0.0:
        raise ValueError("the windowed sinc sums to zero or is not finite")
    return h / s


def kaiser_beta(atten_db: float) -> float:
    """Kaiser's rule for beta from the stop-band attenuation in dB."""
    a = float(atten_db)
    if a > 50.0:
        return 0.1102 * (a - 8.7)
    if a >= 21.0:
        return 0.5842 * (a - 21.0) ** 0.4 + 0.07886 * (a - 21.0)
    return 0.0
