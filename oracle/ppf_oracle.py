"""FP64 CPU oracle of the polyphase filter bank (PPF).

TEST INFRASTRUCTURE ONLY. Nothing on the product path imports, calls or
links this module: only the tests, the smoke check and the CPU-baseline leg
of the benchmark do. It shares no code with the HIP library: no kernels,
headers, tables, helpers or pre/post-processing.

What it computes is the plain definition of the PPF, written out without
any blocking, fusion or reordering:

* FIR presum (section 2, Eq. 1, with the per-channel taps of the PPF over N
  channels, section 2 first paragraph, and the spectra x channels x taps
  multiply-accumulate of Algorithm 1):

      u[m][c] = sum_{t=0}^{T-1} h[t*N + c] * x[(m+t)*N + c]

  for 0 <= m < M and 0 <= c < N, where the input holds (M+T-1)*N samples.

* DFT of each presummed block (section 2, the channels become DFT bins;
  section 3, a library FFT follows the FIR):

      X[m][k] = sum_{c=0}^{N-1} u[m][c] * exp(-2 pi i ((c*k) mod N) / N)

Readings of the paper this oracle fixes (the paper leaves them open):

* Tap direction: segment t of the prototype weights block m+t (a windowed
  presum). Per channel this is Eq. 1 with b_i = h[(T-1-i)*N + c] and
  n = m+T-1, i.e. the newest block meets the last segment.
* Output count: only "valid" spectra are produced; M = L/N - T + 1 for an
  input of L samples. Streams start from a zero history.
* DFT sign and scale: forward transform with exp(-2 pi i ck/N), no 1/N
  factor, bins in natural order (the forward default of the FFT libraries
  the paper calls).
* Precision: everything is upcast exactly to FP64 / complex128 first; FP32,
  FP16 and int8 inputs are all exactly representable.

Steps run in the order above: upcast, view as blocks, presum summing taps
t = 0 .. T-1 in order, then a matrix product with the explicit DFT matrix
(a BLAS zgemm serves as the matrix-product step, in column slices so the
matrix is never held whole at large N).
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "as_complex128", "n_spectra", "twiddles", "dft_matrix_columns",
    "fir_presum", "dft", "ppf", "ppf_stream",
]

# Largest DFT-matrix column slice, in complex128 elements (256 MiB).
_SLICE_ELEMS = 1 << 24


def as_complex128(x) -> np.ndarray:
    """Exact upcast of a stored complex signal to a flat complex128 array.

    Accepts complex arrays, or real arrays of shape (L, 2) holding (re, im)
    pairs (int8 and float16 storage).
    """
    a = np.asarray(x)
    if np.iscomplexobj(a):
        return a.astype(np.complex128, copy=False).reshape(-1)
    if a.ndim == 2 and a.shape[1] == 2:
        re = a[:, 0].astype(np.float64)
        im = a[:, 1].astype(np.float64)
        return re + 1j * im
    raise ValueError("expected a complex array or (L, 2) real pairs")


def n_spectra(n_samples: int, n_channels: int, taps: int) -> int:
    """Number of valid output spectra for an input of n_samples samples."""
    return max(0, n_samples // n_channels - taps + 1)


def twiddles(n: int) -> np.ndarray:
    """W[p] = exp(-2 pi i p / n) for 0 <= p < n, in FP64.

    cos and sin are evaluated on the exactly reduced angle 2 pi p/n; the
    points that lie on an axis (p a multiple of n/4) are set to their exact
    values 1, -i, -1, i, which the library cos/sin only approximate to
    about 1e-16.
    """
    p = np.arange(n, dtype=np.int64)
    ang = 2.0 * np.pi * p.astype(np.float64) / n
    w = np.cos(ang) - 1j * np.sin(ang)
    axis = (4 * p) % n == 0
    quarter = ((4 * p[axis]) // n) % 4
    w[axis] = np.array([1.0, -1j, -1.0, 1j])[quarter]
    return w


def dft_matrix_columns(n: int, k0: int, k1: int, w: np.ndarray | None = None) -> np.ndarray:
    """Columns k0..k1-1 of F[c][k] = W[(c*k) mod n], shape (n, k1-k0)."""
    if w is None:
        w = twiddles(n)
    c = np.arange(n, dtype=np.int64)[:, None]
    k = np.arange(k0, k1, dtype=np.int64)[None, :]
    return w[(c * k) % n]


def fir_presum(x, h, n_channels: int, taps: int, spectra=None) -> np.ndarray:
    """u[m][c] = sum_t h[t*N + c] * x[(m+t)*N + c] (Eq. 1 per channel).

    ``spectra``: optional iterable of output indices m to compute (all valid
    ones by default). Returns complex128 of shape (len(spectra), N).
    """
    n, t_count = int(n_channels), int(taps)
    xs = as_complex128(x)
    hs = np.asarray(h, dtype=np.float64).reshape(-1)
    if hs.size != n * t_count:
        raise ValueError("h must hold taps*n_channels values")
    m_total = n_spectra(xs.size, n, t_count)
    m_idx = np.arange(m_total) if spectra is None else np.asarray(list(spectra), dtype=np.int64)
    if m_idx.size and (m_idx.min() < 0 or m_idx.max() >= m_total):
        raise IndexError("spectrum index out of range")
    blocks = xs[: (m_total + t_count - 1) * n].reshape(-1, n)
    u = np.zeros((m_idx.size, n), dtype=np.complex128)
    for t in range(t_count):
        u += hs[t * n:(t + 1) * n][None, :] * blocks[m_idx + t]
    return u


def dft(u: np.ndarray) -> np.ndarray:
    """X[m][k] = sum_c u[m][c] exp(-2 pi i ck/N) as u @ F, F in column slices."""
    u = np.asarray(u, dtype=np.complex128)
    n = u.shape[-1]
    w = twiddles(n)
    out = np.empty_like(u)
    step = max(1, min(n, _SLICE_ELEMS // n))
    for k0 in range(0, n, step):
        k1 = min(n, k0 + step)
        out[:, k0:k1] = u @ dft_matrix_columns(n, k0, k1, w)
    return out


def ppf(x, h, n_channels: int, taps: int, spectra=None) -> np.ndarray:
    """The PPF: FIR presum over N channels, then the N-point DFT.

    Returns complex128 of shape (M, N), or (len(spectra), N).
    """
    return dft(fir_presum(x, h, n_channels, taps, spectra))


def ppf_stream(chunks, h, n_channels: int, taps: int) -> list[np.ndarray]:
    """Stream form: each chunk of S*N samples yields S spectra.

    The stream starts with (T-1)*N zero samples of history; the outputs are
    the batch PPF over zeros ++ chunk_1 ++ chunk_2 ++ ..., cut at the chunk
    boundaries.
    """
    n, t_count = int(n_channels), int(taps)
    parts = [as_complex128(c) for c in chunks]
    for p in parts:
        if p.size % n:
            raise ValueError("chunk length must be a multiple of N")
    whole = np.concatenate([np.zeros((t_count - 1) * n, dtype=np.complex128)] + parts)
    spectra = ppf(whole, h, n, t_count)
    out, at = [], 0
    for p in parts:
        s = p.size // n
        out.append(spectra[at:at + s])
        at += s
    return out


def ppf_power(x, h, n_channels: int, taps: int, k_int: int) -> np.ndarray:
    """Detected and integrated spectra: the power |X|^2 of each bin summed
    over groups of k_int consecutive spectra (the screening step that follows
    the filter bank in the pipeline of section 1).

        P[j][k] = sum_{i=0}^{k_int-1} |X[j*k_int + i][k]|^2,  0 <= j < M // k_int

    Spectra beyond the last whole group are not used.
    """
    k_int = int(k_int)
    if k_int < 1:
        raise ValueError("k_int must be >= 1")
    spectra = ppf(x, h, n_channels, taps)
    groups = spectra.shape[0] // k_int
    power = np.abs(spectra[:groups * k_int]) ** 2
    return power.reshape(groups, k_int, spectra.shape[1]).sum(axis=1)
