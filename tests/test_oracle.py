"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each pin checks the oracle against something other than itself: exact
Gaussian-integer brute force, numpy's FFT as a library special case, the
impulse response, a closed form for tones, linearity, Parseval, Hermitian
symmetry and shift invariance. The mutation tests at the end plant a
mistake in a private copy of the oracle (on the CPU) and require that at
least one pin catches it.
"""

from __future__ import annotations

import importlib.util
import pathlib
import types

import numpy as np
import pytest

import oracle.ppf_oracle as ORACLE
from paper_1411_3656_amd import signals

ORACLE_SRC = pathlib.Path(ORACLE.__file__).read_text()


# ---------------------------------------------------------------------------
# independent references used by the pins
# ---------------------------------------------------------------------------

def _mul_pow_minus_i(a: int, b: int, q: int):
    """(a + ib) * (-i)^q with Python integers."""
    q %= 4
    if q == 0:
        return a, b
    if q == 1:
        return b, -a
    if q == 2:
        return -a, -b
    return -b, a


def brute_force_gaussian(xr, xi, h, n, taps):
    """Exact PPF for N in {1, 2, 4} over Gaussian integers (Python ints).

    For these N every DFT twiddle exp(-2 pi i p/N) is a power of -i, so the
    whole transform is exact integer arithmetic.
    """
    assert n in (1, 2, 4)
    m_total = len(xr) // n - taps + 1
    out = []
    for m in range(m_total):
        row = []
        for k in range(n):
            sr = si = 0
            for c in range(n):
                ur = ui = 0
                for t in range(taps):
                    hv = h[t * n + c]
                    ur += hv * xr[(m + t) * n + c]
                    ui += hv * xi[(m + t) * n + c]
                q = ((c * k) % n) * (4 // n)
                pr, pi = _mul_pow_minus_i(ur, ui, q)
                sr += pr
                si += pi
            row.append((sr, si))
        out.append(row)
    return out


def response(h, nu):
    """H(nu) = sum_j h_j exp(-2 pi i nu j): the prototype's frequency response."""
    j = np.arange(len(h), dtype=np.float64)
    return np.exp(-2j * np.pi * np.asarray(nu, dtype=np.float64)[..., None] * j) @ np.asarray(h, np.float64)


def _rms(a):
    return float(np.sqrt(np.mean(np.abs(a) ** 2)))


# ---------------------------------------------------------------------------
# pins, written against an oracle module so that mutants can be checked too
# ---------------------------------------------------------------------------

def pin_p1_bruteforce(mod):
    rng = np.random.default_rng(1)
    for n in (1, 2, 4):
        for taps in (1, 2, 3):
            for m_total in (1, 2, 5):
                length = (m_total + taps - 1) * n
                xr = [int(v) for v in rng.integers(-9, 10, length)]
                xi = [int(v) for v in rng.integers(-9, 10, length)]
                h = [int(v) for v in rng.integers(-5, 6, taps * n)]
                want = np.array(brute_force_gaussian(xr, xi, h, n, taps), dtype=np.float64)
                want = want[..., 0] + 1j * want[..., 1]
                x = np.array(xr, np.float64) + 1j * np.array(xi, np.float64)
                got = mod.ppf(x, np.array(h, np.float64), n, taps)
                assert got.shape == want.shape
                assert np.array_equal(got, want), (n, taps, m_total)
                # the same signal stored as int8 (re, im) pairs
                pairs = np.stack([np.array(xr), np.array(xi)], axis=1).astype(np.int8)
                got8 = mod.ppf(pairs, np.array(h, np.float64), n, taps)
                assert np.array_equal(got8, want), ("int8", n, taps, m_total)


def pin_p2_library_fft(mod):
    rng = np.random.default_rng(2)
    for n in (8, 64, 256):
        m_total = 7
        x = rng.standard_normal(m_total * n) + 1j * rng.standard_normal(m_total * n)
        want = np.fft.fft(x.reshape(m_total, n), axis=1)
        got = mod.ppf(x, np.ones(n), n, 1)
        assert np.max(np.abs(got - want)) <= 1e-12 * _rms(want) * np.sqrt(n)
        w = signals.window(n, "hamming")
        want_w = np.fft.fft(x.reshape(m_total, n) * w[None, :], axis=1)
        got_w = mod.ppf(x, w, n, 1)
        assert np.max(np.abs(got_w - want_w)) <= 1e-12 * _rms(want_w) * np.sqrt(n)


def pin_p3_impulse(mod):
    rng = np.random.default_rng(3)
    n, taps, m_total = 16, 4, 9
    h = rng.standard_normal(taps * n)          # asymmetric on purpose
    t0, c0 = 5, 3
    x = np.zeros((m_total + taps - 1) * n, dtype=np.complex128)
    x[t0 * n + c0] = 1.0
    got = mod.ppf(x, h, n, taps)
    k = np.arange(n)
    phase = np.exp(-2j * np.pi * c0 * k / n)
    for m in range(m_total):
        if t0 - taps + 1 <= m <= t0:
            want = h[(t0 - m) * n + c0] * phase
        else:
            want = np.zeros(n)
        assert np.max(np.abs(got[m] - want)) <= 1e-14, m


def pin_p4_single_segment(mod):
    rng = np.random.default_rng(4)
    n, taps, t_star, m_total = 32, 5, 2, 6
    g = rng.standard_normal(n)
    h = np.zeros(taps * n)
    h[t_star * n:(t_star + 1) * n] = g
    x = rng.standard_normal((m_total + taps - 1) * n) + 1j * rng.standard_normal((m_total + taps - 1) * n)
    blocks = x.reshape(-1, n)
    want = np.fft.fft(blocks[t_star:t_star + m_total] * g[None, :], axis=1)
    got = mod.ppf(x, h, n, taps)
    assert np.max(np.abs(got - want)) <= 1e-12 * _rms(want) * np.sqrt(n)


def pin_p5_tone(mod):
    n, taps, m_total = 64, 8, 6
    h = signals.design_coeffs(n, taps, "hamming")
    length = (m_total + taps - 1) * n
    k = np.arange(n)
    for num, den, phi in [(11, n, 0.3), (2 * 37 + 1, 2 * n, 1.9)]:
        f = num / den
        x = signals.tones(length, [(num, den, phi)])
        got = mod.ppf(x, h, n, taps)
        hk = response(h, k / n - f)
        for m in range(m_total):
            shift = np.exp(2j * np.pi * ((m * n * num) % den) / den)
            want = np.exp(1j * phi) * shift * hk
            assert np.max(np.abs(got[m] - want)) <= 1e-12, (num, den, m)
        if den == n:                               # bin centre: the tone sits in its bin
            assert np.allclose(got[:, num], np.exp(1j * phi), atol=1e-12)
        else:                                      # half bin: two equal neighbours
            kk = num // 2
            assert np.allclose(np.abs(got[:, kk]), np.abs(got[:, kk + 1]), atol=1e-12)
            assert abs(np.abs(got[0, kk]) - 0.50036) < 5e-4


def pin_p6_linearity(mod):
    rng = np.random.default_rng(6)
    n, taps, m_total = 32, 3, 5
    length = (m_total + taps - 1) * n
    a = rng.standard_normal(length) + 1j * rng.standard_normal(length)
    b = rng.standard_normal(length) + 1j * rng.standard_normal(length)
    h = rng.standard_normal(taps * n)
    al, be = 0.7 - 1.3j, -2.1 + 0.4j
    lhs = mod.ppf(al * a + be * b, h, n, taps)
    rhs = al * mod.ppf(a, h, n, taps) + be * mod.ppf(b, h, n, taps)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * _rms(lhs) * np.sqrt(n)


def pin_p7_parseval(mod):
    n, taps, m_total = 256, 8, 400
    h = signals.design_coeffs(n, taps, "hamming")
    x = signals.complex_gaussian((m_total + taps - 1) * n, 1.0, seed=77, dtype=np.complex128)
    u = mod.fir_presum(x, h, n, taps)
    got = mod.ppf(x, h, n, taps)
    lhs = np.sum(np.abs(got) ** 2, axis=1)
    rhs = n * np.sum(np.abs(u) ** 2, axis=1)
    assert np.max(np.abs(lhs - rhs) / rhs) <= 1e-12
    # white noise, sigma 1 per component: E|X|^2 = 2 sum h^2
    expect = 2.0 * np.sum(h ** 2)
    assert abs(np.mean(np.abs(got) ** 2) / expect - 1.0) < 0.05
    assert abs(_rms(got) - 0.0840) < 0.004          # N=256, T=8, Hamming


def pin_p8_hermitian(mod):
    rng = np.random.default_rng(8)
    n, taps, m_total = 64, 4, 5
    x = rng.standard_normal((m_total + taps - 1) * n).astype(np.complex128)
    h = rng.standard_normal(taps * n)
    got = mod.ppf(x, h, n, taps)
    k = np.arange(1, n)
    assert np.max(np.abs(got[:, n - k] - np.conj(got[:, k]))) <= 1e-12 * _rms(got) * np.sqrt(n)
    assert np.max(np.abs(got[:, 0].imag)) <= 1e-12 * _rms(got) * np.sqrt(n)


def pin_p9_shift(mod):
    rng = np.random.default_rng(9)
    n, taps, m_total = 16, 3, 6
    x = rng.standard_normal((m_total + taps) * n) + 1j * rng.standard_normal((m_total + taps) * n)
    h = rng.standard_normal(taps * n)
    full = mod.ppf(x, h, n, taps)
    shifted = mod.ppf(x[n:], h, n, taps)
    assert full.shape[0] == m_total + 1 and shifted.shape[0] == m_total
    assert np.max(np.abs(full[1:] - shifted)) <= 1e-12 * _rms(full) * np.sqrt(n)


def pin_p10_stream(mod):
    rng = np.random.default_rng(10)
    n, taps = 8, 3
    h = rng.standard_normal(taps * n)
    lens = [1, 4, 2, 7]
    chunks = [rng.standard_normal(s * n) + 1j * rng.standard_normal(s * n) for s in lens]
    outs = mod.ppf_stream(chunks, h, n, taps)
    assert [o.shape[0] for o in outs] == lens
    # first spectrum: the two zero history blocks contribute nothing, so only
    # the last segment (t = T-1) meets the first chunk block
    first = np.fft.fft(h[(taps - 1) * n:] * chunks[0][:n])
    assert np.max(np.abs(outs[0][0] - first)) <= 1e-12 * _rms(first) * np.sqrt(n)
    # once T-1 blocks have arrived the stream equals the batch PPF
    whole = np.concatenate(chunks)
    batch = mod.ppf(whole, h, n, taps)
    streamed = np.concatenate(outs)[taps - 1:]
    assert np.max(np.abs(streamed - batch)) <= 1e-12 * _rms(batch) * np.sqrt(n)


def pin_p11_power_tone_exact(mod):
    """Detected power of a bin-centred tone through one rectangular tap:
    X[m][k0] = N A e^(i phi) in every spectrum, so each group of K spectra
    holds K N^2 A^2 in bin k0 and nothing elsewhere."""
    n, amp, phi, k0 = 64, 0.75, 0.4, 9
    for k_int in (1, 3, 8):
        m_total = 2 * k_int + 1                     # one spectrum beyond the last group
        t = np.arange(m_total * n)
        x = amp * np.exp(2j * np.pi * k0 * t / n + 1j * phi)
        p = mod.ppf_power(x, np.ones(n), n, 1, k_int)
        assert p.shape == (m_total // k_int, n)
        want = k_int * n * n * amp * amp
        assert np.allclose(p[:, k0], want, rtol=1e-12), (k_int, p[:, k0], want)
        others = np.delete(p, k0, axis=1)
        assert np.max(others) <= 1e-18 * want * n


def pin_p12_power_parseval(mod):
    """Per group, the summed power over bins is N times the presum energy of
    its K spectra (Parseval), with the presum from the FIR step alone."""
    rng = np.random.default_rng(12)
    n, taps, k_int, m_total = 32, 4, 5, 17
    x = rng.standard_normal((m_total + taps - 1) * n) + 1j * rng.standard_normal((m_total + taps - 1) * n)
    h = rng.standard_normal(taps * n)
    p = mod.ppf_power(x, h, n, taps, k_int)
    u = mod.fir_presum(x, h, n, taps)
    assert p.shape == (m_total // k_int, n)
    for j in range(p.shape[0]):
        energy = 0.0
        for i in range(k_int):
            energy += float(np.sum(np.abs(u[j * k_int + i]) ** 2))
        assert np.isclose(p[j].sum(), n * energy, rtol=1e-10), j


def pin_p13_power_noise_level(mod):
    """White complex noise of variance 2 sigma^2 per sample: the expected
    detected power of a bin is K N 2 sigma^2 sum_t h_c^2 averaged over c,
    i.e. K * 2 sigma^2 * sum(h^2) per bin for the prototype normalised by
    sum over all T*N taps."""
    rng = np.random.default_rng(13)
    n, taps, k_int, m_total, sigma = 128, 4, 4, 400, 1.5
    x = sigma * (rng.standard_normal((m_total + taps - 1) * n) + 1j * rng.standard_normal((m_total + taps - 1) * n))
    h = rng.uniform(0.5, 1.5, taps * n)
    p = mod.ppf_power(x, h, n, taps, k_int)
    expect = k_int * 2 * sigma * sigma * np.sum(h * h)       # per bin, averaged over channels (times N / N)
    assert abs(p.mean() / expect - 1.0) < 0.02, p.mean() / expect


PINS = [pin_p1_bruteforce, pin_p2_library_fft, pin_p3_impulse, pin_p4_single_segment,
        pin_p5_tone, pin_p6_linearity, pin_p7_parseval, pin_p8_hermitian, pin_p9_shift,
        pin_p10_stream, pin_p11_power_tone_exact, pin_p12_power_parseval, pin_p13_power_noise_level]


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_pin_holds_for_oracle(pin):
    pin(ORACLE)


def test_twiddles_exact_on_axes_and_accurate_elsewhere():
    for n in (1, 2, 4, 8, 1024):
        w = ORACLE.twiddles(n)
        p = np.arange(n)
        ref = np.exp(-2j * np.pi * p / n)
        assert np.max(np.abs(w - ref)) <= 4e-16
        if n % 4 == 0:
            assert w[n // 4] == -1j and w[n // 2] == -1 and w[3 * n // 4] == 1j


def test_sampled_spectra_match_full():
    rng = np.random.default_rng(11)
    n, taps, m_total = 32, 4, 20
    x = rng.standard_normal((m_total + taps - 1) * n) + 1j * rng.standard_normal((m_total + taps - 1) * n)
    h = rng.standard_normal(taps * n)
    full = ORACLE.ppf(x, h, n, taps)
    pick = [0, 7, 19]
    assert np.array_equal(ORACLE.ppf(x, h, n, taps, spectra=pick), full[pick])


def test_dft_column_slices_match_single_slice(monkeypatch):
    rng = np.random.default_rng(12)
    u = rng.standard_normal((3, 64)) + 1j * rng.standard_normal((3, 64))
    whole = ORACLE.dft(u)
    monkeypatch.setattr(ORACLE, "_SLICE_ELEMS", 64 * 5)   # 5 columns per slice
    sliced = ORACLE.dft(u)
    assert np.max(np.abs(whole - sliced)) <= 1e-13


def test_empty_and_degenerate_inputs():
    h = np.ones(4 * 8)
    assert ORACLE.ppf(np.zeros(3 * 8, np.complex128), h, 8, 4).shape == (0, 8)
    one = ORACLE.ppf(np.arange(5, dtype=np.complex128), np.array([2.0]), 1, 1)
    assert np.array_equal(one[:, 0], 2.0 * np.arange(5))


# ---------------------------------------------------------------------------
# planted mistakes: every mutant must be caught by at least one pin
# ---------------------------------------------------------------------------

MUTANTS = {
    "tap_direction_flipped": ("hs[t * n:(t + 1) * n][None, :]",
                              "hs[(t_count - 1 - t) * n:(t_count - t) * n][None, :]"),
    "last_tap_dropped": ("for t in range(t_count):", "for t in range(max(1, t_count - 1)):"),
    "blocks_reversed": ("blocks[m_idx + t]", "blocks[m_idx + t_count - 1 - t]"),
    "channels_reversed": ("hs[t * n:(t + 1) * n][None, :]", "hs[t * n:(t + 1) * n][None, ::-1]"),
    "dft_sign_flipped": ("w = np.cos(ang) - 1j * np.sin(ang)", "w = np.cos(ang) + 1j * np.sin(ang)"),
    "axis_table_wrong": ("np.array([1.0, -1j, -1.0, 1j])", "np.array([1.0, 1j, -1.0, -1j])"),
    "dft_index_off": ("return w[(c * k) % n]", "return w[(c * (k + 1)) % n]"),
    "dft_scaled": ("out[:, k0:k1] = u @ dft_matrix_columns(n, k0, k1, w)",
                   "out[:, k0:k1] = (u @ dft_matrix_columns(n, k0, k1, w)) / n"),
    "pairs_conjugated": ("return re + 1j * im", "return re - 1j * im"),
    "stream_history_long": ("np.zeros((t_count - 1) * n", "np.zeros(t_count * n"),
    "spectra_count_off": ("return max(0, n_samples // n_channels - taps + 1)",
                          "return max(0, n_samples // n_channels - taps)"),
    "power_not_squared": ("np.abs(spectra[:groups * k_int]) ** 2", "np.abs(spectra[:groups * k_int])"),
    "power_mean_not_sum": (".sum(axis=1)\n", ".mean(axis=1)\n"),
    "power_groups_shifted": ("spectra[:groups * k_int]", "spectra[1:groups * k_int + 1]"),
    "power_group_short": ("groups = spectra.shape[0] // k_int", "groups = spectra.shape[0] // k_int\n    k_int = max(1, k_int - 1)"),
}


def _mutant(name: str) -> types.ModuleType:
    old, new = MUTANTS[name]
    assert ORACLE_SRC.count(old) >= 1, f"mutation site for {name} not found"
    src = ORACLE_SRC.replace(old, new)
    spec = importlib.util.spec_from_loader(f"oracle_mutant_{name}", loader=None)
    mod = importlib.util.module_from_spec(spec)
    exec(compile(src, f"<mutant {name}>", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    mod = _mutant(name)
    caught = []
    for pin in PINS:
        try:
            pin(mod)
        except Exception:                  # noqa: BLE001 - a failing pin is the point
            caught.append(pin.__name__)
    assert caught, f"no pin catches the mutant {name}"
