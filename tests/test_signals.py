"""Checks of the input generators: coefficient design and seeded signals."""

import numpy as np
import pytest

from paper_1411_3656_amd import signals


def _resp(h, nu):
    j = np.arange(h.size)
    return abs(np.exp(-2j * np.pi * nu * j) @ h)


@pytest.mark.parametrize("n", [256, 1024])
def test_sinc_hamming_prototype(n):
    taps = 8
    h = signals.design_coeffs(n, taps, "hamming")
    assert h.shape == (taps * n,)
    assert abs(h.sum() - 1.0) < 1e-12                 # unit DC gain
    assert np.max(np.abs(h - h[::-1])) < 1e-15          # symmetric
    assert abs(_resp(h, 0.0) - 1.0) < 1e-12
    assert abs(_resp(h, 0.5 / n) - 0.50036) < 1e-4       # -6 dB at half a channel
    assert _resp(h, 1.0 / n) < 1e-3                      # one channel away
    assert int(np.argmax(h)) in (taps * n // 2 - 1, taps * n // 2)


def test_windows():
    for kind in ("hamming", "hann", "rect", "kaiser"):
        w = signals.window(33, kind)
        assert np.allclose(w, w[::-1])
        assert abs(w[16] - 1.0) < 1e-12
    assert abs(signals.window(33, "hamming")[0] - 0.08) < 1e-12
    assert signals.window(33, "hann")[0] == 0.0
    assert np.array_equal(signals.window(1, "hann"), [1.0])


def test_fp16_coefficients_scale_is_exact_power_of_two():
    h = signals.design_coeffs(4096, 16, "hamming")
    h16, s = signals.coeffs_fp16(h)
    assert h16.dtype == np.float16 and s > 0
    assert np.max(np.abs(h16.astype(np.float64))) < 2.0 ** 14
    back = h16.astype(np.float64) * 2.0 ** -s
    big = np.abs(h) > 1e-6
    assert np.max(np.abs(back[big] - h[big]) / np.abs(h[big])) < 2.0 ** -10


def test_generators_are_seeded_and_shaped():
    a = signals.plain_input(256, 4096, seed=5)
    b = signals.plain_input(256, 4096, seed=5)
    assert a.dtype == np.complex64 and np.array_equal(a, b)
    assert not np.array_equal(a, signals.plain_input(256, 4096, seed=6))
    noise = signals.complex_gaussian(1 << 18, 16.0, seed=3)
    assert abs(noise.real.std() / 16.0 - 1) < 0.01 and abs(noise.imag.std() / 16.0 - 1) < 0.01
    q = signals.int8_input(1 << 16, seed=4)
    assert q.dtype == np.int8 and q.shape == (1 << 16, 2)
    assert q.min() >= -127 and q.max() <= 127


def test_tone_plan_places_tones_as_specified():
    for n in (64, 256, 1024):
        plan = signals.tone_plan(n, seed=9)
        assert len(plan) == 3
        bins = [num for num, den, _ in plan[:2]] + [plan[2][0] // 2]
        assert plan[2][1] == 2 * n and plan[2][0] % 2 == 1
        assert all(n // 8 <= k < 7 * n // 8 for k in bins)
        assert min(abs(a - b) for i, a in enumerate(bins) for b in bins[i + 1:]) >= 4
    x = signals.tones(1000, [(3, 16, 0.5)])
    assert np.allclose(np.abs(x), 1.0)
    assert np.allclose(x[16], x[0])                     # period 16 for f = 3/16
