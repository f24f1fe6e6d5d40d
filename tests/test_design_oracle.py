"""Pins of the prototype-filter design oracle (windowed sinc, Kaiser window).

Each pin checks the oracle against something other than itself: an
independent library routine (scipy's windows, scipy's I0, which uses
Chebyshev expansions rather than the power series, and scipy's Kaiser rule),
a closed form, or a property of the designed filter that the design rule
fixes (unit DC gain, half amplitude at the channel edge, Kaiser's
attenuation). Every planted mistake below must fail at least one pin.
"""

import importlib.util
import pathlib
import types

import numpy as np
import pytest
import scipy.signal
import scipy.special

from oracle import design as DESIGN

DESIGN_SRC = pathlib.Path(DESIGN.__file__).read_text()


def _response(h, oversample=16):
    """|H(w)| on a dense grid of w in [0, pi], by a zero-padded FFT."""
    f = oversample * h.size * 8
    mag = np.abs(np.fft.rfft(h, f))
    w = 2.0 * np.pi * np.arange(mag.size) / f
    return w, mag


def pin_d1_bessel_against_scipy(mod):
    x = np.concatenate([np.linspace(0.0, 2.0, 41), np.linspace(2.5, 60.0, 116)])
    got = mod.bessel_i0(x)
    want = scipy.special.i0(x)
    assert np.max(np.abs(got / want - 1.0)) < 1e-13
    assert mod.bessel_i0(np.array([0.0]))[0] == 1.0


def pin_d2_windows_against_scipy(mod):
    for length in (1, 2, 7, 64, 1000):
        sym = dict(sym=True)
        pairs = [("rect", None, scipy.signal.windows.boxcar(length, **sym)),
                 ("hamming", None, scipy.signal.windows.hamming(length, **sym)),
                 ("hann", None, scipy.signal.windows.hann(length, **sym)),
                 ("kaiser", 0.0, np.ones(length)),
                 ("kaiser", 5.0, scipy.signal.windows.kaiser(length, 5.0, **sym)),
                 ("kaiser", 14.0, scipy.signal.windows.kaiser(length, 14.0, **sym))]
        for kind, beta, want in pairs:
            got = mod.window(length, kind, beta)
            assert got.shape == (length,)
            assert np.max(np.abs(got - want)) < 1e-13, (kind, beta, length)
    user = np.linspace(0.25, 2.0, 9)
    assert np.array_equal(mod.window(9, "user", None, user), user)


def pin_d3_kaiser_rule_against_scipy(mod):
    for a in (0.0, 10.0, 20.99, 21.0, 30.0, 40.0, 50.0, 50.01, 60.0, 80.0, 120.0):
        assert abs(mod.kaiser_beta(a) - scipy.signal.kaiser_beta(a)) < 1e-12, a


def pin_d4_prototype_shape(mod):
    # T = N = 1: the single coefficient 1
    assert np.array_equal(mod.prototype(1, 1, "rect"), np.array([1.0]))
    # rectangular window, T = 1: the sinc over one block is sampled within
    # |u| < 1/2, so every coefficient is positive; the sum is 1
    h = mod.prototype(16, 1, "rect")
    assert np.all(h > 0) and abs(h.sum() - 1.0) < 1e-15
    for kind, beta in (("hamming", None), ("hann", None), ("kaiser", 8.0)):
        h = mod.prototype(32, 8, kind, beta)
        assert h.shape == (256,)
        assert abs(h.sum() - 1.0) < 1e-14
        assert np.max(np.abs(h - h[::-1])) < 1e-14 * np.max(np.abs(h))   # symmetric
        assert np.argmax(h) in (127, 128)                      # peak at the centre
    # the sinc's zeros: with a rectangular window and an odd length, the
    # centre falls on a sample and every N-th sample away from it is zero
    # (up to the rounding of pi in sin(pi k))
    h = mod.prototype(1, 9, "rect")
    assert np.max(np.abs(h - np.array([0, 0, 0, 0, 1.0, 0, 0, 0, 0]))) < 1e-15
    h = mod.prototype(3, 5, "rect")                            # L = 15, centre 7
    assert np.max(np.abs(h[[1, 4, 10, 13]])) < 1e-15
    assert np.all(np.abs(np.delete(h, [1, 4, 10, 13])) > 1e-3)


def pin_d5_channel_response(mod):
    # unit DC gain, half amplitude at the channel edge (half a bin), and
    # Kaiser's rule: the stop band starts half a transition width beyond
    # the edge and is at least (A - 2) dB down
    for n, taps, a in ((64, 8, 60.0), (256, 8, 80.0), (16, 16, 40.0), (1024, 4, 50.0)):
        h = mod.prototype(n, taps, "kaiser", mod.kaiser_beta(a))
        w, mag = _response(h)
        assert abs(mag[0] - 1.0) < 1e-12
        wc = np.pi / n
        assert abs(np.interp(wc, w, mag) - 0.5) < 5e-3, (n, taps, a)
        dw = (a - 8.0) / (2.285 * (h.size - 1))
        stop = mag[w >= wc + dw / 2].max()
        assert 20 * np.log10(stop) < -(a - 2.0), (n, taps, a, 20 * np.log10(stop))
    # Hamming, T = 8: about 0.5 at the edge and below 1e-3 beyond one bin
    h = mod.prototype(256, 8, "hamming")
    w, mag = _response(h)
    assert abs(np.interp(np.pi / 256, w, mag) - 0.5) < 2e-3
    assert mag[w >= 3 * np.pi / 256].max() < 1e-3


def pin_d6_user_window(mod):
    # a user window equal to a built-in one gives the same prototype; a
    # scaled window gives the same prototype (the sum normalises it)
    ham = scipy.signal.windows.hamming(512, sym=True)
    a = mod.prototype(64, 8, "hamming")
    b = mod.prototype(64, 8, "user", None, 3.0 * ham)
    assert np.max(np.abs(a - b)) < 1e-16
    with pytest.raises(ValueError):
        mod.prototype(4, 2, "user", None, np.zeros(8))


PINS = [pin_d1_bessel_against_scipy, pin_d2_windows_against_scipy, pin_d3_kaiser_rule_against_scipy,
        pin_d4_prototype_shape, pin_d5_channel_response, pin_d6_user_window]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_design_oracle_pin(pin):
    pin(DESIGN)


MUTANTS = {
    "i0_not_squared": ("term = term * q / (k * k)", "term = term * q / k"),
    "i0_half_argument": ("q = 0.25 * x * x", "q = 0.5 * x * x"),
    "kaiser_no_sqrt": ("np.sqrt(np.maximum(0.0, 1.0 - r * r))", "np.maximum(0.0, 1.0 - r * r)"),
    "kaiser_not_normalised": (") / bessel_i0(beta)", ")"),
    "hamming_coefficients": ("0.54 - 0.46 * np.cos", "0.5 - 0.46 * np.cos"),
    "window_periodic": ("np.cos(2.0 * np.pi * j / (length - 1))\n    if kind == \"hann\"",
                        "np.cos(2.0 * np.pi * j / length)\n    if kind == \"hann\""),
    "sinc_without_pi": ("np.sin(np.pi * u[nz]) / (np.pi * u[nz])", "np.sin(u[nz]) / u[nz]"),
    "sinc_off_centre": ("(j - (length - 1) / 2.0) / n", "(j - length / 2.0) / n"),
    "cutoff_two_bins": ("(j - (length - 1) / 2.0) / n", "2.0 * (j - (length - 1) / 2.0) / n"),
    "not_normalised": ("return h / s", "return h"),
    "rule_high_slope": ("return 0.1102 * (a - 8.7)", "return 0.1102 * (a - 7.8)"),
    "rule_mid_exponent": ("(a - 21.0) ** 0.4", "(a - 21.0) ** 0.5"),
    "rule_boundary": ("if a > 50.0:", "if a > 40.0:"),
}


def _mutant(name: str) -> types.ModuleType:
    old, new = MUTANTS[name]
    assert DESIGN_SRC.count(old) >= 1, f"mutation site for {name} not found"
    src = DESIGN_SRC.replace(old, new)
    spec = importlib.util.spec_from_loader(f"design_mutant_{name}", loader=None)
    mod = importlib.util.module_from_spec(spec)
    exec(compile(src, f"<mutant {name}>", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_design_planted_mistake_is_caught(name):
    mod = _mutant(name)
    caught = []
    for pin in PINS:
        try:
            pin(mod)
        except Exception:                  # noqa: BLE001 - a failing pin is the point
            caught.append(pin.__name__)
    assert caught, f"no pin catches the mutant {name}"
