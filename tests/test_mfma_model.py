"""The error bar of the matrix-core precision form, derived (CPU).

tests/mfma_model.py rounds where the matrix-core kernel rounds (FP16
presums, stage inputs and DFT matrices; FP32 sums and twiddles). Without
its roundings it must reproduce the FP64 oracle (so the three-stage
factorisation and the scaling are right); with them it gives the SNR that
the GPU's FP16 arithmetic can reach on the C4 workload's statistics
(complex int8, sigma 16, FP16 sinc x Hamming, T = 16). The GPU tests then
require at least that SNR less 1.7 dB (66 dB) and a largest error of at
most about 3x the modelled one (4e-3 of the output RMS).
"""

from __future__ import annotations

import numpy as np

import oracle
from paper_1411_3656_amd import signals
from tests import mfma_model

N, TAPS = 4096, 16


def _case(m_total=24, seed=signals.SEED_BASE + 3):
    x = signals.int8_input((m_total + TAPS - 1) * N, seed=seed, sigma=16.0)
    h16, shift = signals.coeffs_fp16(signals.design_coeffs(N, TAPS, "hamming"))
    idx = list(range(m_total))
    ref = oracle.ppf(x, h16.astype(np.float64) * 2.0 ** -shift, N, TAPS, spectra=idx)
    return x, h16, shift, idx, ref


def snr_db(got, ref):
    return float(10.0 * np.log10(np.sum(np.abs(ref) ** 2) / np.sum(np.abs(got - ref) ** 2)))


def test_model_without_rounding_is_the_dft():
    x, h16, shift, idx, ref = _case(m_total=6)
    got = mfma_model.model(x, h16, shift, TAPS, idx, exact=True)
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    assert float(np.max(np.abs(got - ref))) / rms < 1e-12


def test_modelled_snr_sets_the_bar():
    x, h16, shift, idx, ref = _case()
    got = mfma_model.model(x, h16, shift, TAPS, idx)
    snr = snr_db(got, ref)
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    max_err = float(np.max(np.abs(got - ref))) / rms
    print(f"modelled matrix-core SNR {snr:.2f} dB, max err / rms {max_err:.2e}")
    # about u/sqrt(3) .. u/2 relative RMS error (u = 2^-11) at each of about
    # six rounding points: 10 log10(1 / (6 * (2^-11 / 2)^2)) = 64.4 .. 68 dB
    assert 66.0 + 1.5 <= snr <= 69.5
    assert max_err <= 4e-3 / 2


def _case_n(n, taps, m_total, fp16=False, seed=signals.SEED_BASE + 9):
    if fp16:
        x = signals.to_complex_fp16(signals.complex_gaussian((m_total + taps - 1) * n, 1.0, seed))
    else:
        x = signals.int8_input((m_total + taps - 1) * n, seed=seed, sigma=16.0)
    h16, shift = signals.coeffs_fp16(signals.design_coeffs(n, taps, "hamming"))
    idx = list(range(m_total))
    ref = oracle.ppf(x, h16.astype(np.float64) * 2.0 ** -shift, n, taps, spectra=idx)
    return x, h16, shift, idx, ref


import pytest  # noqa: E402


@pytest.mark.parametrize("n,taps", [(1024, 8), (1024, 16), (256, 8), (256, 13)])
def test_small_n_model_without_rounding_is_the_dft(n, taps):
    """N = 1024 (radix 4 over p, then 16, 16) and N = 256 (16, 16): the
    factorisations and twiddle indices reproduce the plain DFT."""
    x, h16, shift, idx, ref = _case_n(n, taps, 7)
    got = mfma_model.model(x, h16, shift, taps, idx, exact=True)
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    assert float(np.max(np.abs(got - ref))) / rms < 1e-12


@pytest.mark.parametrize("fp16", [False, True], ids=["int8", "fp16"])
@pytest.mark.parametrize("n,taps", [(1024, 8), (256, 8)])
def test_small_n_modelled_snr(n, taps, fp16):
    """Fewer FP16 rounding points than at N = 4096 (two matrix-core stages;
    at N = 1024 the radix-4 stage is FP32): the modelled SNR is at least
    the N = 4096 bar."""
    x, h16, shift, idx, ref = _case_n(n, taps, 40, fp16)
    got = mfma_model.model(x, h16, shift, taps, idx)
    snr = snr_db(got, ref)
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    max_err = float(np.max(np.abs(got - ref))) / rms
    print(f"N={n} T={taps} fp16={fp16}: modelled SNR {snr:.2f} dB, max err / rms {max_err:.2e}")
    assert 66.0 + 1.5 <= snr <= 75.0
    assert max_err <= 4e-3 / 2
