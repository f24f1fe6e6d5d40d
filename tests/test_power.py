"""Detection in the transform's epilogue: |X|^2 summed over K consecutive
spectra, against the oracle's ppf_power.

Bar, derived from the FP32 spectra bar (max |dX| <= 1e-5 RMS(X)): each of
the K terms changes by at most (2|X| + |dX|)|dX| and |X| stays below about
6 RMS(X) for these sizes, so max |P - P_ref| <= K * 12 * 1e-5 RMS(X)^2 =
1.2e-4 * mean(P_ref).
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1411_3656_amd import ppf, signals

pytestmark = pytest.mark.gpu
BAR = 1.2e-4


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("n,taps,k_int,m_total,path", [
    (256, 8, 4, 64, ppf.PPF_PATH_AUTO),
    (1024, 16, 1, 24, ppf.PPF_PATH_AUTO),
    (64, 3, 7, 70, ppf.PPF_PATH_AUTO),
    (2048, 8, 2, 40, ppf.PPF_PATH_AUTO),
    (1024, 8, 6, 36, ppf.PPF_PATH_TWO_PASS),
    (4096, 16, 8, 32, ppf.PPF_PATH_AUTO),       # two-pass: power in the FFT pass
    (4096, 8, 5, 600, ppf.PPF_PATH_FUSED),      # fused N=4096: coefficients in LDS
    (4096, 4, 3, 300, ppf.PPF_PATH_FUSED),      # fused N=4096: coefficients in registers
    (1024, 32, 5, 40, ppf.PPF_PATH_AUTO),
    (16384, 4, 3, 9, ppf.PPF_PATH_AUTO),
])
def test_power_matches_oracle(n, taps, k_int, m_total, path):
    torch = _torch()
    print(f"case power N={n} T={taps} K={k_int} M={m_total} path={path}", flush=True)
    rng = np.random.default_rng(n * 3 + taps + k_int)
    h = rng.standard_normal(taps * n).astype(np.float32)
    x = signals.complex_gaussian((m_total + taps - 1) * n, 1.0, seed=n + k_int)
    plan = ppf.Plan(n, taps, h, path)
    got = plan.execute_power(torch.from_numpy(x).cuda(), k_int)
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.float64)
    plan.close()
    ref = oracle.ppf_power(x, h, n, taps, k_int)
    assert got.shape == ref.shape
    err = float(np.max(np.abs(got - ref))) / float(np.mean(ref))
    print(f"  max|dP|/mean(P) = {err:.2e}")
    assert err <= BAR, err


def test_power_int8_two_pass():
    torch = _torch()
    n, taps, k_int, m_total = 512, 8, 2, 30
    h16, shift = signals.coeffs_fp16(signals.design_coeffs(n, taps))
    x = signals.int8_input((m_total + taps - 1) * n, seed=17, sigma=16.0)
    plan = ppf.Plan(n, taps, h16, in_type=ppf.PPF_CI8, coeff_shift=shift)
    got = plan.execute_power(torch.from_numpy(x).cuda(), k_int)
    torch.cuda.synchronize()
    plan.close()
    ref = oracle.ppf_power(x, h16.astype(np.float64) * 2.0 ** -shift, n, taps, k_int)
    err = float(np.max(np.abs(got.cpu().numpy() - ref))) / float(np.mean(ref))
    assert err <= BAR, err


def test_power_argument_errors():
    torch = _torch()
    plan = ppf.Plan(256, 4, np.ones(1024, np.float32))
    x = torch.zeros(20 * 256, dtype=torch.complex64, device="cuda")
    out = torch.zeros((17, 256), dtype=torch.float32, device="cuda")
    with pytest.raises(ppf.PPFError) as ei:
        ppf.ppf_execute_power(plan.handle, x, out, 17, 4)          # 17 is not a multiple of 4
    assert ei.value.status == ppf.PPF_ERR_INVALID
    with pytest.raises(ppf.PPFError) as ei:
        ppf.ppf_execute_power(plan.handle, x, out, 16, 0)
    assert ei.value.status == ppf.PPF_ERR_INVALID
    assert ppf.ppf_execute_power(plan.handle, x, out, 0, 3) == ppf.PPF_OK
    plan.close()
    h16, shift = signals.coeffs_fp16(signals.design_coeffs(4096, 16))
    mplan = ppf.Plan(4096, 16, h16, in_type=ppf.PPF_CI8, coeff_shift=shift, fft_mode=ppf.PPF_FFT_MFMA_F16)
    xi = torch.zeros((31 * 4096, 2), dtype=torch.int8, device="cuda")
    po = torch.zeros((16, 4096), dtype=torch.float32, device="cuda")
    # the matrix-core mode detects in its own epilogue, with the same rules
    with pytest.raises(ppf.PPFError) as ei:
        ppf.ppf_execute_power(mplan.handle, xi, po, 16, 3)
    assert ei.value.status == ppf.PPF_ERR_INVALID
    po.fill_(float("nan"))
    assert ppf.ppf_execute_power(mplan.handle, xi, po, 16, 1) == ppf.PPF_OK
    torch.cuda.synchronize()
    assert bool((po == 0).all())                                   # zero input, zero power
    mplan.close()


def test_power_c2_full_size_sampled():
    """The N=1024, T=8 workload (2^27 samples) detected with K=16 in the
    benchmark's launch configuration. Every 97th power spectrum plus the
    first and last two are checked, each against the oracle on the input
    blocks of its own K spectra. The bar above holds at this size: the
    largest |X| among ~1.3e8 complex Gaussian bins is about 4.3 RMS(X)."""
    torch = _torch()
    n, taps, k_int = 1024, 8, 16
    n_samples = 1 << 27
    m_total = (oracle.n_spectra(n_samples, n, taps) // k_int) * k_int
    groups = m_total // k_int
    print(f"case power C2 N={n} T={taps} K={k_int} M={m_total}", flush=True)
    h32 = signals.design_coeffs(n, taps, "hamming").astype(np.float32)
    x = signals.complex_gaussian(n_samples, 1.0, seed=signals.SEED_BASE + 1)
    plan = ppf.Plan(n, taps, h32)
    try:
        got = plan.execute_power(torch.from_numpy(x).cuda(), k_int, nspectra=m_total)
        torch.cuda.synchronize()
    finally:
        plan.close()
    assert tuple(got.shape) == (groups, n)
    pick = sorted(set(range(0, groups, 97)) | {0, 1, groups - 2, groups - 1})
    got = got[torch.tensor(pick, device=got.device)].cpu().numpy().astype(np.float64)
    ref = np.empty_like(got)
    for i, j in enumerate(pick):
        xs = x[j * k_int * n:(j * k_int + k_int + taps - 1) * n]
        ref[i] = oracle.ppf_power(xs, h32, n, taps, k_int)[0]
    err = float(np.max(np.abs(got - ref))) / float(np.mean(ref))
    print(f"  checked {len(pick)} of {groups} power spectra, max|dP|/mean(P) = {err:.2e}", flush=True)
    assert err <= BAR, err
