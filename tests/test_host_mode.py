"""Single mode (host-resident input and output; the PCIe-inclusive M_b
measure of section 3): chunked copies to the device, the PPF, and copies
back overlap on three streams. The spectra must equal the batch PPF's."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1411_3656_amd import ppf, signals

TOL = 1e-5


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel_err(got, ref):
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    return float(np.max(np.abs(got - ref))) / rms


@pytest.mark.gpu
@pytest.mark.parametrize("n,taps,m_total,chunk,path", [
    (256, 8, 100, 7, ppf.PPF_PATH_AUTO),      # many chunks, ragged last one
    (1024, 16, 61, 20, ppf.PPF_PATH_AUTO),
    (1024, 8, 50, 0, ppf.PPF_PATH_AUTO),      # default chunk: one chunk
    (4096, 16, 23, 5, ppf.PPF_PATH_AUTO),     # two-pass path per chunk
    (512, 3, 40, 1, ppf.PPF_PATH_TWO_PASS),   # one spectrum per chunk
])
def test_host_mode_matches_oracle(n, taps, m_total, chunk, path):
    torch = _torch()
    print(f"case host-mode N={n} T={taps} M={m_total} chunk={chunk}", flush=True)
    rng = np.random.default_rng(n + taps)
    h = rng.standard_normal(taps * n).astype(np.float32)
    x = signals.complex_gaussian((m_total + taps - 1) * n, 1.0, seed=60 + n)
    xin = torch.from_numpy(x).pin_memory()
    out = torch.full((m_total, n), float("nan"), dtype=torch.complex64).pin_memory()
    plan = ppf.Plan(n, taps, h, path)
    plan.execute_host(xin, out, chunk_spectra=chunk)
    torch.cuda.current_stream().synchronize()
    got = out.numpy()
    plan.close()
    ref = oracle.ppf(x, h, n, taps)
    assert rel_err(got, ref) <= TOL


@pytest.mark.gpu
def test_host_mode_int8_and_repeat_equal_device_path():
    """int8 input through the single mode equals the device-resident path bit
    for bit, also on a second call that reuses the staging buffers."""
    torch = _torch()
    n, taps, m_total = 1024, 8, 70
    h16, shift = signals.coeffs_fp16(signals.design_coeffs(n, taps))
    x = signals.int8_input((m_total + taps - 1) * n, seed=8, sigma=16.0)
    plan = ppf.Plan(n, taps, h16, in_type=ppf.PPF_CI8, coeff_shift=shift)
    dev = plan.execute(torch.from_numpy(x).cuda())
    xin = torch.from_numpy(x).pin_memory()
    for chunk in (9, 30):
        out = torch.empty((m_total, n), dtype=torch.complex64).pin_memory()
        plan.execute_host(xin, out, chunk_spectra=chunk)
        torch.cuda.current_stream().synchronize()
        assert torch.equal(out, dev.cpu())
    plan.close()


def test_host_mode_validates_before_device_work():
    """Argument errors come back before any HIP call (runs without a GPU)."""
    L = ppf.lib()
    buf = np.zeros(4096, dtype=np.complex64)
    assert L.ppf_execute_host(None, buf.ctypes.data, buf.ctypes.data, 4, 0) == ppf.PPF_ERR_INVALID


@pytest.mark.gpu
def test_host_mode_c2_full_size_default_chunks():
    """The N=1024, T=8 workload (2^27 samples) from page-locked host memory
    with the default chunking (several 192 MiB chunks through three staging
    pairs), as the single-mode benchmark runs it. Every 97th spectrum and
    the first and last 2T are checked against the oracle; the whole output
    must have been written (no NaN left from the fill)."""
    torch = _torch()
    n, taps = 1024, 8
    n_samples = 1 << 27
    m_total = oracle.n_spectra(n_samples, n, taps)
    print(f"case host-mode C2 N={n} T={taps} M={m_total} default chunks", flush=True)
    h32 = signals.design_coeffs(n, taps, "hamming").astype(np.float32)
    x = signals.complex_gaussian(n_samples, 1.0, seed=signals.SEED_BASE + 1)
    xin = torch.from_numpy(x).pin_memory()
    out = torch.full((m_total, n), float("nan"), dtype=torch.complex64).pin_memory()
    plan = ppf.Plan(n, taps, h32)
    try:
        plan.execute_host(xin, out)
        torch.cuda.current_stream().synchronize()
    finally:
        plan.close()
    got = out.numpy()
    assert np.isfinite(got).all()
    pick = sorted(set(range(0, m_total, 97)) | set(range(2 * taps)) | set(range(m_total - 2 * taps, m_total)))
    ref = oracle.ppf(x, h32, n, taps, spectra=pick)
    err = rel_err(got[pick], ref)
    print(f"host-mode C2 checked {len(pick)} spectra, max err / rms = {err:.3e}", flush=True)
    assert err <= TOL
