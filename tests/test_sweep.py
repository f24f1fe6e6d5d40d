"""The shape sweep at full size against the FP64 oracle: N in {64, 512,
4096, 16384} x T in {4, 8, 16, 32}, 2^28 complex FP32 Gaussian samples per
N, sinc x Hann prototype, in the launch configuration the benchmark times.

Each point is checked on every 97th spectrum plus the first and last 2T
spectra (the oracle computes them one by one), to the tolerance
max |X - X_ref| <= 1e-5 * RMS(X_ref) over the checked spectra. The whole
output is also checked to be finite, and its mean power to match the
white-noise level 2 sigma^2 sum(h^2) within 2%.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1411_3656_amd import ppf, signals

pytestmark = pytest.mark.gpu

TOL = 1e-5
SWEEP_N = [64, 512, 4096, 16384]
SWEEP_T = [4, 8, 16, 32]
SAMPLES = 1 << 28
POINTS = [(i, n, t) for i, n in enumerate(SWEEP_N) for t in SWEEP_T]


@pytest.fixture(scope="module")
def inputs():
    """One N's input at a time (host and device): points run grouped by N."""
    cache = {}
    yield cache
    cache.clear()


def _input(cache, i, n):
    import torch
    if cache.get("n") != n:
        cache.clear()
        torch.cuda.empty_cache()
        x = signals.complex_gaussian(SAMPLES, 1.0, seed=signals.SEED_BASE + 2 + 100 * i)
        cache.update(n=n, x=x, xd=torch.from_numpy(x).cuda())
    return cache["x"], cache["xd"]


def _pick(m_total, taps, every=97):
    idx = set(range(0, m_total, every))
    idx.update(range(0, min(2 * taps, m_total)))
    idx.update(range(max(0, m_total - 2 * taps), m_total))
    return sorted(idx)


@pytest.mark.parametrize("i,n,taps", POINTS, ids=[f"n{n}_t{t}" for _, n, t in POINTS])
def test_sweep_point_full_size_sampled(inputs, i, n, taps):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m_total = SAMPLES // n - taps + 1
    print(f"case sweep N={n} T={taps} M={m_total}", flush=True)
    x, xd = _input(inputs, i, n)
    h32 = signals.design_coeffs(n, taps, "hann").astype(np.float32)
    plan = ppf.Plan(n, taps, h32)
    try:
        out = plan.execute(xd, nspectra=m_total)
        torch.cuda.synchronize()
        path = plan.path
    finally:
        plan.close()
    pick = _pick(m_total, taps)
    got = out[torch.tensor(pick, device=out.device)].cpu().numpy()
    finite = bool(torch.isfinite(torch.view_as_real(out)).all().item())
    power = float(out.abs().pow(2).mean().item())
    del out
    ref = oracle.ppf(x, h32, n, taps, spectra=pick)
    err = float(np.max(np.abs(got - ref))) / float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    print(f"sweep N={n} T={taps} path={path} checked {len(pick)} spectra, max err / rms = {err:.3e}", flush=True)
    assert err <= TOL
    assert finite
    expect = 2.0 * float(np.sum(h32.astype(np.float64) ** 2))
    assert abs(power / expect - 1.0) < 0.02
