"""Largest batches: more spectra than one kernel launch takes.

A batch of more than 2^28 spectra is split into several launches, each
starting at its own input block. This runs N=16, T=4 over 2^28 + 777
spectra (34 GB in, 34 GB out, resident in HBM) and checks, against the
FP64 oracle, the spectra on both sides of the split, at both ends and
spread over the batch. The oracle gets only the T input blocks of each
checked spectrum. The whole output must be finite with the white-noise
power sum(h^2) E|x|^2.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1411_3656_amd import ppf, signals

pytestmark = pytest.mark.gpu

TOL = 1e-5
SPLIT = 1 << 28          # spectra per launch of the batch kernels


def test_batch_split_across_launches():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n, taps = 16, 4
    m_total = SPLIT + 777
    in_bytes = (m_total + taps - 1) * n * 8
    free, _ = torch.cuda.mem_get_info()
    if free < 2 * in_bytes + (4 << 30):
        pytest.skip(f"needs {2 * in_bytes / 1e9:.0f} GB of device memory, {free / 1e9:.0f} GB free")
    print(f"case max-size N={n} T={taps} M={m_total}", flush=True)
    h32 = signals.design_coeffs(n, taps, "hamming").astype(np.float32)
    gen = torch.Generator(device="cuda").manual_seed(signals.SEED_BASE + 50)
    x = torch.randn((m_total + taps - 1) * n, dtype=torch.complex64, device="cuda", generator=gen)
    plan = ppf.Plan(n, taps, h32)
    try:
        out = plan.execute(x, nspectra=m_total)
        torch.cuda.synchronize()
        path = plan.path
    finally:
        plan.close()
    pick = sorted(set(range(0, 3)) | set(range(SPLIT - 4, SPLIT + 4)) | set(range(m_total - 3, m_total))
                  | set(range(0, m_total, 1 << 24)))
    got = out[torch.tensor(pick, device="cuda")].cpu().numpy()
    ref = np.empty((len(pick), n), np.complex128)
    for i, m in enumerate(pick):
        xs = x[m * n:(m + taps) * n].cpu().numpy()
        ref[i] = oracle.ppf(xs, h32, n, taps)[0]
    finite = bool(torch.isfinite(torch.view_as_real(out)).all().item())
    power = float(out.abs().pow(2).mean(dtype=torch.float64).item())
    del out, x
    torch.cuda.empty_cache()
    err = float(np.max(np.abs(got - ref))) / float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    print(f"max-size path={path} checked {len(pick)} spectra, max err / rms = {err:.3e}", flush=True)
    assert err <= TOL
    assert finite
    expect = float(np.sum(h32.astype(np.float64) ** 2))      # E|x|^2 = 1
    assert abs(power / expect - 1.0) < 0.01
