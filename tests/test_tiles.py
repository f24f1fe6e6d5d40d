"""Batches cut into more tiles than group slots, against the FP64 oracle.

For N <= 256 a batch launch cuts the batch into several tiles per resident
group slot, and for N = 512 and 1024 (T <= 8) no tile is longer than 2 MiB
of input, so large batches run several tiles per slot. These cases run
such batches (2^26 samples for N = 16..256, 2^28 for N = 1024) and check
every 61st spectrum plus the first and last 2T against the oracle (section
2, Eq. 1), to max |X - X_ref| <= 1e-5 * RMS(X_ref); the whole output must
be finite. A wrong tile start or halo would show in the checked spectra.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1411_3656_amd import ppf, signals

pytestmark = pytest.mark.gpu

TOL = 1e-5
CASES = [(16, 4, 26), (32, 8, 26), (128, 4, 26), (256, 8, 26), (256, 3, 26), (1024, 8, 28), (1024, 5, 28)]


def _pick(m_total, taps, every=61):
    idx = set(range(0, m_total, every))
    idx.update(range(0, min(2 * taps, m_total)))
    idx.update(range(max(0, m_total - 2 * taps), m_total))
    return sorted(idx)


@pytest.mark.parametrize("n,taps,log2s", CASES, ids=[f"n{n}_t{t}_2p{s}" for n, t, s in CASES])
def test_many_tiles_per_slot_sampled(n, taps, log2s):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    samples = 1 << log2s
    m_total = samples // n - taps + 1
    print(f"case tiles N={n} T={taps} M={m_total}", flush=True)
    x = signals.complex_gaussian(samples, 1.0, seed=signals.SEED_BASE + 60 + n + taps)
    xd = torch.from_numpy(x).cuda()
    h32 = signals.design_coeffs(n, taps, "hamming").astype(np.float32)
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
    del out, xd
    torch.cuda.empty_cache()
    ref = oracle.ppf(x, h32, n, taps, spectra=pick)
    err = float(np.max(np.abs(got - ref))) / float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    print(f"tiles N={n} T={taps} path={path} checked {len(pick)} spectra, max err / rms = {err:.3e}", flush=True)
    assert path == ppf.PPF_PATH_FUSED
    assert err <= TOL
    assert finite
