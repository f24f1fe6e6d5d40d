"""ppf_execute_noalloc through the C ABI: the same spectra as ppf_execute
on two calls in a row (the second with a smaller input), for two-pass plans
(whose presums go through the static workspace) and a fused plan; a batch
beyond the workspace is refused before any work. Both sides are also
checked against the FP64 oracle."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1411_3656_amd import ppf, signals

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel_err(got, ref):
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    return float(np.max(np.abs(got - ref))) / rms


@pytest.mark.parametrize("n,taps,sizes", [
    (1024, 24, [4000, 1000]),      # two-pass; 4000 spectra = 31.25 MiB of presums
    (4096, 16, [1024, 300]),       # two-pass at the workspace's limit (32 MiB)
    (256, 8, [5000, 77]),          # fused: no workspace
])
def test_noalloc_matches_execute(n, taps, sizes):
    torch = _torch()
    h = np.random.default_rng(n + taps).standard_normal(taps * n).astype(np.float32)
    plan = ppf.Plan(n, taps, h)
    ppf.ppf_set_stream(plan.handle, torch.cuda.current_stream().cuda_stream)
    for call, m_total in enumerate(sizes):
        x = signals.complex_gaussian((m_total + taps - 1) * n, 1.0, seed=40 + call)
        xd = torch.from_numpy(x).cuda()
        want = torch.empty((m_total, n), dtype=torch.complex64, device="cuda")
        got = torch.full((m_total, n), float("nan"), dtype=torch.complex64, device="cuda")
        print(f"case noalloc N={n} T={taps} path={plan.path} call {call} M={m_total}", flush=True)
        ppf.ppf_execute(plan.handle, xd, want, m_total)
        ppf.ppf_execute_noalloc(plan.handle, xd, got, m_total)
        torch.cuda.synchronize()
        g, w = got.cpu().numpy(), want.cpu().numpy()
        assert np.array_equal(g, w), (call, m_total)
        idx = sorted(set(range(0, m_total, 37)) | {m_total - 1})
        assert rel_err(g[idx], oracle.ppf(x, h, n, taps, spectra=idx)) <= TOL
    plan.close()


def test_noalloc_refuses_batches_beyond_the_workspace():
    torch = _torch()
    n, taps = 4096, 16
    plan = ppf.Plan(n, taps, np.ones(n * taps, np.float32))
    assert plan.path == ppf.PPF_PATH_TWO_PASS
    m_total = ppf.PPF_NOALLOC_SCRATCH_BYTES // (n * 8) + 1
    xd = torch.zeros((m_total + taps - 1) * n, dtype=torch.complex64, device="cuda")
    out = torch.full((m_total, n), 7.0, dtype=torch.complex64, device="cuda")
    with pytest.raises(ppf.PPFError) as ei:
        ppf.ppf_execute_noalloc(plan.handle, xd, out, m_total)
    assert ei.value.status == ppf.PPF_ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())          # nothing was launched
    plan.close()
