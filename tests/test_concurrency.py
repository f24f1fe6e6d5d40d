"""A plan shared by host threads: each thread binds its own HIP stream
(ppf_set_stream is per thread) and executes concurrently; the two-pass
path gives every stream its own workspace, so results stay exact. Also the
detection bounds on K."""

from __future__ import annotations

import threading

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


@pytest.mark.parametrize("n,taps", [(1024, 24), (4096, 8), (256, 8)])
def test_threads_share_a_plan(n, taps):
    torch = _torch()
    h = np.random.default_rng(n + taps).standard_normal(taps * n).astype(np.float32)
    plan = ppf.Plan(n, taps, h)
    m_total = 300
    n_threads, reps = 3, 12
    xs = [signals.complex_gaussian((m_total + taps - 1) * n, 1.0, seed=500 + i) for i in range(n_threads)]
    refs = [oracle.ppf(x, h, n, taps) for x in xs]
    xds = [torch.from_numpy(x).cuda() for x in xs]
    outs = [[torch.empty((m_total, n), dtype=torch.complex64, device="cuda") for _ in range(reps)]
            for _ in range(n_threads)]
    streams = [torch.cuda.Stream() for _ in range(n_threads)]
    torch.cuda.synchronize()
    errors = []
    barrier = threading.Barrier(n_threads)
    print(f"case shared plan N={n} T={taps} path={plan.path} threads={n_threads}", flush=True)

    def worker(i):
        try:
            ppf.ppf_set_stream(plan.handle, streams[i].cuda_stream)
            barrier.wait()
            for r in range(reps):
                ppf.ppf_execute(plan.handle, xds[i], outs[i][r], m_total)
            streams[i].synchronize()
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(i,)) for i in range(n_threads)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for i in range(n_threads):
        for r in range(reps):
            err = rel_err(outs[i][r].cpu().numpy(), refs[i])
            assert err <= TOL, (i, r, err)
    if plan.path == ppf.PPF_PATH_TWO_PASS:
        # one workspace per HIP stream the plan ran on
        assert ppf.ppf_plan_query(plan.handle, ppf.PPF_Q_WORKSPACE_BYTES) >= n_threads * (128 << 20)
    plan.close()


def test_power_k_bounds():
    torch = _torch()
    x = torch.zeros(64 * 64, dtype=torch.complex64, device="cuda")
    out = torch.zeros(64 * 64, dtype=torch.float32, device="cuda")
    fused = ppf.Plan(64, 8, np.ones(512, np.float32))
    with pytest.raises(ppf.PPFError) as ei:
        ppf.ppf_execute_power(fused.handle, x, out, (1 << 28) + 1, (1 << 28) + 1)
    assert ei.value.status == ppf.PPF_ERR_UNSUPPORTED
    two = ppf.Plan(4096, 32, np.ones(4096 * 32, np.float32))
    assert two.path == ppf.PPF_PATH_TWO_PASS
    with pytest.raises(ppf.PPFError) as ei:
        ppf.ppf_execute_power(two.handle, x, out, 8192, 8192)      # K*N = 2^25
    assert ei.value.status == ppf.PPF_ERR_UNSUPPORTED
    fused.close()
    two.close()


@pytest.mark.parametrize("n,taps,mib", [(4096, 16, 128), (16384, 8, 512), (8192, 32, 512)])
def test_two_pass_workspace_size(n, taps, mib):
    """The two-pass workspace of a stream is one chunk: 128 MiB, and 512 MiB
    for N >= 8192 (longer chunks there re-read fewer tap windows); the
    small batch run through it still matches the oracle."""
    torch = _torch()
    m_total = 40
    h = np.random.default_rng(n + taps).standard_normal(n * taps).astype(np.float32)
    x = signals.complex_gaussian((m_total + taps - 1) * n, 1.0, seed=n + 3 * taps)
    print(f"case workspace N={n} T={taps} M={m_total}", flush=True)
    plan = ppf.Plan(n, taps, h)
    try:
        assert plan.path == ppf.PPF_PATH_TWO_PASS
        assert ppf.ppf_plan_query(plan.handle, ppf.PPF_Q_WORKSPACE_BYTES) == 0
        got = plan.execute(torch.from_numpy(x).cuda())
        torch.cuda.synchronize()
        assert ppf.ppf_plan_query(plan.handle, ppf.PPF_Q_WORKSPACE_BYTES) == mib << 20
        err = rel_err(got.cpu().numpy(), oracle.ppf(x, h, n, taps))
    finally:
        plan.close()
    assert err <= TOL, err
