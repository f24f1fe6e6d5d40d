"""Stream form on the GPU: chunked outputs equal the oracle's stream PPF
(the batch PPF over the zero-prefixed concatenation), whatever the chunking,
and a saved history resumes a stream exactly."""

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


def push_all(torch, plan, stream, chunks):
    outs = []
    for i, c in enumerate(chunks):
        s = c.size // plan.N
        xd = torch.from_numpy(c).cuda()
        od = torch.empty((s, plan.N), dtype=torch.complex64, device="cuda")
        ppf.ppf_stream_push(stream, xd, od, s, tag=i)
        outs.append((xd, od))
    torch.cuda.synchronize()
    return [o.cpu().numpy() for _, o in outs]


@pytest.mark.parametrize("n,taps,path", [
    (256, 8, ppf.PPF_PATH_FUSED),
    (1024, 8, ppf.PPF_PATH_FUSED),
    (64, 3, ppf.PPF_PATH_FUSED),
    (512, 1, ppf.PPF_PATH_FUSED),
    (1024, 8, ppf.PPF_PATH_TWO_PASS),
    (4096, 16, ppf.PPF_PATH_AUTO),
    (4096, 8, ppf.PPF_PATH_FUSED),
])
def test_chunk_split_matches_oracle(n, taps, path):
    torch = _torch()
    rng = np.random.default_rng(n + taps)
    h32 = rng.standard_normal(taps * n).astype(np.float32)
    lens = [1, 2, 3, 17, 1, 40, 5] if n <= 1024 else [1, 3, 9, 2]
    x = signals.complex_gaussian(sum(lens) * n, 1.0, seed=3 * n + taps)
    chunks, at = [], 0
    for s in lens:
        chunks.append(x[at * n:(at + s) * n])
        at += s
    print(f"case stream N={n} T={taps} path={path} chunks={lens}", flush=True)
    plan = ppf.Plan(n, taps, h32, path)
    ppf.ppf_set_stream(plan.handle, torch.cuda.current_stream().cuda_stream)
    st = ppf.ppf_stream_create(plan.handle)
    got = push_all(torch, plan, st, chunks)
    assert ppf.ppf_stream_position(st) == sum(lens)
    ref = oracle.ppf_stream(chunks, h32, n, taps)
    for g, r in zip(got, ref):
        assert g.shape == r.shape
    err = rel_err(np.concatenate(got), np.concatenate(ref))
    assert err <= TOL, err
    # the same samples pushed as one chunk give the same spectra
    st2 = ppf.ppf_stream_create(plan.handle)
    whole = push_all(torch, plan, st2, [x])[0]
    assert rel_err(whole, np.concatenate(ref)) <= TOL
    ppf.ppf_stream_destroy(st)
    ppf.ppf_stream_destroy(st2)
    plan.close()


def test_history_checkpoint_restore_is_exact():
    torch = _torch()
    n, taps = 256, 8
    h32 = signals.design_coeffs(n, taps).astype(np.float32)
    a = signals.complex_gaussian(37 * n, 1.0, seed=21)
    b = signals.complex_gaussian(11 * n, 1.0, seed=22)
    plan = ppf.Plan(n, taps, h32)
    ppf.ppf_set_stream(plan.handle, torch.cuda.current_stream().cuda_stream)
    s1 = ppf.ppf_stream_create(plan.handle)
    push_all(torch, plan, s1, [a])
    hist = np.empty((taps - 1) * n, dtype=np.complex64)
    ppf.ppf_stream_get_history(s1, hist)
    assert np.array_equal(hist, a[-(taps - 1) * n:])        # the last T-1 blocks
    out1 = push_all(torch, plan, s1, [b])[0]
    s2 = ppf.ppf_stream_create(plan.handle)
    ppf.ppf_stream_set_history(s2, hist)
    out2 = push_all(torch, plan, s2, [b])[0]
    assert np.array_equal(out1, out2)
    ppf.ppf_stream_destroy(s1)
    ppf.ppf_stream_destroy(s2)
    plan.close()


def test_short_chunks_shift_history():
    torch = _torch()
    n, taps = 128, 8
    h32 = signals.design_coeffs(n, taps).astype(np.float32)
    plan = ppf.Plan(n, taps, h32)
    ppf.ppf_set_stream(plan.handle, torch.cuda.current_stream().cuda_stream)
    st = ppf.ppf_stream_create(plan.handle)
    chunks = [signals.complex_gaussian(n, 1.0, seed=40 + i) for i in range(12)]   # one spectrum each
    got = push_all(torch, plan, st, chunks)
    ref = oracle.ppf_stream(chunks, h32, n, taps)
    assert rel_err(np.concatenate(got), np.concatenate(ref)) <= TOL
    hist = np.empty((taps - 1) * n, dtype=np.complex64)
    ppf.ppf_stream_get_history(st, hist)
    assert np.array_equal(hist, np.concatenate(chunks[-(taps - 1):]))
    ppf.ppf_stream_destroy(st)
    plan.close()


def test_stream_argument_errors():
    torch = _torch()
    plan = ppf.Plan(256, 4, np.ones(1024, np.float32))
    st = ppf.ppf_stream_create(plan.handle)
    buf = torch.zeros(8 * 256, dtype=torch.complex64, device="cuda")
    with pytest.raises(ppf.PPFError) as ei:
        ppf.ppf_stream_push(st, buf.data_ptr() + 8, torch.empty_like(buf), 2)
    assert ei.value.status == ppf.PPF_ERR_ALIGN
    with pytest.raises(ppf.PPFError) as ei:
        ppf.ppf_stream_push(st, buf, buf, 2)
    assert ei.value.status == ppf.PPF_ERR_INVALID
    assert ppf.ppf_stream_push(st, buf, torch.empty_like(buf), 0) == ppf.PPF_OK
    assert ppf.ppf_stream_position(st) == 0
    ppf.ppf_stream_destroy(st)
    plan.close()
