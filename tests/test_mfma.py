"""Matrix-core reduced-precision form on the GPU (N = 4096 = 16^3, taps <= 16,
complex int8 input, FP16 coefficients): FIR in FP32 from exact FP16
operands, then three radix-16 DFT stages on FP16 MFMA with FP32
accumulation and FP32 twiddles, stage inputs rounded to FP16.

Parity is against the FP64 oracle fed the identical int8 samples and the
FP16 coefficients exactly as stored (times 2^-shift). The arithmetic rounds
each of the three stage inputs and the DFT-16 matrix entries to FP16 (unit
roundoff u = 2^-11). The rounding-point model of tests/mfma_model.py,
checked in tests/test_mfma_model.py, gives 67.7 dB on the C4 statistics;
the bar is SNR >= 66 dB and a largest error of at most 4e-3 of the output
RMS. On the same input the GPU must also stay close to the model itself
(the difference well below the FP16 error), which checks that the kernel
rounds where the model says.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1411_3656_amd import ppf, signals

pytestmark = pytest.mark.gpu
N = 4096
MIN_SNR_DB = 66.0
MAX_ERR_OVER_RMS = 4e-3


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def snr_db(got, ref):
    return float(10.0 * np.log10(np.sum(np.abs(ref) ** 2) / np.sum(np.abs(got - ref) ** 2)))


def rel_err(got, ref):
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    return float(np.max(np.abs(got - ref))) / rms


def fp16_coeffs(taps, kind="hamming"):
    h16, shift = signals.coeffs_fp16(signals.design_coeffs(N, taps, kind))
    return h16, shift, h16.astype(np.float64) * 2.0 ** -shift


def mfma_plan(h16, taps, shift):
    return ppf.Plan(N, taps, h16, in_type=ppf.PPF_CI8, coeff_shift=shift, fft_mode=ppf.PPF_FFT_MFMA_F16)


def check(got, ref, label):
    s, e = snr_db(got, ref), rel_err(got, ref)
    print(f"  {label}: SNR {s:.1f} dB, max err/rms {e:.2e}", flush=True)
    assert s >= MIN_SNR_DB, (label, s)
    assert e <= MAX_ERR_OVER_RMS, (label, e)


@pytest.mark.parametrize("taps,m_total", [(16, 1), (16, 37), (16, 300), (9, 37), (1, 20)])
def test_matches_oracle(taps, m_total):
    torch = _torch()
    print(f"case mfma N={N} T={taps} M={m_total}", flush=True)
    h16, shift, h_exact = fp16_coeffs(taps)
    x = signals.int8_input((m_total + taps - 1) * N, seed=700 + taps + m_total, sigma=16.0)
    plan = mfma_plan(h16, taps, shift)
    assert plan.path == ppf.PPF_PATH_FUSED
    got = plan.execute(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    plan.close()
    pick = list(range(m_total)) if m_total <= 40 else sorted(set(range(0, m_total, 7)) | {1, 2, m_total - 2, m_total - 1})
    ref = oracle.ppf(x, h_exact, N, taps, spectra=pick)
    assert np.all(np.isfinite(got))
    check(got[pick], ref, f"T={taps} M={m_total}")


def test_long_tiles_sampled():
    """More spectra per workgroup tile than the 16-step unrolled loop
    (4500 spectra over at most 256 tiles), sampled at tile edges."""
    torch = _torch()
    taps, m_total = 16, 4500
    print(f"case mfma long tiles M={m_total}", flush=True)
    h16, shift, h_exact = fp16_coeffs(taps)
    x = signals.int8_input((m_total + taps - 1) * N, seed=77, sigma=16.0)
    plan = mfma_plan(h16, taps, shift)
    got = plan.execute(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    plan.close()
    s = -(-m_total // 256)
    edges = {e for k in range(1, 256) for e in (k * s - 1, k * s) if k * s < m_total}
    pick = sorted(set(range(0, m_total, 97)) | set(range(0, m_total, 61)) | set(list(edges)[:40])
                  | {0, 15, 16, 17, m_total - 1})
    ref = oracle.ppf(x, h_exact, N, taps, spectra=pick)
    check(got[pick].cpu().numpy(), ref, "long tiles")


def test_stream_chunks_match_oracle_stream():
    torch = _torch()
    taps = 16
    h16, shift, h_exact = fp16_coeffs(taps)
    lens = [3, 1, 17, 2, 20]
    x = signals.int8_input(sum(lens) * N, seed=91, sigma=16.0)
    plan = mfma_plan(h16, taps, shift)
    ppf.ppf_set_stream(plan.handle, torch.cuda.current_stream().cuda_stream)
    st = ppf.ppf_stream_create(plan.handle)
    chunks, outs, at = [], [], 0
    for s in lens:
        c = x[at * N:(at + s) * N]
        chunks.append(c)
        xd = torch.from_numpy(np.ascontiguousarray(c)).cuda()
        od = torch.empty((s, N), dtype=torch.complex64, device="cuda")
        ppf.ppf_stream_push(st, xd, od, s)
        outs.append((xd, od))
        at += s
    torch.cuda.synchronize()
    got = np.concatenate([o.cpu().numpy() for _, o in outs])
    ref = np.concatenate(oracle.ppf_stream(chunks, h_exact, N, taps))
    check(got, ref, "stream")
    ppf.ppf_stream_destroy(st)
    plan.close()


def test_deterministic_and_path_fixed():
    torch = _torch()
    taps = 16
    h16, shift, _ = fp16_coeffs(taps)
    x = torch.from_numpy(signals.int8_input((40 + taps - 1) * N, seed=5, sigma=16.0)).cuda()
    plan = mfma_plan(h16, taps, shift)
    a = plan.execute(x)
    b = plan.execute(x)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    with pytest.raises(ppf.PPFError) as ei:
        ppf.ppf_plan_set_path(plan.handle, ppf.PPF_PATH_TWO_PASS)
    assert ei.value.status == ppf.PPF_ERR_UNSUPPORTED
    assert ppf.ppf_plan_query(plan.handle, ppf.PPF_Q_FFT_MODE) == ppf.PPF_FFT_MFMA_F16
    plan.close()


def test_matches_the_rounding_model():
    """GPU against the rounding-point model on the C4 statistics: the two
    round at the same points, so they differ by much less than either
    differs from the exact result (only the FP32 summation order inside a
    matrix-core instruction and single FP16 roundings that flip differ)."""
    torch = _torch()
    from tests import mfma_model
    taps, m_total = 16, 40
    x = signals.int8_input((m_total + taps - 1) * N, seed=signals.SEED_BASE + 3, sigma=16.0)
    h16, shift, h_exact = fp16_coeffs(taps)
    plan = mfma_plan(h16, taps, shift)
    got = plan.execute(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.complex128)
    plan.close()
    idx = list(range(m_total))
    ref = oracle.ppf(x, h_exact, N, taps, spectra=idx)
    mod = mfma_model.model(x, h16, shift, taps, idx)
    s_gpu, s_mod = snr_db(got, ref), snr_db(mod, ref)
    s_gap = snr_db(got, mod)
    print(f"  GPU {s_gpu:.2f} dB, model {s_mod:.2f} dB, GPU vs model {s_gap:.2f} dB", flush=True)
    assert abs(s_gpu - s_mod) <= 0.5
    assert s_gap >= s_mod + 6.0


def _fp16_input(n_samples, seed):
    return signals.to_complex_fp16(signals.complex_gaussian(n_samples, 1.0, seed))


def mfma_plan_in(h16, taps, shift, in_type):
    return ppf.Plan(N, taps, h16, in_type=in_type, coeff_shift=shift, fft_mode=ppf.PPF_FFT_MFMA_F16)


@pytest.mark.parametrize("taps,m_total", [(16, 37), (16, 300), (8, 41)])
def test_fp16_input(taps, m_total):
    """Complex FP16 input on the matrix-core stages: any finite FP16 sample
    is admitted (the scale is set for |x| <= 65504, so no stage input can
    overflow); at sigma 1 the same bars hold, and the FP32 path on the same
    FP16 values is reported beside it."""
    torch = _torch()
    from tests import mfma_model
    print(f"case mfma fp16 input T={taps} M={m_total}", flush=True)
    h16, shift, h_exact = fp16_coeffs(taps)
    x = _fp16_input((m_total + taps - 1) * N, seed=800 + taps + m_total)
    xd = torch.from_numpy(x).cuda()
    plan = mfma_plan_in(h16, taps, shift, ppf.PPF_C16)
    got = plan.execute(xd)
    plan32 = ppf.Plan(N, taps, h16, in_type=ppf.PPF_C16, coeff_shift=shift)     # FP32 DFT stages
    got32 = plan32.execute(xd)
    torch.cuda.synchronize()
    plan.close()
    plan32.close()
    pick = list(range(m_total)) if m_total <= 41 else sorted(set(range(0, m_total, 7)) | {1, m_total - 1})
    ref = oracle.ppf(x, h_exact, N, taps, spectra=pick)
    g = got.cpu().numpy()[pick]
    check(g, ref, f"fp16 input T={taps}")
    mod = mfma_model.model(x, h16, shift, taps, pick)
    print(f"  model {snr_db(mod, ref):.2f} dB; FP32 DFT path on the same input: "
          f"SNR {snr_db(got32.cpu().numpy()[pick], ref):.1f} dB, max err/rms {rel_err(got32.cpu().numpy()[pick], ref):.2e}",
          flush=True)
    assert abs(snr_db(g, ref) - snr_db(mod, ref)) <= 0.5
    assert rel_err(got32.cpu().numpy()[pick], ref) <= 1e-5


def test_fp16_input_extremes_do_not_overflow():
    """FP16 samples at the format's largest magnitude give finite spectra
    (the scale bounds every stage input below the FP16 range)."""
    torch = _torch()
    taps, m_total = 16, 20
    h16, shift, h_exact = fp16_coeffs(taps)
    rng = np.random.default_rng(3)
    x = np.empty(((m_total + taps - 1) * N, 2), np.float16)
    x[:] = rng.choice(np.array([65504.0, -65504.0], np.float16), size=x.shape)
    plan = mfma_plan_in(h16, taps, shift, ppf.PPF_C16)
    got = plan.execute(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    plan.close()
    got = got.cpu().numpy()
    assert np.isfinite(got).all()
    ref = oracle.ppf(x, h_exact, N, taps)
    s = snr_db(got, ref)
    print(f"  full-scale FP16 input: SNR {s:.1f} dB", flush=True)
    assert s >= MIN_SNR_DB


@pytest.mark.parametrize("in_type,k_int,m_total", [(ppf.PPF_CI8, 16, 320), (ppf.PPF_C16, 4, 100), (ppf.PPF_CI8, 3, 60)])
def test_detection_in_matrix_core_mode(in_type, k_int, m_total):
    """|X|^2 summed over K spectra in the matrix-core kernel's epilogue,
    against the oracle's detected power on the same input; its error is that
    of the modelled matrix-core spectra, detected the same way."""
    torch = _torch()
    from tests import mfma_model
    taps = 16
    print(f"case mfma detection in={in_type} K={k_int} M={m_total}", flush=True)
    h16, shift, h_exact = fp16_coeffs(taps)
    n_samples = (m_total + taps - 1) * N
    x = signals.int8_input(n_samples, seed=900 + k_int, sigma=16.0) if in_type == ppf.PPF_CI8 \
        else _fp16_input(n_samples, seed=900 + k_int)
    plan = mfma_plan_in(h16, taps, shift, in_type)
    got = plan.execute_power(torch.from_numpy(x).cuda(), k_int)
    torch.cuda.synchronize()
    plan.close()
    got = got.cpu().numpy().astype(np.float64)
    ref = oracle.ppf_power(x, h_exact, N, taps, k_int)
    mod_x = mfma_model.model(x, h16, shift, taps, range(m_total))
    mod = (np.abs(mod_x) ** 2).reshape(m_total // k_int, k_int, N).sum(axis=1)
    rel = lambda p: float(np.sqrt(np.mean((p - ref) ** 2)) / np.sqrt(np.mean(ref ** 2)))
    print(f"  detected power: rms rel error GPU {rel(got):.2e}, model {rel(mod):.2e}", flush=True)
    assert got.shape == ref.shape
    assert rel(got) <= 1.5 * rel(mod) + 1e-6


# ---- N = 256 and N = 1024 on the matrix cores ------------------------------

def _coeffs_n(n, taps):
    h16, shift = signals.coeffs_fp16(signals.design_coeffs(n, taps, "hamming"))
    return h16, shift, h16.astype(np.float64) * 2.0 ** -shift


def _input_n(kind, n_samples, seed):
    if kind == ppf.PPF_CI8:
        return signals.int8_input(n_samples, seed=seed, sigma=16.0)
    return signals.to_complex_fp16(signals.complex_gaussian(n_samples, 1.0, seed))


@pytest.mark.parametrize("kind", [ppf.PPF_CI8, ppf.PPF_C16], ids=["ci8", "c16"])
@pytest.mark.parametrize("n,taps,m_total", [(1024, 8, 700), (1024, 16, 333), (1024, 3, 41),
                                            (256, 8, 2100), (256, 16, 901), (256, 1, 37)])
def test_small_n_matches_oracle_and_model(n, taps, m_total, kind):
    """N = 1024 (radix 4 in FP32, two DFT-16 stages on the matrix cores) and
    N = 256 (two matrix-core stages): several tiles per workgroup group and
    a ragged tail, against the same-input FP64 oracle at the matrix-core bar,
    against the rounding model, and beside the FP32 DFT path."""
    torch = _torch()
    from tests import mfma_model
    print(f"case mfma small N={n} T={taps} M={m_total} in={kind}", flush=True)
    h16, shift, h_exact = _coeffs_n(n, taps)
    x = _input_n(kind, (m_total + taps - 1) * n, seed=1300 + n + taps + kind)
    xd = torch.from_numpy(x).cuda()
    plan = ppf.Plan(n, taps, h16, in_type=kind, coeff_shift=shift, fft_mode=ppf.PPF_FFT_MFMA_F16)
    assert plan.path == ppf.PPF_PATH_FUSED
    got = plan.execute(xd)
    plan32 = ppf.Plan(n, taps, h16, in_type=kind, coeff_shift=shift)
    got32 = plan32.execute(xd)
    torch.cuda.synchronize()
    plan.close()
    plan32.close()
    got = got.cpu().numpy()
    assert np.isfinite(got).all()
    pick = sorted(set(range(0, m_total, 13)) | set(range(m_total - 20, m_total)) | {0, 1, 7, 8, 15, 16})
    ref = oracle.ppf(x, h_exact, n, taps, spectra=pick)
    check(got[pick], ref, f"N={n} T={taps} in={kind}")
    mod = mfma_model.model(x, h16, shift, taps, pick)
    agree = snr_db(got[pick], mod)
    g32 = got32.cpu().numpy()[pick]
    print(f"  model {snr_db(mod, ref):.2f} dB, GPU vs model {agree:.1f} dB; FP32 DFT path: SNR "
          f"{snr_db(g32, ref):.1f} dB, max err/rms {rel_err(g32, ref):.2e}", flush=True)
    assert abs(snr_db(got[pick], ref) - snr_db(mod, ref)) <= 0.5
    assert agree >= 85.0
    assert rel_err(g32, ref) <= 1e-5


@pytest.mark.parametrize("n,kind,k_int,m_total", [(1024, ppf.PPF_CI8, 16, 640), (256, ppf.PPF_C16, 5, 300),
                                                  (1024, ppf.PPF_C16, 3, 99)])
def test_small_n_detection(n, kind, k_int, m_total):
    torch = _torch()
    from tests import mfma_model
    taps = 8
    print(f"case mfma small detection N={n} in={kind} K={k_int} M={m_total}", flush=True)
    h16, shift, h_exact = _coeffs_n(n, taps)
    x = _input_n(kind, (m_total + taps - 1) * n, seed=1500 + n + k_int)
    plan = ppf.Plan(n, taps, h16, in_type=kind, coeff_shift=shift, fft_mode=ppf.PPF_FFT_MFMA_F16)
    got = plan.execute_power(torch.from_numpy(x).cuda(), k_int)
    torch.cuda.synchronize()
    plan.close()
    got = got.cpu().numpy().astype(np.float64)
    ref = oracle.ppf_power(x, h_exact, n, taps, k_int)
    mod_x = mfma_model.model(x, h16, shift, taps, range(m_total))
    mod = (np.abs(mod_x) ** 2).reshape(m_total // k_int, k_int, n).sum(axis=1)
    rel = lambda p: float(np.sqrt(np.mean((p - ref) ** 2)) / np.sqrt(np.mean(ref ** 2)))
    print(f"  detected power: rms rel error GPU {rel(got):.2e}, model {rel(mod):.2e}", flush=True)
    assert got.shape == ref.shape
    assert rel(got) <= 1.5 * rel(mod) + 1e-6


@pytest.mark.parametrize("n", [256, 1024])
def test_small_n_stream_chunks(n):
    torch = _torch()
    taps = 8
    h16, shift, h_exact = _coeffs_n(n, taps)
    lens = [3, 1, 17, 2, 40, 9]
    x = signals.int8_input(sum(lens) * n, seed=91 + n, sigma=16.0)
    plan = ppf.Plan(n, taps, h16, in_type=ppf.PPF_CI8, coeff_shift=shift, fft_mode=ppf.PPF_FFT_MFMA_F16)
    ppf.ppf_set_stream(plan.handle, torch.cuda.current_stream().cuda_stream)
    st = ppf.ppf_stream_create(plan.handle)
    chunks, outs, at = [], [], 0
    for s in lens:
        c = x[at * n:(at + s) * n]
        chunks.append(c)
        xd = torch.from_numpy(np.ascontiguousarray(c)).cuda()
        od = torch.empty((s, n), dtype=torch.complex64, device="cuda")
        ppf.ppf_stream_push(st, xd, od, s)
        outs.append((xd, od))
        at += s
    torch.cuda.synchronize()
    got = np.concatenate([o.cpu().numpy() for _, o in outs])
    ppf.ppf_stream_destroy(st)
    plan.close()
    ref = np.concatenate(oracle.ppf_stream(chunks, h_exact, n, taps))
    check(got, ref, f"stream N={n}")
