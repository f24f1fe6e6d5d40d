"""Reduced-precision form on the GPU: complex int8 / FP16 input and FP16
coefficients, widened to FP32 in registers with FP32 accumulation.

Two errors are reported (reading of the precision-form reference):
(i) arithmetic error against the FP64 oracle fed the identical stored
inputs and the FP16 coefficients exactly as stored (times 2^-shift); the
arithmetic is FP32, so the FP32 tolerance applies;
(ii) end-to-end error against the oracle with the FP64 coefficients, stated
as SNR = 10 log10(sum |X_ref|^2 / sum |X - X_ref|^2) with the max error over
the RMS; it measures coefficient quantisation, so it is reported, not bounded
by the FP32 tolerance.
"""

from __future__ import annotations

import json
import os

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


def snr_db(got, ref):
    return 10.0 * np.log10(np.sum(np.abs(ref) ** 2) / np.sum(np.abs(got - ref) ** 2))


def make_input(kind, n_samples, seed):
    if kind == ppf.PPF_CI8:
        return signals.int8_input(n_samples, seed, sigma=16.0)
    if kind == ppf.PPF_C16:
        return signals.to_complex_fp16(signals.complex_gaussian(n_samples, 1.0, seed))
    return signals.complex_gaussian(n_samples, 1.0, seed)


def stored_coeffs(h64, half):
    if half:
        h16, shift = signals.coeffs_fp16(h64)
        return h16, shift, h16.astype(np.float64) * 2.0 ** -shift
    h32 = h64.astype(np.float32)
    return h32, None, h32.astype(np.float64)


@pytest.mark.parametrize("half", [True, False], ids=["h16", "h32"])
@pytest.mark.parametrize("kind", [ppf.PPF_CI8, ppf.PPF_C16], ids=["ci8", "c16"])
@pytest.mark.parametrize("n,taps", [(256, 8), (1024, 3), (4096, 16), (64, 16)])
def test_reduced_precision_inputs(n, taps, kind, half):
    torch = _torch()
    m_total = 97 if n < 4096 else 29
    x = make_input(kind, (m_total + taps - 1) * n, seed=n + taps + kind)
    h64 = signals.design_coeffs(n, taps, "hamming")
    h, shift, h_exact = stored_coeffs(h64, half)
    print(f"case precision N={n} T={taps} in={kind} half={half}", flush=True)
    plan = ppf.Plan(n, taps, h, in_type=kind, coeff_shift=shift)
    got = plan.execute(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    plan.close()
    ref = oracle.ppf(x, h_exact, n, taps)
    assert got.shape == ref.shape
    err = rel_err(got, ref)
    assert err <= TOL, err
    ref64 = oracle.ppf(x, h64, n, taps)
    print(f"  arithmetic err/rms {err:.2e}; end-to-end SNR {snr_db(got, ref64):.1f} dB")


@pytest.mark.parametrize("kind", [ppf.PPF_CI8, ppf.PPF_C16], ids=["ci8", "c16"])
@pytest.mark.parametrize("n,taps,m_total", [(16, 3, 700), (64, 16, 300), (256, 1, 257), (512, 8, 611),
                                            (1024, 8, 300), (2048, 5, 129), (4096, 8, 300), (4096, 4, 41)])
def test_widened_fused_and_two_pass(n, taps, m_total, kind):
    """The fused kernels widen FP16 / int8 samples as they load them; the
    two-pass form widens in its FIR pass. Both against the same-input
    oracle at the FP32 bar, over several tiles and a ragged tail."""
    torch = _torch()
    x = make_input(kind, (m_total + taps - 1) * n, seed=3 * n + taps + kind)
    h16, shift, h_exact = stored_coeffs(signals.design_coeffs(n, taps, "hann"), True)
    idx = sorted(set(range(0, m_total, 11)) | set(range(m_total - 2 * taps, m_total)) | {1, 2})
    ref = oracle.ppf(x, h_exact, n, taps, spectra=idx)
    xd = torch.from_numpy(x).cuda()
    for path in (ppf.PPF_PATH_FUSED, ppf.PPF_PATH_TWO_PASS):
        print(f"case widened N={n} T={taps} M={m_total} in={kind} path={path}", flush=True)
        plan = ppf.Plan(n, taps, h16, path, in_type=kind, coeff_shift=shift)
        assert plan.path == path
        got = plan.execute(xd)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        plan.close()
        assert np.isfinite(got).all()
        err = rel_err(got[idx], ref)
        print(f"  path {path}: max err/rms {err:.2e}", flush=True)
        assert err <= TOL, (path, err)


def test_int8_stream_split_matches_oracle():
    torch = _torch()
    n, taps = 512, 8
    h16, shift, h_exact = stored_coeffs(signals.design_coeffs(n, taps), True)
    plan = ppf.Plan(n, taps, h16, in_type=ppf.PPF_CI8, coeff_shift=shift)
    ppf.ppf_set_stream(plan.handle, torch.cuda.current_stream().cuda_stream)
    st = ppf.ppf_stream_create(plan.handle)
    lens = [3, 1, 9, 2]
    x = signals.int8_input(sum(lens) * n, seed=31)
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
    ref = np.concatenate(oracle.ppf_stream(chunks, h_exact, n, taps))
    assert rel_err(got, ref) <= TOL
    hist = np.empty(((taps - 1) * n, 2), dtype=np.int8)
    ppf.ppf_stream_get_history(st, hist)
    assert np.array_equal(hist, x[-(taps - 1) * n:])
    ppf.ppf_stream_destroy(st)
    plan.close()


def test_c4_precision_form_full_size_sampled():
    """N=4096, T=16, 2^28 complex int8 samples (sigma 16), FP16 sinc x Hamming:
    FP32 DFT stages and FP16 matrix-core DFT stages, and the FP32 path."""
    torch = _torch()
    n, taps, n_samples = 4096, 16, 1 << 28
    m_total = oracle.n_spectra(n_samples, n, taps)
    print(f"case C4 N={n} T={taps} M={m_total}", flush=True)
    x = signals.int8_input(n_samples, seed=signals.SEED_BASE + 3, sigma=16.0)
    h64 = signals.design_coeffs(n, taps, "hamming")
    h16, shift, h_exact = stored_coeffs(h64, True)
    xd = torch.from_numpy(x).cuda()
    plan = ppf.Plan(n, taps, h16, in_type=ppf.PPF_CI8, coeff_shift=shift)
    got = plan.execute(xd)
    torch.cuda.synchronize()
    plan.close()
    # the same inputs with the radix-16 DFT stages on FP16 matrix cores
    plan_m = ppf.Plan(n, taps, h16, in_type=ppf.PPF_CI8, coeff_shift=shift, fft_mode=ppf.PPF_FFT_MFMA_F16)
    got_m = plan_m.execute(xd)
    torch.cuda.synchronize()
    plan_m.close()
    # the FP32 path on the same values (int8 widened, FP32 coefficients)
    x32 = torch.view_as_complex(xd.to(torch.float32).contiguous())
    plan32 = ppf.Plan(n, taps, h64.astype(np.float32))
    got32 = plan32.execute(x32)
    torch.cuda.synchronize()
    plan32.close()
    pick = sorted(set(range(0, m_total, 97)) | set(range(2 * taps)) | set(range(m_total - 2 * taps, m_total)))
    g = got[pick].cpu().numpy()
    g32 = got32[pick].cpu().numpy()
    gm = got_m[pick].cpu().numpy()
    ref = oracle.ppf(x, h_exact, n, taps, spectra=pick)
    ref64 = oracle.ppf(x, h64, n, taps, spectra=pick)
    err = rel_err(g, ref)
    report = {
        "workload": "precision_n4096_t16_int8_2p28", "spectra_checked": len(pick),
        "int8_fp16coef": {"arith_max_err_over_rms": err, "arith_snr_db": float(snr_db(g, ref)),
                          "e2e_snr_db": float(snr_db(g, ref64)), "e2e_max_err_over_rms": rel_err(g, ref64)},
        "int8_fp16coef_mfma_f16": {"arith_max_err_over_rms": rel_err(gm, ref), "arith_snr_db": float(snr_db(gm, ref)),
                                   "e2e_snr_db": float(snr_db(gm, ref64)), "e2e_max_err_over_rms": rel_err(gm, ref64)},
        "fp32_path": {"e2e_snr_db": float(snr_db(g32, ref64)), "e2e_max_err_over_rms": rel_err(g32, ref64)},
    }
    print(json.dumps(report))
    out = os.environ.get("PPF_REPORT_DIR")
    if out:
        with open(os.path.join(out, "precision_c4.json"), "w") as f:
            json.dump(report, f, indent=1)
    assert err <= TOL
    assert rel_err(g32, ref64) <= TOL
    # matrix-core DFT stages: FP16 rounding bar (derived in test_mfma_model)
    assert snr_db(gm, ref) >= 66.0 and rel_err(gm, ref) <= 4e-3
