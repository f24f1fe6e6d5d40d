"""Throughput benchmark of the MI355X polyphase filter bank.

Default workload (one GPU): the SKA-LFAA-like single channel, N=1024
channels, T=8 taps, 2^27 complex FP32 input samples (1 GiB), sinc x Hamming
coefficients; a step is one ppf_execute over the whole batch (FIR presum and
FFT of all 131065 spectra) with the input already in HBM.

Prints one JSON line: input GB/s (the metric), the real-time multiple of
the 6.5 GB/s single-channel rate (the paper's Eq. 2, streaming mode M_c),
the roofline of the dominant kernel and the FP64 CPU oracle timed on a
bounded sample of the same workload.

Other workloads (--workload): c1 (N=256, T=8, 16384 spectra), sweep (the
shape sweep N in {64, 512, 4096, 16384} x T in {4, 8, 16, 32}, one line per
point). They print the same fields.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import pathlib
import sys
import time

import numpy as np

ROOT = pathlib.Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

from paper_1411_3656_amd import metrics, ppf, signals  # noqa: E402

METRIC = "PPF input GB/s (×6.5 GB/s real-time), % HBM peak; p99 stream chunk latency"
PROFILES = ROOT / "profiles"
CSRC = ROOT / "paper_1411_3656_amd" / "csrc"
# the kernel source each workload's dominant kernel is built from
KERNEL_SOURCES = {"c4": [CSRC / "ppf_mfma.hip"]}
DEFAULT_KERNEL_SOURCES = [CSRC / "ppf_kernels.hip", CSRC / "ppf_engine.h", CSRC / "ppf_fourstep.hip"]

WORKLOADS = {
    "c1": dict(name="plain_n256_t8_16384spectra", N=256, T=8, window="hamming", spectra=16384, tones=True,
               seed=signals.SEED_BASE + 0),
    "c2": dict(name="ska_lfaa_n1024_t8_2p27", N=1024, T=8, window="hamming", samples=1 << 27, tones=False,
               seed=signals.SEED_BASE + 1),
}
# The paper's Table 2 (its hardware; context, never the target): streaming
# (data in device memory) and single mode (PCIe included) real-time multiples.
PAPER_MC = {"2x Xeon E5-2650": 1.92, "Xeon Phi 5110P": 2.25, "GTX 580": 5.65, "Tesla K40": 6.89,
            "GTX 750 Ti": 2.39}
PAPER_MB = {"2x Xeon E5-2650": 1.92, "Xeon Phi 5110P": 0.40, "GTX 580": 0.37, "Tesla K40": 1.38,
            "GTX 750 Ti": 0.82}
SWEEP_N = [64, 512, 4096, 16384]
SWEEP_T = [4, 8, 16, 32]


def kernel_hash(workload: str = "c2") -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES.get(workload, DEFAULT_KERNEL_SOURCES):
        h.update(p.read_bytes())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary.

    The summary records the kernel-source hash it was taken with; a
    different hash means the kernel changed since, and traffic is null.
    """
    f = PROFILES / f"traffic_{workload}.json"
    if not f.exists():
        return None
    try:
        rec = json.loads(f.read_text())
    except ValueError:
        return None
    if rec.get("kernel_hash") != kernel_hash(workload):
        return None
    return rec.get("bytes_per_launch")


def cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, h32, budget_s: float = 12.0):
    """FP64 oracle on a bounded sample: whole spectra of the same workload."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:  # noqa: BLE001
        cores = os.cpu_count() or 1
    n, taps = cfg["N"], cfg["T"]
    spectra = 1024
    total_s, done = 0.0, 0
    x = signals.complex_gaussian((spectra + taps - 1) * n, 1.0, seed=cfg["seed"] + 77)
    oracle.ppf(x[: (16 + taps - 1) * n], h32, n, taps)            # warm the BLAS pools
    while total_s < budget_s and done < 4096:
        t0 = time.perf_counter()
        oracle.ppf(x, h32, n, taps)
        total_s += time.perf_counter() - t0
        done += 1
    rate = done * spectra * n * 8 / total_s / 1e9
    return {"value": round(rate, 4), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} x {spectra} spectra of N={n}, T={taps} ({done * spectra * n} input samples), "
                      f"{total_s:.1f} s of FP64 numpy/BLAS",
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}


def run_point(torch, n, taps, m_total, x_dev, h32, steps, warmup, path=ppf.PPF_PATH_AUTO, windows=0,
              in_type=ppf.PPF_C32, coeff_shift=None, fft_mode=ppf.PPF_FFT_F32):
    """Average ms per execute over `steps` after `warmup`; with windows > 0
    also the average of each of `windows` consecutive slices of the steps."""
    plan = ppf.Plan(n, taps, h32, path, in_type=in_type, coeff_shift=coeff_shift, fft_mode=fft_mode)
    out = torch.empty((m_total, n), dtype=torch.complex64, device="cuda")
    stream = torch.cuda.current_stream()
    ppf.ppf_set_stream(plan.handle, stream.cuda_stream)
    for _ in range(warmup):
        ppf.ppf_execute(plan.handle, x_dev, out, m_total)
    torch.cuda.synchronize()
    nwin = max(1, windows)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(nwin + 1)]
    bounds = [round(i * steps / nwin) for i in range(nwin + 1)]
    marks[0].record(stream)
    for w in range(nwin):
        for _ in range(bounds[w + 1] - bounds[w]):
            ppf.ppf_execute(plan.handle, x_dev, out, m_total)
        marks[w + 1].record(stream)
    torch.cuda.synchronize()
    ms = marks[0].elapsed_time(marks[-1]) / steps
    win_ms = [marks[w].elapsed_time(marks[w + 1]) / max(1, bounds[w + 1] - bounds[w]) for w in range(nwin)]
    used_path = plan.path
    plan.close()
    del out
    return (ms, used_path, win_ms) if windows else (ms, used_path)


def serve(load: float, seconds: float, warmup: float = 1.0) -> dict:
    """Serving workload: 64 streams, N in {256, 1024, 4096}, T in {8, 16},
    Poisson chunk arrivals of 1..64 spectra at `load` x 6.5 GB/s offered,
    32 GB state budget; run by the native load generator."""
    import subprocess
    exe = ROOT / "paper_1411_3656_amd" / "ppf_serve_bench"
    if not exe.exists():
        return {"error": f"{exe} is not built"}
    cmd = [str(exe), "--load", str(load), "--seconds", str(seconds), "--warmup", str(warmup), "--streams", "64",
           "--seed", str(signals.SEED_BASE + 4), "--budget", "32e9", "--inflight", "2"]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=seconds + warmup + 120)
    if res.returncode != 0:
        return {"error": "load generator failed", "stderr": res.stderr[-2000:], "stdout": res.stdout[-2000:]}
    s = json.loads(res.stdout.strip().splitlines()[-1])
    return {
        "metric": METRIC, "value": s["sustained_gbps"], "unit": "GB/s", "n_gpus": 1,
        "steps": s["chunks"], "warmup": warmup, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "realtime_multiple": s["realtime_multiple"],
        "config": {"workload": s["workload"], "streams": 64, "N": [256, 1024, 4096], "taps": [8, 16],
                   "chunk_spectra": [1, 64], "arrivals": "poisson", "offered_load_multiple": load,
                   "offered_gbps": s["offered_gbps"], "state_budget_bytes": 32e9, "seconds": seconds},
        "serving": {k: s[k] for k in ("p50_us", "p99_us", "max_us", "mean_us", "chunks", "batches",
                                      "mean_batch_chunks", "chunk_rate_per_s", "late_submits", "mean_n")},
    }


def line(workload, n, taps, m_total, ms, used_path, steps, warmup, traffic=None, cpu=None):
    in_bytes = metrics.input_bytes(n, m_total)
    gbps = in_bytes / (ms * 1e-3) / 1e9
    alg = metrics.algorithmic_bytes(n, taps, m_total)
    achieved = alg / (ms * 1e-3) / 1e9
    peak = metrics.HBM_PEAK_BYTES_PER_S / 1e9
    rec = {
        "metric": METRIC,
        "value": round(gbps, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "realtime_multiple": round(metrics.realtime_multiple(gbps * 1e9), 2),
        "config": {"workload": workload, "N": n, "taps": taps, "nspectra": m_total,
                   "input_samples": (m_total + taps - 1) * n,
                   "path": {1: "fused", 2: "two_pass"}.get(used_path, str(used_path))},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": peak, "unit": "GB/s",
                     "frac": round(achieved / peak, 4),
                     "traffic": None if traffic is None else int(traffic),
                     "algorithmic_bytes": alg},
    }
    if cpu is not None:
        rec["cpu_baseline"] = cpu
    rec["paper_context_mc"] = PAPER_MC
    return rec


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2",
                    choices=["c1", "c2", "c2_reduced", "c4", "sweep", "copy", "serve", "serve_sweep", "mb", "detect"])
    ap.add_argument("--k-int", type=int, default=16, help="detect: spectra integrated per power spectrum")
    ap.add_argument("--load", type=float, default=50.0, help="serving: offered load in multiples of 6.5 GB/s")
    ap.add_argument("--seconds", type=float, default=10.0, help="serving: measured seconds")
    ap.add_argument("--path", default="auto", choices=["auto", "fused", "two_pass"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="c2: skip the short serving leg")
    ap.add_argument("--point", default="",
                    help="sweep: run only the point 'N,T' (e.g. 512,8)")
    ap.add_argument("--chunk-mib", type=int, default=0,
                    help="mb: input MiB per pipeline chunk (0: the library's default)")
    ap.add_argument("--windows", type=int, default=0,
                    help="also report the mean step time of this many consecutive slices of the timed steps")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        return 2

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        return 1
    path = {"auto": ppf.PPF_PATH_AUTO, "fused": ppf.PPF_PATH_FUSED, "two_pass": ppf.PPF_PATH_TWO_PASS}[args.path]

    if args.workload in ("serve", "serve_sweep"):
        loads = [args.load] if args.workload == "serve" else [50, 100, 150, 200, 300, 400]
        for load in loads:
            rec = serve(load, args.seconds)
            print(json.dumps(rec), flush=True)
            if rec.get("error"):
                return 1
        return 0

    if args.workload == "c4":
        # precision form: complex int8 input (sigma 16), FP16 coefficients with
        # a 2^s scale, FP32 FIR accumulation, radix-16 DFT stages on FP16 matrix
        # cores with FP32 accumulation. Beside it: the same int8/FP16 input with
        # FP32 DFT stages, and the FP32 path on the same values.
        n, taps, n_samples = 4096, 16, 1 << 28
        m_total = n_samples // n - taps + 1
        x = signals.int8_input(n_samples, seed=signals.SEED_BASE + 3, sigma=16.0)
        x_dev = torch.from_numpy(x).cuda()
        del x
        h64 = signals.design_coeffs(n, taps, "hamming")
        h16, shift = signals.coeffs_fp16(h64)
        msm, usedm = run_point(torch, n, taps, m_total, x_dev, h16, args.steps, args.warmup,
                               in_type=ppf.PPF_CI8, coeff_shift=shift, fft_mode=ppf.PPF_FFT_MFMA_F16)
        rec = line("precision_n4096_t16_int8_fp16coef_2p28", n, taps, m_total, msm, usedm, args.steps,
                   args.warmup, measured_traffic("c4"))
        in_b = metrics.input_bytes(n, m_total, 2)
        rec["value"] = round(in_b / (msm * 1e-3) / 1e9, 3)
        rec["realtime_multiple"] = round(metrics.realtime_multiple(rec["value"] * 1e9), 2)
        rec["dtype"] = "ci8_in/f16_coef/f32_fir/f16_mfma_f32_acc"
        rec["config"]["fft"] = "mfma_f16_radix16"
        alg = metrics.algorithmic_bytes(n, taps, m_total, in_bytes=2, out_bytes=8, coeff_bytes=2)
        rec["roofline"].update({"achieved": round(alg / (msm * 1e-3) / 1e9, 2), "algorithmic_bytes": alg})
        rec["roofline"]["frac"] = round(rec["roofline"]["achieved"] / rec["roofline"]["peak"], 4)
        rec["samples_per_s"] = round(n * m_total / (msm * 1e-3), 1)
        ms8, used8 = run_point(torch, n, taps, m_total, x_dev, h16, args.steps, args.warmup,
                               in_type=ppf.PPF_CI8, coeff_shift=shift)
        rec["int8_fp32_fft_path"] = {"ms_per_step": round(ms8, 5),
                                     "input_gbps_int8": round(in_b / (ms8 * 1e-3) / 1e9, 3),
                                     "path": {1: "fused", 2: "two_pass"}.get(used8)}
        x32 = torch.view_as_complex(x_dev.to(torch.float32).contiguous())
        del x_dev
        ms32, used32 = run_point(torch, n, taps, m_total, x32, h64.astype(np.float32), args.steps, args.warmup)
        rec["fp32_path_same_values"] = {"ms_per_step": round(ms32, 5),
                                        "input_gbps_fp32": round(metrics.input_bytes(n, m_total) / (ms32 * 1e-3) / 1e9, 3),
                                        "samples_per_s": round(n * m_total / (ms32 * 1e-3), 1),
                                        "path": {1: "fused", 2: "two_pass"}.get(used32)}
        print(json.dumps(rec), flush=True)
        return 0

    if args.workload == "c2_reduced":
        # C2's shape (N=1024, T=8, 2^27 samples) with complex int8 and complex
        # FP16 input and FP16 coefficients, widened to FP32 in the fused
        # kernel's loads: input bytes 2 or 4 per sample instead of 8.
        n, taps, n_samples = 1024, 8, 1 << 27
        m_total = n_samples // n - taps + 1
        h64 = signals.design_coeffs(n, taps, "hamming")
        h16, shift = signals.coeffs_fp16(h64)
        for kind, name, sb, seed, fft in ((ppf.PPF_CI8, "int8", 2, 5, ppf.PPF_FFT_F32),
                                          (ppf.PPF_C16, "fp16", 4, 6, ppf.PPF_FFT_F32),
                                          (ppf.PPF_CI8, "int8", 2, 5, ppf.PPF_FFT_MFMA_F16),
                                          (ppf.PPF_C16, "fp16", 4, 6, ppf.PPF_FFT_MFMA_F16)):
            if kind == ppf.PPF_CI8:
                x = signals.int8_input(n_samples, seed=signals.SEED_BASE + seed, sigma=16.0)
            else:
                x = signals.to_complex_fp16(signals.complex_gaussian(n_samples, 1.0, seed=signals.SEED_BASE + seed))
            x_dev = torch.from_numpy(x).cuda()
            del x
            ms, used = run_point(torch, n, taps, m_total, x_dev, h16, args.steps, args.warmup, path,
                                 in_type=kind, coeff_shift=shift, fft_mode=fft)
            mc = fft == ppf.PPF_FFT_MFMA_F16
            rec = line(f"ska_lfaa_n1024_t8_2p27_{name}_in" + ("_mfma" if mc else ""), n, taps, m_total, ms, used,
                       args.steps, args.warmup)
            rec["config"]["fft"] = "mfma_f16_radix4_16_16" if mc else "f32"
            in_b = metrics.input_bytes(n, m_total, sb)
            rec["value"] = round(in_b / (ms * 1e-3) / 1e9, 3)
            rec["realtime_multiple"] = round(metrics.realtime_multiple(rec["value"] * 1e9), 2)
            rec["dtype"] = f"{'ci8' if sb == 2 else 'c16'}_in/f16_coef/f32" + ("_fir/f16_mfma_f32_acc" if mc else "")
            alg = metrics.algorithmic_bytes(n, taps, m_total, in_bytes=sb, out_bytes=8, coeff_bytes=2)
            rec["roofline"].update({"achieved": round(alg / (ms * 1e-3) / 1e9, 2), "algorithmic_bytes": alg})
            rec["roofline"]["frac"] = round(rec["roofline"]["achieved"] / rec["roofline"]["peak"], 4)
            rec["samples_per_s"] = round(n * m_total / (ms * 1e-3), 1)
            print(json.dumps(rec), flush=True)
            del x_dev
            torch.cuda.empty_cache()
        return 0

    if args.workload == "detect":
        # C2 with detection in the epilogue: |X|^2 summed over K spectra; the
        # output shrinks from 8 B per bin and spectrum to 4 B per bin per K
        cfg = WORKLOADS["c2"]
        n, taps, k_int = cfg["N"], cfg["T"], args.k_int
        m_total = (cfg["samples"] // n - taps + 1) // k_int * k_int
        h32 = signals.design_coeffs(n, taps, cfg["window"]).astype(np.float32)
        x = signals.complex_gaussian((m_total + taps - 1) * n, 1.0, seed=cfg["seed"])
        x_dev = torch.from_numpy(x).cuda()
        del x
        plan = ppf.Plan(n, taps, h32)
        out = torch.empty((m_total // k_int, n), dtype=torch.float32, device="cuda")
        stream = torch.cuda.current_stream()
        ppf.ppf_set_stream(plan.handle, stream.cuda_stream)
        for _ in range(args.warmup):
            ppf.ppf_execute_power(plan.handle, x_dev, out, m_total, k_int)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.steps):
            ppf.ppf_execute_power(plan.handle, x_dev, out, m_total, k_int)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        used = plan.path
        plan.close()
        in_b = metrics.input_bytes(n, m_total)
        gbps = in_b / (ms * 1e-3) / 1e9
        alg = (m_total + taps - 1) * n * 8 + (m_total // k_int) * n * 4 + taps * n * 4
        peak = metrics.HBM_PEAK_BYTES_PER_S / 1e9
        print(json.dumps({
            "metric": METRIC, "value": round(gbps, 3), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "realtime_multiple": round(metrics.realtime_multiple(gbps * 1e9), 2),
            "config": {"workload": f"detect_k{k_int}_n1024_t8_2p27", "N": n, "taps": taps, "nspectra": m_total,
                       "K": k_int, "path": {1: "fused", 2: "two_pass"}.get(used)},
            "roofline": {"bound": "hbm", "achieved": round(alg / (ms * 1e-3) / 1e9, 2), "peak": peak, "unit": "GB/s",
                         "frac": round(alg / (ms * 1e-3) / 1e9 / peak, 4), "traffic": None,
                         "algorithmic_bytes": alg}}), flush=True)
        return 0

    if args.workload == "mb":
        # single mode (M_b of section 3): C2's input and output in page-locked
        # host memory, moved over PCIe by the chunked pipeline
        cfg = WORKLOADS["c2"]
        n, taps = cfg["N"], cfg["T"]
        m_total = cfg["samples"] // n - taps + 1
        h32 = signals.design_coeffs(n, taps, cfg["window"]).astype(np.float32)
        x = signals.complex_gaussian((m_total + taps - 1) * n, 1.0, seed=cfg["seed"])
        xin = torch.from_numpy(x).pin_memory()
        del x
        out = torch.empty((m_total, n), dtype=torch.complex64).pin_memory()
        plan = ppf.Plan(n, taps, h32)
        # spectra per pipeline chunk: 0 is the library's default (192 MiB of input)
        chunk = (args.chunk_mib << 20) // (n * 8) if args.chunk_mib > 0 else 0
        stream = torch.cuda.current_stream()
        steps = min(args.steps, 20)
        warm = min(args.warmup, 2)
        for _ in range(warm):
            plan.execute_host(xin, out, chunk_spectra=chunk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(steps):
            plan.execute_host(xin, out, chunk_spectra=chunk)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        ms = ev0.elapsed_time(ev1) / steps
        plan.close()
        in_b = metrics.input_bytes(n, m_total)
        gbps = in_b / (ms * 1e-3) / 1e9
        pcie = (in_b + m_total * n * 8) / (ms * 1e-3) / 1e9
        # the link's own rates with the same page-locked buffers, copied in
        # 128 MiB pieces as the pipeline does: each direction alone, and
        # both at once on two streams
        dev_in = torch.empty(xin.shape, dtype=xin.dtype, device="cuda")
        dev_out = torch.empty(out.shape, dtype=out.dtype, device="cuda")
        s_in, s_out = torch.cuda.Stream(), torch.cuda.Stream()
        piece = (128 << 20) // 8
        flat_in, flat_dev_in = xin.reshape(-1), dev_in.reshape(-1)
        flat_out, flat_dev_out = out.reshape(-1), dev_out.reshape(-1)

        def timed(fn, reps=3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t) / reps

        def h2d(i):
            with torch.cuda.stream(s_in):
                flat_dev_in[i:i + piece].copy_(flat_in[i:i + piece], non_blocking=True)

        def d2h(i):
            with torch.cuda.stream(s_out):
                flat_out[i:i + piece].copy_(flat_dev_out[i:i + piece], non_blocking=True)

        def both():
            for i in range(0, max(flat_in.numel(), flat_out.numel()), piece):
                if i < flat_in.numel():
                    h2d(i)
                if i < flat_out.numel():
                    d2h(i)

        t_h2d = timed(lambda: [h2d(i) for i in range(0, flat_in.numel(), piece)])
        t_d2h = timed(lambda: [d2h(i) for i in range(0, flat_out.numel(), piece)])
        t_both = timed(both)
        link = {"h2d_gbps": round(in_b / t_h2d / 1e9, 2), "d2h_gbps": round(out.numel() * 8 / t_d2h / 1e9, 2),
                "both_directions_gbps": round((in_b + out.numel() * 8) / t_both / 1e9, 2)}
        del dev_in, dev_out
        print(json.dumps({
            "metric": METRIC, "value": round(gbps, 3), "unit": "GB/s", "n_gpus": 1, "steps": steps, "warmup": warm,
            "ms_per_step": round(ms, 4), "host_wall_ms_per_step": round(wall * 1e3, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "realtime_multiple_mb": round(metrics.realtime_multiple(gbps * 1e9), 2),
            "pcie_gbps_in_plus_out": round(pcie, 2),
            "pcie_copy_only": link,
            "pcie_frac_of_copy_only": round(pcie / link["both_directions_gbps"], 3),
            "config": {"workload": "single_mode_host_resident_n1024_t8_2p27", "N": n, "taps": taps,
                       "nspectra": m_total, "host_memory": "page-locked",
                       "chunk_input_bytes": (chunk * n * 8) if chunk else 192 << 20},
            "paper_context_mb": PAPER_MB}), flush=True)
        return 0

    if args.workload == "copy":
        # plain device copies of known size: the yardstick for the HBM byte
        # counters (FETCH_SIZE, WRITE_SIZE) and the achievable copy rate, by
        # the native copy program (long warm-up) and by torch
        import subprocess
        exe = ROOT / "paper_1411_3656_amd" / "ppf_copy_bench"
        if exe.exists():
            res = subprocess.run([str(exe), "--mib", "1024", "--reps", str(max(20, args.steps)), "--warmup", "300"],
                                 capture_output=True, text=True, timeout=300)
            sys.stdout.write(res.stdout)
            if res.returncode != 0:
                sys.stderr.write(res.stderr)
                return 1
        nbytes = 1 << 30
        src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(args.warmup):
            dst.copy_(src)
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(args.steps):
            dst.copy_(src)
        end.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(end) / args.steps
        print(json.dumps({"workload": "copy_1GiB_torch", "bytes_read": nbytes, "bytes_written": nbytes,
                          "ms_per_copy": round(ms, 5), "GBps_moved": round(2 * nbytes / ms / 1e6, 1)}),
              flush=True)
        return 0

    if args.workload == "sweep":
        only = tuple(int(v) for v in args.point.split(",")) if args.point else None
        for i, n in enumerate(SWEEP_N):
            if only and n != only[0]:
                continue
            x = signals.complex_gaussian(1 << 28, 1.0, seed=signals.SEED_BASE + 2 + 100 * i)
            x_dev = torch.from_numpy(x).cuda()
            del x
            for taps in SWEEP_T:
                if only and taps != only[1]:
                    continue
                h32 = signals.design_coeffs(n, taps, "hann").astype(np.float32)
                m_total = (1 << 28) // n - taps + 1
                ms, used = run_point(torch, n, taps, m_total, x_dev, h32, args.steps, args.warmup, path)
                rec = line(f"sweep_n{n}_t{taps}_2p28", n, taps, m_total, ms, used, args.steps, args.warmup,
                           measured_traffic(f"sweep_n{n}_t{taps}"))
                print(json.dumps(rec), flush=True)
            del x_dev
            torch.cuda.empty_cache()
        return 0

    cfg = WORKLOADS[args.workload]
    n, taps = cfg["N"], cfg["T"]
    if "samples" in cfg:
        m_total = cfg["samples"] // n - taps + 1
    else:
        m_total = cfg["spectra"]
    n_samples = (m_total + taps - 1) * n
    h32 = signals.design_coeffs(n, taps, cfg["window"]).astype(np.float32)
    if cfg["tones"]:
        x = signals.plain_input(n, n_samples, seed=cfg["seed"])
    else:
        x = signals.complex_gaussian(n_samples, 1.0, seed=cfg["seed"])
    x_dev = torch.from_numpy(x).cuda()
    del x
    res = run_point(torch, n, taps, m_total, x_dev, h32, args.steps, args.warmup, path, args.windows)
    ms, used = res[0], res[1]
    cpu = None if args.no_cpu_baseline else cpu_baseline(cfg, h32)
    rec = line(cfg["name"], n, taps, m_total, ms, used, args.steps, args.warmup,
               measured_traffic(args.workload), cpu)
    if args.windows:
        rec["window_ms_per_step"] = [round(w, 5) for w in res[2]]
    if args.workload == "c2" and not args.no_serving:
        # the metric's p99 chunk latency: a short run of the 64-stream
        # serving mix at 100 x the real-time rate, after the timed region
        del x_dev
        torch.cuda.empty_cache()
        sv = serve(100.0, 3.0, warmup=0.5)
        if sv.get("error"):
            rec["serving"] = {"error": sv["error"]}
        else:
            rec["serving"] = {"p50_us": sv["serving"]["p50_us"], "p99_us": sv["serving"]["p99_us"],
                              "sustained_gbps": sv["value"], "realtime_multiple": sv["realtime_multiple"],
                              "offered_load_multiple": 100.0, "seconds": 3.0,
                              "workload": sv["config"]["workload"], "chunks": sv["serving"]["chunks"]}
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
