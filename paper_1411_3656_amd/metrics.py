"""Throughput accounting for the PPF: bytes, real-time multiples, roofline.

The real-time multiple is the paper's Eq. 2 (section 3): one second of data
divided by the time taken to process it, one second being 6.5 GB of the
single-SKA-LFAA-channel stream. M_c counts only device time (data resident);
M_b would include host transfers.
"""

from __future__ import annotations

REALTIME_BYTES_PER_S = 6.5e9     # section 1 / section 3: 6.5 GB/s per SKA-LFAA channel
HBM_PEAK_BYTES_PER_S = 8.0e12    # MI355X HBM3E

#: bytes per stored complex sample, by input type name
SAMPLE_BYTES = {"c32": 8, "c16": 4, "ci8": 2}


def realtime_multiple(input_bytes_per_s: float) -> float:
    """Eq. 2: multiples of real time for a given input byte rate."""
    return input_bytes_per_s / REALTIME_BYTES_PER_S


def input_bytes(n_channels: int, nspectra: int, in_bytes: int = 8) -> int:
    """Input consumed by nspectra spectra: N new samples per spectrum."""
    return int(n_channels) * int(nspectra) * int(in_bytes)


def algorithmic_bytes(n_channels: int, taps: int, nspectra: int,
                      in_bytes: int = 8, out_bytes: int = 8, coeff_bytes: int = 4) -> int:
    """Compulsory HBM bytes of one batch PPF launch.

    Every input sample once ((M+T-1)*N of them), every output bin once
    (M*N complex FP32) and the T*N coefficients once. Re-reads of
    overlapping tap blocks and any intermediate round trip are not counted.
    """
    n, t, m = int(n_channels), int(taps), int(nspectra)
    return (m + t - 1) * n * in_bytes + m * n * out_bytes + t * n * coeff_bytes


def unfused_bytes_per_input_byte(in_bytes: int = 8, out_bytes: int = 8) -> float:
    """HBM bytes per input byte when FIR and FFT are separate passes.

    FIR reads x and writes u, the FFT reads u and writes X: 4x the input
    for complex FP32 in and out. The paper's streaming-mode bandwidth is
    about four times its input rate on every platform (Table 2).
    """
    return (in_bytes + out_bytes + out_bytes + out_bytes) / in_bytes


def transfer_bytes_per_input_byte(in_bytes: int = 8, out_bytes: int = 8) -> float:
    """Host<->device bytes per input byte in single mode: input in, spectra out."""
    return (in_bytes + out_bytes) / in_bytes


def roofline(achieved: float, peak: float) -> float:
    return achieved / peak if peak else float("nan")
