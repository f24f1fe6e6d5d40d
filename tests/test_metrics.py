"""The byte accounting and real-time multiple against the paper's Table 1/2."""

import csv
import pathlib

import pytest

from paper_1411_3656_amd import metrics

GOLDEN = pathlib.Path(__file__).parent / "golden" / "paper_tables.csv"


def _rows():
    lines = [ln for ln in GOLDEN.read_text().splitlines() if ln and not ln.startswith("#")]
    return list(csv.DictReader(lines))


def test_golden_table_is_complete():
    assert [r["platform"] for r in _rows()] == [
        "xeon_e5_2650_x2", "xeon_phi_5110p", "gtx_580", "tesla_k40", "gtx_750_ti"]


@pytest.mark.parametrize("row", _rows(), ids=lambda r: r["platform"])
def test_streaming_bandwidth_is_four_times_the_input_rate(row):
    # M_c * 6.5 GB/s is the input rate; the unfused FIR + FFT moves 4x that
    input_rate = float(row["m_c"]) * metrics.REALTIME_BYTES_PER_S
    ratio = float(row["bw_gbs"]) * 1e9 / input_rate
    assert abs(ratio - metrics.unfused_bytes_per_input_byte()) < 0.1


@pytest.mark.parametrize("row", [r for r in _rows() if r["pcie_gbs"]], ids=lambda r: r["platform"])
def test_single_mode_pcie_carries_input_plus_equal_output(row):
    input_rate = float(row["m_b"]) * metrics.REALTIME_BYTES_PER_S
    ratio = float(row["pcie_gbs"]) * 1e9 / input_rate
    assert abs(ratio - metrics.transfer_bytes_per_input_byte()) < 0.02


@pytest.mark.parametrize("row", _rows(), ids=lambda r: r["platform"])
def test_bandwidth_percent_of_peak(row):
    frac = metrics.roofline(float(row["bw_gbs"]), float(row["peak_bw_gbs"]))
    assert abs(100 * frac - float(row["bw_pct"])) <= 1.0


def test_realtime_multiple_and_cpu_ratio():
    rows = {r["platform"]: r for r in _rows()}
    assert metrics.realtime_multiple(6.5e9) == 1.0
    # conclusions: the best CPU is 3.6x slower than the K40
    assert round(float(rows["tesla_k40"]["m_c"]) / float(rows["xeon_e5_2650_x2"]["m_c"]), 1) == 3.6


def test_algorithmic_bytes():
    # N=1024, T=8, 2^27 input samples: 131065 spectra
    m = (1 << 27) // 1024 - 8 + 1
    b = metrics.algorithmic_bytes(1024, 8, m)
    assert b == (1 << 27) * 8 + m * 1024 * 8 + 8 * 1024 * 4
    assert metrics.input_bytes(1024, m) == m * 1024 * 8
