"""The C ABI without a GPU: the library loads, exports every declared symbol,
and rejects invalid arguments before making any HIP call."""

import ctypes
import pathlib
import re

import numpy as np
import pytest

from paper_1411_3656_amd import ppf

ROOT = pathlib.Path(__file__).resolve().parents[1]
HEADERS = sorted((ROOT / "include").glob("*.h"))


def declared_functions():
    names = []
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", h.read_text(), flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        for m in re.finditer(r"\b(ppf_[a-z0-9_]+)\s*\(", text):
            names.append(m.group(1))
    return sorted(set(names))


def test_headers_exist_and_declare_the_boundary():
    names = declared_functions()
    for required in ("ppf_plan", "ppf_execute", "ppf_destroy", "ppf_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ppf.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    bound = {name for name, _, _ in ppf._SIGNATURES}
    assert set(declared_functions()) <= bound


def test_status_strings():
    assert ppf.status_str(ppf.PPF_OK) == "PPF_OK"
    assert ppf.status_str(ppf.PPF_ERR_ALIGN) == "PPF_ERR_ALIGN"
    assert ppf.status_str(-99) == "PPF_ERR_UNKNOWN"


def _raw_plan(n, t, coeffs_ptr):
    return ppf.lib().ppf_plan(n, t, coeffs_ptr)


@pytest.mark.parametrize("n,t,status", [
    (100, 8, ppf.PPF_ERR_UNSUPPORTED),     # not a power of two
    (8, 8, ppf.PPF_ERR_UNSUPPORTED),       # below 16
    (32768, 8, ppf.PPF_ERR_UNSUPPORTED),   # above 16384
    (256, 65, ppf.PPF_ERR_UNSUPPORTED),    # too many taps
    (256, 0, ppf.PPF_ERR_INVALID),
    (0, 8, ppf.PPF_ERR_INVALID),
])
def test_plan_rejects_unsupported_sizes(n, t, status):
    h = np.ones(max(1, n * max(t, 1)), dtype=np.float32)
    assert not _raw_plan(n, t, h.ctypes.data)
    assert ppf.last_error()[0] == status


def test_plan_rejects_null_coefficients():
    assert not _raw_plan(256, 8, None)
    code, msg = ppf.last_error()
    assert code == ppf.PPF_ERR_INVALID and "coeffs" in msg


def test_plan_ex_validates_types():
    h = np.ones(256 * 8, dtype=np.float32)
    L = ppf.lib()
    assert not L.ppf_plan_ex(256, 8, h.ctypes.data, 7, 0, ppf.PPF_C32, ppf.PPF_FFT_F32)
    assert ppf.last_error()[0] == ppf.PPF_ERR_INVALID
    assert not L.ppf_plan_ex(256, 8, h.ctypes.data, ppf.PPF_R32, 3, ppf.PPF_C32, ppf.PPF_FFT_F32)
    assert ppf.last_error()[0] == ppf.PPF_ERR_INVALID
    assert not L.ppf_plan_ex(256, 8, h.ctypes.data, ppf.PPF_R32, 0, 9, ppf.PPF_FFT_F32)
    assert ppf.last_error()[0] == ppf.PPF_ERR_INVALID
    assert not L.ppf_plan_ex(256, 8, h.ctypes.data, ppf.PPF_R32, 0, ppf.PPF_C32, 5)
    assert ppf.last_error()[0] == ppf.PPF_ERR_INVALID


def test_matrix_core_mode_validates_its_domain():
    """The FP16 matrix-core mode is built for N = 256, 1024 and 4096, taps
    <= 16, complex int8 or FP16 input and FP16 coefficients; anything else
    is rejected before any device call."""
    L = ppf.lib()
    h16 = np.ones(4096 * 16, dtype=np.float16)
    h32 = np.ones(4096 * 16, dtype=np.float32)
    mf = ppf.PPF_FFT_MFMA_F16
    cases = [
        (2048, 16, h16, ppf.PPF_R16, ppf.PPF_CI8),     # N not built
        (512, 8, h16, ppf.PPF_R16, ppf.PPF_C16),
        (64, 4, h16, ppf.PPF_R16, ppf.PPF_CI8),
        (1024, 17, np.ones(1024 * 17, np.float16), ppf.PPF_R16, ppf.PPF_CI8),
        (4096, 17, np.ones(4096 * 17, np.float16), ppf.PPF_R16, ppf.PPF_CI8),   # more than 16 taps
        (4096, 16, h32, ppf.PPF_R32, ppf.PPF_CI8),     # FP32 coefficients
        (4096, 16, h16, ppf.PPF_R16, ppf.PPF_C32),
    ]
    for n, taps, h, ct, it in cases:
        assert not L.ppf_plan_ex(n, taps, h.ctypes.data, ct, 0, it, mf)
        code, msg = ppf.last_error()
        assert code == ppf.PPF_ERR_UNSUPPORTED and "MFMA" in msg, (n, taps, ct, it, msg)


def test_null_handles():
    L = ppf.lib()
    assert L.ppf_execute(None, None, None, 4) == ppf.PPF_ERR_INVALID
    assert L.ppf_set_stream(None, None) == ppf.PPF_ERR_INVALID
    assert L.ppf_plan_set_path(None, 1) == ppf.PPF_ERR_INVALID
    v = ctypes.c_longlong(0)
    assert L.ppf_plan_query(None, 0, ctypes.byref(v)) == ppf.PPF_ERR_INVALID
    assert L.ppf_destroy(None) == ppf.PPF_OK


def test_error_raises_in_binding():
    with pytest.raises(ppf.PPFError) as ei:
        ppf.ppf_plan(100, 8, np.ones(800, np.float32))
    assert ei.value.status == ppf.PPF_ERR_UNSUPPORTED


def test_server_entry_points_reject_null_handles():
    L = ppf.lib()
    p50, p99, gb = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    assert L.ppf_server_stats(None, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(gb)) == ppf.PPF_ERR_INVALID
    h = ctypes.c_void_p()
    assert L.ppf_server_open_stream(None, None, ctypes.byref(h)) == ppf.PPF_ERR_INVALID
    assert L.ppf_server_open_stream_ex(None, None, ppf.PPF_OPEN_NOWAIT, ctypes.byref(h)) == ppf.PPF_ERR_INVALID
    assert L.ppf_server_submit(None, None, -1) == ppf.PPF_ERR_INVALID
    assert L.ppf_server_stream_admitted(None) == ppf.PPF_ERR_INVALID
    assert L.ppf_server_close_stream(None) == ppf.PPF_ERR_INVALID
    assert L.ppf_server_poll(None, None, 0) == ppf.PPF_ERR_INVALID
    assert L.ppf_server_drain(None, 1.0) == ppf.PPF_ERR_INVALID
    assert L.ppf_server_destroy(None) == ppf.PPF_OK
    assert L.ppf_stream_push(None, None) == ppf.PPF_ERR_INVALID
    assert L.ppf_stream_destroy(None) == ppf.PPF_OK
    assert L.ppf_execute_power(None, None, None, 16, 4) == ppf.PPF_ERR_INVALID
