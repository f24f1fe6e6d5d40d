"""Thin ctypes binding of libppf.so (include/ppf.h), same names as the C ABI.

Every function here only marshals arguments: all PPF arithmetic runs in the
HIP library. Device buffers are passed as integer addresses (torch's
``tensor.data_ptr()``) and HIP streams as integer handles (torch's
``stream.cuda_stream``). Failures raise :class:`PPFError`; a missing
library raises at load time, never falling back to anything else.
"""

from __future__ import annotations

import ctypes
import os
import pathlib

# PPF_LIBRARY selects another build of the same library (tuning variants).
_LIB_PATH = pathlib.Path(os.environ.get("PPF_LIBRARY") or pathlib.Path(__file__).resolve().with_name("libppf.so"))
_lib = None

# status codes (enum ppf_status)
PPF_OK = 0
PPF_ERR_INVALID = -1
PPF_ERR_UNSUPPORTED = -2
PPF_ERR_ALIGN = -3
PPF_ERR_NOMEM = -4
PPF_ERR_BUDGET = -5
PPF_ERR_HIP = -6
PPF_ERR_BUSY = -7

# element types (enum ppf_dtype)
PPF_C32, PPF_C16, PPF_CI8, PPF_R32, PPF_R16 = 0, 1, 2, 3, 4
# FFT modes, paths, queries
PPF_FFT_F32, PPF_FFT_MFMA_F16 = 0, 1
PPF_PATH_AUTO, PPF_PATH_FUSED, PPF_PATH_TWO_PASS = 0, 1, 2
(PPF_Q_N, PPF_Q_TAPS, PPF_Q_PATH, PPF_Q_WORKSPACE_BYTES, PPF_Q_IN_TYPE, PPF_Q_FFT_MODE,
 PPF_Q_COEFF_SHIFT, PPF_Q_FUSED_AVAILABLE) = range(8)

# windows of the prototype-filter designer (enum ppf_window)
PPF_WIN_RECT, PPF_WIN_HAMMING, PPF_WIN_HANN, PPF_WIN_KAISER, PPF_WIN_USER = range(5)
WINDOWS = {"rect": PPF_WIN_RECT, "hamming": PPF_WIN_HAMMING, "hann": PPF_WIN_HANN, "kaiser": PPF_WIN_KAISER,
           "user": PPF_WIN_USER}

SAMPLE_BYTES = {PPF_C32: 8, PPF_C16: 4, PPF_CI8: 2}

_c_ll = ctypes.c_longlong
_c_vp = ctypes.c_void_p
_c_int = ctypes.c_int


class ppf_chunk(ctypes.Structure):  # noqa: N801 - the C name
    _fields_ = [("in_", _c_vp), ("out", _c_vp), ("nspectra", _c_ll), ("tag", ctypes.c_ulonglong)]


# flags of ppf_server_open_stream_ex
PPF_OPEN_QUEUE, PPF_OPEN_NOWAIT = 0, 1


class ppf_server_stats_t(ctypes.Structure):  # noqa: N801 - the C name
    _fields_ = [(n, _c_ll) for n in ("chunks_done", "spectra_done", "bytes_in_done", "batches", "admitted",
                                     "rejected", "queued_admissions", "state_bytes_used", "tags_dropped")] + \
               [(n, ctypes.c_double) for n in ("p50_us", "p99_us", "max_us", "mean_us", "elapsed_s",
                                               "input_gbps", "mean_batch_chunks", "mean_batch_gpu_us",
                                               "mean_form_us", "mean_launch_us")]


class PPFError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_str(status)} ({status}): {message}")
        self.status = status


# (name, restype, argtypes) of every exported function
_SIGNATURES = [
    ("ppf_plan", _c_vp, [_c_int, _c_int, _c_vp]),
    ("ppf_plan_ex", _c_vp, [_c_int, _c_int, _c_vp, _c_int, _c_int, _c_int, _c_int]),
    ("ppf_set_stream", _c_int, [_c_vp, _c_vp]),
    ("ppf_plan_set_path", _c_int, [_c_vp, _c_int]),
    ("ppf_plan_query", _c_int, [_c_vp, _c_int, ctypes.POINTER(_c_ll)]),
    ("ppf_execute", _c_int, [_c_vp, _c_vp, _c_vp, _c_ll]),
    ("ppf_execute_noalloc", _c_int, [_c_vp, _c_vp, _c_vp, _c_ll]),
    ("ppf_execute_host", _c_int, [_c_vp, _c_vp, _c_vp, _c_ll, _c_ll]),
    ("ppf_execute_power", _c_int, [_c_vp, _c_vp, _c_vp, _c_ll, _c_int]),
    ("ppf_destroy", _c_int, [_c_vp]),
    ("ppf_design_coeffs", _c_int, [_c_int, _c_int, _c_int, ctypes.c_double, _c_vp, _c_vp]),
    ("ppf_kaiser_beta", _c_int, [ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    ("ppf_stream_create", _c_vp, [_c_vp]),
    ("ppf_stream_push", _c_int, [_c_vp, _c_vp]),
    ("ppf_stream_get_history", _c_int, [_c_vp, _c_vp]),
    ("ppf_stream_set_history", _c_int, [_c_vp, _c_vp]),
    ("ppf_stream_position", _c_ll, [_c_vp]),
    ("ppf_stream_destroy", _c_int, [_c_vp]),
    ("ppf_clock_ns", _c_ll, []),
    ("ppf_server_create", _c_vp, [ctypes.c_size_t, _c_int]),
    ("ppf_server_open_stream", _c_int, [_c_vp, _c_vp, ctypes.POINTER(_c_vp)]),
    ("ppf_server_open_stream_ex", _c_int, [_c_vp, _c_vp, _c_int, ctypes.POINTER(_c_vp)]),
    ("ppf_server_stream_admitted", _c_int, [_c_vp]),
    ("ppf_server_submit", _c_int, [_c_vp, _c_vp, _c_ll]),
    ("ppf_server_poll", _c_int, [_c_vp, ctypes.POINTER(ctypes.c_ulonglong), _c_int]),
    ("ppf_server_drain", _c_int, [_c_vp, ctypes.c_double]),
    ("ppf_server_close_stream", _c_int, [_c_vp]),
    ("ppf_server_stats", _c_int, [_c_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]),
    ("ppf_server_get_stats", _c_int, [_c_vp, _c_vp]),
    ("ppf_server_reset_stats", _c_int, [_c_vp]),
    ("ppf_server_destroy", _c_int, [_c_vp]),
    ("ppf_last_error", _c_int, []),
    ("ppf_last_error_message", ctypes.c_char_p, []),
    ("ppf_status_str", ctypes.c_char_p, [_c_int]),
]


def lib() -> ctypes.CDLL:
    """Load libppf.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            raise RuntimeError(f"{_LIB_PATH} is not built: run `python -m paper_1411_3656_amd.build`")
        # torch ships its own HIP runtime. Loaded first, it is the runtime the
        # library's HIP calls bind to as well; if the library loads the
        # system runtime first, torch later finds no devices. torch provides
        # the device memory and streams, so it goes first.
        import torch  # noqa: F401
        handle = ctypes.CDLL(str(_LIB_PATH))
        for name, res, args in _SIGNATURES:
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def library_path() -> pathlib.Path:
    return _LIB_PATH


def status_str(status: int) -> str:
    try:
        return lib().ppf_status_str(int(status)).decode()
    except Exception:  # noqa: BLE001 - used while formatting an error
        return str(status)


def last_error() -> tuple[int, str]:
    L = lib()
    return int(L.ppf_last_error()), L.ppf_last_error_message().decode(errors="replace")


def _check(status: int) -> int:
    if status != PPF_OK:
        code, msg = last_error()
        raise PPFError(status, msg)
    return status


def _handle(h):
    if not h:
        code, msg = last_error()
        raise PPFError(code, msg)
    return h


def _addr(buf) -> int | None:
    """Address of a buffer: an int, an object with data_ptr() (a tensor), or
    a numpy array."""
    if buf is None:
        return None
    if isinstance(buf, int):
        return buf
    if hasattr(buf, "data_ptr"):
        return int(buf.data_ptr())
    return int(buf.ctypes.data)


# ---------------------------------------------------------------------------
# the C ABI, name for name
# ---------------------------------------------------------------------------

def ppf_plan(n_channels: int, taps: int, coeffs) -> int:
    """coeffs: host float32 array of taps*n_channels values (copied)."""
    import numpy as np
    h = np.ascontiguousarray(coeffs, dtype=np.float32)
    if h.size != n_channels * taps:
        raise ValueError("coeffs must hold taps*n_channels values")
    return _handle(lib().ppf_plan(int(n_channels), int(taps), h.ctypes.data))


def ppf_plan_ex(n_channels: int, taps: int, coeffs, coeff_type: int, coeff_shift: int,
                in_type: int, fft_mode: int) -> int:
    import numpy as np
    dt = np.float32 if coeff_type == PPF_R32 else np.float16
    h = np.ascontiguousarray(coeffs, dtype=dt)
    return _handle(lib().ppf_plan_ex(int(n_channels), int(taps), h.ctypes.data, int(coeff_type),
                                     int(coeff_shift), int(in_type), int(fft_mode)))


def ppf_set_stream(plan: int, hip_stream) -> int:
    return _check(lib().ppf_set_stream(plan, _addr(hip_stream) if hip_stream else None))


def ppf_plan_set_path(plan: int, path: int) -> int:
    return _check(lib().ppf_plan_set_path(plan, int(path)))


def ppf_plan_query(plan: int, key: int) -> int:
    v = _c_ll(0)
    _check(lib().ppf_plan_query(plan, int(key), ctypes.byref(v)))
    return int(v.value)


def ppf_execute(plan: int, inp, out, nspectra: int) -> int:
    return _check(lib().ppf_execute(plan, _addr(inp), _addr(out), int(nspectra)))


def ppf_execute_noalloc(plan: int, inp, out, nspectra: int) -> int:
    return _check(lib().ppf_execute_noalloc(plan, _addr(inp), _addr(out), int(nspectra)))


PPF_NOALLOC_SCRATCH_BYTES = 32 << 20


def ppf_execute_host(plan: int, host_in, host_out, nspectra: int, chunk_spectra: int = 0) -> int:
    return _check(lib().ppf_execute_host(plan, _addr(host_in), _addr(host_out), int(nspectra), int(chunk_spectra)))


def ppf_execute_power(plan: int, inp, out_power, nspectra: int, k_int: int) -> int:
    return _check(lib().ppf_execute_power(plan, _addr(inp), _addr(out_power), int(nspectra), int(k_int)))


def ppf_destroy(plan: int) -> int:
    return _check(lib().ppf_destroy(plan))


def ppf_design_coeffs(n_channels: int, taps: int, window, beta: float = 0.0, user_window=None):
    """Prototype coefficients (host float32, taps*n_channels values) designed
    on the GPU. window: a ppf_window value or one of WINDOWS' names."""
    import numpy as np
    w = WINDOWS[window] if isinstance(window, str) else int(window)
    out = np.empty(max(0, int(n_channels) * int(taps)), dtype=np.float32)
    user = None if user_window is None else np.ascontiguousarray(user_window, dtype=np.float64)
    if user is not None and user.size != out.size:
        raise ValueError("user_window must hold taps*n_channels values")
    _check(lib().ppf_design_coeffs(int(n_channels), int(taps), w, float(beta), _addr(user),
                                   _addr(out) if out.size else None))
    return out


def ppf_kaiser_beta(atten_db: float) -> float:
    beta = ctypes.c_double()
    _check(lib().ppf_kaiser_beta(float(atten_db), ctypes.byref(beta)))
    return beta.value


def ppf_stream_create(plan: int) -> int:
    return _handle(lib().ppf_stream_create(plan))


def ppf_stream_push(stream: int, inp, out, nspectra: int, tag: int = 0) -> int:
    ch = ppf_chunk(_addr(inp), _addr(out), int(nspectra), int(tag))
    return _check(lib().ppf_stream_push(stream, ctypes.byref(ch)))


def ppf_stream_get_history(stream: int, host_dst) -> int:
    """host_dst: writable numpy array of (T-1)*N samples of the input type."""
    return _check(lib().ppf_stream_get_history(stream, host_dst.ctypes.data))


def ppf_stream_set_history(stream: int, host_src) -> int:
    import numpy as np
    src = np.ascontiguousarray(host_src)
    return _check(lib().ppf_stream_set_history(stream, src.ctypes.data))


def ppf_stream_position(stream: int) -> int:
    v = int(lib().ppf_stream_position(stream))
    if v < 0:
        _check(last_error()[0])
    return v


def ppf_stream_destroy(stream: int) -> int:
    return _check(lib().ppf_stream_destroy(stream))


def ppf_clock_ns() -> int:
    return int(lib().ppf_clock_ns())


def ppf_server_create(hbm_budget_bytes: int, max_inflight: int = 2) -> int:
    return _handle(lib().ppf_server_create(int(hbm_budget_bytes), int(max_inflight)))


def ppf_server_open_stream(server: int, plan: int) -> int:
    """A server stream handle (waits in line for budget if needed)."""
    h = _c_vp()
    _check(lib().ppf_server_open_stream(server, plan, ctypes.byref(h)))
    return int(h.value)


def ppf_server_open_stream_ex(server: int, plan: int, flags: int) -> int:
    h = _c_vp()
    _check(lib().ppf_server_open_stream_ex(server, plan, int(flags), ctypes.byref(h)))
    return int(h.value)


def ppf_server_stream_admitted(stream: int) -> bool:
    r = int(lib().ppf_server_stream_admitted(stream))
    if r < 0:
        _check(r)
    return r == 1


def ppf_server_submit(stream: int, inp, out, nspectra: int, tag: int = 0, arrival_ns: int = -1) -> int:
    ch = ppf_chunk(_addr(inp), _addr(out), int(nspectra), int(tag))
    return _check(lib().ppf_server_submit(stream, ctypes.byref(ch), int(arrival_ns)))


def ppf_server_poll(server: int, max_tags: int = 4096) -> list[int]:
    buf = (ctypes.c_ulonglong * max_tags)()
    n = int(lib().ppf_server_poll(server, buf, int(max_tags)))
    if n < 0:
        _check(n)
    return [int(buf[i]) for i in range(n)]


def ppf_server_drain(server: int, timeout_s: float = 60.0) -> int:
    return _check(lib().ppf_server_drain(server, float(timeout_s)))


def ppf_server_close_stream(stream: int) -> int:
    return _check(lib().ppf_server_close_stream(stream))


def ppf_server_stats(server: int) -> tuple[float, float, float]:
    """(p50 us, p99 us, input GB/s) of the chunks since the last reset."""
    p50, p99, gbps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().ppf_server_stats(server, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(gbps)))
    return float(p50.value), float(p99.value), float(gbps.value)


def ppf_server_get_stats(server: int) -> dict:
    st = ppf_server_stats_t()
    _check(lib().ppf_server_get_stats(server, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in ppf_server_stats_t._fields_}


def ppf_server_reset_stats(server: int) -> int:
    return _check(lib().ppf_server_reset_stats(server))


def ppf_server_destroy(server: int) -> int:
    return _check(lib().ppf_server_destroy(server))


# ---------------------------------------------------------------------------
# torch convenience (device memory and streams only)
# ---------------------------------------------------------------------------

class Plan:
    """Owning wrapper of a ppf_plan_t bound to torch's current stream.

    coeffs: float32 (any precision input) or float16 with ``coeff_shift``
    (stored values are h * 2^coeff_shift). in_type: PPF_C32, PPF_C16 or
    PPF_CI8; complex FP16/int8 inputs are (L, 2) tensors of (re, im).
    """

    def __init__(self, n_channels: int, taps: int, coeffs, path: int = PPF_PATH_AUTO,
                 in_type: int = PPF_C32, coeff_shift: int | None = None, fft_mode: int = PPF_FFT_F32):
        import numpy as np
        self.N, self.T = int(n_channels), int(taps)
        self.in_type = int(in_type)
        h = np.asarray(coeffs)
        if h.dtype == np.float16:
            self.handle = ppf_plan_ex(self.N, self.T, h, PPF_R16, int(coeff_shift or 0), self.in_type, fft_mode)
        elif self.in_type == PPF_C32 and fft_mode == PPF_FFT_F32:
            self.handle = ppf_plan(self.N, self.T, h)
        else:
            self.handle = ppf_plan_ex(self.N, self.T, h.astype(np.float32), PPF_R32, 0, self.in_type, fft_mode)
        if path != PPF_PATH_AUTO:
            ppf_plan_set_path(self.handle, path)

    @property
    def path(self) -> int:
        return ppf_plan_query(self.handle, PPF_Q_PATH)

    def execute(self, x, out=None, nspectra: int | None = None, stream=None):
        """x: complex64 CUDA tensor of (M+T-1)*N samples; returns (M, N) complex64."""
        import torch
        if nspectra is None:
            samples = x.numel() if x.is_complex() else x.shape[0]
            nspectra = samples // self.N - self.T + 1
        if out is None:
            out = torch.empty((nspectra, self.N), dtype=torch.complex64, device=x.device)
        st = torch.cuda.current_stream(x.device) if stream is None else stream
        ppf_set_stream(self.handle, st.cuda_stream)
        ppf_execute(self.handle, x, out, nspectra)
        return out

    def execute_power(self, x, k_int: int, out=None, nspectra: int | None = None, stream=None):
        """Detected power |X|^2 summed over k_int spectra: (M // k_int, N) float32."""
        import torch
        if nspectra is None:
            samples = x.numel() if x.is_complex() else x.shape[0]
            nspectra = samples // self.N - self.T + 1
        if out is None:
            out = torch.empty((nspectra // k_int, self.N), dtype=torch.float32, device=x.device)
        st = torch.cuda.current_stream(x.device) if stream is None else stream
        ppf_set_stream(self.handle, st.cuda_stream)
        ppf_execute_power(self.handle, x, out, nspectra, k_int)
        return out

    def execute_host(self, x, out, nspectra: int | None = None, chunk_spectra: int = 0, stream=None):
        """Single mode: x and out are host tensors (page-locked for full
        speed); the call is asynchronous on the plan's stream, which
        completes once every spectrum is in out."""
        import torch
        if nspectra is None:
            samples = x.numel() if x.is_complex() else x.shape[0]
            nspectra = samples // self.N - self.T + 1
        st = torch.cuda.current_stream() if stream is None else stream
        ppf_set_stream(self.handle, st.cuda_stream)
        ppf_execute_host(self.handle, x, out, nspectra, chunk_spectra)
        return out

    def close(self):
        if self.handle:
            ppf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass
