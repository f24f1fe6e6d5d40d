"""FP64 CPU oracle of the polyphase filter bank: test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package; the product path never does.
"""
from .ppf_oracle import (as_complex128, dft, dft_matrix_columns, fir_presum,  # noqa: F401
                         n_spectra, ppf, ppf_power, ppf_stream, twiddles)
from . import design  # noqa: F401,E402  (prototype-filter design)
