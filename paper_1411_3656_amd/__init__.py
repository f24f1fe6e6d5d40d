"""MI355X-native polyphase filter bank (PPF).

The compute path lives in the HIP library ``libppf.so`` (built from
``csrc/``); :mod:`paper_1411_3656_amd.ppf` is its thin ctypes binding and
:mod:`paper_1411_3656_amd.signals` makes seeded synthetic inputs. Importing
the package does not load the library; the binding does, and raises if it
is missing.
"""
__all__ = ["signals"]
