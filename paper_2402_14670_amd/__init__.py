"""Looking Forward track following (arXiv 2402.14670) on AMD MI355X.

The hot path lives in the HIP library ``liblf_hip.so`` (sources in
``csrc/``, C ABI in ``include/lf.h``); ``lf`` is its ctypes binding.
"""
from . import lf  # noqa: F401
from .lf import Forward  # noqa: F401
