"""MI355X-native tensor-network circuit contraction executor.

The compute path lives in the HIP shared library ``libtcx.so`` (sources in
``csrc/``, ABI in ``include/tcx.h``); this package only marshals arguments.
"""
from . import _lib  # noqa: F401
