"""MI355X-native lattice Boltzmann stream-collide on structured blocks.

The compute path lives in the HIP library ``libwlb.so`` (sources under
``csrc/``, C ABI declared in ``include/wlb.h``); ``wlb`` is its ctypes
binding.  Importing this package does not load the library; ``wlb`` does,
and raises if it has not been built.
"""
__all__ = ["wlb", "inputs"]
