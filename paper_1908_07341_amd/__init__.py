"""MI355X-native shaken dynamics (arXiv:1908.07341): HIP kernels behind a C ABI.

The package exposes the C ABI of include/shaken.h through a ctypes binding with
the same names; see binding.py.
"""
from .binding import *  # noqa: F401,F403
from .binding import ShakenError, lib, lib_path, new_lattice  # noqa: F401
