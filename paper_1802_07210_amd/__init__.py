"""ELAS dense-stereo hot path on AMD Instinct MI355X (gfx950).

The compute lives in libelas_mi355x.so (HIP kernels + host mesh step behind
the C-ABI of include/elas.h); `elas` is its ctypes binding.
"""
from .elas import Elas, ElasError, Server, default_params, triangulate  # noqa: F401
