"""MicSA (microcanonical simulated annealing) for the 3D Edwards-Anderson
+-J spin glass on AMD MI355X: HIP kernels behind the C ABI of libmicsa.

The binding module ``micsa`` loads the in-tree libmicsa.so lazily; nothing
here imports torch or touches the GPU at import time.
"""
from . import micsa  # noqa: F401

__all__ = ["micsa"]
