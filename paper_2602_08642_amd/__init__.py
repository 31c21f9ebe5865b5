"""MI355X (gfx950) implementation of the sub-1-spp adaptive-sampling hot path.

The computation lives in libaps.so (HIP kernels behind a C ABI, include/aps.h); this package
loads it with ctypes (`_lib`), wraps it for torch device tensors (`ops`), and sequences a
frame or a training step (`pipeline`).  Importing never builds; use
`python -m paper_2602_08642_amd.build`.
"""
from . import _lib  # noqa: F401

__version__ = "1.0.0"
