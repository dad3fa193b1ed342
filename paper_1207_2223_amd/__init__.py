"""MI355X-native (gfx950) Wilson-Dirac operator, conjugate-gradient solver and
two-flavour HMC pieces (arXiv:1207.2223), behind the C-ABI of include/wd.h.

The compute path is the HIP library libwd.so built from csrc/; wd.py is its
ctypes binding.
"""
from . import wd  # noqa: F401

__version__ = "0.1"
