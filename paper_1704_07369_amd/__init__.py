"""MI355X (gfx950) library for the entropic Fourier method collision operator.

The compute path is libefm.so (hand-written HIP); this package holds its
sources (csrc/), the build script and a ctypes binding with the C-ABI names.
Importing the package does not load the library; the first call does, and
fails loudly if it has not been built.
"""
from ._binding import *  # noqa: F401,F403
from . import _binding as binding  # noqa: F401
from .batch import Batch, Plan, pack, unpack  # noqa: F401
