"""Independent FP64 CPU oracle of the entropic Fourier method.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
CPU-baseline leg of bench.py.  The product library never imports it and it
never imports the product library.
"""
from .efm import *  # noqa: F401,F403
from . import efm  # noqa: F401
