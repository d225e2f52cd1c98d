"""MI355X (gfx950) fractional Adams-Bashforth-Moulton history-sum library.

``libabm.so`` (HIP, built by ``build.py``) does the work behind the C ABI of
``include/abm.h``; ``abm`` is its ctypes binding and ``inputs`` the seeded
synthetic workloads.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "abm", "build"]
