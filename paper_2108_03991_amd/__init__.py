"""MI355X implementation of the SLIM system matrix-vector product and GMRES solve.

The work is done by libslim.so (HIP, gfx950); `slim` is its ctypes binding.
"""
from . import slim  # noqa: F401
