"""MI355X-native coupled EM/TM stress + IR-drop hot path (EMSpice 3 method).

The work runs in libem.so (HIP kernels for gfx950, C ABI in include/em.h);
``Batch`` is its ctypes binding and ``synth`` builds seeded synthetic grids.
"""
from ._binding import API, MLP, Batch, EmError, lib  # noqa: F401

__all__ = ["Batch", "MLP", "EmError", "lib", "API"]
