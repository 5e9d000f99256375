"""MI355X-native DeepABM-COVID daily transmission-and-progression step.

The compute path is libabm.so (hand-written HIP for gfx950 behind the C ABI in
include/abm.h); this package is its thin Python binding.  Importing the package does
not load the library; the first Simulator (or ``_lib.lib()``) does, and fails loudly
if it was not built.
"""
__all__ = ["Simulator", "philox"]


def __getattr__(name):
    if name in ("Simulator", "philox"):
        from . import sim
        return getattr(sim, name)
    raise AttributeError(name)
