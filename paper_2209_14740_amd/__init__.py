"""MI355X-native stochastic-Galerkin Helmholtz solver (HIP for gfx950).

The compute path lives in ``libsg.so`` (built by ``paper_2209_14740_amd.build``);
``paper_2209_14740_amd.sg`` is its ctypes binding.  Importing this package loads
nothing native; ``sg.lib()`` loads the library and raises if it was not built.
"""
__all__ = ["sg", "build"]
