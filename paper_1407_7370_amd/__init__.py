"""MI355X (gfx950) Lanczos short-time propagator for the 2D Dirac equation.

Beerwerth & Bauke, "Krylov subspace methods for the Dirac equation",
arXiv:1407.7370.  The computation runs in the HIP library
``libdirac_lanczos.so`` (C ABI in ``include/dirac_lanczos.h``); this package
holds its ctypes binding (``binding``), the seeded workload/packet generators
(``packets``) and the build script (``build``).
"""

__all__ = ["Propagator", "load_library", "packets"]


def __getattr__(name):
    if name in ("Propagator", "load_library"):
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
