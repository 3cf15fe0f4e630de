"""MI355X-native GRMHD right-hand side and SSP-RK3 time update.

The numerical work runs in the HIP library ``libgrmhd.so`` (built for gfx950
by ``build.py``) behind the C ABI of ``include/grmhd.h``; this package only
marshals arguments (``_lib``) and holds device memory in torch tensors
(``grid.Grid``).  There is no CPU fallback: without the built library every
entry point raises.
"""
__all__ = ["Grid", "load_library"]


def load_library():
    from ._lib import lib
    return lib()


def __getattr__(name):
    if name == "Grid":
        from .grid import Grid
        return Grid
    raise AttributeError(name)
