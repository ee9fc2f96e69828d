"""MI355X (gfx950) implementation of the ViSta visibility-domain stacking hot path.

The product is the C-ABI library ``_build/libvista.so`` (declared in ``include/vista.h``);
``vista`` is its ctypes binding and ``build`` compiles it with hipcc.
"""
from . import vista  # noqa: F401

__all__ = ["vista"]
