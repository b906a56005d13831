"""MI355X (gfx950) emission-spectrum forward model of Helios-r2 (arXiv:1910.01070).

The product is ``libhr2.so`` (C ABI in ``include/hr2.h``); ``hr2`` is its
ctypes binding.  Importing this package loads nothing; ``hr2.load()`` loads
the library and fails loudly when it has not been built.
"""
from . import hr2  # noqa: F401

__all__ = ["hr2"]
