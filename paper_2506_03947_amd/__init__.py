"""alphacirc: block alpha-circulant preconditioned all-at-once diffusion solves on
AMD Instinct MI355X (gfx950), behind the C ABI of include/alphacirc.h.

Import the binding from ``paper_2506_03947_amd.api``; it loads
``libalphacirc.so`` built in-tree by ``python -m paper_2506_03947_amd.build``
and raises if the library is missing.
"""

from ._lib import LIB_PATH  # noqa: F401

__all__ = ["LIB_PATH"]
