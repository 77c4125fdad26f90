"""MI355X (gfx950) GateKeeper-GPU pre-alignment filter.

The filter itself runs in the HIP library libgk.so (C ABI in include/gk.h);
``paper_2103_14978_amd.gk`` is its Python binding.
"""
from . import gk  # noqa: F401
