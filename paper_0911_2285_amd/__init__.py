"""MI355X (gfx950) incremental eigBiCG: C-ABI HIP library + thin Python binding.

``paper_0911_2285_amd.ebicg`` loads ``libebicg.so`` (built in-tree by
``paper_0911_2285_amd.build``) and exposes the calls of ``include/ebicg.h``.
"""
from . import ebicg  # noqa: F401  (loads nothing until a call needs the library)

__all__ = ["ebicg"]
