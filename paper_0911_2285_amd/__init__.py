"""MI355X (gfx950) incremental eigBiCG: C-ABI HIP library + thin Python binding.

``paper_0911_2285_amd.ebicg`` loads ``libebicg.so`` (built in-tree by
``paper_0911_2285_amd.build``) and exposes the calls of ``include/ebicg.h``;
``paper_0911_2285_amd.serve`` is the request loop that serves solves over
several resident operators through the library's sessions.
"""
from . import ebicg  # noqa: F401  (loads nothing until a call needs the library)
from . import serve  # noqa: F401

__all__ = ["ebicg", "serve"]
