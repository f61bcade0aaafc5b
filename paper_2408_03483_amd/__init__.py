"""MI355X (gfx950) tensor-train finite-volume solver for the 2-D shallow water equations.

The compute path is libttfv.so (hand-written HIP, built by paper_2408_03483_amd.build);
``paper_2408_03483_amd.ttfv`` is its Python binding.
"""
from . import ttfv  # noqa: F401
