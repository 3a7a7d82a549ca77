"""MI355X-native QBX (Quadrature by Expansion) hot path: 2D Helmholtz S and D.

The computation lives in libqbx.so (hand-written HIP for gfx950, C ABI in
include/qbx.h); ``paper_1207_4461_amd.qbx`` is the PyTorch-facing binding.
"""
from . import inputs  # noqa: F401  (pure data generator, no GPU needed)

__all__ = ["inputs"]
