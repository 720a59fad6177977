"""MI355X-native VESIS hot path (arXiv 2208.05524): density sums, binary
level-set flips, energies, forces and adaptive-mobility steps in HIP for
gfx950 behind the C ABI of include/vesis.h."""
from ._lib import VesisError, load  # noqa: F401
from .vesis import Batch, Context, default_mobility  # noqa: F401

__all__ = ["Batch", "Context", "VesisError", "default_mobility", "load"]
