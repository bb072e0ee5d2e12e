"""MI355X (gfx950) rank-2 Galerkin ROM of staggered LTI systems.

The computation lives in the HIP library ``librom.so`` (C ABI declared in
``include/rom.h``); this package only marshals arguments to it.
"""
from ._lib import RomError, load as load_library, LIB_PATH  # noqa: F401

__all__ = ["RomError", "load_library", "LIB_PATH", "Rom", "RomQoI", "run_grouped", "GroupPlan", "AffineFamily",
           "Fom", "pod"]


def __getattr__(name):
    # torch is imported lazily so the CPU-only ABI checks stay light
    if name in ("Rom", "RomQoI", "run_grouped", "GroupPlan", "AffineFamily", "Fom", "pod"):
        from . import rom
        return getattr(rom, name)
    raise AttributeError(name)
