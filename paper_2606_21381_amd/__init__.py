"""MI355X-native OSOG renderer: SoA particles -> OPD canvas -> wave-optics image.

The compute path is the C-ABI library ``libosog.so`` (hand-written HIP for
gfx950); this package only marshals arguments to it.  Submodules load the
library on first use and raise if it is missing.
"""
__all__ = ["workloads"]
