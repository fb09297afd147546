"""M1 radiative-transfer subcycle on MI355X (gfx950): HIP kernels behind a C
ABI (``include/rt.h``) and a ctypes binding of it (``paper_2404_17630_amd.rt``).

Zier et al. (2024), "Adapting AREPO-RT for Exascale Computing: GPU
Acceleration and Efficient Communication", Sections 2.2-2.3 and 4.1.
"""
from . import rt  # noqa: F401  (the binding loads the library lazily, on first call)

__all__ = ["rt"]
