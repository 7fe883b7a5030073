"""START on MI355X: photoionization rates of SPH particles from many
radiation sources with the tree acceleration of Hasegawa & Umemura (2010),
as hand-written HIP kernels for gfx950 behind the C-ABI of include/start.h.
"""
from .binding import (Box, Context, EXPORTS, FP32C, FP64, LUM_KERNEL_MEAN, LUM_KERNEL_VOLUME,  # noqa: F401
                      GasGrid, LibraryMissing, SourceTree, StartError, estimate_bytes, lib)

__all__ = ["Box", "Context", "GasGrid", "SourceTree", "StartError", "LibraryMissing", "estimate_bytes", "lib",
           "FP64", "FP32C", "LUM_KERNEL_MEAN", "LUM_KERNEL_VOLUME", "EXPORTS"]
