"""MI355X-native polarized subsurface BRDF of flat particulate layers (discrete ordinates).

The solver itself is the HIP library libvbrdf.so (C-ABI in include/vbrdf.h); ``binding`` wraps it
with ctypes and ``api.BRDFSolver`` adds torch-managed device buffers. Importing this package does
not load the library; the first call into ``binding`` does.
"""

__all__ = ["binding", "api", "build"]
