"""MI355X (gfx950) solver for boundary integral equations with the generalized
Neumann kernel: the trapezoidal Nystrom systems of (I - N) mu = -M gamma (with
h = [M mu - (I - N) gamma]/2) and of (I + N* + J) mu = gamma, solved by
device-resident restarted GMRES over direct Cauchy sums and FFT circulant
blocks, all in the HIP library libgnk.so (C ABI in include/gnk.h).

The Python layer only marshals arguments; the library must be built
(``python -m paper_1308_5351_amd.build``).
"""
from .gnk import (FP64, MIXED, OP_FB, OP_FB_T, OP_FC, OP_FC_T, OP_GB, OP_GB_T, OP_LHAT, Context,
                  DeviceDomain, GnkError, LIB_PATH, load_library)

__all__ = ["Context", "DeviceDomain", "GnkError", "LIB_PATH", "load_library", "FP64", "MIXED",
           "OP_FB", "OP_FC", "OP_GB", "OP_FB_T", "OP_FC_T", "OP_GB_T", "OP_LHAT"]
