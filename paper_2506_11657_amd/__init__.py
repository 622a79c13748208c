"""MI355X (gfx950) library for TEM forward modelling with a shared-pole
rational approximant of exp(-t M^-1 K) (HIP kernels behind the C ABI in
include/tem.h).  The Python side only marshals arguments: see ``tem``."""
from . import tem  # noqa: F401
