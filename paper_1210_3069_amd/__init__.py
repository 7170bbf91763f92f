"""MI355X-native SHT+MG lens-plane solver and multiple-plane ray tracer
after Becker (2013), CALCLENS (arXiv:1210.3069).

The computation lives in libcalclens_mi.so (HIP for gfx950, C ABI declared
in include/calclens_mi.h); `clm` is its thin ctypes binding and `inputs`
the seeded synthetic-input recipe."""
from . import inputs  # noqa: F401
