"""MI355X-native sparse FFT (Hassanieh, Indyk, Katabi, Price, "Nearly Optimal
Sparse Fourier Transform"): HIP kernels for gfx950 behind a C ABI
(include/sfft.h), with a thin ctypes binding in ``sfft``."""
from . import sfft  # noqa: F401
from .sfft import Plan, load  # noqa: F401
