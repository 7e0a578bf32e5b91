"""MI355X (gfx950) three-phonon linewidths: HIP kernels behind a C ABI
(libkaldo.so, declared in include/kaldo.h) and a thin ctypes binding."""
from . import kaldo  # noqa: F401
