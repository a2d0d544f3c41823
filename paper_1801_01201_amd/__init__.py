"""MI355X-native multi-implicit SDC (MISDC / MISDCQ / concurrent CISDCQ-nu)
for low-Mach reacting flow: HIP kernels for gfx950 behind a C ABI
(include/misdc.h, libmisdc.so) with a thin ctypes binding (``native``).

Submodules are imported lazily so that building does not need the library.
"""
__all__ = ["native", "flame", "build"]
