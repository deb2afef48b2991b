"""MI355X-native multi-reference alignment (MRA) hot path.

The compute lives in ``libmra.so`` (HIP kernels for gfx950 behind a C ABI
declared in ``include/mra.h``); ``mra`` is a thin ctypes binding over it.
Submodules are imported lazily so that ``synth`` (input generation) can be
used without loading the native library.
"""

__all__ = ["mra", "synth", "serve"]
