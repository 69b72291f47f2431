"""MI355X (gfx950) Wilson-Dirac operator and Krylov solvers.

The compute path is the HIP library libwilson.so (C ABI in include/wilson.h), reached
through the ctypes binding in `_lib` (imported lazily, so that `inputs` and `counts`
are usable without a GPU).
"""
__all__ = ["inputs", "counts"]
