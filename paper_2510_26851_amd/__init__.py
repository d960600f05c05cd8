"""MI355X-native Friends-of-Friends hot path: hand-written HIP kernels for gfx950 behind the
C ABI of include/fof.h (libfof.so), with a thin Python front end.

Importing the package loads libfof.so and raises ImportError when it has not been built.
"""
from . import _lib

_lib.load()

from .fof import Plan, Stream, find_groups, trim  # noqa: E402

__all__ = ["Plan", "Stream", "find_groups", "trim"]
