"""MI355X-native directional distance field hot path (arXiv 2306.16142).

``api`` holds the PyTorch binding of libddf.so (C ABI in include/ddf.h); the library is
loaded on first use and its absence is an error.
"""
from . import _lib  # noqa: F401
from . import api  # noqa: F401

__all__ = ["api"]
