"""MI355X-native deep copy of pointer-linked struct trees and pointer-chain
leaf kernels (arXiv 1906.01128), behind the C ABI of include/dc.h.

The compute path is libdc.so (hand-written HIP for gfx950); `dc` is its
ctypes binding. Importing `dc` fails if the library has not been built.
"""
from . import dc  # noqa: F401
from .dc import (ChainCopy, Context, DcError, Graph, Plan, Schema, Server, Tree, load, version)  # noqa: F401
