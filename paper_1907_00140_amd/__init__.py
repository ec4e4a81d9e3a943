"""PLaNT construction of the Canonical Hub Labeling on MI355X (gfx950).

The work runs in libchl.so (hand-written HIP kernels behind the C-ABI of
include/chl.h); ``chl`` is its Python binding. Build the library with
``python -m paper_1907_00140_amd.build``.
"""
# the labeling build itself is chl.build: the name "build" in this package is
# the submodule that compiles the library
from .chl import ChlError, Labels, TorchAllocator, load  # noqa: F401

__all__ = ["ChlError", "Labels", "TorchAllocator", "load"]
