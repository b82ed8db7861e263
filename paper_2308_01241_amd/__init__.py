"""MI355X partition simulator for the conductance-LIF network of
"Digital Twin Brain" (arXiv 2308.01241): Python binding of libdtb.so.

The binding only marshals arguments; every step runs in the library's HIP
kernels for gfx950.  Importing works without a GPU, but creating a handle
needs the compiled library and a GPU (no CPU fallback exists)."""
from ._lib import DtbError, load
from .net import Net, enkf_analysis, pack_bits, unpack_bits
from .surrogate import MLP, topk

__all__ = ["DtbError", "load", "Net", "MLP", "topk", "enkf_analysis", "pack_bits", "unpack_bits"]
