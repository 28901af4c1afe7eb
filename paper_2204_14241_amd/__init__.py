"""MI355X (gfx950) HIP implementation of the Hybrid Monte Carlo hot path for the O(3)
spin-fermion model of Lunts, Albergo and Lindsey (arXiv:2204.14241).

The product is the C-ABI shared library libhmc.so (include/hmc.h) built from csrc/;
`hmc` is its Python binding (argument marshalling only) and `autograd` wraps the
pseudofermion action as a torch.autograd.Function whose backward is the library's
hand-written gradient kernel.
"""
from ._lib import load, LIB_PATH  # noqa: F401

__all__ = ["load", "LIB_PATH"]
