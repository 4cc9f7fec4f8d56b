"""MI355X (gfx950) implementation of FGFRFT's online operator update
(arXiv 2602.20870): HIP kernels behind a C ABI (include/fgfrft.h), with a
thin PyTorch binding.  Importing the package does not load the library;
the first call does, and fails loudly if it has not been built.
"""
from ._lib import FGFRFTError, LIB_PATH, lib  # noqa: F401


def __getattr__(name):
    if name in ("Plan", "apply_operator", "gfrft_exact"):
        from . import ops
        return getattr(ops, name)
    if name == "FGFRFTFunction":
        from .autograd import FGFRFTFunction
        return FGFRFTFunction
    raise AttributeError(name)
