"""MI355X (gfx950) t-SVDM library: tube transforms, facewise truncated SVD and
the structured apply of the tensor-based matrix approximation, behind the C
ABI in include/tsvdm.h.  ``tsvdm`` is the ctypes binding; ``api`` holds the
PyTorch-facing helpers.  Nothing here computes on the CPU."""
from . import tsvdm  # noqa: F401
