"""MI355X (gfx950) library for the variational deterministic-particle scheme
and its POD reduction.  The compute path is libvds.so (HIP); this package is its
ctypes binding.  Importing it without the built library raises ImportError."""
from . import _vds
from ._vds import Batch, Context, Mlp, Rom, VDSError, make_problem

__all__ = ["Batch", "Context", "Mlp", "Rom", "VDSError", "make_problem", "_vds"]
