"""MI355X-native batched range-only tracking environment (arXiv 2505.08222).

The compute path is the HIP library `libmilrauv.so` built from `csrc/`; the
Python modules here only marshal arguments (torch tensors supply device memory
and streams). Importing the package does not load the library; the first call
that needs it does, and it raises if the library is missing.
"""
from . import configs  # noqa: F401

__all__ = ["configs"]
