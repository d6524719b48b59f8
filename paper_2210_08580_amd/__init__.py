"""MI355X-native filtered fast direct solver for the 2D TE-EFIE / TE-MFIE.

The numerical work lives in libfds.so (HIP for gfx950, C ABI in include/fds.h);
`binding` marshals arguments to it and `workloads` generates seeded inputs.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "binding"]
