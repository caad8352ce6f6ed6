"""MI355X (gfx950) Newton-step linear solver for monolithic ALE fluid-structure
interaction: FGMRES + geometric multigrid with an additive Vanka smoother,
plus the condensed deformation update and the ALE extension solve.

The numerical work runs in the HIP library ``libfsimg.so`` (C ABI in
``include/fsimg.h``); ``fsimg`` is its ctypes binding and ``problems`` adapts
the seeded input generator's matrices to the library's level descriptors.
"""
from . import fsimg  # noqa: F401
