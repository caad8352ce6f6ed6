"""FP64 CPU oracle of the Newton-step linear solve (TEST INFRASTRUCTURE ONLY).

Plain, slow, obviously-correct NumPy/SciPy implementation of what the GPU
library computes: block-CSR products, the additive Vanka smoother (eq. vanka,
Sec. 4.3), the block ILU(0) smoother (Sec. 5.5's comparison smoother), Q2 grid transfers, the geometric multigrid V-cycle (Sec. 4.3 (II)),
flexible GMRES (Sec. 4.3 (I)), the condensed deformation update (Sec. 3.1,
eq. problem:2), the ALE extension solve (eq. problem:3), and the approximate
Newton loop around them (eq. newton: the condensed residual of eq. aletime:2,
its Jacobian by the complex step, Jacobian reuse and line search), and the
benchmark's time step and its drag / lift in residual form (Sec. 5).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library; both receive
their inputs from the separate input generator ``fsigen``.

Every function here is pinned by a ``-m "not gpu"`` test against something
other than itself (closed forms, library routines, invariants); see
``tests/test_oracle_pins.py``, ``tests/test_oracle_newton.py`` and
``tests/test_oracle_channel.py``.
"""
from .linalg import to_csr, matvec, masked_residual
from .patches import element_patches, patch_dofs
from .vanka import local_matrices, local_inverses, vanka_sweep, VankaData
from .transfer import prolongation_1d, prolongation
from .mg import Hierarchy, vcycle
from .ilu import BlockILU, ilu_sweep
from .fgmres import fgmres
from .deform import deform_update
from .step import newton_step_solve
from . import fsi

__all__ = ["to_csr", "matvec", "masked_residual", "element_patches", "patch_dofs",
           "local_matrices", "local_inverses", "vanka_sweep", "VankaData", "prolongation_1d",
           "prolongation", "Hierarchy", "vcycle", "BlockILU", "ilu_sweep", "fgmres", "deform_update",
           "newton_step_solve", "fsi"]
