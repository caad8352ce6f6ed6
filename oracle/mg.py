"""Geometric multigrid V-cycle used as the preconditioner of the outer Krylov
iteration (Sec. 4.3 (II)).  Every level has its own re-discretised matrix
(the paper assembles the matrices on all multigrid levels); the smoother is
the additive Vanka iteration (or block ILU(0), oracle.ilu); the coarsest level is solved exactly by a dense
LU with partial pivoting (the paper does not name its coarse solver).

V-cycle(l, r), returning an approximation of A_l^{-1} r:
    l coarsest:  x = LU solve of A_l x = r
    otherwise:   x = 0
                 nu_pre Vanka steps on A_l x = r
                 x += P V-cycle(l+1, R (r - A_l x))
                 nu_post Vanka steps on A_l x = r
Identity (Dirichlet) dofs of the correction are kept at zero on every level
(after the restriction, after the prolongation, and on the result)."""
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from .linalg import to_csr
from .transfer import prolongation
from .vanka import VankaData, vanka_sweep
from .ilu import BlockILU, ilu_sweep


@dataclass
class MGLevel:
    A: object
    mask: np.ndarray
    cells: tuple
    vanka: VankaData = None
    ilu: BlockILU = None
    P: object = None      # prolongation from the next coarser level
    lu: tuple = None      # coarsest level only


class Hierarchy:
    def __init__(self, mats, cells_per_level, omega=0.8, nu_pre=2, nu_post=2, weighting="plain",
                 patches="element", cell_solid=None, smoother="vanka", omega_ilu=1.0):
        """mats: per-level block-CSR systems (finest first), cells_per_level:
        cells per axis on each level; patches "element" or "block" (2 x 2 (x 2)
        element blocks, in 3D solid only: cell_solid per level); smoother
        "vanka" or "ilu" (block ILU(0), damping omega_ilu)."""
        self.nu_pre, self.nu_post = nu_pre, nu_post
        self.smoother, self.omega_ilu = smoother, omega_ilu
        self.levels = []
        L = len(mats)
        for l, (m, cells) in enumerate(zip(mats, cells_per_level)):
            lev = MGLevel(A=to_csr(m), mask=m.dirichlet.astype(bool), cells=tuple(cells))
            if l < L - 1:
                if smoother == "ilu":
                    lev.ilu = BlockILU(m)
                else:
                    lev.vanka = VankaData.build(m, cells, omega=omega, weighting=weighting,
                                                patches=patches,
                                                cell_solid=None if cell_solid is None else cell_solid[l])
                lev.P = prolongation(tuple(cells_per_level[l + 1]), m.b)
            else:
                lev.lu = sla.lu_factor(lev.A.toarray())
            self.levels.append(lev)

    def coarse_solve(self, r):
        lev = self.levels[-1]
        x = sla.lu_solve(lev.lu, r)
        x[lev.mask] = 0.0
        return x


def vcycle(H: Hierarchy, r: np.ndarray, l: int = 0) -> np.ndarray:
    lev = H.levels[l]
    r = r.copy()
    r[lev.mask] = 0.0
    if l == len(H.levels) - 1:
        return H.coarse_solve(r)
    x = np.zeros_like(r)
    for s in range(H.nu_pre):
        x = smooth(H, lev, r, x, d=r if s == 0 else None)
    d = r - lev.A @ x
    d[lev.mask] = 0.0
    rc = lev.P.T @ d
    xc = vcycle(H, rc, l + 1)
    x = x + lev.P @ xc
    x[lev.mask] = 0.0
    for _ in range(H.nu_post):
        x = smooth(H, lev, r, x)
    return x


def smooth(H: Hierarchy, lev: MGLevel, r: np.ndarray, x: np.ndarray, d: np.ndarray = None):
    """One step of the hierarchy's smoother on A_l x = r."""
    if H.smoother == "ilu":
        return ilu_sweep(lev.A, r, x, lev.ilu, lev.mask, omega=H.omega_ilu, d=d)
    return vanka_sweep(lev.A, r, x, lev.vanka, lev.mask, d=d)
