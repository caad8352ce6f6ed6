"""Additive (Jacobi) Vanka smoother, eq. (vanka) of Sec. 4.3:

    d = b - A x
    x <- x + omega * sum_i R_i^T A_i^{-1} R_i d,      A_i = R_i A R_i^T,

with the local matrices inverted exactly (the paper uses a dense LU; here
LAPACK through numpy.linalg.inv, i.e. LU with partial pivoting).

Reading of the sum over overlapping element patches (the paper prints a plain
sum with omega ~ 0.8): ``weighting="plain"`` adds every patch correction as
printed; ``weighting="mult"`` divides the summed correction at each dof by the
number of patches that contain it (an averaging of the overlapping local
solutions).  Which one the solver uses is fixed by the caller.
"""
from dataclasses import dataclass

import numpy as np

from .patches import patch_dofs


def local_matrices(m, cells, patches=None) -> np.ndarray:
    """A_i = R_i A R_i^T for element patches: [npatch, n_p, n_p] (dense, FP64).

    Looks every (row node, column node) block up in the block-CSR structure;
    a block absent from the structure is zero."""
    from .patches import element_patches
    nodes = element_patches(cells)
    if patches is not None:
        nodes = nodes[patches]
    b = m.b
    n = m.rowptr.shape[0] - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(m.rowptr))
    keys = rows * n + m.colind.astype(np.int64)
    nl = nodes.shape[1]
    out = np.zeros((nodes.shape[0], nl * b, nl * b))
    vals = np.asarray(m.vals, dtype=np.float64)
    for a in range(nl):
        k = nodes[:, a][:, None] * n + nodes  # [npatch, nl] keys of row node a
        pos = np.searchsorted(keys, k)
        pos = np.minimum(pos, keys.shape[0] - 1)
        found = keys[pos] == k
        blk = np.where(found[:, :, None, None], vals[pos], 0.0)  # [npatch, nl, b, b]
        # rows a*b..a*b+b-1, columns node-major then component
        out[:, a * b:(a + 1) * b, :] = blk.transpose(0, 2, 1, 3).reshape(nodes.shape[0], b, nl * b)
    return out


def local_inverses(m, cells, chunk: int = 4096) -> np.ndarray:
    """A_i^{-1} for every element patch: [npatch, n_p, n_p]."""
    ncell = int(np.prod(cells))
    b = m.b
    npp = 3 ** len(cells) * b
    out = np.empty((ncell, npp, npp))
    for s in range(0, ncell, chunk):
        idx = np.arange(s, min(ncell, s + chunk))
        out[idx] = np.linalg.inv(local_matrices(m, cells, idx))
    return out


@dataclass
class VankaData:
    dofs: np.ndarray      # [npatch, n_p]
    inv: np.ndarray       # [npatch, n_p, n_p]
    scale: np.ndarray     # [n] per-dof factor applied to the summed correction
    omega: float

    @staticmethod
    def build(m, cells, omega: float = 0.8, weighting: str = "plain") -> "VankaData":
        dofs = patch_dofs(cells, m.b)
        n = (m.rowptr.shape[0] - 1) * m.b
        if weighting == "plain":
            scale = np.ones(n)
        elif weighting == "mult":
            mult = np.bincount(dofs.ravel(), minlength=n).astype(np.float64)
            scale = 1.0 / np.maximum(mult, 1.0)
        else:
            raise ValueError(weighting)
        return VankaData(dofs=dofs, inv=local_inverses(m, cells), scale=scale, omega=omega)


def vanka_sweep(A, b: np.ndarray, x: np.ndarray, V: VankaData, mask: np.ndarray,
                d: np.ndarray = None) -> np.ndarray:
    """One additive Vanka step; returns the new x.  ``d`` may pass a residual
    b - A x that is already known.  Identity rows keep their value."""
    if d is None:
        d = b - A @ x
    d = d.copy()
    d[mask] = 0.0
    loc = np.matmul(V.inv, d[V.dofs][:, :, None])[:, :, 0]  # A_i^{-1} R_i d
    corr = np.bincount(V.dofs.ravel(), weights=loc.ravel(), minlength=x.shape[0])
    xn = x + V.omega * V.scale * corr
    xn[mask] = x[mask]
    return xn
