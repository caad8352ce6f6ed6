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
    """A_i = R_i A R_i^T for element patches: [npatch, n_p, n_p] (dense, FP64)."""
    from .patches import element_patches
    nodes = element_patches(cells)
    if patches is not None:
        nodes = nodes[patches]
    return local_matrices_nodes(m, nodes)


def local_matrices_nodes(m, nodes) -> np.ndarray:
    """A_i = R_i A R_i^T for patches given by their node lists [npatch, nl].

    Looks every (row node, column node) block up in the block-CSR structure;
    a block absent from the structure is zero."""
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
    def build(m, cells, omega: float = 0.8, weighting: str = "plain", patches: str = "element",
              cell_solid=None):
        """patches="element": one VankaData of the one-element patches.
        patches="block": a list of VankaData, one per patch size (2 x 2 (x 2)
        element blocks, see patches.block_patch_groups), sharing one scale:
        the multiplicity counts the patches of every group."""
        n = (m.rowptr.shape[0] - 1) * m.b
        if patches == "element":
            groups = [(patch_dofs(cells, m.b), None)]
        elif patches == "block":
            from .patches import block_patch_groups
            groups = []
            for nodes, _ in block_patch_groups(cells, cell_solid):
                if nodes.shape[0]:
                    dofs = (nodes[:, :, None] * m.b + np.arange(m.b)).reshape(nodes.shape[0], -1)
                    groups.append((dofs, nodes))
        else:
            raise ValueError(patches)
        if weighting == "plain":
            scale = np.ones(n)
        elif weighting == "mult":
            mult = np.zeros(n)
            for dofs, _ in groups:
                mult += np.bincount(dofs.ravel(), minlength=n)
            scale = 1.0 / np.maximum(mult, 1.0)
        else:
            raise ValueError(weighting)
        if patches == "element":
            return VankaData(dofs=groups[0][0], inv=local_inverses(m, cells), scale=scale, omega=omega)
        return [VankaData(dofs=dofs, inv=np.linalg.inv(local_matrices_nodes(m, nodes)), scale=scale,
                          omega=omega) for dofs, nodes in groups]


def vanka_sweep(A, b: np.ndarray, x: np.ndarray, V, mask: np.ndarray,
                d: np.ndarray = None) -> np.ndarray:
    """One additive Vanka step; returns the new x.  ``V`` is a VankaData or a
    list of them (patch groups of different sizes, one shared scale).  ``d``
    may pass a residual b - A x that is already known.  Identity rows keep
    their value."""
    if d is None:
        d = b - A @ x
    d = d.copy()
    d[mask] = 0.0
    groups = V if isinstance(V, list) else [V]
    corr = np.zeros(x.shape[0])
    for g in groups:
        loc = np.matmul(g.inv, d[g.dofs][:, :, None])[:, :, 0]  # A_i^{-1} R_i d
        corr += np.bincount(g.dofs.ravel(), weights=loc.ravel(), minlength=x.shape[0])
    V0 = groups[0]
    xn = x + V0.omega * V0.scale * corr
    xn[mask] = x[mask]
    return xn
