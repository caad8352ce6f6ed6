"""Vanka patches P_i: in the simplest case one patch holds every degree of
freedom of one mesh element (Sec. 4.3).  For Q2 that is 3^d nodes times n_c
components: n_p = 27 (2D momentum), 108 (3D momentum), 18 / 81 (ALE and
deformation, n_c = d).  R_i restricts a block vector to those dofs, ordered
node-major (element-local lexicographic node order, x fastest) then by
component."""
import numpy as np


def element_patches(cells) -> np.ndarray:
    """[ncells, 3^d] node indices of every element, elements lexicographic
    (x fastest), nodes lexicographic inside the element."""
    dim = len(cells)
    nn = [2 * c + 1 for c in cells]
    eidx = np.indices(cells[::-1]).reshape(dim, -1)[::-1]  # per axis element coordinate, x first
    loc = np.indices([3] * dim).reshape(dim, -1)[::-1]     # local node offsets, x fastest
    out = np.zeros((eidx.shape[1], loc.shape[1]), dtype=np.int64)
    stride = 1
    for a in range(dim):
        out += stride * (2 * eidx[a][:, None] + loc[a][None, :])
        stride *= nn[a]
    return out


def patch_dofs(cells, b: int) -> np.ndarray:
    """[ncells, 3^d * b] global dof indices of every element patch."""
    nodes = element_patches(cells)
    return (nodes[:, :, None] * b + np.arange(b)[None, None, :]).reshape(nodes.shape[0], -1)
