"""Vanka patches P_i: in the simplest case one patch holds every degree of
freedom of one mesh element (Sec. 4.3).  For Q2 that is 3^d nodes times n_c
components: n_p = 27 (2D momentum), 108 (3D momentum), 18 / 81 (ALE and
deformation, n_c = d).  R_i restricts a block vector to those dofs, ordered
node-major (patch-local lexicographic node order, x fastest) then by
component.

Larger patches (Sec. 5.5.1, the patch-size study): a patch may instead hold
the 5^d nodes of a 2 x 2 (x 2) block of elements -- in 2D every such block
(n_p = 75 for the momentum system), in 3D only blocks of solid elements
(n_p = 500); elements outside such blocks keep their one-element patch."""
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


def _box_nodes(lo, width, cells) -> np.ndarray:
    """[n_box, (2*width+1)^d] node indices of the node boxes of `width`
    elements per axis starting at element coordinates lo ([n_box, d])."""
    dim = len(cells)
    nn = [2 * c + 1 for c in cells]
    loc = np.indices([2 * width + 1] * dim).reshape(dim, -1)[::-1]  # x fastest
    out = np.zeros((lo.shape[0], loc.shape[1]), dtype=np.int64)
    stride = 1
    for a in range(dim):
        out += stride * (2 * lo[:, a][:, None] + loc[a][None, :])
        stride *= nn[a]
    return out


def block_patch_groups(cells, cell_solid=None):
    """Patch groups with 2 x 2 (x 2) element blocks.  2D: every aligned block
    (element coordinates 2i, 2i+1 per axis); 3D: aligned blocks whose eight
    elements are all solid.  Returns [(nodes [n, 3^d], elements [n]),
    (nodes [m, 5^d], first elements [m])]: the one-element patches of the
    elements not covered by a block, then the block patches, each in
    lexicographic order of their (first) element."""
    dim = len(cells)
    ncell = int(np.prod(cells))
    ecoord = np.indices(cells[::-1]).reshape(dim, -1)[::-1].T  # [ncell, d], x first
    covered = np.zeros(ncell, dtype=bool)
    blocks = []
    nb = [c // 2 for c in cells]
    for bi in np.indices(nb[::-1]).reshape(dim, -1)[::-1].T:
        lo = 2 * bi
        members = []
        for off in np.indices([2] * dim).reshape(dim, -1)[::-1].T:
            e = lo + off
            idx = 0
            stride = 1
            for a in range(dim):
                idx += int(e[a]) * stride
                stride *= cells[a]
            members.append(idx)
        if dim == 3 and (cell_solid is None or not all(cell_solid[m] for m in members)):
            continue
        covered[members] = True
        blocks.append((members[0], lo))
    elem = np.nonzero(~covered)[0]
    groups = [(element_patches(cells)[elem], elem)]
    if blocks:
        firsts = np.array([b[0] for b in blocks], dtype=np.int64)
        lo = np.array([b[1] for b in blocks], dtype=np.int64)
        groups.append((_box_nodes(lo, 2, cells), firsts))
    return groups
