"""Grid transfers between nested Q2 meshes.  The paper names a geometric
multigrid on nested, interface-resolving meshes (Sec. 4.3 (II)) without
giving the transfer operators; the reading used here is the canonical one:
the prolongation P interpolates a coarse Q2 function at the fine nodes
(exact for every coarse Q2 function), applied component-wise, and the
restriction is its transpose R = P^T.

1D: a coarse cell with nodes at reference positions 0, 1/2, 1 is bisected; the
fine nodes sit at 0, 1/4, 1/2, 3/4, 1.  Coincident nodes take weight 1; the
quarter points take the quadratic Lagrange basis values there:
(3/8, 3/4, -1/8) at 1/4 and (-1/8, 3/4, 3/8) at 3/4.  On a graded mesh every
coarse cell is bisected, so the weights are the same in every cell."""
import numpy as np
import scipy.sparse as sp


def prolongation_1d(n_coarse_cells: int) -> sp.csr_matrix:
    """[(4 nc + 1) x (2 nc + 1)] interpolation matrix along one axis."""
    nc = n_coarse_cells
    nf_nodes, nc_nodes = 4 * nc + 1, 2 * nc + 1
    rows, cols, vals = [], [], []

    def quad(xi):  # quadratic Lagrange basis on nodes 0, 1/2, 1
        return [2 * (xi - 0.5) * (xi - 1.0), 4 * xi * (1.0 - xi), 2 * xi * (xi - 0.5)]

    for e in range(nc):
        for loc, xi in ((0, 0.0), (1, 0.25), (2, 0.5), (3, 0.75), (4, 1.0)):
            i = 4 * e + loc
            if loc == 4 and e < nc - 1:
                continue  # shared vertex, written by the next cell
            for c, w in enumerate(quad(xi)):
                if w != 0.0:
                    rows.append(i)
                    cols.append(2 * e + c)
                    vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf_nodes, nc_nodes))


def prolongation(coarse_cells, b: int) -> sp.csr_matrix:
    """P for block vectors (node-major, b components) from the coarse level with
    ``coarse_cells`` cells per axis to its uniform refinement."""
    dim = len(coarse_cells)
    P = prolongation_1d(coarse_cells[0])
    for a in range(1, dim):
        P = sp.kron(prolongation_1d(coarse_cells[a]), P)  # later axes vary slower
    return sp.kron(P, sp.identity(b)).tocsr()
