"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, a library routine solving the same problem, or an invariant, chosen so
that a dropped term, a wrong index or a transposed operand fails."""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from fsigen import make_problem
from fsigen.problem import SOLID_2D, SOLID_3D
from oracle import (Hierarchy, VankaData, deform_update, element_patches, fgmres,
                    local_matrices, patch_dofs, prolongation, prolongation_1d, to_csr,
                    vanka_sweep, vcycle)
from oracle.step import newton_step_solve, solve_system

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ transfers
def test_prolongation_1d_matches_closed_form_weights():
    tab = np.loadtxt(os.path.join(GOLDEN, "q2_prolongation_1d.txt"))
    P = prolongation_1d(1).toarray()
    np.testing.assert_array_equal(P, tab[:, 1:])


@pytest.mark.parametrize("dim", [2, 3])
def test_prolongation_reproduces_q2_functions(dim):
    """P I_H q = I_h q for every coarse Q2 function q (graded coarse mesh)."""
    from fsigen.problem import graded_axis, _nodes_from_verts
    rng = np.random.default_rng(0)
    verts = [graded_axis(4, 0.3, 0.7, 2) for _ in range(dim)]
    coarse = [_nodes_from_verts(v[1]) for v in verts]
    fine = [_nodes_from_verts(v[0]) for v in verts]
    b = 2
    P = prolongation(tuple([4] * dim), b)
    # the tensor Q2 space on a graded mesh is piecewise; a global tensor quadratic is in it
    coef = rng.standard_normal((b, dim, 3))

    def ev(coords):
        X = np.meshgrid(*coords[::-1], indexing="ij")[::-1]
        out = []
        for c in range(b):
            val = np.ones_like(X[0])
            for a in range(dim):
                val = val * (coef[c, a, 0] + coef[c, a, 1] * X[a] + coef[c, a, 2] * X[a] ** 2)
            out.append(val.ravel())
        return np.stack(out, axis=1).ravel()
    np.testing.assert_allclose(P @ ev(coarse), ev(fine), rtol=0, atol=1e-13)
    # restriction is the transpose
    R = P.T
    y = rng.standard_normal(P.shape[0])
    z = rng.standard_normal(P.shape[1])
    assert abs(y @ (P @ z) - z @ (R @ y)) < 1e-12


# ---------------------------------------------------------------- local matrices
def test_local_matrices_match_dense_submatrix(prob_t2):
    m = prob_t2.levels[0].systems["mom"]
    cells = prob_t2.levels[0].cells
    A = to_csr(m).toarray()
    dofs = patch_dofs(cells, m.b)
    loc = local_matrices(m, cells)
    for i in (0, 5, 37, len(dofs) - 1):
        np.testing.assert_array_equal(loc[i], A[np.ix_(dofs[i], dofs[i])])
    # a sparse-pattern (compressed) system: missing blocks are zero
    ma = prob_t2.levels[0].systems["ale"]
    Aa = to_csr(ma).toarray()
    da = patch_dofs(cells, ma.b)
    la = local_matrices(ma, cells)
    for i in range(len(da)):
        np.testing.assert_array_equal(la[i], Aa[np.ix_(da[i], da[i])])


def test_element_patches_nodes():
    # 2 x 1 cells in 2D: 5 x 3 nodes
    p = element_patches((2, 1))
    np.testing.assert_array_equal(p[0], [0, 1, 2, 5, 6, 7, 10, 11, 12])
    np.testing.assert_array_equal(p[1], [2, 3, 4, 7, 8, 9, 12, 13, 14])


# ---------------------------------------------------------------------- Vanka
def _system(prob, name="mom"):
    m = prob.levels[0].systems[name]
    return m, to_csr(m), m.dirichlet.astype(bool), prob.levels[0].cells


def test_single_patch_step_is_exact_local_solve(prob_t3):
    """One patch, omega = 1: after the update the patch residual vanishes."""
    m, A, mask, cells = _system(prob_t3)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(A.shape[0])
    b[mask] = 0.0
    x = rng.standard_normal(A.shape[0])
    x[mask] = 0.0
    full = VankaData.build(m, cells, omega=1.0, weighting="plain")
    for i in (0, 77, 200):
        V1 = VankaData(dofs=full.dofs[i:i + 1], inv=full.inv[i:i + 1], scale=np.ones_like(b), omega=1.0)
        xn = vanka_sweep(A, b, x, V1, mask)
        r = b - A @ xn
        free = full.dofs[i][~mask[full.dofs[i]]]
        assert np.abs(r[free]).max() < 1e-10 * np.abs(b).max()
        # dofs outside the patch are untouched
        out = np.setdiff1d(np.arange(b.shape[0]), full.dofs[i])
        np.testing.assert_array_equal(xn[out], x[out])


@pytest.mark.parametrize("solid", [False, True])
def test_one_element_mesh_vanka_is_direct_solve(solid):
    """On a one-element mesh the only patch is the whole system: one Vanka step
    with omega = 1 is numpy.linalg.solve(A, b)."""
    from fsigen.problem import make_level, PARAMS_DEFAULT
    rng = np.random.default_rng(4)
    coords = [np.array([0.0, 0.5, 1.0])] * 2
    st = {k: rng.standard_normal((9, 2)) * 0.01 for k in ("v_old", "u_old", "v_cur")}
    st["u_cur"] = st["u_old"] + 0.005 * (st["v_cur"] + st["v_old"])
    box = ((0.2, 0.2), (0.8, 0.8)) if solid else ((0.6, 0.6), (0.7, 0.7))
    lev = make_level(2, (1, 1), coords, box, st, PARAMS_DEFAULT)
    assert lev.cell_solid[0] == int(solid)
    for name in ("mom", "ale", "mass"):
        m = lev.systems[name]
        A = to_csr(m)
        mask = m.dirichlet.astype(bool)
        b = rng.standard_normal(A.shape[0])
        b[mask] = 0.0
        for wt in ("plain", "mult"):
            V = VankaData.build(m, lev.cells, omega=1.0, weighting=wt)
            x = vanka_sweep(A, b, np.zeros_like(b), V, mask)
            ref = np.linalg.solve(A.toarray(), b)
            np.testing.assert_allclose(x, ref, rtol=0, atol=1e-12 * max(np.abs(ref).max(), 1e-300))


def test_vanka_additive_order_independent_and_weights(prob_t3):
    m, A, mask, cells = _system(prob_t3)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(A.shape[0])
    b[mask] = 0.0
    V = VankaData.build(m, cells, omega=0.8, weighting="mult")
    x1 = vanka_sweep(A, b, np.zeros_like(b), V, mask)
    perm = rng.permutation(V.dofs.shape[0])
    Vp = VankaData(dofs=V.dofs[perm], inv=V.inv[perm], scale=V.scale, omega=V.omega)
    x2 = vanka_sweep(A, b, np.zeros_like(b), Vp, mask)
    np.testing.assert_allclose(x2, x1, rtol=0, atol=1e-13 * np.abs(x1).max())
    # multiplicities: a 3D interior vertex is in 8 element patches, an edge midpoint
    # in 4, a face midpoint in 2, a cell centre in 1
    nn = [2 * c + 1 for c in cells]

    def node(i, j, k):
        return i + nn[0] * (j + nn[1] * k)
    for (ijk, mult) in (((2, 2, 2), 8), ((1, 2, 2), 4), ((1, 1, 2), 2), ((1, 1, 1), 1)):
        assert V.scale[node(*ijk) * m.b] == pytest.approx(1.0 / mult)


# ---------------------------------------------------------------- multigrid
@pytest.mark.parametrize("dim,n", [(2, 8), (2, 16), (3, 6)])
def test_two_level_mg_fgmres_matches_superlu(dim, n):
    """Two levels, exact coarse solve, FGMRES to 1e-10 -> SuperLU's answer to
    1e-10 (SuperLU's own relative residual on these saddle-point systems is
    ~1e-11, so a tighter solver tolerance is not attainable in FP64)."""
    box = SOLID_2D if dim == 2 else SOLID_3D
    P = make_problem(dim, n, 2, box, seed=1)
    cells = [l.cells for l in P.levels]
    for name in ("mom", "ale"):
        mats = P.system(name)
        A = to_csr(mats[0])
        mask = mats[0].dirichlet.astype(bool)
        b = P.rhs[name]
        x0 = np.zeros_like(b)
        if name == "ale":  # interface / solid data carried in by x0
            x0[mask] = np.random.default_rng(5).standard_normal(int(mask.sum())) * 1e-2
        x, info, _ = solve_system(mats, cells, b, x0=x0, rtol=1e-10, weighting="mult")
        assert info["converged"]
        bb = b.copy()
        bb[mask] = x0[mask]
        xref = spla.splu(A.tocsc()).solve(bb)
        assert np.linalg.norm(x - xref) <= 1e-10 * np.linalg.norm(xref)


def test_vcycle_coarse_level_is_exact_and_galerkin_projection(prob_t2):
    """On the coarsest level the V-cycle is an exact solve; with the coarse
    matrix replaced by R A P the coarse correction I - P Ac^-1 R A is a
    projection (idempotent)."""
    mats = prob_t2.system("mom")
    cells = [l.cells for l in prob_t2.levels]
    H = Hierarchy(mats, cells, weighting="mult")
    Ac = H.levels[-1].A
    maskc = H.levels[-1].mask
    r = np.random.default_rng(0).standard_normal(Ac.shape[0])
    r[maskc] = 0.0
    np.testing.assert_allclose(Ac @ vcycle(H, r, l=1), r, atol=1e-10 * np.abs(r).max())
    # Galerkin projection invariant on the transfer operators
    A = H.levels[0].A.toarray()
    Pm = H.levels[0].P.toarray()
    mask = H.levels[0].mask
    Pm[mask, :] = 0.0
    Pm[:, maskc] = 0.0
    Ag = Pm.T @ A @ Pm
    Ag[np.ix_(maskc, maskc)] = np.eye(int(maskc.sum()))
    C = np.eye(A.shape[0]) - Pm @ np.linalg.solve(Ag, Pm.T @ A)
    np.testing.assert_allclose(C @ C, C, atol=1e-8 * np.abs(C).max())


# ------------------------------------------------------------------- FGMRES
def test_fgmres_exact_preconditioner_one_iteration(prob_t2):
    m, A, mask, cells = _system(prob_t2)
    lu = spla.splu(A.tocsc())
    b = prob_t2.rhs["mom"]
    x, info = fgmres(A, b, np.zeros_like(b), lambda v: lu.solve(v), mask, rtol=1e-10)
    assert info["iters"] == 1 and info["converged"]


def test_fgmres_unpreconditioned_matches_dense_and_orthogonal():
    rng = np.random.default_rng(7)
    n = 60
    A = sp.csr_matrix(np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3)
    b = rng.standard_normal(n)
    mask = np.zeros(n, dtype=bool)
    x, info = fgmres(A, b, np.zeros(n), lambda v: v.copy(), mask, rtol=1e-12, restart=n)
    np.testing.assert_allclose(x, np.linalg.solve(A.toarray(), b), rtol=1e-10, atol=1e-12)
    # Arnoldi basis orthonormal while the residual is far above rounding level
    # (MGS loses orthogonality in proportion to eps * kappa * ||r0|| / ||r_k||)
    _, info_b = fgmres(A, b, np.zeros(n), lambda v: v.copy(), mask, rtol=1e-3, restart=n,
                       return_basis=True)
    V = info_b["V"]
    assert V.shape[0] > 5
    assert np.abs(V @ V.T - np.eye(V.shape[0])).max() < 1e-12
    h = np.array(info["res_hist"])
    assert np.all(np.diff(h) <= 1e-14 * h[0])  # GMRES residuals never increase
    # restarted form still converges
    x2, info2 = fgmres(A, b, np.zeros(n), lambda v: v.copy(), mask, rtol=1e-12, restart=5,
                       maxiter=400)
    assert info2["converged"] and info2["restarts"] > 1


# -------------------------------------------------------- mesh independence
def test_mg_contraction_mesh_independent():
    """FGMRES-MG iteration counts to 1e-8 on 2, 3, 4 levels over a fixed coarse
    mesh grow by at most 3 per level (the paper reports counts that rise only
    slightly under refinement, Sec. 5.5.2)."""
    its = []
    for n, nl in ((16, 2), (32, 3), (64, 4)):
        P = make_problem(2, n, nl, SOLID_2D, seed=0)
        cells = [l.cells for l in P.levels]
        _, info, _ = solve_system(P.system("mom"), cells, P.rhs["mom"], rtol=1e-8, weighting="mult")
        assert info["converged"]
        its.append(info["iters"])
    assert its[-1] <= 25
    assert all(its[i + 1] - its[i] <= 3 for i in range(len(its) - 1))


# ---------------------------------------------------------------- deformation
def test_condensation_identity_and_mass_solve(prob_t3):
    """u_n = u_{n-1} + k/2 (v_n + v_{n-1}) for Crank-Nicolson (Sec. 3.1), and the
    deformation system (eq. problem:2) solved with the MG machinery gives the
    same increment as the vector addition."""
    P = prob_t3
    k, th = P.params["k"], P.params["theta"]
    assert th == 0.5
    lev = P.levels[0]
    mask = lev.node_solid.astype(bool)
    un = deform_update(mask, k, th, P.v_cur, u_old=P.u_old, v_old=P.v_old)
    ref = P.u_old + 0.5 * k * (P.v_cur + P.v_old)
    np.testing.assert_allclose(un[mask], ref[mask], rtol=1e-14, atol=1e-17)
    assert np.all(un[~mask] == 0.0)
    out = newton_step_solve(P, rtol=1e-11, mass_solve=True, weighting="mult")
    assert out["info_mom"]["converged"] and out["info_ale"]["converged"]
    dv = out["dv"].reshape(lev.nnodes, 4)[:, 1:]
    du_add = deform_update(mask, k, th, dv)
    np.testing.assert_allclose(out["du_mass"].reshape(-1, 3)[mask], du_add[mask], rtol=0,
                               atol=1e-10 * np.abs(du_add).max())
    # the ALE solution keeps the interface / solid increments and solves the fluid rows
    du = out["du"].reshape(-1, 3)
    np.testing.assert_array_equal(du[mask], du_add[mask])
    Aa = to_csr(lev.systems["ale"])
    amask = lev.systems["ale"].dirichlet.astype(bool)
    r = P.rhs["ale"] - Aa @ out["du"]
    r[amask] = 0.0
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(
        np.where(amask, 0.0, P.rhs["ale"] - Aa @ out["lift"]))


def test_vanka_sum_reading_plain_diverges_averaged_contracts(prob_t2):
    """Reading of the overlapping sum in eq. (vanka): as a stationary
    multigrid iteration x += Vcycle(b - A x), the printed plain sum with
    omega = 0.8 diverges on element patches, the multiplicity-averaged sum
    contracts."""
    mats = prob_t2.system("mom")
    cells = [lv.cells for lv in prob_t2.levels]
    b = prob_t2.rhs["mom"]
    rates = {}
    for wt in ("plain", "mult"):
        H = Hierarchy(mats, cells, omega=0.8, weighting=wt)
        A, mask = H.levels[0].A, H.levels[0].mask
        x = np.zeros_like(b)
        for _ in range(8):
            r = b - A @ x
            r[mask] = 0.0
            x = x + vcycle(H, r)
        r = b - A @ x
        r[mask] = 0.0
        rates[wt] = (np.linalg.norm(r) / np.linalg.norm(b)) ** (1 / 8)
    assert rates["plain"] > 1.0
    assert rates["mult"] < 0.6


# ------------------------------------------------------------ block patches
def test_block_patch_groups_partition_and_shapes():
    """2 x 2 (x 2) element blocks (Sec. 5.5.1): in 2D every aligned block, in
    3D only all-solid blocks; the patches of both groups cover every element
    exactly once and a block holds the 5^d nodes of its node box."""
    from oracle.patches import block_patch_groups
    cells2 = (4, 6)
    g = block_patch_groups(cells2)
    assert g[0][0].shape[0] == 0 and g[1][0].shape == (6, 25)
    nn = [2 * c + 1 for c in cells2]
    allnodes = np.unique(g[1][0])
    assert allnodes.size == nn[0] * nn[1]
    # odd cell counts leave a strip of one-element patches
    g = block_patch_groups((5, 4))
    assert g[1][0].shape[0] == 4 and g[0][0].shape[0] == 4
    # 3D: solid cells (x 2..5, y 4..5, z 4..5 of 8^3) give two blocks
    cells3 = (8, 8, 8)
    sol = np.zeros(512, dtype=np.uint8)
    for k in range(4, 6):
        for j in range(4, 6):
            for i in range(2, 6):
                sol[i + 8 * (j + 8 * k)] = 1
    g = block_patch_groups(cells3, sol)
    assert g[1][0].shape == (2, 125)
    assert g[0][0].shape[0] == 512 - 16
    covered = np.zeros(512, int)
    covered[g[0][1]] += 1
    for f in g[1][1]:
        i, j, k = f % 8, (f // 8) % 8, f // 64
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    covered[(i + dx) + 8 * ((j + dy) + 8 * (k + dz))] += 1
    assert np.all(covered == 1)


def test_block_patch_on_a_two_by_two_mesh_is_direct_solve():
    """A 2 x 2 element mesh is one block patch: one step with omega = 1 is
    numpy.linalg.solve(A, b)."""
    from fsigen.problem import make_level, PARAMS_DEFAULT
    rng = np.random.default_rng(5)
    coords = [np.linspace(0.0, 1.0, 5)] * 2
    st = {k: rng.standard_normal((25, 2)) * 0.01 for k in ("v_old", "u_old", "v_cur")}
    st["u_cur"] = st["u_old"] + 0.005 * (st["v_cur"] + st["v_old"])
    lev = make_level(2, (2, 2), coords, ((0.3, 0.3), (0.7, 0.7)), st, PARAMS_DEFAULT)
    for name in ("mom", "ale"):
        m = lev.systems[name]
        A = to_csr(m)
        mask = m.dirichlet.astype(bool)
        b = rng.standard_normal(A.shape[0])
        b[mask] = 0.0
        V = VankaData.build(m, lev.cells, omega=1.0, weighting="mult", patches="block")
        assert len(V) == 1 and V[0].dofs.shape == (1, 25 * m.b)
        x = vanka_sweep(A, b, np.zeros_like(b), V, mask)
        ref = np.linalg.solve(A.toarray(), b)
        np.testing.assert_allclose(x, ref, rtol=0, atol=1e-12 * max(np.abs(ref).max(), 1e-300))


def test_block_multiplicity_counts_patches(prob_t2):
    """With blocks a node inside a 2 x 2 block belongs to that one patch; the
    averaged weighting divides by the number of patches, not elements."""
    m = prob_t2.levels[0].systems["mom"]
    cells = prob_t2.levels[0].cells
    V = VankaData.build(m, cells, omega=0.8, weighting="mult", patches="block")
    n = m.nrows * m.b
    mult = np.zeros(n)
    for g in V:
        mult += np.bincount(g.dofs.ravel(), minlength=n)
    np.testing.assert_array_equal(V[0].scale, 1.0 / np.maximum(mult, 1.0))
    nx = 2 * cells[0] + 1
    centre = (2 + 2 * nx) * m.b   # node (2, 2): centre of the first block
    corner = (4 + 4 * nx) * m.b   # node (4, 4): shared by four blocks
    assert mult[centre] == 1 and mult[corner] == 4


def test_block_patches_converge_where_element_patches_stall():
    """Nearly incompressible solid (lambda / mu = 40): the V-cycle with
    one-element patches does not reduce the residual, the one with 2 x 2
    blocks converges (the paper chooses the larger solid patches, Sec. 5.5.1)."""
    from fsigen.problem import make_problem, SOLID_2D
    from oracle.fgmres import fgmres
    from oracle.mg import vcycle
    P = make_problem(2, 16, 3, SOLID_2D, seed=0, params=dict(mu_s=5e4, lambda_s=2e6),
                     systems=("mom",))
    mats = [lv.systems["mom"] for lv in P.levels]
    cells = [lv.cells for lv in P.levels]
    solid = [lv.cell_solid for lv in P.levels]
    b = P.rhs["mom"]
    its = {}
    for patches in ("element", "block"):
        H = Hierarchy(mats, cells, omega=0.8, weighting="mult", patches=patches, cell_solid=solid)
        lev = H.levels[0]
        x, info = fgmres(lev.A, b, np.zeros_like(b), lambda v: vcycle(H, v), lev.mask, rtol=1e-8,
                         maxiter=120, restart=20)
        its[patches] = (info["iters"], info["converged"])
    assert its["block"][1] and its["block"][0] <= 40
    assert not its["element"][1]


# ------------------------------------------------------------ block ILU(0) smoother
class _BSR:
    def __init__(self, rowptr, colind, vals, b):
        self.rowptr, self.colind, self.vals, self.b = rowptr, colind, vals, b
        self.nrows = rowptr.shape[0] - 1


def _bsr_from_blocks(blocks, n, b):
    """blocks: dict (i, j) -> b x b array."""
    rows = [sorted(j for (i, j) in blocks if i == r) for r in range(n)]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum([len(r) for r in rows])
    colind = np.array([j for r in rows for j in r], dtype=np.int64)
    vals = np.stack([blocks[(r, j)] for r in range(n) for j in rows[r]]).reshape(-1)
    return _BSR(rowptr, colind, vals, b)


def test_ilu_is_exact_lu_without_fill_in():
    """A block-tridiagonal pattern produces no fill-in, so ILU(0) is the
    exact block LU and one undamped ILU step from zero solves the system."""
    from oracle import BlockILU, ilu_sweep
    rng = np.random.default_rng(21)
    n, b = 30, 3
    blocks = {}
    for i in range(n):
        blocks[(i, i)] = rng.standard_normal((b, b)) + 6.0 * np.eye(b)
        if i > 0:
            blocks[(i, i - 1)] = rng.standard_normal((b, b))
            blocks[(i - 1, i)] = rng.standard_normal((b, b))
    m = _bsr_from_blocks(blocks, n, b)
    A = to_csr(m)
    rhs = rng.standard_normal(n * b)
    ref = np.linalg.solve(A.toarray(), rhs)
    ilu = BlockILU(m)
    assert np.linalg.norm(ilu.solve(rhs) - ref) <= 1e-12 * np.linalg.norm(ref)
    x = ilu_sweep(A, rhs, np.zeros(n * b), ilu, np.zeros(n * b, dtype=bool))
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


def test_ilu_block_diagonal_is_block_jacobi():
    from oracle import BlockILU
    rng = np.random.default_rng(22)
    n, b = 12, 4
    blocks = {(i, i): rng.standard_normal((b, b)) + 5.0 * np.eye(b) for i in range(n)}
    m = _bsr_from_blocks(blocks, n, b)
    d = rng.standard_normal(n * b)
    ref = np.concatenate([np.linalg.solve(blocks[(i, i)], d[i * b:(i + 1) * b]) for i in range(n)])
    assert np.abs(BlockILU(m).solve(d) - ref).max() <= 1e-13 * np.abs(ref).max()


def test_ilu_product_reproduces_the_matrix_on_its_pattern():
    """The defining property of ILU(0): (L U)_ij = A_ij on every block of the
    pattern (the discarded fill-in lies outside it), on a 2D Q2 momentum
    matrix with Dirichlet rows; L unit block-lower, U block-upper."""
    from oracle import BlockILU
    P = make_problem(2, 8, 2, SOLID_2D, seed=0, systems=("mom",))
    m = P.levels[0].systems["mom"]
    A = to_csr(m).toarray()
    L, U = BlockILU(m).lower_upper_dense()
    b = m.b
    assert np.allclose(np.tril(L, -1) + np.eye(L.shape[0]), L)  # unit lower
    LU = L @ U
    on = np.zeros_like(A, dtype=bool)
    for i in range(m.nrows):
        for p in range(m.rowptr[i], m.rowptr[i + 1]):
            j = m.colind[p]
            on[i * b:(i + 1) * b, j * b:(j + 1) * b] = True
    assert np.abs(LU - A)[on].max() <= 1e-11 * np.abs(A).max()
    assert np.abs(LU - A)[~on].max() > 1e-8 * np.abs(A).max()  # fill-in was dropped


def test_ilu_smoothed_mg_converges_mesh_independently():
    """FGMRES with an ILU-smoothed V-cycle reaches 1e-8 (true residual checked
    with SciPy) in few, mesh-independent iterations, no more than with Vanka."""
    its = []
    for n, nl in ((16, 2), (32, 3)):
        P = make_problem(2, n, nl, SOLID_2D, seed=0, systems=("mom",))
        cells = [l.cells for l in P.levels]
        mats = P.system("mom")
        H = Hierarchy(mats, cells, smoother="ilu")
        x, info, _ = solve_system(mats, cells, P.rhs["mom"], rtol=1e-8, H=H)
        A = to_csr(mats[0])
        r = P.rhs["mom"] - A @ x
        r[mats[0].dirichlet.astype(bool)] = 0.0
        assert info["converged"] and np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(P.rhs["mom"])
        _, info_v, _ = solve_system(mats, cells, P.rhs["mom"], rtol=1e-8, weighting="mult")
        assert info["iters"] <= info_v["iters"]
        its.append(info["iters"])
    assert its[1] - its[0] <= 2 and its[1] <= 12
