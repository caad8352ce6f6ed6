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
