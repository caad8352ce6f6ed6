"""Pins of the input generator (fsigen): the assembled matrices are what the
paper's discretisation defines (Sec. 3.1 / 3.2 / 4.2)."""
import numpy as np
import pytest
import scipy.sparse as sp

from fsigen import graded_axis, make_problem
from fsigen.problem import SOLID_2D, SOLID_3D, make_level, residual_momentum, _nodes_from_verts


def _csr(m):
    n = m.rowptr.shape[0] - 1
    return sp.bsr_matrix((m.vals, m.colind, m.rowptr), shape=(n * m.b, n * m.b)).tocsr()


def test_graded_axis_counts():
    # coarse cell shares: 2D 8 cells -> 3/3/2 (x), 4/1/3 (y); 3D 4 cells -> 1/2/1, 2/1/1
    def counts(v, lo, hi):
        return [int(np.sum((v[1:] <= lo + 1e-12))), int(np.sum((v[1:] > lo + 1e-12) & (v[1:] <= hi + 1e-12))),
                int(np.sum(v[1:] > hi + 1e-12))]
    assert counts(graded_axis(8, 0.3, 0.7, 1)[0], 0.3, 0.7) == [3, 3, 2]
    assert counts(graded_axis(8, 0.45, 0.55, 1)[0], 0.45, 0.55) == [4, 1, 3]
    assert counts(graded_axis(4, 0.3, 0.7, 1)[0], 0.3, 0.7) == [1, 2, 1]
    assert counts(graded_axis(4, 0.4, 0.6, 1)[0], 0.4, 0.6) == [2, 1, 1]
    fine = graded_axis(4, 0.3, 0.7, 3)
    assert [len(v) - 1 for v in fine] == [16, 8, 4]
    assert np.any(np.isclose(fine[0], 0.3)) and np.any(np.isclose(fine[0], 0.7))


def _flat_level(dim, n):
    verts = [graded_axis(n // 2, 0.3, 0.7, 2)[0] for _ in range(dim)]
    coords = [_nodes_from_verts(v) for v in verts]
    nn = int(np.prod([len(c) for c in coords]))
    z = np.zeros((nn, dim))
    st = dict(v_old=z, u_old=z, v_cur=z, u_cur=z)
    box = SOLID_2D if dim == 2 else SOLID_3D
    return make_level(dim, tuple([n] * dim), coords, box, st, dict(
        rho_f=1e3, nu_f=1e-3, rho_s=1e3, mu_s=5e5, lambda_s=2e6, k=0.01, theta=0.5, alpha0=1.0),
        need_smass=True)


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_sums_to_volume(dim):
    lev = _flat_level(dim, 8)
    assert abs(lev.systems["smass"].vals.sum() - 1.0) < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_laplace_rows_and_quadratic_exactness(dim):
    """ALE rows of fluid-only interior nodes: the Q2 Laplacian, whose rows sum to
    zero and which reproduces -Laplace(q) = -2d for q = |x|^2 exactly."""
    lev = _flat_level(dim, 8)
    A = _csr(lev.systems["ale"])
    M = _csr(lev.systems["smass"])
    X = np.stack(np.meshgrid(*lev.coords[::-1], indexing="ij")[::-1], axis=-1).reshape(-1, dim)
    q = np.sum(X * X, axis=1)
    rows = np.nonzero((lev.node_solid == 0) & (lev.node_bdry == 0))[0]
    u = np.repeat(q[:, None], dim, axis=1).ravel()
    ones = np.ones(lev.nnodes * dim)
    lhs = (A @ u).reshape(-1, dim)[rows]
    rhs = -2.0 * dim * (M @ np.ones(lev.nnodes))[rows]
    assert np.abs((A @ ones).reshape(-1, dim)[rows]).max() < 1e-12
    assert np.abs(lhs - rhs[:, None]).max() < 1e-11 * np.abs(rhs).max()


@pytest.mark.parametrize("name,dim", [("t2", 2), ("t3", 3)])
def test_momentum_jacobian_finite_differences(name, dim, request):
    """The momentum matrix is the Jacobian of the condensed residual with all
    derivatives w.r.t. the ALE deformation dropped (Sec. 4.2): central finite
    differences of an independently coded residual agree to O(eps^2)."""
    P = request.getfixturevalue("prob_" + name)
    lev = P.levels[0]
    A = lev.systems["mom"]
    n, b = lev.nnodes, dim + 1
    M = _csr(A)
    rng = np.random.default_rng(1)
    delta = rng.standard_normal(n * b)
    mask = A.dirichlet.astype(bool)
    delta[mask] = 0.0
    pres = rng.standard_normal(n)

    def R(eps):
        dv = delta.reshape(n, b)
        return residual_momentum(lev, P.params, P.v_old, P.u_old, P.u_cur,
                                 P.v_cur + eps * dv[:, 1:], pres + eps * dv[:, 0])
    Jd = M @ delta
    errs = []
    for eps in (1e-3, 1e-4):
        fd = (R(eps) - R(-eps)) / (2 * eps)
        errs.append(np.abs(fd - Jd)[~mask].max() / np.abs(Jd[~mask]).max())
    assert errs[1] < 1e-7
    assert errs[1] < errs[0] / 50  # second-order convergence of the difference quotient


def test_condensed_state_and_flags(prob_t3):
    P = prob_t3
    k, th = P.params["k"], P.params["theta"]
    np.testing.assert_allclose(P.u_cur, P.u_old + k * th * P.v_cur + k * (1 - th) * P.v_old,
                               rtol=0, atol=1e-15)
    lev = P.levels[0]
    # pressure identity rows exactly at solid-interior nodes
    mom = lev.systems["mom"]
    pmask = mom.dirichlet.reshape(-1, 4)[:, 0].astype(bool)
    np.testing.assert_array_equal(pmask, (lev.node_solid == 1) & (lev.node_fluid == 0))
    # every level resolves the solid box: solid volume identical on all levels
    vols = []
    for L in P.levels:
        h = [np.diff(c[::2]) for c in L.coords]
        cv = np.multiply.outer(np.multiply.outer(h[2], h[1]), h[0]).ravel()
        vols.append(float(cv[L.cell_solid == 1].sum()))
    np.testing.assert_allclose(vols, 0.4 * 0.2 * 0.2, rtol=1e-12)


def test_rhs_recipe(prob_t2):
    P = prob_t2
    for key, name in (("mom", "mom"), ("ale", "ale")):
        b = P.rhs[key]
        assert abs(np.linalg.norm(b) - 1.0) < 1e-12
        assert np.all(b[P.levels[0].systems[name].dirichlet.astype(bool)] == 0.0)
    P2 = make_problem(2, 16, 2, SOLID_2D, seed=0)
    np.testing.assert_array_equal(P2.rhs["mom"], P.rhs["mom"])  # seeded
