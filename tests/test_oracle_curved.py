"""The curved benchmark channel (Sec. 5: a cylinder of radius 0.05 cut from
the channel) on isoparametric Q2 cells, and the oracle's residual on such
cells, pinned by what the geometry and the mathematics fix exactly:

* the map keeps the channel's walls, puts the obstacle's surface and the
  beam's root on the circle and inverts no cell on any level;
* the mesh's cells tile the channel box, so their quadrature areas sum to
  its area exactly (det(dx/dxi) of a Q2 map is a polynomial of degree <= 5
  per reference axis, which 3-point Gauss integrates exactly), and the
  obstacle's area converges to pi r^2 under refinement;
* isoparametric Q2 reproduces functions linear in the physical coordinates,
  so the closed forms of the residual on affine states (constant pressure,
  affine solid deformation, ALE divergence, the divergence-theorem force)
  hold exactly with the cells' areas;
* the oracle's complex-step Jacobian equals the input generator's
  independently coded matrix on a curved mesh at a seeded state.
"""
import numpy as np
import pytest

from fsigen import make_channel
from fsigen.problem import (CHANNEL_BEAM, CHANNEL_ENDS, CHANNEL_OBSTACLE, CYL_CENTER, CYL_RADIUS,
                            _grid_coords, channel_map, make_level)
from oracle.fsi import Mesh, force, jacobian_bsr, operator_value, point_weights


@pytest.fixture(scope="module", params=[2, 3])
def curved(request):
    return make_channel(request.param, 2, params=dict(mu_s=5e5, lambda_s=2e6), curved=True)


def _box_area(dim):
    return float(np.prod([CHANNEL_ENDS[a][-1] for a in range(dim)]))


def _cell_areas(m):
    return point_weights(m).sum(axis=1)


def test_map_keeps_walls_and_puts_the_obstacle_on_the_circle():
    for dim in (2, 3):
        for nlev in (2, 3) if dim == 2 else (2,):
            C = make_channel(dim, nlev, curved=True)
            lev = C.problem.levels[0]
            X, R = lev.node_coords, _grid_coords(lev.coords, dim)
            for a in range(dim):
                for v in (CHANNEL_ENDS[a][0], CHANNEL_ENDS[a][-1]):
                    on = R[:, a] == v
                    assert np.array_equal(X[on, a], R[on, a])  # the wall stays a wall
            if dim == 3:
                assert np.array_equal(X[:, 2], R[:, 2])
            # nodes on the square obstacle's boundary land on the circle
            lo, hi = CHANNEL_OBSTACLE[0], CHANNEL_OBSTACLE[1]
            sinf = np.maximum(np.abs(R[:, 0] - CYL_CENTER[0]), np.abs(R[:, 1] - CYL_CENTER[1]))
            on_sq = np.abs(sinf - (hi[0] - lo[0]) / 2) < 1e-12
            r = np.hypot(X[on_sq, 0] - CYL_CENTER[0], X[on_sq, 1] - CYL_CENTER[1])
            assert on_sq.sum() >= 8 and np.abs(r - CYL_RADIUS).max() < 1e-14
            # the probe point B is unchanged
            assert np.array_equal(X[C.probe_node], [0.9, 0.2, 0.3][:dim])
            # every row stays ordered in y at every x (no fold)
            for l, lv in enumerate(C.problem.levels):
                Y = lv.node_coords[:, 1].reshape([len(c) for c in lv.coords[::-1]])
                assert np.all(np.diff(Y, axis=-2) > 0)
                assert Mesh(lv).detJ.min() > 0.0, l


def test_map_is_the_identity_far_from_obstacle_and_beam():
    R = np.array([[1.0, 0.17], [0.45, 0.33], [0.8, 0.1]])
    np.testing.assert_array_equal(channel_map(R), R)
    # rows of even height at the inflow: breaks 0.15 .. 0.25 -> 0.082 .. 0.328
    Y = channel_map(np.array([[0.0, 0.15], [0.0, 0.19], [0.0, 0.21], [0.0, 0.25]]))[:, 1]
    np.testing.assert_allclose(Y, [0.082, 0.164, 0.246, 0.328], rtol=0, atol=1e-15)


def test_cells_tile_the_box_exactly(curved):
    for lv in curved.problem.levels:
        m = Mesh(lv)
        assert abs(_cell_areas(m).sum() - _box_area(m.dim)) <= 1e-13 * _box_area(m.dim)


def test_obstacle_area_converges_to_the_disc():
    """2D: the obstacle cells' area -> pi r^2 at O(h^4) (Q2 interpolation of
    the circle); the error drops by >= 8 per refinement."""
    errs = []
    for nlev in (2, 3, 4):
        C = make_channel(2, nlev, curved=True)
        m = Mesh(C.problem.levels[0])
        rigid = np.isin(np.arange(m.nodes.shape[0]),
                        np.nonzero(np.all(np.isin(m.nodes, C.force_nodes), axis=1))[0])
        errs.append(abs(_cell_areas(m)[rigid].sum() - np.pi * CYL_RADIUS ** 2))
    assert errs[0] < 1e-4 and errs[1] <= errs[0] / 8 and errs[2] <= errs[1] / 8, errs


def _states(m, n, d):
    return np.zeros(n * (d + 1)), np.zeros(n * d)


def test_constant_pressure_closed_form(curved):
    """p = c, v = 0, F = I: the momentum rows summed against the node
    coordinates x_b give -k c delta_ab |Omega_f| (|Omega_f|: the fluid
    cells' quadrature area)."""
    P = curved.problem
    lev = P.levels[0]
    m = Mesh(lev)
    n, d = m.nnodes, m.dim
    c = 3.5
    x = np.zeros((n, d + 1)); x[:, 0] = c
    z, zu = _states(m, n, d)
    r = operator_value(m, P.params, x.ravel(), zu, z, zu).reshape(n, d + 1)
    got = lev.node_coords.T @ r[:, 1:]
    want = -P.params["k"] * c * _cell_areas(m)[~m.solid].sum() * np.eye(d)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-14 * abs(want).max())


def test_solid_first_piola_closed_form(curved):
    """u_old = A x (physical x), v = 0: the solid rows tested against x_b
    give k (F Sigma)_ab |Omega_s| (St. Venant-Kirchhoff)."""
    P = curved.problem
    lev = P.levels[0]
    m = Mesh(lev)
    n, d = m.nnodes, m.dim
    A = 0.05 * np.random.default_rng(7).standard_normal((d, d))
    X = lev.node_coords
    uo = (X @ A.T).ravel()
    z = np.zeros(n * (d + 1))
    r = operator_value(m, P.params, z, uo, z, uo).reshape(n, d + 1)
    F = np.eye(d) + A
    E = 0.5 * (F.T @ F - np.eye(d))
    S = 2 * P.params["mu_s"] * E + P.params["lambda_s"] * np.trace(E) * np.eye(d)
    want = P.params["k"] * (F @ S) * _cell_areas(m)[m.solid].sum()
    got = (X.T @ r[:, 1:]).T
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-12 * np.abs(want).max())


def test_fluid_divergence_closed_form(curved):
    """u = A x, v = v_old = B x, p = 0: the divergence rows sum to
    k det(F) tr(B F^-1) |Omega_f| -- needs (dx/dxi)^-T applied correctly."""
    P = curved.problem
    lev = P.levels[0]
    m = Mesh(lev)
    n, d = m.nnodes, m.dim
    rng = np.random.default_rng(8)
    A = 0.05 * rng.standard_normal((d, d))
    B = rng.standard_normal((d, d))
    X = lev.node_coords
    x = np.zeros((n, d + 1)); x[:, 1:] = X @ B.T
    u = (X @ A.T).ravel()
    r = operator_value(m, P.params, x.ravel(), u, x.ravel(), u).reshape(n, d + 1)
    F = np.eye(d) + A
    want = P.params["k"] * np.linalg.det(F) * np.trace(B @ np.linalg.inv(F)) * _cell_areas(m)[~m.solid].sum()
    assert abs(r[:, 0].sum() - want) <= 1e-12 * abs(want)


def _edge_weight(y0, y1, y2):
    """int_0^1 L_0(xi) y'(xi) dxi for the Q2 curve y(xi) = sum_k y_k L_k(xi):
    -y0/2 + 2 y1/3 - y2/6 (L_0 = 1 at the first node)."""
    return -y0 / 2 + 2 * y1 / 3 - y2 / 6


def test_force_closed_form_on_the_curved_obstacle():
    """p = c, v = (a y, 0[, 0]), solid stiffness zero: the force is
    (c G, -rho nu a G[, 0]) with G = int over the fluid of d psi_h / dx, which
    the divergence theorem turns into boundary integrals of psi_h n_x: the
    wetted obstacle surface (psi = 1) gives the y-extent s of the beam's
    root (now a circular arc between mapped nodes) times the depth, and the
    beam's top and bottom faces, curved near the root, add depth times the
    Q2 edge integrals of L_0(xi) dy/dxi over their first cells.  With psi
    extended over the beam the closed surface gives zero."""
    for dim in (2, 3):
        C = make_channel(dim, 2, params=dict(mu_s=0.0, lambda_s=0.0), curved=True)
        P = C.problem
        lev = P.levels[0]
        X = lev.node_coords
        R = _grid_coords(lev.coords, dim)
        n = lev.nnodes
        c, a = 3.7, 2.3
        x = np.zeros((n, dim + 1)); x[:, 0] = c; x[:, 1] = a * X[:, 1]
        u = np.zeros(n * dim)
        m = Mesh(lev)
        F = force(m, P.params, x.ravel(), u, x.ravel(), u, C.force_nodes)
        b0, b1 = CHANNEL_BEAM
        xs = lev.coords[0]
        i0 = int(np.argmin(np.abs(xs - b0[0])))          # the root's node column
        assert abs(xs[i0] - b0[0]) < 1e-15

        def node(ix, y):
            hit = (R[:, 0] == xs[ix]) & (np.abs(R[:, 1] - y) < 1e-15)
            if dim == 3:
                hit &= R[:, 2] == lev.coords[2][0]       # the map does not depend on z
            return np.nonzero(hit)[0][0]

        top = [X[node(i0 + j, b1[1]), 1] for j in range(3)]
        bot = [X[node(i0 + j, b0[1]), 1] for j in range(3)]
        depth = (b1[2] - b0[2]) if dim == 3 else 1.0
        G = depth * ((top[0] - bot[0]) + _edge_weight(*top) - _edge_weight(*bot))
        assert 0.0195 < (top[0] - bot[0]) < 0.02 and G != depth * (top[0] - bot[0])
        exp = [c * G, -P.params["rho_f"] * P.params["nu_f"] * a * G] + [0.0] * (dim - 2)
        assert np.allclose(F, exp, rtol=0, atol=1e-12 * c), (F, exp)
        beam_nodes = np.nonzero(lev.node_solid)[0]
        F2 = force(m, P.params, x.ravel(), u, x.ravel(), u, np.union1d(C.force_nodes, beam_nodes))
        assert np.allclose(F2, 0.0, atol=1e-12 * c)


@pytest.mark.parametrize("dim", [2, 3])
def test_complex_step_jacobian_equals_generator_matrix_on_curved_cells(dim):
    """A curved channel level assembled by the generator at a seeded state
    (velocities, deformations, the solid condensed): the oracle's derivative
    of its own residual reproduces the generator's hand-coded matrix."""
    C = make_channel(dim, 2, curved=True)
    lv0 = C.problem.levels[1]  # the coarser level: a smaller seeded check
    n = lv0.nnodes
    rng = np.random.default_rng(11)
    st = {k: a * rng.standard_normal((n, dim)) for k, a in
          (("v_old", 0.1), ("u_old", 5e-4), ("v_cur", 0.1), ("u_cur", 5e-4))}
    # at solid and interface nodes the deformation is the condensed one (Sec. 3.1)
    k, th = C.problem.params["k"], C.problem.params["theta"]
    ns = lv0.node_solid.astype(bool)
    st["u_cur"][ns] = (st["u_old"] + k * th * st["v_cur"] + k * (1 - th) * st["v_old"])[ns]
    cells = tuple(lv0.cells)
    lev = make_level(dim, cells, lv0.coords, (CHANNEL_BEAM[0][:dim], CHANNEL_BEAM[1][:dim]), st,
                     C.problem.params, systems=("mom",),
                     rigid_box=(CHANNEL_OBSTACLE[0][:dim], CHANNEL_OBSTACLE[1][:dim]),
                     node_coords=lv0.node_coords)
    A = lev.systems["mom"]
    m = Mesh(lev)
    x = np.zeros((n, dim + 1)); x[:, 1:] = st["v_cur"]
    xo = np.zeros((n, dim + 1)); xo[:, 1:] = st["v_old"]
    vals = jacobian_bsr(m, C.problem.params, x.ravel(), st["u_cur"].ravel(), xo.ravel(),
                        st["u_old"].ravel(), A.rowptr, A.colind, A.dirichlet)
    assert np.abs(vals - A.vals).max() <= 1e-13 * np.abs(A.vals).max()
