"""The benchmark channel (Sec. 5) and the residual form of its drag and lift:
the generator's graded breaks, inflow profile and start-up factor against
their definitions, the oracle's force against closed forms from the
divergence theorem, and time steps from rest (invariants of a converged
step, independence of the force from the test function's extension)."""
import numpy as np
import pytest

from fsigen import graded_breaks, inflow_profile, inflow_ramp, make_channel
from fsigen.problem import CHANNEL_BEAM, CHANNEL_ENDS, _grid_coords
from oracle import to_csr
from oracle.fsi import Mesh, force, time_step


@pytest.fixture(scope="module")
def ch2():
    return make_channel(2, 2)


def test_graded_breaks_resolve_every_break_on_every_level():
    for a, ends in enumerate(CHANNEL_ENDS):
        lv = graded_breaks((7, 5, 3)[a], ends, 3)
        assert len(lv[-1]) - 1 == (7, 5, 3)[a]
        for v in lv:
            for e in ends:
                assert np.min(np.abs(v - e)) < 1e-15
            assert np.all(np.diff(v) > 0)
        for f, c in zip(lv[:-1], lv[1:]):
            assert np.array_equal(f[0::2], c)        # nested: coarse vertices kept


def test_graded_breaks_share_rule():
    """[0, 1, 3, 10] with 10 cells: shares 1, 2, 7 exactly."""
    v = graded_breaks(10, [0.0, 1.0, 3.0, 10.0], 1)[0]
    assert np.allclose(v, [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10])
    with pytest.raises(ValueError):
        graded_breaks(2, [0.0, 1.0, 2.0, 3.0], 1)


@pytest.mark.parametrize("dim", [2, 3])
def test_inflow_profile_has_mean_vbar_and_vanishes_on_the_walls(dim):
    """Simpson's rule on the Q2 nodes of the inflow face integrates the
    (bi)quadratic profile exactly: the mean is vbar (Sec. 5)."""
    C = make_channel(dim, 2)
    lev = C.problem.levels[0]
    H = CHANNEL_ENDS[1][-1]

    def simpson_weights(x):
        w = np.zeros_like(x)
        for c in range(0, len(x) - 2, 2):
            h = x[c + 2] - x[c]
            w[c:c + 3] += h / 6.0 * np.array([1.0, 4.0, 1.0])
        return w

    wy = simpson_weights(lev.coords[1])
    if dim == 2:
        vals = inflow_profile(2, lev.coords[1], vbar=C.vbar)
        mean = wy @ vals / H
    else:
        wz = simpson_weights(lev.coords[2])
        Y, Z = np.meshgrid(lev.coords[1], lev.coords[2], indexing="ij")
        mean = wy @ inflow_profile(3, Y, Z, vbar=C.vbar) @ wz / H ** 2
    assert abs(mean - C.vbar) < 1e-12 * C.vbar
    # the generator's rows carry the same values, zero on the walls
    X = _grid_coords(lev.coords, dim)
    node = C.inflow_rows // (dim + 1)
    assert np.all(X[node, 0] == 0.0)
    assert np.allclose(C.inflow_vals, inflow_profile(dim, X[node, 1], X[node, 2] if dim == 3 else None,
                                                     C.vbar), rtol=0, atol=0)
    on_wall = (X[node, 1] == 0) | (X[node, 1] == H)
    if dim == 3:
        on_wall |= (X[node, 2] == 0) | (X[node, 2] == H)
    assert np.all(C.inflow_vals[on_wall] == 0.0) and np.all(C.inflow_vals[~on_wall] > 0)
    # every inflow row is held
    assert np.all(lev.systems["mom"].dirichlet[C.inflow_rows] == 1)


@pytest.mark.parametrize("dim", [2, 3])
def test_probe_node_is_on_the_beams_back_face(dim):
    C = make_channel(dim, 2)
    lev = C.problem.levels[0]
    X = _grid_coords(lev.coords, dim)
    assert np.abs(X[C.probe_node] - np.array([0.9, 0.2, 0.3][:dim])).max() <= 1e-12
    # on the interface: touches the beam and the fluid, its velocity is free
    assert lev.node_solid[C.probe_node] and lev.node_fluid[C.probe_node]
    assert not lev.node_rigid[C.probe_node]
    assert np.all(lev.systems["mom"].dirichlet.reshape(-1, dim + 1)[C.probe_node, 1:] == 0)


def test_ramp_definition():
    assert inflow_ramp(0.0) == 0.0
    assert abs(inflow_ramp(0.5) - 0.5) < 1e-15
    assert abs(inflow_ramp(1.0 - 1e-12) - 1.0) < 1e-15 and inflow_ramp(1.0) == 1.0 == inflow_ramp(7.0)
    assert abs(inflow_ramp(0.25) - (1 - np.sqrt(0.5)) / 2) < 1e-15


def test_obstacle_is_held_and_beam_is_free(ch2):
    lev = ch2.problem.levels[0]
    d = 2
    m = lev.systems["mom"].dirichlet.reshape(-1, d + 1)
    assert np.all(m[ch2.force_nodes, 1:] == 1)
    X = _grid_coords(lev.coords, d)
    b0, b1 = CHANNEL_BEAM[0], CHANNEL_BEAM[1]
    inner = ((X[:, 0] > b0[0]) & (X[:, 0] < b1[0]) & (X[:, 1] > b0[1]) & (X[:, 1] < b1[1]))
    assert inner.any() and np.all(m[inner, 1:] == 0)
    assert np.all(lev.cell_solid.sum() > 0)


@pytest.mark.parametrize("dim", [2, 3])
def test_force_closed_form(dim):
    """State p = c, v = (a y, 0[, 0]) everywhere, u = 0, v_old = v, solid
    stiffness zero: the force has no inertia, convection or solid part; by
    the divergence theorem the pressure gives c times the beam's root
    section (the part of the obstacle's back face the fluid does not wet)
    in x, the symmetric viscous stress rho nu a (e_x e_y + e_y e_x) gives
    -rho nu a times the same section in y, and nothing else survives."""
    C = make_channel(dim, 2, params=dict(mu_s=0.0, lambda_s=0.0))
    P = C.problem
    lev = P.levels[0]
    prm = P.params
    n = lev.nnodes
    X = _grid_coords(lev.coords, dim)
    c, a = 3.7, 2.3
    x = np.zeros((n, dim + 1))
    x[:, 0] = c
    x[:, 1] = a * X[:, 1]
    u = np.zeros(n * dim)
    F = force(Mesh(lev), prm, x.ravel(), u, x.ravel(), u, C.force_nodes)
    exp = [c * C.root_area, -prm["rho_f"] * prm["nu_f"] * a * C.root_area] + [0.0] * (dim - 2)
    assert np.allclose(F, exp, rtol=0, atol=1e-13 * c)
    # the test function on the obstacle and the beam: no unwetted section left
    beam_nodes = np.nonzero(lev.node_solid)[0]
    F2 = force(Mesh(lev), prm, x.ravel(), u, x.ravel(), u, np.union1d(C.force_nodes, beam_nodes))
    assert np.allclose(F2, 0.0, atol=1e-13 * c)


def _steps(C, nsteps, k):
    P = C.problem
    lev = P.levels[0]
    A, E = lev.systems["mom"], lev.systems["ale"]
    M = Mesh(lev)
    d, n = P.dim, lev.nnodes
    x, u = np.zeros(n * (d + 1)), np.zeros(n * d)
    out, jac = [], None
    for s in range(1, nsteps + 1):
        x, u, xo, uo, info, jac = time_step(M, P.params, (A.rowptr, A.colind), A.dirichlet, to_csr(E),
                                            E.dirichlet, x, u, C.inflow_rows, C.inflow_vals,
                                            inflow_ramp(s * k), jac=jac, rtol=1e-10, atol=1e-10,
                                            max_steps=30)
        out.append((x, u, xo, uo, info))
    return M, out


def test_rest_is_a_fixed_point(ch2):
    P = ch2.problem
    lev = P.levels[0]
    A, E = lev.systems["mom"], lev.systems["ale"]
    n, d = lev.nnodes, 2
    x, u, _, _, info, _ = time_step(Mesh(lev), P.params, (A.rowptr, A.colind), A.dirichlet, to_csr(E),
                                    E.dirichlet, np.zeros(n * (d + 1)), np.zeros(n * d), ch2.inflow_rows,
                                    ch2.inflow_vals, 0.0)
    assert info["status"] == "ok" and info["steps"] == 0
    assert not x.any() and not u.any()


def test_time_steps_from_rest():
    """Three steps of the start-up (k = 0.05): each converges; the inflow
    rows carry the ramped profile, the obstacle stays at rest; the drag
    grows with the inflow; and at a converged state the force does not
    depend on how the test function is extended into free nodes (here: onto
    the beam and the fluid nodes next to the obstacle), which is what makes
    the residual form exact (Sec. 5)."""
    k = 0.05
    C = make_channel(2, 2, params=dict(k=k, theta=0.5 + 2 * k))
    M, out = _steps(C, 3, k)
    lev = C.problem.levels[0]
    d = 2
    drags = []
    for s, (x, u, xo, uo, info) in enumerate(out, start=1):
        assert info["status"] == "ok"
        X = x.reshape(-1, d + 1)
        assert np.array_equal(x[C.inflow_rows], inflow_ramp(s * k) * C.inflow_vals)
        assert np.all(X[C.force_nodes, 1:] == 0.0)
        # the deformation there comes out of the direct ALE solve: zero up to
        # its rounding (1e-27 against 1e-5 elsewhere)
        assert np.abs(u.reshape(-1, d)[C.force_nodes]).max() <= 1e-20
        F = force(M, C.problem.params, x, u, xo, uo, C.force_nodes)
        drags.append(F[0])
        # extension of psi into free rows
        near = np.nonzero(np.isin(M.nodes, C.force_nodes).any(axis=1))[0]
        ext = np.unique(M.nodes[near])
        free = ext[lev.systems["mom"].dirichlet.reshape(-1, d + 1)[ext, 1] == 0]
        assert free.size > 10
        F2 = force(M, C.problem.params, x, u, xo, uo, np.union1d(C.force_nodes, free))
        assert np.allclose(F2, F, rtol=0, atol=1e-7 * abs(F[0]))
    assert 0 < drags[0] < drags[1] < drags[2]
