"""Pins of the Newton-loop oracle (oracle.fsi): the condensed residual of the
theta time step (eq. aletime:2, eq. defgrad), its complex-step Jacobian
(eq. problem:1) and the approximate Newton iteration (eq. newton, Sec. 5.5's
Jacobian reuse rule), checked against closed forms, against the generator's
independently coded matrices and residual, and against invariants of the
converged state."""
import numpy as np
import pytest

from fsigen import make_problem
from fsigen.problem import SOLID_2D, SOLID_3D, residual_momentum
from oracle import to_csr
from oracle.fsi import Mesh, inject, jacobian_bsr, newton, operator_value


def _box3():
    """3D 4^3 cells, one level: small enough for the complex step."""
    return make_problem(3, 4, 1, SOLID_3D, seed=3)


def _state(P):
    n, d = P.levels[0].nnodes, P.dim
    x = np.zeros((n, d + 1)); x[:, 1:] = P.v_cur
    xo = np.zeros((n, d + 1)); xo[:, 1:] = P.v_old
    return x.ravel(), P.u_cur.ravel(), xo.ravel(), P.u_old.ravel()


def _xyz(mesh):
    g = np.meshgrid(*mesh.coords[::-1], indexing="ij")[::-1]
    return np.stack([a.ravel() for a in g], axis=1)


def _volume(mesh, solid):
    return float(np.prod(mesh.h, axis=1)[mesh.solid == solid].sum())


@pytest.mark.parametrize("which", ["t2", "box3"])
def test_complex_step_jacobian_equals_generator_matrix(which, prob_t2):
    """The generator's momentum matrix is the hand-derived approximate
    Jacobian (itself checked by central differences of its own residual);
    the oracle's derivative of its own residual reproduces it."""
    P = prob_t2 if which == "t2" else _box3()
    lev = P.levels[0]
    A = lev.systems["mom"]
    vals = jacobian_bsr(Mesh(lev), P.params, *_state(P), A.rowptr, A.colind, A.dirichlet)
    assert np.abs(vals - A.vals).max() <= 1e-13 * np.abs(A.vals).max()


@pytest.mark.parametrize("which", ["t2", "box3"])
def test_residual_differences_equal_generator_residual(which, prob_t2):
    """The generator's residual omits the old-time terms; differences of two
    states with one old state cancel them."""
    P = prob_t2 if which == "t2" else _box3()
    lev = P.levels[0]
    d, n = P.dim, lev.nnodes
    m = Mesh(lev)
    x, u, xo, uo = _state(P)
    rng = np.random.default_rng(5)
    x2 = x.reshape(n, d + 1).copy()
    x2[:, 0] = 10 * rng.standard_normal(n)
    x2[:, 1:] += 0.01 * rng.standard_normal((n, d))
    ra = operator_value(m, P.params, x2.ravel(), u, xo, uo) - operator_value(m, P.params, x, u, xo, uo)
    X = x.reshape(n, d + 1)
    rb = (residual_momentum(lev, P.params, P.v_old, P.u_old, P.u_cur, x2[:, 1:], x2[:, 0])
          - residual_momentum(lev, P.params, P.v_old, P.u_old, P.u_cur, X[:, 1:], X[:, 0]))
    assert np.abs(ra - rb).max() <= 1e-12 * np.abs(rb).max()


def test_rest_and_uniform_motion_have_zero_residual(prob_t2):
    """At rest nothing acts; a uniform velocity with an undeformed fluid mesh
    and zero pressure has no inertia (v = v_old), no convection or viscous
    stress (grad v = 0) and a rigidly translated solid (F = I)."""
    P = prob_t2
    m = Mesh(P.levels[0])
    n, d = m.nnodes, m.dim
    z = np.zeros(n * (d + 1))
    assert np.abs(operator_value(m, P.params, z, np.zeros(n * d), z, np.zeros(n * d))).max() == 0.0
    x = np.zeros((n, d + 1)); x[:, 1:] = [0.3, -0.2]
    r = operator_value(m, P.params, x.ravel(), np.zeros(n * d), x.ravel(), np.zeros(n * d))
    assert np.abs(r).max() < 1e-13


def test_constant_pressure_term(prob_t2):
    """p = c, v = 0, F = I: the momentum rows are -k c (div phi_i) on the
    fluid; summed against the nodal coordinates x_b they give
    -k c delta_ab |Omega_f| (Q2 reproduces linear functions)."""
    P = prob_t2
    m = Mesh(P.levels[0])
    n, d = m.nnodes, m.dim
    c = 3.5
    x = np.zeros((n, d + 1)); x[:, 0] = c
    r = operator_value(m, P.params, x.ravel(), np.zeros(n * d), np.zeros(n * (d + 1)),
                       np.zeros(n * d)).reshape(n, d + 1)
    X = _xyz(m)
    got = X.T @ r[:, 1:]                       # [b, a]
    want = -P.params["k"] * c * _volume(m, False) * np.eye(d)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-14)
    assert np.abs(r[:, 1:].sum(axis=0)).max() < 1e-13


@pytest.mark.parametrize("which", ["t2", "box3"])
def test_solid_first_piola_stress_closed_form(which, prob_t2):
    """Affine deformation u_old = A x, v = v_old = 0: the fluid terms vanish
    and the solid rows tested against x_b give k (F Sigma)_ab |Omega_s| with
    F = I + A, Sigma = 2 mu E + lambda tr(E) I, E = (F^T F - I) / 2 (St.
    Venant-Kirchhoff, Sec. 2)."""
    P = prob_t2 if which == "t2" else _box3()
    m = Mesh(P.levels[0])
    n, d = m.nnodes, m.dim
    rng = np.random.default_rng(7)
    A = 0.05 * rng.standard_normal((d, d))
    X = _xyz(m)
    uo = (X @ A.T).ravel()
    z = np.zeros(n * (d + 1))
    r = operator_value(m, P.params, z, uo, z, uo).reshape(n, d + 1)
    F = np.eye(d) + A
    E = 0.5 * (F.T @ F - np.eye(d))
    S = 2 * P.params["mu_s"] * E + P.params["lambda_s"] * np.trace(E) * np.eye(d)
    want = P.params["k"] * (F @ S) * _volume(m, True)
    got = (X.T @ r[:, 1:]).T                   # [a, b]
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-12 * np.abs(want).max())


def test_fluid_divergence_closed_form(prob_t2):
    """Affine u = A x and v = v_old = B x, p = 0: the divergence rows sum to
    k det(F) tr(B F^-1) |Omega_f| (F = I + A) -- the ALE divergence
    J tr(grad v F^-1) of eq. aletime:1.5."""
    P = prob_t2
    m = Mesh(P.levels[0])
    n, d = m.nnodes, m.dim
    rng = np.random.default_rng(8)
    A = 0.05 * rng.standard_normal((d, d))
    B = rng.standard_normal((d, d))
    X = _xyz(m)
    x = np.zeros((n, d + 1)); x[:, 1:] = X @ B.T
    u = (X @ A.T).ravel()
    r = operator_value(m, P.params, x.ravel(), u, x.ravel(), u).reshape(n, d + 1)
    F = np.eye(d) + A
    want = P.params["k"] * np.linalg.det(F) * np.trace(B @ np.linalg.inv(F)) * _volume(m, False)
    assert abs(r[:, 0].sum() - want) <= 1e-12 * abs(want)


def test_injection_takes_coincident_nodes(prob_t2):
    P = prob_t2
    mf, mc = Mesh(P.levels[0]), Mesh(P.levels[1])
    Xf, Xc = _xyz(mf), _xyz(mc)
    np.testing.assert_array_equal(inject(mf, mc, Xf.ravel(), mf.dim).reshape(-1, mf.dim), Xc)


def _newton(P, gamma, jac=None, state=None):
    lev = P.levels[0]
    A, Ea = lev.systems["mom"], lev.systems["ale"]
    x, u, xo, uo = state if state is not None else _state(P)
    return newton(Mesh(lev), P.params, (A.rowptr, A.colind), A.dirichlet, to_csr(Ea), Ea.dirichlet,
                  x, u, xo, uo, gamma=gamma, jac=jac), (xo, uo)


def test_newton_converged_state_solves_the_time_step(prob_t2):
    """At convergence the momentum residual is below 1e-8 of the initial one,
    the ALE extension holds at the fluid rows, the interface and solid
    deformation obeys the condensation relation (eq. problem:2) and the
    identity-row data are untouched."""
    P = prob_t2
    (x, u, info, _), (xo, uo) = _newton(P, 0.05)
    assert info["status"] == "ok" and info["res"][-1] <= 1e-8 * info["res"][0]
    lev = P.levels[0]
    m = Mesh(lev)
    d, n = P.dim, lev.nnodes
    E = to_csr(lev.systems["ale"])
    amask = lev.systems["ale"].dirichlet.astype(bool)
    assert np.abs((E @ u)[~amask]).max() <= 1e-8 * info["res"][0]
    k, th = P.params["k"], P.params["theta"]
    v = x.reshape(n, d + 1)[:, 1:]
    cond = uo.reshape(n, d) + k * th * v + k * (1 - th) * xo.reshape(n, d + 1)[:, 1:]
    np.testing.assert_allclose(u.reshape(n, d)[m.node_solid], cond[m.node_solid], atol=1e-14)
    mmask = lev.systems["mom"].dirichlet.astype(bool)
    x0 = _state(P)[0]
    np.testing.assert_array_equal(x[mmask], x0[mmask])


def test_newton_jacobian_reuse_rule(prob_t2):
    """gamma = 0 reassembles in every step (full approximate Newton, fewest
    steps); a large gamma keeps the first Jacobian; a Jacobian carried into
    the next time step is reused until the rate exceeds gamma."""
    P = prob_t2
    (_, _, i0, _), _ = _newton(P, 0.0)
    (_, _, i1, _), _ = _newton(P, 2.0)
    assert i0["jacobians"] == i0["steps"]
    assert i1["jacobians"] == 1 and i1["steps"] >= i0["steps"]
    (x, u, i2, jac), _ = _newton(P, 0.05)
    (_, _, i3, _), _ = _newton(P, 2.0, jac=jac, state=(x, u, x, u))
    assert i3["jacobians"] == 0 and i3["status"] == "ok"


def test_time_steps_from_the_previous_state_stay_bounded(prob_t2):
    """Successive time steps, each started from the last converged state
    (u = u_old, which violates the condensation relation by k v_old): the
    deformation increment carries that residual (eq. problem:2 with its
    right-hand side), every step converges, the condensation holds at the
    end of each step, and the Crank-Nicolson solution stays bounded.  (With
    the increment k theta dv alone, u loses k v_old per step and the same
    run grows by a factor ~2.7 per step.)"""
    P = prob_t2
    lev = P.levels[0]
    m = Mesh(lev)
    d, n = P.dim, lev.nnodes
    k, th = P.params["k"], P.params["theta"]
    (x, u, info, jac), (xo, uo) = _newton(P, 0.05)
    vmax = [np.abs(x.reshape(n, d + 1)[:, 1:]).max()]
    for _ in range(4):
        xo, uo = x.copy(), u.copy()
        (x, u, info, jac), _ = _newton(P, 0.05, jac=jac, state=(x, u, xo, uo))
        assert info["status"] == "ok"
        v = x.reshape(n, d + 1)[:, 1:]
        cond = uo.reshape(n, d) + k * th * v + k * (1 - th) * xo.reshape(n, d + 1)[:, 1:]
        np.testing.assert_allclose(u.reshape(n, d)[m.node_solid], cond[m.node_solid], atol=1e-12)
        vmax.append(np.abs(v).max())
    assert max(vmax) < 2.0 * vmax[0]


def test_element_subset_rows_are_complete(prob_t2):
    """Rows of sampled nodes assembled over only the cells that contain them
    equal the full assembly's rows (the full-size GPU checks rely on it)."""
    from oracle.fsi import cells_of_nodes, element_subset
    P = prob_t2
    m = Mesh(P.levels[0])
    x, u, xo, uo = _state(P)
    rng = np.random.default_rng(11)
    nodes = rng.choice(m.nnodes, 12, replace=False)
    sub = element_subset(m, cells_of_nodes(m, nodes))
    d = m.dim
    full = operator_value(m, P.params, x, u, xo, uo).reshape(-1, d + 1)
    part = operator_value(sub, P.params, x, u, xo, uo).reshape(-1, d + 1)
    np.testing.assert_array_equal(part[nodes], full[nodes])
    A = P.levels[0].systems["mom"]
    Jf = to_csr(type("M", (), dict(rowptr=A.rowptr, colind=A.colind, b=d + 1,
                                   vals=jacobian_bsr(m, P.params, x, u, xo, uo, A.rowptr, A.colind,
                                                     A.dirichlet))))
    Js = to_csr(type("M", (), dict(rowptr=A.rowptr, colind=A.colind, b=d + 1,
                                   vals=jacobian_bsr(sub, P.params, x, u, xo, uo, A.rowptr, A.colind,
                                                     A.dirichlet))))
    rows = (nodes[:, None] * (d + 1) + np.arange(d + 1)).ravel()
    assert abs(Jf[rows] - Js[rows]).max() == 0.0
