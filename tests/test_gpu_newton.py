"""The Newton loop on the GPU (include/fsimg_newton.h) against the oracle
(oracle.fsi): the condensed residual element by element, the assembled
approximate Jacobian on every multigrid level (its action on random vectors,
against the oracle's complex-step Jacobian at the injected state), and whole
Newton time steps (residual histories, Jacobian reuse decisions, the final
state) against the oracle's Newton loop with direct solves."""
import numpy as np
import pytest

from fsigen import config_problem
from oracle import to_csr
from oracle.fsi import Mesh, inject, jacobian_bsr, newton, newton_residual

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1904_02401_amd import fsimg  # noqa: E402
from paper_1904_02401_amd.problems import fsi_levels, fsi_state, level_dicts  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fsimg.fsimg_ctx_create(0)
    yield c
    fsimg.fsimg_ctx_destroy(c)


@pytest.fixture(scope="module")
def probs():
    return {name: config_problem(name, seed=0) for name in ("t2", "t3")}


class Fsi:
    """momentum + ALE hierarchies and the Newton object of a problem."""

    def __init__(self, ctx, P, precision=fsimg.FSIMG_FP64, rtol=1e-10, ale=True):
        o = fsimg.fsimg_default_opts(precision=precision, rtol=rtol)
        self.mom = fsimg.fsimg_hier_create(ctx, level_dicts(P, "mom"), o)
        self.ale = fsimg.fsimg_hier_create(ctx, level_dicts(P, "ale"), o) if ale else None
        self.f = fsimg.fsimg_fsi_create(self.mom, self.ale, fsi_levels(P), P.params)

    def close(self):
        fsimg.fsimg_fsi_destroy(self.f)
        fsimg.fsimg_hier_destroy(self.mom)
        if self.ale:
            fsimg.fsimg_hier_destroy(self.ale)


def _perturbed(P, seed):
    """the generator's state with a pressure field and perturbed velocity and
    fluid deformation (a state off the generator's own)."""
    x, u, xo, uo = fsi_state(P)
    d, n = P.dim, P.levels[0].nnodes
    rng = np.random.default_rng(seed)
    X = x.reshape(n, d + 1).copy()
    X[:, 0] = rng.standard_normal(n)
    X[:, 1:] += 0.02 * rng.standard_normal((n, d))
    mask = P.levels[0].systems["mom"].dirichlet.astype(bool)
    Xf = X.ravel()
    Xf[mask] = x[mask]
    u2 = u + 1e-3 * rng.standard_normal(u.size)
    return Xf, u2, xo, uo


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV, dtype=torch.float64)


@pytest.mark.parametrize("name", ["t2", "t3"])
def test_residual_matches_oracle(ctx, probs, name):
    P = probs[name]
    lev = P.levels[0]
    mask = lev.systems["mom"].dirichlet
    S = Fsi(ctx, P, ale=False)
    try:
        for seed in (0, 1):
            x, u, xo, uo = _perturbed(P, seed) if seed else fsi_state(P)
            ref = newton_residual(Mesh(lev), P.params, x, u, xo, uo, mask)
            res = torch.empty(x.size, device=DEV, dtype=torch.float64)
            fsimg.fsimg_fsi_residual(S.f, _t(x), _t(u), _t(xo), _t(uo), res)
            got = res.cpu().numpy()
            assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
            assert np.all(got[mask.astype(bool)] == 0.0)
    finally:
        S.close()


@pytest.mark.parametrize("name", ["t2", "t3"])
def test_jacobian_matches_oracle_on_every_level(ctx, probs, name):
    """The assembled Jacobian's action y = J_l z on three random vectors per
    level equals the oracle's complex-step Jacobian at the state injected to
    that level, with the level's identity rows."""
    P = probs[name]
    d = P.dim
    x, u, xo, uo = _perturbed(P, 2)
    S = Fsi(ctx, P, ale=False)
    try:
        fsimg.fsimg_fsi_jacobian(S.f, _t(x), _t(u), _t(xo), _t(uo))
        meshes = [Mesh(lv) for lv in P.levels]
        st = [x, u, xo, uo]
        rng = np.random.default_rng(3)
        for l, lv in enumerate(P.levels):
            if l > 0:
                st = [inject(meshes[l - 1], meshes[l], a, c)
                      for a, c in zip(st, (d + 1, d, d + 1, d))]
            A = lv.systems["mom"]
            vals = jacobian_bsr(meshes[l], P.params, *st, A.rowptr, A.colind, A.dirichlet)
            J = to_csr(type("M", (), dict(rowptr=A.rowptr, colind=A.colind, vals=vals, b=d + 1)))
            for _ in range(3):
                z = rng.standard_normal(J.shape[0])
                y = torch.empty(z.size, device=DEV, dtype=torch.float64)
                fsimg.fsimg_level_apply(S.mom, l, fsimg.FSIMG_FP64, _t(z), y)
                torch.cuda.synchronize()
                ref = J @ z
                assert np.abs(y.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max(), l
    finally:
        S.close()


def _oracle_newton(P, gamma, state=None, jac=None):
    lev = P.levels[0]
    A, E = lev.systems["mom"], lev.systems["ale"]
    x, u, xo, uo = state if state is not None else fsi_state(P)
    return newton(Mesh(lev), P.params, (A.rowptr, A.colind), A.dirichlet, to_csr(E), E.dirichlet,
                  x, u, xo, uo, gamma=gamma, jac=jac)


@pytest.mark.parametrize("name,gamma", [("t2", 0.05), ("t2", 0.0), ("t3", 0.05)])
def test_newton_time_step_matches_oracle(ctx, probs, name, gamma):
    """One time step: the same number of Newton steps and Jacobian
    assemblies, residual histories within the linear-solve tolerance, and
    the same converged state (the oracle solves its linear systems directly,
    the GPU by FGMRES + multigrid to 1e-10)."""
    P = probs[name]
    xr, ur, info, _ = _oracle_newton(P, gamma)
    x, u, xo, uo = fsi_state(P)
    S = Fsi(ctx, P)
    try:
        X, U = _t(x), _t(u)
        st = fsimg.fsimg_fsi_newton(S.f, X, U, _t(xo), _t(uo),
                                    fsimg.fsimg_default_newton_opts(gamma=gamma))
        torch.cuda.synchronize()
    finally:
        S.close()
    assert st["status"] == fsimg.FSIMG_OK and info["status"] == "ok"
    assert st["steps"] == info["steps"] and st["jacobians"] == info["jacobians"]
    h_gpu, h_ref = np.array(st["res_hist"]), np.array(info["res"])
    big = h_ref > 1e-5 * h_ref[0]
    np.testing.assert_allclose(h_gpu[big], h_ref[big], rtol=1e-5)
    assert st["omega_hist"] == info["omegas"]
    xg, ug = X.cpu().numpy(), U.cpu().numpy()
    assert np.abs(xg - xr).max() <= 1e-7 * np.abs(xr).max()
    assert np.abs(ug - ur).max() <= 1e-7 * np.abs(ur).max()


def test_newton_reuses_jacobian_across_time_steps(ctx, probs):
    """A Jacobian carried into the next time step is kept while the rate
    stays below gamma (here: always), as in the oracle."""
    P = probs["t2"]
    x1, u1, _, jac = _oracle_newton(P, 0.05)
    _, _, info2, _ = _oracle_newton(P, 2.0, state=(x1, u1, x1, u1), jac=jac)
    x, u, xo, uo = fsi_state(P)
    S = Fsi(ctx, P)
    try:
        X, U = _t(x), _t(u)
        fsimg.fsimg_fsi_newton(S.f, X, U, _t(xo), _t(uo), fsimg.fsimg_default_newton_opts(gamma=0.05))
        Xo, Uo = X.clone(), U.clone()
        st = fsimg.fsimg_fsi_newton(S.f, X, U, Xo, Uo, fsimg.fsimg_default_newton_opts(gamma=2.0))
        torch.cuda.synchronize()
    finally:
        S.close()
    assert info2["jacobians"] == 0 and st["jacobians"] == 0
    assert st["steps"] == info2["steps"]


def test_newton_mixed_precision_reaches_the_fp64_state(ctx, probs):
    """FP32 V-cycles inside FP64 FGMRES and FP64 residuals: the same
    converged time step."""
    P = probs["t3"]
    out = {}
    for prec in (fsimg.FSIMG_FP64, fsimg.FSIMG_MIXED):
        x, u, xo, uo = fsi_state(P)
        S = Fsi(ctx, P, precision=prec, rtol=1e-8)
        try:
            X, U = _t(x), _t(u)
            st = fsimg.fsimg_fsi_newton(S.f, X, U, _t(xo), _t(uo))
            torch.cuda.synchronize()
            assert st["status"] == fsimg.FSIMG_OK
            out[prec] = (X.cpu().numpy(), U.cpu().numpy())
        finally:
            S.close()
    for a, b in zip(out[fsimg.FSIMG_FP64], out[fsimg.FSIMG_MIXED]):
        assert np.abs(a - b).max() <= 1e-6 * np.abs(a).max()


def test_newton_refusals(ctx, probs):
    P = probs["t2"]
    S = Fsi(ctx, P, ale=False)
    try:
        x, u, xo, uo = (_t(a) for a in fsi_state(P))
        with pytest.raises(fsimg.FsimgError) as ei:
            fsimg.fsimg_fsi_newton(S.f, x, u, xo, uo)
        assert ei.value.status == fsimg.FSIMG_ERR_ARG
        with pytest.raises(fsimg.FsimgError) as ei:
            fsimg.fsimg_fsi_create(S.mom, None, fsi_levels(P), dict(P.params, k=0.0))
        assert ei.value.status == fsimg.FSIMG_ERR_ARG
        # an inverted fluid deformation (u_1 = -2 x_1: det F = -1) is reported
        X1 = np.stack(np.meshgrid(*P.levels[0].coords[::-1], indexing="ij")[::-1], axis=-1).reshape(-1, 2)
        ub = np.zeros_like(X1)
        ub[:, 0] = -2.0 * X1[:, 0]
        bad = _t(ub.ravel())
        res = torch.empty_like(x)
        with pytest.raises(fsimg.FsimgError) as ei:
            fsimg.fsimg_fsi_residual(S.f, x, bad, xo, uo, res)
        assert ei.value.status == fsimg.FSIMG_ERR_SINGULAR
    finally:
        S.close()


def test_successive_time_steps_match_oracle(ctx, probs):
    """Three time steps, each from the last converged state (u = u_old at
    the start: the deformation increment carries the condensation residual),
    with the Jacobian carried across steps: per step the same Newton and
    Jacobian counts as the oracle and the same state."""
    P = probs["t2"]
    xr, ur, xor, uor = fsi_state(P)
    jac = None
    x, u, xo, uo = (_t(a) for a in fsi_state(P))
    S = Fsi(ctx, P)
    try:
        for step in range(3):
            if step:
                xor, uor = xr.copy(), ur.copy()
                xo.copy_(x)
                uo.copy_(u)
            xr, ur, info, jac = _oracle_newton(P, 0.05, state=(xr, ur, xor, uor), jac=jac)
            st = fsimg.fsimg_fsi_newton(S.f, x, u, xo, uo, fsimg.fsimg_default_newton_opts(gamma=0.05))
            torch.cuda.synchronize()
            assert st["status"] == fsimg.FSIMG_OK and info["status"] == "ok"
            assert (st["steps"], st["jacobians"]) == (info["steps"], info["jacobians"]), step
            assert np.abs(x.cpu().numpy() - xr).max() <= 1e-7 * np.abs(xr).max()
            assert np.abs(u.cpu().numpy() - ur).max() <= 1e-7 * np.abs(ur).max()
    finally:
        S.close()


def test_c2_full_size_sampled_rows_match_oracle(ctx):
    """3D 32^3 (the size and launch configuration `bench.py --newton` times,
    mixed precision): residual rows and Jacobian rows (finest and first
    coarse level) at sampled fluid, solid and interface nodes against the
    oracle assembled over the cells around them; then one GPU Newton time
    step, whose final state the oracle's own residual confirms at those rows."""
    from oracle.fsi import cells_of_nodes, element_subset
    P = config_problem("c2", seed=0)
    d = P.dim
    lev0 = P.levels[0]
    rng = np.random.default_rng(12)
    ns, nf = lev0.node_solid.astype(bool), lev0.node_fluid.astype(bool)
    nodes = np.concatenate([rng.choice(np.nonzero(ns & ~nf)[0], 6, replace=False),
                            rng.choice(np.nonzero(ns & nf)[0], 6, replace=False),
                            rng.choice(np.nonzero(nf & ~ns)[0], 12, replace=False)])
    S = Fsi(ctx, P, precision=fsimg.FSIMG_MIXED, rtol=1e-8)
    try:
        x, u, xo, uo = _perturbed(P, 4)
        m0 = Mesh(lev0)
        sub = element_subset(m0, cells_of_nodes(m0, nodes))
        ref = newton_residual(sub, P.params, x, u, xo, uo, lev0.systems["mom"].dirichlet)
        res = torch.empty(x.size, device=DEV, dtype=torch.float64)
        fsimg.fsimg_fsi_residual(S.f, _t(x), _t(u), _t(xo), _t(uo), res)
        rows = (nodes[:, None] * (d + 1) + np.arange(d + 1)).ravel()
        got = res.cpu().numpy()[rows]
        assert np.abs(got - ref[rows]).max() <= 1e-12 * np.abs(ref[rows]).max()
        # Jacobian rows on levels 0 and 1
        fsimg.fsimg_fsi_jacobian(S.f, _t(x), _t(u), _t(xo), _t(uo))
        st = [x, u, xo, uo]
        meshes = [m0, Mesh(P.levels[1])]
        for l in (0, 1):
            lv = P.levels[l]
            if l == 1:
                st = [inject(meshes[0], meshes[1], a, c) for a, c in zip(st, (d + 1, d, d + 1, d))]
                nl = np.unique(rng.choice(lv.nnodes, 24, replace=False))
            else:
                nl = nodes
            subl = element_subset(meshes[l], cells_of_nodes(meshes[l], nl))
            A = lv.systems["mom"]
            vals = jacobian_bsr(subl, P.params, *st, A.rowptr, A.colind, A.dirichlet)
            J = to_csr(type("M", (), dict(rowptr=A.rowptr, colind=A.colind, vals=vals, b=d + 1)))
            z = rng.standard_normal(J.shape[0])
            y = torch.empty(z.size, device=DEV, dtype=torch.float64)
            fsimg.fsimg_level_apply(S.mom, l, fsimg.FSIMG_FP64, _t(z), y)
            torch.cuda.synchronize()
            rl = (nl[:, None] * (d + 1) + np.arange(d + 1)).ravel()
            yr = (J @ z)[rl]
            assert np.abs(y.cpu().numpy()[rl] - yr).max() <= 1e-12 * np.abs(yr).max(), l
        # one Newton time step from the seeded state
        x0, u0, xo0, uo0 = fsi_state(P)
        X, U = _t(x0), _t(u0)
        stn = fsimg.fsimg_fsi_newton(S.f, X, U, _t(xo0), _t(uo0))
        torch.cuda.synchronize()
        assert stn["status"] == fsimg.FSIMG_OK
        xf, uf = X.cpu().numpy(), U.cpu().numpy()
        rf = newton_residual(sub, P.params, xf, uf, xo0, uo0, lev0.systems["mom"].dirichlet)
        assert np.abs(rf[rows]).max() <= 1e-7 * stn["res0"]
    finally:
        S.close()


def test_jacobian_on_a_general_block_pattern(ctx, probs):
    """A finest-level pattern that is not exactly the Q2 stencil (one extra
    block outside it) takes the search path for block positions: the result
    still equals the oracle's, and the extra block stays zero."""
    P = probs["t2"]
    d, b = P.dim, P.dim + 1
    levels = level_dicts(P, "mom")
    L0 = dict(levels[0])
    rp, ci, vals = L0["rowptr"], L0["colind"], L0["vals"]
    far = P.levels[0].nnodes - 1
    assert far not in ci[rp[0]:rp[1]]
    L0["colind"] = np.insert(ci, rp[1], far).astype(np.int32)
    L0["vals"] = np.insert(vals, rp[1], 0.0, axis=0)
    L0["rowptr"] = np.concatenate([rp[:1], rp[1:] + 1]).astype(np.int32)
    levels[0] = L0
    o = fsimg.fsimg_default_opts(precision=fsimg.FSIMG_FP64)
    mom = fsimg.fsimg_hier_create(ctx, levels, o)
    f = fsimg.fsimg_fsi_create(mom, None, fsi_levels(P), P.params)
    try:
        x, u, xo, uo = _perturbed(P, 5)
        fsimg.fsimg_fsi_jacobian(f, _t(x), _t(u), _t(xo), _t(uo))
        A = P.levels[0].systems["mom"]
        ref_vals = jacobian_bsr(Mesh(P.levels[0]), P.params, x, u, xo, uo, L0["rowptr"], L0["colind"],
                                A.dirichlet)
        J = to_csr(type("M", (), dict(rowptr=L0["rowptr"], colind=L0["colind"], vals=ref_vals, b=b)))
        rng = np.random.default_rng(6)
        z = rng.standard_normal(J.shape[0])
        y = torch.empty(z.size, device=DEV, dtype=torch.float64)
        fsimg.fsimg_level_apply(mom, 0, fsimg.FSIMG_FP64, _t(z), y)
        torch.cuda.synchronize()
        ref = J @ z
        assert np.abs(y.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
        # the extra block contributes nothing: a vector supported on the far node
        z2 = np.zeros(J.shape[0])
        z2[far * b:(far + 1) * b] = 1.0
        fsimg.fsimg_level_apply(mom, 0, fsimg.FSIMG_FP64, _t(z2), y)
        torch.cuda.synchronize()
        assert np.all(y.cpu().numpy()[:b] == 0.0)
    finally:
        fsimg.fsimg_fsi_destroy(f)
        fsimg.fsimg_hier_destroy(mom)


@pytest.mark.parametrize("tolerances", ["same", "mixed"])
def test_served_newton_requests_equal_solo_runs(ctx, probs, tolerances):
    """Three Newton requests (2D and 3D, different seeds) served together for
    two time steps each, their momentum and ALE solves batched (per distinct
    tolerance when the requests ask for different momentum / ALE
    tolerances): every final state is bitwise the one fsimg_fsi_newton gives
    the request alone over the same two time steps, with the same Newton and
    Jacobian counts."""
    Ps = [probs["t2"], config_problem("t2", seed=1), probs["t3"]]
    opts = fsimg.fsimg_default_opts(precision=fsimg.FSIMG_MIXED)
    if tolerances == "same":
        nall = [fsimg.fsimg_default_newton_opts()] * 3
    else:
        nall = [fsimg.fsimg_default_newton_opts(),
                fsimg.fsimg_default_newton_opts(lin_rtol=1e-4, ale_rtol=1e-4, atol=1e-8, max_steps=40),
                fsimg.fsimg_default_newton_opts(ale_rtol=1e-6, max_steps=40)]
    solo = []
    for P, nopts in zip(Ps, nall):
        mom = fsimg.fsimg_hier_create(ctx, level_dicts(P, "mom"), opts)
        ale = fsimg.fsimg_hier_create(ctx, level_dicts(P, "ale"), opts)
        f = fsimg.fsimg_fsi_create(mom, ale, fsi_levels(P), P.params)
        try:
            x, u, xo, uo = (_t(a) for a in fsi_state(P))
            sts = []
            for t in range(2):
                if t:
                    xo.copy_(x)
                    uo.copy_(u)
                sts.append(fsimg.fsimg_fsi_newton(f, x, u, xo, uo, nopts))
            torch.cuda.synchronize()
            solo.append((x.cpu().numpy(), u.cpu().numpy(), sts))
        finally:
            fsimg.fsimg_fsi_destroy(f)
            fsimg.fsimg_hier_destroy(mom)
            fsimg.fsimg_hier_destroy(ale)
    srv = fsimg.fsimg_server_create(ctx, opts)
    try:
        datas = [fsimg.NewtonRequestData(level_dicts(P, "mom"), level_dicts(P, "ale"), fsi_levels(P),
                                         P.params, *fsi_state(P)) for P in Ps]
        ids = [fsimg.fsimg_server_submit_newton(srv, dd, 2, no) for dd, no in zip(datas, nall)]
        for _ in range(200):
            active, queued = fsimg.fsimg_server_step(srv)
            if active == 0 and queued == 0:
                break
        assert active == 0 and queued == 0
        for P, rid, (xs, us, sts) in zip(Ps, ids, solo):
            assert fsimg.fsimg_server_request_status(srv, rid) == fsimg.FSIMG_OK
            n = P.levels[0].nnodes
            xm, xa = fsimg.fsimg_server_result(srv, rid, n * (P.dim + 1), n * P.dim)
            np.testing.assert_array_equal(xm, xs)
            np.testing.assert_array_equal(xa, us)
            acc = fsimg.fsimg_server_newton_stats(srv, rid)
            assert acc["steps"] == sum(s["steps"] for s in sts)
            assert acc["jacobians"] == sum(s["jacobians"] for s in sts)
            assert acc["lin_iters_mom"] == sum(s["lin_iters_mom"] for s in sts)
            assert acc["lin_iters_ale"] == sum(s["lin_iters_ale"] for s in sts)
    finally:
        fsimg.fsimg_server_destroy(srv)


@pytest.mark.parametrize("name", ["t2", "t3"])
def test_inexact_momentum_solves_reach_the_same_time_step(ctx, probs, name):
    """With the paper's setting (each momentum solve reduces the error by
    1e-4, Newton stops at a relative or absolute 1e-8, Sec. 5.5) the loop
    converges to the oracle's time step (solved with exact linear solves) to
    within the Newton tolerance."""
    P = probs[name]
    xr, ur, info, _ = _oracle_newton(P, 0.05)
    x, u, xo, uo = fsi_state(P)
    S = Fsi(ctx, P, rtol=1e-8)
    try:
        X, U = _t(x), _t(u)
        st = fsimg.fsimg_fsi_newton(S.f, X, U, _t(xo), _t(uo),
                                    fsimg.fsimg_default_newton_opts(lin_rtol=1e-4, atol=1e-8, max_steps=40))
        torch.cuda.synchronize()
    finally:
        S.close()
    assert st["status"] == fsimg.FSIMG_OK
    assert st["res"] <= max(1e-8 * st["res0"], 1e-8)
    assert np.abs(X.cpu().numpy() - xr).max() <= 1e-6 * np.abs(xr).max()
    assert np.abs(U.cpu().numpy() - ur).max() <= 1e-6 * np.abs(ur).max()


@pytest.mark.parametrize("variant", ["block_patches", "ilu"])
def test_newton_with_other_momentum_smoothers(ctx, probs, variant):
    """The Newton loop does not depend on the smoother of the momentum
    hierarchy: with 2 x 2 block Vanka patches or the block ILU(0) smoother it
    reaches the oracle's time step (exact linear solves) to within the Newton
    tolerance."""
    P = probs["t2"]
    xr, ur, info, _ = _oracle_newton(P, 0.05)
    over = (dict(vanka_patches=fsimg.FSIMG_PATCH_BLOCK) if variant == "block_patches"
            else dict(smoother=fsimg.FSIMG_SMOOTHER_ILU))
    o = fsimg.fsimg_default_opts(precision=fsimg.FSIMG_FP64, rtol=1e-10, **over)
    mom = fsimg.fsimg_hier_create(ctx, level_dicts(P, "mom"), o)
    ale = fsimg.fsimg_hier_create(ctx, level_dicts(P, "ale"), fsimg.fsimg_default_opts(rtol=1e-10))
    f = fsimg.fsimg_fsi_create(mom, ale, fsi_levels(P), P.params)
    try:
        X, U, Xo, Uo = (_t(a) for a in fsi_state(P))
        st = fsimg.fsimg_fsi_newton(f, X, U, Xo, Uo)
        torch.cuda.synchronize()
    finally:
        fsimg.fsimg_fsi_destroy(f)
        fsimg.fsimg_hier_destroy(mom)
        fsimg.fsimg_hier_destroy(ale)
    assert st["status"] == fsimg.FSIMG_OK
    assert (st["steps"], st["jacobians"]) == (info["steps"], info["jacobians"])
    assert np.abs(X.cpu().numpy() - xr).max() <= 1e-7 * np.abs(xr).max()
    assert np.abs(U.cpu().numpy() - ur).max() <= 1e-7 * np.abs(ur).max()
