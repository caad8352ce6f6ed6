"""Block ILU(0) smoother on the GPU against the FP64 oracle (oracle.ilu):
the factors element by element, one smoothing step, one V-cycle, solves to
1e-8 with the oracle's iteration counts, the mixed path, the footprint, and
the calls that refuse ILU hierarchies."""
import numpy as np
import pytest

from fsigen import config_problem
from oracle import BlockILU, Hierarchy, ilu_sweep, to_csr, vcycle
from oracle.step import solve_system

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1904_02401_amd import fsimg  # noqa: E402
from paper_1904_02401_amd.problems import level_dicts  # noqa: E402

DEV = "cuda:0"
ILU = dict(smoother=fsimg.FSIMG_SMOOTHER_ILU)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fsimg.fsimg_ctx_create(0)
    yield c
    fsimg.fsimg_ctx_destroy(c)


@pytest.fixture(scope="module")
def probs():
    return {name: config_problem(name, seed=0) for name in ("t2", "t3", "c1")}


class Hier:
    def __init__(self, ctx, P, system, **opts):
        self.h = fsimg.fsimg_hier_create(ctx, level_dicts(P, system), fsimg.fsimg_default_opts(**opts))

    def __enter__(self):
        return self.h

    def __exit__(self, *a):
        fsimg.fsimg_hier_destroy(self.h)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("name,system", [("t2", "mom"), ("t2", "ale"), ("t3", "mom"), ("t3", "ale")])
def test_ilu_factors_match_oracle(ctx, probs, name, system):
    P = probs[name]
    m = P.levels[0].systems[system]
    ref = BlockILU(m).F
    with Hier(ctx, P, system, **ILU) as h:
        fsimg.fsimg_factor(h)
        got = fsimg.fsimg_ilu_factors(h, 0, m.colind.size, m.b)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < 1e-12, err


@pytest.mark.parametrize("name,system", [("t2", "mom"), ("t3", "mom"), ("t3", "ale")])
def test_ilu_step_fp64_matches_oracle(ctx, probs, name, system):
    P = probs[name]
    m = P.levels[0].systems[system]
    A = to_csr(m)
    mask = m.dirichlet.astype(bool)
    rng = np.random.default_rng(31)
    b = rng.standard_normal(A.shape[0])
    b[mask] = 0.0
    x0 = rng.standard_normal(A.shape[0]) * 0.1
    ref = ilu_sweep(A, b, x0, BlockILU(m), mask)
    with Hier(ctx, P, system, **ILU) as h:
        fsimg.fsimg_factor(h)
        x = torch.tensor(x0, device=DEV)
        fsimg.fsimg_ilu_step(h, 0, fsimg.FSIMG_FP64, torch.tensor(b, device=DEV), x)
        torch.cuda.synchronize()
        got = x.cpu().numpy()
    assert _rel(got - x0, ref - x0) < 1e-11
    assert np.array_equal(got[mask], x0[mask])


def test_ilu_step_mixed_close_to_fp64(ctx, probs):
    P = probs["t3"]
    m = P.levels[0].systems["mom"]
    A = to_csr(m)
    mask = m.dirichlet.astype(bool)
    rng = np.random.default_rng(32)
    b = rng.standard_normal(A.shape[0])
    b[mask] = 0.0
    ref = ilu_sweep(A, b, np.zeros_like(b), BlockILU(m), mask)
    with Hier(ctx, P, "mom", precision=fsimg.FSIMG_MIXED, **ILU) as h:
        fsimg.fsimg_factor(h)
        x = torch.zeros(A.shape[0], device=DEV, dtype=torch.float32)
        fsimg.fsimg_ilu_step(h, 0, fsimg.FSIMG_MIXED, torch.tensor(b, device=DEV, dtype=torch.float32), x)
        torch.cuda.synchronize()
        assert _rel(x.double().cpu().numpy(), ref) < 1e-4


@pytest.mark.parametrize("name", ["t2", "t3"])
def test_ilu_vcycle_fp64_matches_oracle(ctx, probs, name):
    P = probs[name]
    mats = P.system("mom")
    cells = [lv.cells for lv in P.levels]
    Ho = Hierarchy(mats, cells, smoother="ilu")
    rng = np.random.default_rng(33)
    r = rng.standard_normal(mats[0].nrows * mats[0].b)
    r[mats[0].dirichlet.astype(bool)] = 0.0
    with Hier(ctx, P, "mom", **ILU) as h:
        fsimg.fsimg_factor(h)
        z = torch.empty(r.size, device=DEV, dtype=torch.float64)
        fsimg.fsimg_vcycle(h, fsimg.FSIMG_FP64, torch.tensor(r, device=DEV), z)
        torch.cuda.synchronize()
        assert _rel(z.cpu().numpy(), vcycle(Ho, r)) < 1e-10


@pytest.mark.parametrize("precision", [fsimg.FSIMG_FP64, fsimg.FSIMG_MIXED])
@pytest.mark.parametrize("name,system", [("t2", "mom"), ("t3", "mom"), ("t3", "ale"), ("c1", "mom")])
def test_ilu_solve_converges_like_the_oracle(ctx, probs, name, system, precision):
    P = probs[name]
    mats = P.system(system)
    cells = [lv.cells for lv in P.levels]
    Ho = Hierarchy(mats, cells, smoother="ilu")
    _, info, _ = solve_system(mats, cells, P.rhs[system], H=Ho, rtol=1e-8)
    with Hier(ctx, P, system, precision=precision, **ILU) as h:
        fsimg.fsimg_factor(h)
        b = torch.tensor(P.rhs[system], device=DEV)
        x = torch.zeros_like(b)
        st = fsimg.fsimg_solve(h, b, x)
        torch.cuda.synchronize()
    A = to_csr(mats[0])
    res = P.rhs[system] - A @ x.cpu().numpy()
    res[mats[0].dirichlet.astype(bool)] = 0.0
    assert st["status"] == fsimg.FSIMG_OK
    assert np.linalg.norm(res) <= 1.01e-8 * np.linalg.norm(P.rhs[system])
    assert abs(st["iters"] - info["iters"]) <= 1


def test_ilu_footprint_and_refactor(ctx, probs):
    P = probs["t3"]
    opts = fsimg.fsimg_default_opts(precision=fsimg.FSIMG_MIXED, **ILU)
    levels = level_dicts(P, "mom")
    need = fsimg.fsimg_hier_footprint(levels, opts)
    before = fsimg.fsimg_ctx_bytes_in_use(ctx)
    h = fsimg.fsimg_hier_create(ctx, levels, opts)
    try:
        assert fsimg.fsimg_ctx_bytes_in_use(ctx) - before <= need
        fsimg.fsimg_factor(h)
        held = fsimg.fsimg_ctx_bytes_in_use(ctx)
        m = P.levels[0].systems["mom"]
        f1 = fsimg.fsimg_ilu_factors(h, 0, m.colind.size, m.b)
        fsimg.fsimg_factor(h)  # refactoring allocates nothing and reproduces the factors
        assert fsimg.fsimg_ctx_bytes_in_use(ctx) == held
        assert np.array_equal(f1, fsimg.fsimg_ilu_factors(h, 0, m.colind.size, m.b))
    finally:
        fsimg.fsimg_hier_destroy(h)
    assert fsimg.fsimg_ctx_bytes_in_use(ctx) == before


def test_calls_that_refuse_ilu_hierarchies(ctx, probs):
    P = probs["t2"]
    with Hier(ctx, P, "mom", **ILU) as hi, Hier(ctx, P, "mom") as hv:
        fsimg.fsimg_factor(hi)
        fsimg.fsimg_factor(hv)
        b = torch.tensor(P.rhs["mom"], device=DEV)
        x = torch.zeros_like(b)
        with pytest.raises(fsimg.FsimgError) as ei:
            fsimg.fsimg_solve_batch([hi], [b], [x])
        assert ei.value.status == fsimg.FSIMG_ERR_ARG
        with pytest.raises(fsimg.FsimgError) as ei:
            fsimg.fsimg_vanka_step(hi, 0, fsimg.FSIMG_FP64, b, x)
        assert ei.value.status == fsimg.FSIMG_ERR_STATE
        with pytest.raises(fsimg.FsimgError) as ei:
            fsimg.fsimg_ilu_step(hv, 0, fsimg.FSIMG_FP64, b, x)
        assert ei.value.status == fsimg.FSIMG_ERR_STATE
        fsimg.fsimg_hier_tune(hi)  # times the SpMV shapes only: no patch inverses exist
    with pytest.raises(fsimg.FsimgError) as ei:
        fsimg.fsimg_server_create(ctx, fsimg.fsimg_default_opts(**ILU))
    assert ei.value.status == fsimg.FSIMG_ERR_ARG


@pytest.mark.parametrize("precision", [fsimg.FSIMG_FP64, fsimg.FSIMG_MIXED])
def test_ilu_graph_replays_equal_eager_launches(ctx, probs, precision):
    """The captured level sweeps, replayed in several solves in a row (eager
    work and synchronisation between them), give bitwise the eager result."""
    P = probs["t3"]
    b = torch.tensor(P.rhs["mom"], device=DEV)
    out = {}
    for graphs in (0, 1):
        with Hier(ctx, P, "mom", precision=precision, graphs=graphs, **ILU) as h:
            fsimg.fsimg_factor(h)
            res = []
            for _ in range(3):
                x = torch.zeros_like(b)
                fsimg.fsimg_solve(h, b, x)
                torch.cuda.synchronize()
                res.append(x.cpu().numpy())
            out[graphs] = res
    for r in out[1]:
        np.testing.assert_array_equal(r, out[0][0])
    for r in out[0]:
        np.testing.assert_array_equal(r, out[0][0])
