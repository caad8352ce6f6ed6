"""Edge cases of the GPU path against the oracle: block rows longer than the
128 blocks of the unrolled SpMV sweep (a general BSR pattern, not a Q2
stencil), zero right-hand sides, and a batch that mixes a zero right-hand
side with ordinary ones."""
import numpy as np
import pytest
import scipy.sparse as sp

from fsigen import config_problem
from oracle import to_csr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1904_02401_amd import fsimg  # noqa: E402
from paper_1904_02401_amd.problems import level_dicts  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fsimg.fsimg_ctx_create(0)
    yield c
    fsimg.fsimg_ctx_destroy(c)


@pytest.fixture(scope="module")
def t3():
    return config_problem("t3", seed=0)


def _long_rows(lev, rng, extra=140, nrows_long=12):
    """Level dict with `extra` random blocks added to some rows whose dofs are
    all free (the pattern stays sorted); returns (dict, scipy CSR of it)."""
    d = dict(lev)
    b = d["block"]
    rp, ci, va = d["rowptr"], d["colind"], d["vals"].reshape(-1, b, b)
    nrows = rp.size - 1
    free = np.nonzero(d["dirichlet"].reshape(nrows, b).max(axis=1) == 0)[0]
    long_rows = set(rng.choice(free, size=nrows_long, replace=False).tolist())
    new_rp, new_ci, new_va = [0], [], []
    for r in range(nrows):
        cols = ci[rp[r]:rp[r + 1]]
        vals = va[rp[r]:rp[r + 1]]
        if r in long_rows:
            cand = np.setdiff1d(np.arange(nrows), cols)
            add = np.sort(rng.choice(cand, size=extra, replace=False))
            cols = np.concatenate([cols, add])
            vals = np.concatenate([vals, rng.standard_normal((extra, b, b))])
            order = np.argsort(cols, kind="stable")
            cols, vals = cols[order], vals[order]
        new_ci.append(cols)
        new_va.append(vals)
        new_rp.append(new_rp[-1] + cols.size)
    d["rowptr"] = np.asarray(new_rp, dtype=np.int32)
    d["colind"] = np.concatenate(new_ci).astype(np.int32)
    d["vals"] = np.concatenate(new_va).reshape(-1)
    n = nrows * b
    A = sp.bsr_matrix((d["vals"].reshape(-1, b, b), d["colind"], d["rowptr"]), shape=(n, n)).tocsr()
    assert np.diff(d["rowptr"]).max() > 128
    return d, A


@pytest.mark.parametrize("system", ["mom", "ale"])
@pytest.mark.parametrize("precision", [fsimg.FSIMG_FP64, fsimg.FSIMG_MIXED])
def test_spmv_rows_longer_than_the_unrolled_sweep(ctx, t3, system, precision):
    rng = np.random.default_rng(7)
    levels = level_dicts(t3, system)
    lev0, A = _long_rows(levels[0], rng)
    h = fsimg.fsimg_hier_create(ctx, [lev0] + levels[1:],
                                fsimg.fsimg_default_opts(precision=precision))
    try:
        n = A.shape[0]
        x = rng.standard_normal(n)
        ref = A @ x
        for prec, dt, tol in ((fsimg.FSIMG_FP64, torch.float64, 1e-13),
                              (fsimg.FSIMG_MIXED, torch.float32, 2e-6)):
            if prec == fsimg.FSIMG_MIXED and precision != fsimg.FSIMG_MIXED:
                continue
            xt = torch.tensor(x, device=DEV, dtype=dt)
            y = torch.zeros_like(xt)
            fsimg.fsimg_level_apply(h, 0, prec, xt, y)
            torch.cuda.synchronize()
            got = y.double().cpu().numpy()
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            assert err <= tol, (prec, err)
            # rows of the long pattern and their neighbours individually
            rows = np.nonzero(np.diff(lev0["rowptr"]) > 128)[0]
            b = lev0["block"]
            for r in rows:
                sl = slice(r * b, (r + 1) * b)
                assert np.allclose(got[sl], ref[sl], rtol=tol * 10, atol=tol * np.abs(ref).max())
    finally:
        fsimg.fsimg_hier_destroy(h)


@pytest.mark.parametrize("precision", [fsimg.FSIMG_FP64, fsimg.FSIMG_MIXED])
def test_zero_rhs_and_mixed_batch(ctx, t3, precision):
    opts = fsimg.fsimg_default_opts(precision=precision)
    hs = [fsimg.fsimg_hier_create(ctx, level_dicts(t3, "mom"), opts) for _ in range(3)]
    try:
        for h in hs:
            fsimg.fsimg_factor(h)
        b = torch.tensor(t3.rhs["mom"], device=DEV)
        zero = torch.zeros_like(b)
        # alone: b = 0 and x0 = 0 -> nothing to do, x stays 0
        x = torch.zeros_like(b)
        st = fsimg.fsimg_solve(hs[0], zero, x)
        torch.cuda.synchronize()
        assert st["iters"] == 0 and st["status"] == fsimg.FSIMG_OK
        assert float(x.abs().max()) == 0.0
        # in a batch with two ordinary right-hand sides
        xs = [torch.zeros_like(b) for _ in hs]
        sts = fsimg.fsimg_solve_batch(hs, [b, zero, b], xs)
        torch.cuda.synchronize()
        assert sts[1]["iters"] == 0 and float(xs[1].abs().max()) == 0.0
        np.testing.assert_array_equal(xs[0].cpu().numpy(), xs[2].cpu().numpy())
        m = t3.levels[0].systems["mom"]
        A = to_csr(m)
        r = t3.rhs["mom"] - A @ xs[0].cpu().numpy()
        r[m.dirichlet.astype(bool)] = 0.0
        assert np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(t3.rhs["mom"])
    finally:
        for h in hs:
            fsimg.fsimg_hier_destroy(h)
