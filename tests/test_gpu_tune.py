"""Launch-shape tuning: shapes change no result bit, the tuner records a
value for every key it measured, and the JSON cache round-trips."""
import json

import numpy as np
import pytest

from fsigen import batch_instance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1904_02401_amd import fsimg  # noqa: E402
from paper_1904_02401_amd.problems import level_dicts  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def insts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return [batch_instance(i, sizes=(8, 12)) for i in range(3)]


def _solve_all(ctx, insts, precision, system="mom"):
    opts = fsimg.fsimg_default_opts(precision=precision)
    hs = [fsimg.fsimg_hier_create(ctx, level_dicts(P, system), opts) for P in insts]
    try:
        for h in hs:
            fsimg.fsimg_factor(h)
        bs = [torch.tensor(P.rhs[system], device=DEV) for P in insts]
        xs = [torch.zeros_like(b) for b in bs]
        fsimg.fsimg_solve_batch(hs, bs, xs)
        x1 = torch.zeros_like(bs[0])
        fsimg.fsimg_solve(hs[0], bs[0], x1)
        torch.cuda.synchronize()
        return [x.cpu().numpy() for x in xs] + [x1.cpu().numpy()]
    finally:
        for h in hs:
            fsimg.fsimg_hier_destroy(h)


@pytest.mark.parametrize("precision", [fsimg.FSIMG_FP64, fsimg.FSIMG_MIXED])
def test_shapes_do_not_change_results(insts, precision):
    word = 8 if precision == fsimg.FSIMG_FP64 else 4
    ctx = fsimg.fsimg_ctx_create(0)
    try:
        ref = _solve_all(ctx, insts, precision)
        for rows, ppw in ((2, 1), (4, 3)):
            for P in insts:
                for lev in P.levels:
                    m = lev.systems["mom"]
                    for w in (word, 8):
                        fsimg.fsimg_tune_set(ctx, fsimg.FSIMG_TUNE_SPMV_ROWS, m.b, w, m.nrows, rows)
                    npatch = max(int(np.prod(lev.cells)), 1)
                    fsimg.fsimg_tune_set(ctx, fsimg.FSIMG_TUNE_VANKA_PPW, 108, word, npatch, ppw)
            got = _solve_all(ctx, insts, precision)
            for a, b in zip(got, ref):
                np.testing.assert_array_equal(a, b)
    finally:
        fsimg.fsimg_ctx_destroy(ctx)


def test_tuner_and_cache(insts, tmp_path):
    ctx = fsimg.fsimg_ctx_create(0)
    try:
        opts = fsimg.fsimg_default_opts(precision=fsimg.FSIMG_MIXED)
        P = insts[0]
        h = fsimg.fsimg_hier_create(ctx, level_dicts(P, "mom"), opts)
        try:
            with pytest.raises(fsimg.FsimgError):
                fsimg.fsimg_hier_tune(h)  # not factored yet
            fsimg.fsimg_factor(h)
            fsimg.fsimg_hier_tune(h)
        finally:
            fsimg.fsimg_hier_destroy(h)
        path = str(tmp_path / "tune.json")
        fsimg.fsimg_tune_save(ctx, path)
        doc = json.load(open(path))
        kinds = {(e["kind"], e["key"], e["word"]) for e in doc["entries"]}
        m = P.levels[0].systems["mom"]
        assert (fsimg.FSIMG_TUNE_SPMV_ROWS, m.b, 4) in kinds      # V-cycle SpMV
        assert (fsimg.FSIMG_TUNE_SPMV_ROWS, m.b, 8) in kinds      # outer FP64 SpMV
        assert (fsimg.FSIMG_TUNE_VANKA_PPW, 108, 4) in kinds
        for e in doc["entries"]:
            assert e["value"] in ((1, 2, 4) if e["kind"] == 0 else range(1, 10))
        # a fresh context takes the file; the values in use agree
        ctx2 = fsimg.fsimg_ctx_create(0)
        try:
            fsimg.fsimg_tune_load(ctx2, path)
            for e in doc["entries"]:
                size = 1 << e["bucket"]
                assert (fsimg.fsimg_tune_get(ctx2, e["kind"], e["key"], e["word"], size) ==
                        fsimg.fsimg_tune_get(ctx, e["kind"], e["key"], e["word"], size) == e["value"])
            # another architecture's file is refused and changes nothing
            doc2 = dict(doc, arch="gfx000")
            bad = str(tmp_path / "other.json")
            json.dump(doc2, open(bad, "w"))
            with pytest.raises(fsimg.FsimgError):
                fsimg.fsimg_tune_load(ctx2, bad)
            # out-of-range values are refused
            with pytest.raises(fsimg.FsimgError):
                fsimg.fsimg_tune_set(ctx2, fsimg.FSIMG_TUNE_SPMV_ROWS, 4, 4, 1000, 3)
            with pytest.raises(fsimg.FsimgError):
                fsimg.fsimg_tune_set(ctx2, fsimg.FSIMG_TUNE_VANKA_PPW, 108, 4, 1000, 10)
        finally:
            fsimg.fsimg_ctx_destroy(ctx2)
    finally:
        fsimg.fsimg_ctx_destroy(ctx)


@pytest.mark.parametrize("precision", [fsimg.FSIMG_FP64, fsimg.FSIMG_MIXED])
def test_schedule_timing(insts, precision):
    """fsimg_tune_schedule times a V-cycle under each Vanka schedule and names
    the fastest; block patches admit only the gather; the context holds no
    memory afterwards."""
    ctx = fsimg.fsimg_ctx_create(0)
    try:
        levels = level_dicts(insts[1], "mom")
        ms, best = fsimg.fsimg_tune_schedule(ctx, levels, fsimg.fsimg_default_opts(precision=precision), reps=3)
        assert all(t > 0 for t in ms), ms
        assert best == int(np.argmin(ms))
        assert fsimg.fsimg_ctx_bytes_in_use(ctx) == 0
        ms, best = fsimg.fsimg_tune_schedule(
            ctx, levels, fsimg.fsimg_default_opts(precision=precision, vanka_patches=fsimg.FSIMG_PATCH_BLOCK),
            reps=2)
        assert ms[0] > 0 and ms[1] == -1 and ms[2] == -1 and best == fsimg.FSIMG_VANKA_GATHER, ms
    finally:
        fsimg.fsimg_ctx_destroy(ctx)
