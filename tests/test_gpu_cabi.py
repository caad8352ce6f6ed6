"""The C ABI from plain C: tests/cabi_driver.c (no Python, no torch in its
process) reads a hierarchy from files, solves it with libfsimg.so and writes
x; the result must equal the Python binding's solve of the same inputs bit
for bit and meet the FP64 residual bound."""
import os
import subprocess

import numpy as np
import pytest

from fsigen import config_problem
from oracle import to_csr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1904_02401_amd import fsimg  # noqa: E402
from paper_1904_02401_amd.build import CABI_DRIVER, build_cabi_driver  # noqa: E402
from paper_1904_02401_amd.problems import level_dicts  # noqa: E402


def _write(P, system, d):
    levels = level_dicts(P, system)
    with open(os.path.join(d, "meta.txt"), "w") as f:
        f.write(f"{len(levels)} {levels[0]['dim']} {levels[0]['block']}\n")
        for l, lv in enumerate(levels):
            cells = list(lv["cells"]) + [1] * (3 - len(lv["cells"]))
            nrows = lv["rowptr"].size - 1
            f.write(f"{cells[0]} {cells[1]} {cells[2]} {nrows} {lv['colind'].size}\n")
            np.ascontiguousarray(lv["rowptr"], dtype=np.int32).tofile(os.path.join(d, f"L{l}_rowptr.bin"))
            np.ascontiguousarray(lv["colind"], dtype=np.int32).tofile(os.path.join(d, f"L{l}_colind.bin"))
            np.ascontiguousarray(lv["vals"], dtype=np.float64).tofile(os.path.join(d, f"L{l}_vals.bin"))
            np.ascontiguousarray(lv["dirichlet"], dtype=np.uint8).tofile(
                os.path.join(d, f"L{l}_dirichlet.bin"))
            np.ascontiguousarray(lv["cell_class"], dtype=np.uint8).tofile(
                os.path.join(d, f"L{l}_cellclass.bin"))
    np.ascontiguousarray(P.rhs[system], dtype=np.float64).tofile(os.path.join(d, "rhs.bin"))
    return levels


@pytest.mark.parametrize("precision", [fsimg.FSIMG_FP64, fsimg.FSIMG_MIXED])
@pytest.mark.parametrize("name,system", [("t2", "mom"), ("t3", "mom"), ("t3", "ale")])
def test_plain_c_client_matches_binding(tmp_path, name, system, precision):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(CABI_DRIVER):
        build_cabi_driver()
    P = config_problem(name, seed=0)
    levels = _write(P, system, str(tmp_path))
    r = subprocess.run([CABI_DRIVER, str(tmp_path), str(precision)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    status, iters, _ = r.stdout.split()
    assert int(status) == fsimg.FSIMG_OK and int(iters) > 0
    xc = np.fromfile(os.path.join(str(tmp_path), "x.bin"), dtype=np.float64)
    # the same solve through the Python binding
    ctx = fsimg.fsimg_ctx_create(0)
    try:
        h = fsimg.fsimg_hier_create(ctx, levels, fsimg.fsimg_default_opts(precision=precision))
        try:
            fsimg.fsimg_factor(h)
            b = torch.tensor(P.rhs[system], device="cuda:0")
            x = torch.zeros_like(b)
            st = fsimg.fsimg_solve(h, b, x)
            torch.cuda.synchronize()
        finally:
            fsimg.fsimg_hier_destroy(h)
    finally:
        fsimg.fsimg_ctx_destroy(ctx)
    np.testing.assert_array_equal(xc, x.cpu().numpy())
    assert st["iters"] == int(iters)
    m = P.levels[0].systems[system]
    res = P.rhs[system] - to_csr(m) @ xc
    res[m.dirichlet.astype(bool)] = 0.0
    assert np.linalg.norm(res) <= 1.01e-8 * np.linalg.norm(P.rhs[system])
