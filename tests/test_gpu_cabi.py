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


def _write_newton(P, d):
    from paper_1904_02401_amd.problems import fsi_state
    mom, ale = level_dicts(P, "mom"), level_dicts(P, "ale")
    with open(os.path.join(d, "meta.txt"), "w") as f:
        f.write(f"{len(mom)} {P.dim}\n")
        for l, (lm, la, lev) in enumerate(zip(mom, ale, P.levels)):
            cells = list(lm["cells"]) + [1] * (3 - len(lm["cells"]))
            f.write(f"{cells[0]} {cells[1]} {cells[2]} {lm['rowptr'].size - 1} {lm['colind'].size} "
                    f"{la['colind'].size}\n")
            for tag, L in (("M", lm), ("A", la)):
                np.ascontiguousarray(L["rowptr"], dtype=np.int32).tofile(os.path.join(d, f"{tag}{l}_rowptr.bin"))
                np.ascontiguousarray(L["colind"], dtype=np.int32).tofile(os.path.join(d, f"{tag}{l}_colind.bin"))
                np.ascontiguousarray(L["vals"], dtype=np.float64).tofile(os.path.join(d, f"{tag}{l}_vals.bin"))
                np.ascontiguousarray(L["dirichlet"], dtype=np.uint8).tofile(
                    os.path.join(d, f"{tag}{l}_dirichlet.bin"))
            for a in range(P.dim):
                np.ascontiguousarray(lev.coords[a], dtype=np.float64).tofile(os.path.join(d, f"G{l}_c{a}.bin"))
            np.ascontiguousarray(lev.cell_solid, dtype=np.uint8).tofile(os.path.join(d, f"G{l}_solid.bin"))
    p = P.params
    np.array([p[k] for k in ("rho_f", "nu_f", "rho_s", "mu_s", "lambda_s", "k", "theta", "alpha0")],
             dtype=np.float64).tofile(os.path.join(d, "phys.bin"))
    vecs = fsi_state(P)
    for name, v in zip(("x", "u", "xo", "uo"), vecs):
        np.ascontiguousarray(v, dtype=np.float64).tofile(os.path.join(d, f"{name}.bin"))
    return mom, ale, vecs


@pytest.mark.parametrize("precision", [fsimg.FSIMG_FP64, fsimg.FSIMG_MIXED])
@pytest.mark.parametrize("name", ["t2", "t3"])
def test_plain_c_newton_client_matches_binding(tmp_path, name, precision):
    """tests/cabi_newton.c runs one Newton time step through
    include/fsimg_newton.h from plain C; the new state equals the Python
    binding's bit for bit."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02401_amd.build import CABI_NEWTON
    from paper_1904_02401_amd.problems import fsi_levels
    if not os.path.exists(CABI_NEWTON):
        build_cabi_driver()
    P = config_problem(name, seed=0)
    mom, ale, vecs = _write_newton(P, str(tmp_path))
    r = subprocess.run([CABI_NEWTON, str(tmp_path), str(precision)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    status, steps, jacs = (int(v) for v in r.stdout.split())
    assert status == fsimg.FSIMG_OK and steps > 0
    xc = np.fromfile(os.path.join(str(tmp_path), "x_out.bin"), dtype=np.float64)
    uc = np.fromfile(os.path.join(str(tmp_path), "u_out.bin"), dtype=np.float64)
    ctx = fsimg.fsimg_ctx_create(0)
    try:
        o = fsimg.fsimg_default_opts(precision=precision)
        hm = fsimg.fsimg_hier_create(ctx, mom, o)
        ha = fsimg.fsimg_hier_create(ctx, ale, o)
        f = fsimg.fsimg_fsi_create(hm, ha, fsi_levels(P), P.params)
        try:
            x, u, xo, uo = (torch.tensor(v, device="cuda:0") for v in vecs)
            st = fsimg.fsimg_fsi_newton(f, x, u, xo, uo)
            torch.cuda.synchronize()
        finally:
            fsimg.fsimg_fsi_destroy(f)
            fsimg.fsimg_hier_destroy(hm)
            fsimg.fsimg_hier_destroy(ha)
    finally:
        fsimg.fsimg_ctx_destroy(ctx)
    np.testing.assert_array_equal(xc, x.cpu().numpy())
    np.testing.assert_array_equal(uc, u.cpu().numpy())
    assert (st["steps"], st["jacobians"]) == (steps, jacs)
