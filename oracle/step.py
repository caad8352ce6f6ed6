"""The linear solve inside one approximate Newton step (Sec. 4.2): the reduced
Jacobian (eq. REDUCEDMATRIX) splits into

  (1) the coupled momentum system in (p, v), eq. problem:1,
  (2) the deformation update on interface and solid dofs, eq. problem:2
      (one vector addition; optionally also solved as a mass-matrix system),
  (3) the ALE extension E_f du_f = b5 - E_i du_i, eq. problem:3.

(1) and (3) are solved by FGMRES preconditioned with the multigrid V-cycle
(Vanka smoother).  For (3) the interface and solid values du come from (2):
they enter as the initial guess at the identity rows, so the first residual
at the fluid rows is exactly b5 - E_i du_i."""
import numpy as np

from .deform import deform_update
from .fgmres import fgmres
from .mg import Hierarchy, vcycle


def solve_system(mats, cells, b, x0=None, rtol=1e-8, restart=20, maxiter=500, omega=0.8,
                 nu_pre=2, nu_post=2, weighting="plain", H=None):
    if H is None:
        H = Hierarchy(mats, cells, omega=omega, nu_pre=nu_pre, nu_post=nu_post,
                      weighting=weighting)
    lev = H.levels[0]
    x0 = np.zeros_like(b) if x0 is None else x0
    x, info = fgmres(lev.A, b, x0, lambda v: vcycle(H, v), lev.mask, rtol=rtol,
                     restart=restart, maxiter=maxiter)
    return x, info, H


def newton_step_solve(problem, rtol=1e-8, mass_solve=False, **kw):
    """Returns dict(dv (momentum solution, [n*(d+1)]), du (ALE solution incl.
    interface/solid values, [n*d]), du_mass (optional), info_mom, info_ale)."""
    d = problem.dim
    cells = [lev.cells for lev in problem.levels]
    out = {}
    x, info, _ = solve_system(problem.system("mom"), cells, problem.rhs["mom"], rtol=rtol, **kw)
    out["dv"], out["info_mom"] = x, info
    fine = problem.levels[0]
    nn = fine.nnodes
    dvel = x.reshape(nn, d + 1)[:, 1:]
    p = problem.params
    lift = deform_update(fine.node_solid.astype(bool), p["k"], p["theta"], dvel)
    if mass_solve:
        mats = problem.system("mass")
        from .linalg import to_csr
        M = to_csr(mats[0])
        rhs = M @ (p["k"] * p["theta"] * dvel).ravel()
        xm, im, _ = solve_system(mats, cells, rhs, rtol=rtol, **kw)
        out["du_mass"], out["info_mass"] = xm, im
    xa, ia, _ = solve_system(problem.system("ale"), cells, problem.rhs["ale"], x0=lift.ravel(),
                             rtol=rtol, **kw)
    out["du"], out["info_ale"], out["lift"] = xa, ia, lift.ravel()
    return out
