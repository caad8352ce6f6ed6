"""Approximate Newton loop of one time step (TEST INFRASTRUCTURE ONLY).

The nonlinear residual of the theta time step in ALE coordinates (Sec. 2,
eq. aletime:2) with the solid deformation condensed into the velocity
(Sec. 3.1, eq. defgrad), its approximate Jacobian (Sec. 4.2: every derivative
with respect to the ALE deformation dropped, eq. REDUCEDMATRIX / problem:1),
and the Newton iteration of eq. newton with the Jacobian reuse rule of
Sec. 5.5 (reassemble when the rate rho_l exceeds gamma_nt) and a halving line
search (a trial state with det F <= 0 at a Gauss point counts as no
decrease).  The Newton increment of the deformation on interface and solid
nodes is k theta times the velocity increment plus the residual of the
condensation relation (eq. problem:2 with its right-hand side b6, b7), so a
time step may start from u = u_{n-1}.

Readings (the same as the input generator's matrices): inertia and convection
carry rho_f; the pressure enters the momentum rows as -k (J p F^-T, grad phi)
and the divergence row as +k (J tr(grad v F^-1), xi); the mesh-transport term
uses vbar = theta v_n + (1 - theta) v_{n-1}; the pressure is stabilised by
s_h(p, xi) = sum_K delta_K (grad p, grad xi)_K with
delta_K = alpha0 k^2 h_K^2 / (rho_f (h_K^2 + k theta nu_f)); the line search
halves omega until the max-norm of the residual decreases.

Cells are rectilinear (per-axis node coordinates) or isoparametric Q2 (node
positions: the cell is the image of the reference cell under
x(xi) = sum_i x_i N_i(xi), gradients by (dx/dxi)^-T, weights by det(dx/dxi) at
each Gauss point; h_K of the stabilisation is then the longest cell edge from
the first corner), which carries the curved cylinder of Sec. 5.

The residual is written out per element and Gauss point in plain NumPy.  The
Jacobian is *defined* as the derivative of that residual: it is taken by the
complex step (Im R(x + i h e_j) / h, exact to rounding for this analytic
residual), element by element, so no hand-derived derivative is involved.
The linear systems of the oracle Newton loop are solved directly (SuperLU).
Everything is FP64 (complex128 inside the complex step)."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .linalg import to_csr

_GP = np.array([0.5 - np.sqrt(0.15), 0.5, 0.5 + np.sqrt(0.15)])  # 3-point Gauss on [0,1]
_GW = np.array([5.0, 8.0, 5.0]) / 18.0


def _lagrange(x):
    """1D quadratic Lagrange basis on the nodes 0, 1/2, 1 and its derivative."""
    L = np.array([2 * (x - 0.5) * (x - 1), 4 * x * (1 - x), 2 * x * (x - 0.5)])
    dL = np.array([4 * x - 3, 4 - 8 * x, 4 * x - 1])
    return L, dL


def reference_tables(dim):
    """N[q, i], dN[q, i, m] on the unit cell and the weights w[q] (sum 1);
    nodes and points lexicographic with x fastest."""
    nn = 3 ** dim
    idx = np.array([[(i // 3 ** a) % 3 for a in range(dim)] for i in range(nn)])
    N = np.ones((nn, nn))
    dN = np.ones((nn, nn, dim))
    w = np.ones(nn)
    for q in range(nn):
        for a in range(dim):
            L, dL = _lagrange(_GP[idx[q, a]])
            w[q] *= _GW[idx[q, a]]
            N[q] *= L[idx[:, a]]
            for m in range(dim):
                dN[q, :, m] *= dL[idx[:, a]] if m == a else L[idx[:, a]]
    return N, dN, w


def element_nodes(cells, dim):
    """[ne, 3^d] global node numbers of every cell (lexicographic cells and
    nodes, x fastest) and the cells' integer coordinates [ne, d]."""
    nnode = [2 * c + 1 for c in cells]
    ec = np.stack(np.meshgrid(*[np.arange(c) for c in cells[::-1]], indexing="ij")[::-1],
                  axis=-1).reshape(-1, dim)
    loc = np.array([[(i // 3 ** a) % 3 for a in range(dim)] for i in range(3 ** dim)])
    g = np.zeros((ec.shape[0], loc.shape[0]), dtype=np.int64)
    stride = 1
    for a in range(dim):
        g += stride * (2 * ec[:, a][:, None] + loc[:, a][None, :])
        stride *= nnode[a]
    return g, ec


class Mesh:
    """Geometry of one level of the Q2 mesh: solid cells, element node lists
    and the map of every cell from the reference cell.  Rectilinear levels
    (per-axis node coordinates) map each cell by x = x_0 + h xi; levels with
    node positions (isoparametric Q2 cells, Sec. 5's curved cylinder) by
    x(xi) = sum_i x_i N_i(xi), whose Jacobian dx/dxi, its inverse and its
    determinant are taken at every Gauss point."""

    def __init__(self, level):
        self.dim = level.dim
        self.cells = tuple(level.cells)
        self.coords = [np.asarray(c, dtype=np.float64) for c in level.coords]
        self.solid = np.asarray(level.cell_solid).astype(bool)
        self.nodes, ec = element_nodes(self.cells, self.dim)
        self.h = np.stack([self.coords[a][2 * ec[:, a] + 2] - self.coords[a][2 * ec[:, a]]
                           for a in range(self.dim)], axis=1)
        self.nnodes = int(np.prod([2 * c + 1 for c in self.cells]))
        self.node_solid = np.zeros(self.nnodes, dtype=bool)
        self.node_solid[self.nodes[self.solid].ravel()] = True
        self.N, self.dNref, self.w = reference_tables(self.dim)
        xyz = getattr(level, "node_coords", None)
        if xyz is None:
            self.Ji = self.detJ = None
            self.hK = self.h.max(axis=1)
        else:
            Xe = np.asarray(xyz, dtype=np.float64)[self.nodes]           # [e, i, c]
            Jg = np.einsum("eic,qim->eqcm", Xe, self.dNref)              # dx_c / dxi_m
            self.detJ = np.linalg.det(Jg)                                # [e, q]
            self.Ji = np.linalg.inv(Jg)                                  # [e, q, m, c] = dxi_m / dx_c
            # h_K: the longest cell edge from the first corner (local nodes 2, 6, 18)
            corner = [2 * 3 ** a for a in range(self.dim)]
            self.hK = np.max([np.linalg.norm(Xe[:, c] - Xe[:, 0], axis=1) for c in corner], axis=0)


def grad_basis(mesh):
    """Physical basis gradients dN[e, q, i, m] = d N_i / d x_m at the Gauss
    points: (dx/dxi)^-T applied to the reference gradients."""
    if mesh.Ji is None:
        return mesh.dNref[None] / mesh.h[:, None, None, :]
    return np.einsum("qik,eqkm->eqim", mesh.dNref, mesh.Ji)


def point_weights(mesh):
    """Quadrature weights times det(dx/dxi): wq[e, q]."""
    if mesh.Ji is None:
        return mesh.w[None, :] * np.prod(mesh.h, axis=1)[:, None]
    return mesh.w[None, :] * mesh.detJ


def _mv(A, x):
    """batched matrix-vector product A x over leading axes."""
    return (A @ x[..., None])[..., 0]


def element_subset(mesh, elems):
    """A view of the mesh restricted to the cells `elems` (node numbering and
    node count unchanged): residuals and Jacobians assembled over it are
    complete in the rows of every node whose cells are all in `elems`."""
    import copy
    sub = copy.copy(mesh)
    elems = np.asarray(elems)
    sub.solid = mesh.solid[elems]
    sub.nodes = mesh.nodes[elems]
    sub.h = mesh.h[elems]
    sub.hK = mesh.hK[elems]
    if mesh.Ji is not None:
        sub.Ji = mesh.Ji[elems]
        sub.detJ = mesh.detJ[elems]
    return sub


def cells_of_nodes(mesh, nodes):
    """The cells that contain any of the given nodes."""
    hit = np.isin(mesh.nodes, np.asarray(nodes)).any(axis=1)
    return np.nonzero(hit)[0]


def _split(x, d):
    """momentum vector [n*(d+1)] (p, v per node) -> p [n], v [n, d]."""
    X = np.asarray(x).reshape(-1, d + 1)
    return X[:, 0], X[:, 1:]


def _fields(mesh, prm, pe, ve, ue, vo, uo):
    """Values and reference-cell gradients at the Gauss points of the
    element's nodal fields, with a leading batch axis of length 1.  Solid
    cells take the deformation from the velocity (eq. defgrad); fluid cells
    use ue."""
    k, th = prm["k"], prm["theta"]
    uc = np.where(mesh.solid[:, None, None], uo + k * th * ve + k * (1 - th) * vo, ue)
    N = mesh.N                                             # [q, i]
    dN = grad_basis(mesh)       # [e, q, i, m]

    def val(f):
        return np.einsum("qi,eic->eqc", N, f)[None]

    def grad(f):
        return np.einsum("eqim,eic->eqcm", dN, f)[None]    # [1, e, q, c, m] = d_m f_c

    return dict(v=val(ve), gv=grad(ve), vo=val(vo), gvo=grad(vo), u=val(uc), gu=grad(uc),
                uo=val(uo), guo=grad(uo), p=np.einsum("qi,ei->eq", N, pe)[None],
                gp=np.einsum("eqim,ei->eqm", dN, pe)[None])


def _fluid_geometry(prm, d, f):
    """What the fluid terms take from the (frozen) deformation and from the
    old time level: J, F^-1, Jbar, the mesh-transport velocity
    Jbar Fbar^-1 (u_n - u_{n-1}), and the explicit k (1 - theta) A_F(U_{n-1})
    parts.  None of it depends on (v_n, p_n) in fluid cells."""
    k, th = prm["k"], prm["theta"]
    rf, nu = prm["rho_f"], prm["nu_f"]
    I = np.eye(d)
    F, Fo = I + f["gu"], I + f["guo"]
    J, Jo = np.linalg.det(F), np.linalg.det(Fo)
    Fi, Foi = np.linalg.inv(F), np.linalg.inv(Fo)
    Jb = 0.5 * (J + Jo)
    Fbi = np.linalg.inv(0.5 * (F + Fo))
    vold, gvo = f["vo"], f["gvo"]
    return dict(J=J, Fi=Fi, Jb=Jb,
                w=Jb[..., None] * _mv(Fbi, f["u"] - f["uo"]),
                vec_o=k * (1 - th) * rf * Jo[..., None] * _mv(gvo, _mv(Foi, vold)),
                ten_o=k * (1 - th) * _visc(rf, nu, gvo, Foi, Jo))


def _visc(rf, nu, gv, Fi, J):
    """rho_f nu_f J (grad v F^-1 + F^-T grad v^T) F^-T."""
    G = gv @ Fi
    return rf * nu * J[..., None, None] * (G + np.swapaxes(G, -1, -2)) @ np.swapaxes(Fi, -1, -2)


def _fluid(prm, d, f, g):
    """Fluid cells (ALE Navier-Stokes): the vector tested with phi, the
    tensor tested with grad phi and the divergence tested with xi; g from
    _fluid_geometry."""
    k, th = prm["k"], prm["theta"]
    rf, nu = prm["rho_f"], prm["nu_f"]
    v, gv, vold, gvo = f["v"], f["gv"], f["vo"], f["gvo"]
    J, Fi, Jb = g["J"], g["Fi"], g["Jb"]
    gvb = th * gv + (1 - th) * gvo                          # grad vbar
    vec = (rf * Jb[..., None] * (v - vold)
           - rf * _mv(gvb, g["w"])
           + k * th * rf * J[..., None] * _mv(gv, _mv(Fi, v))
           + g["vec_o"])
    ten = (k * th * _visc(rf, nu, gv, Fi, J) + g["ten_o"]
           - k * (J * f["p"])[..., None, None] * np.swapaxes(Fi, -1, -2))
    div = k * J * np.trace(gv @ Fi, axis1=-2, axis2=-1)     # k J tr(grad v F^-1)
    return vec, ten, div


def _solid(prm, d, f):
    """Solid cells (St. Venant-Kirchhoff, first Piola F Sigma, deformation
    condensed into the velocity)."""
    k, th = prm["k"], prm["theta"]
    mu, lam = prm["mu_s"], prm["lambda_s"]
    I = np.eye(d)

    def piola(Fx):
        E = 0.5 * (np.swapaxes(Fx, -1, -2) @ Fx - I)
        trE = np.trace(E, axis1=-2, axis2=-1)
        return Fx @ (2 * mu * E + lam * trE[..., None, None] * I)

    vec = prm["rho_s"] * (f["v"] - f["vo"])
    ten = k * th * piola(I + f["gu"]) + k * (1 - th) * piola(I + f["guo"])
    return vec, ten


def _terms(mesh, prm, f, geo=None):
    """The residual of eq. aletime:2 (moved to the left-hand side) tested with
    every local basis function: [B, ne, nn, d+1] for fields with batch axis
    B; row 0 divergence (+ pressure stabilisation), rows 1.. momentum.
    geo: _fluid_geometry of the fluid cells (computed from f if None)."""
    d = mesh.dim
    k, th, rf, nu = prm["k"], prm["theta"], prm["rho_f"], prm["nu_f"]
    N = mesh.N
    dN = grad_basis(mesh)       # [e, q, i, m]
    wq = point_weights(mesh)   # [e, q]
    B, ne, nq = f["p"].shape
    nn = N.shape[1]
    dt = np.result_type(*[a.dtype for a in f.values()])
    vec = np.zeros((B, ne, nq, d), dtype=dt)
    ten = np.zeros((B, ne, nq, d, d), dtype=dt)
    div = np.zeros((B, ne, nq), dtype=dt)
    fl, so = np.nonzero(~mesh.solid)[0], np.nonzero(mesh.solid)[0]
    if fl.size:
        ff = {key: a[:, fl] for key, a in f.items()}
        if geo is None:
            geo = _fluid_geometry(prm, d, ff)
        vec[:, fl], ten[:, fl], div[:, fl] = _fluid(prm, d, ff, geo)
    if so.size:
        vec[:, so], ten[:, so] = _solid(prm, d, {key: a[:, so] for key, a in f.items()})
    hK = mesh.hK
    dK = prm["alpha0"] * k * k * hK ** 2 / (rf * (hK ** 2 + k * th * nu))
    dK = np.where(mesh.solid, 0.0, dK)
    # sum over Gauss points q (and the gradient index b) against the test
    # functions N[q, i] and dN[e, q, i, b], as batched matrix products
    dNr = np.ascontiguousarray(np.transpose(dN, (0, 2, 1, 3)).reshape(ne, nn, nq * d))
    tw = np.swapaxes(wq[..., None, None] * ten, -1, -2).reshape(B, ne, nq * d, d)
    r = np.zeros((B, ne, nn, d + 1), dtype=dt)
    r[..., 1:] = N.T @ (wq[..., None] * vec) + dNr @ tw
    gpw = (wq[..., None] * f["gp"]).reshape(B, ne, nq * d, 1)
    r[..., 0] = (wq * div) @ N + dK[:, None] * (dNr @ gpw)[..., 0]
    return r


def _gather(mesh, x, u, x_old, u_old):
    d = mesh.dim
    p, v = _split(x, d)
    _, vo = _split(x_old, d)
    u = np.asarray(u).reshape(-1, d)
    uo = np.asarray(u_old).reshape(-1, d)
    nd = mesh.nodes
    return p[nd], v[nd], u[nd], vo[nd], uo[nd]


def operator_value(mesh, prm, x, u, x_old, u_old):
    """A(U) of the condensed momentum + divergence rows (eq. system, rows D
    and M), node-major [n*(d+1)], no boundary handling."""
    d = mesh.dim
    r = _terms(mesh, prm, _fields(mesh, prm, *_gather(mesh, x, u, x_old, u_old)))[0]
    out = np.zeros((mesh.nnodes, d + 1))
    np.add.at(out, mesh.nodes.ravel(), r.reshape(-1, d + 1))
    return out.ravel()


def newton_residual(mesh, prm, x, u, x_old, u_old, mask):
    """B - A(U) with B = 0 (no volume forces), zero at identity rows."""
    r = -operator_value(mesh, prm, x, u, x_old, u_old)
    r[np.asarray(mask).astype(bool)] = 0.0
    return r


def element_jacobians(mesh, prm, x, u, x_old, u_old, h=1e-30):
    """K[e, i, a, j, b] = d r_e[i, a] / d x_e[j, b] by the complex step, the
    deformation of fluid cells held fixed (the dropped ALE derivatives).  The
    Gauss-point fields are linear in the nodal values, so a step i h in the
    local dof (j, b) adds i h N_j (value) and i h grad N_j (gradient) to the
    field it belongs to; in solid cells a velocity step also moves the
    condensed deformation by k theta times that.  The d+1 components of one
    node are stepped in separate batch entries of one evaluation."""
    d = mesh.dim
    kt = prm["k"] * prm["theta"]
    base = _fields(mesh, prm, *_gather(mesh, x, u, x_old, u_old))
    fl = np.nonzero(~mesh.solid)[0]
    geo = _fluid_geometry(prm, d, {key: a[:, fl] for key, a in base.items()}) if fl.size else None
    N = mesh.N
    dN = grad_basis(mesh)
    sol = mesh.solid[:, None]
    ne, nn = dN.shape[0], N.shape[1]
    K = np.zeros((ne, nn, d + 1, nn, d + 1))
    B = d + 1
    for j in range(nn):
        f = {key: np.repeat(val.astype(np.complex128), B, axis=0) for key, val in base.items()}
        Nj = 1j * h * np.broadcast_to(N[None, :, j], (ne, N.shape[0]))     # [e, q]
        dNj = 1j * h * dN[:, :, j, :]                                      # [e, q, m]
        f["p"][0] += Nj
        f["gp"][0] += dNj
        for c in range(d):
            f["v"][1 + c, ..., c] += Nj
            f["gv"][1 + c, ..., c, :] += dNj
            f["u"][1 + c, ..., c] += np.where(sol, kt * Nj, 0.0)
            f["gu"][1 + c, ..., c, :] += np.where(sol[..., None], kt * dNj, 0.0)
        r = _terms(mesh, prm, f, geo).imag / h                                  # [B, e, i, a]
        K[:, :, :, j, :] = np.moveaxis(r, 0, -1)
    return K


def jacobian_bsr(mesh, prm, x, u, x_old, u_old, rowptr, colind, mask):
    """The approximate Jacobian assembled into the given block pattern, with
    the identity rows of the momentum system (row and column eliminated,
    diagonal one).  Returns vals [nnzb, d+1, d+1]."""
    d, b = mesh.dim, mesh.dim + 1
    K = element_jacobians(mesh, prm, x, u, x_old, u_old)
    n = mesh.nnodes
    # block position of every (row node, col node) pair via a CSR lookup
    pos = sp.csr_matrix((np.arange(colind.size) + 1, colind, rowptr), shape=(n, n))
    nd = mesh.nodes
    rows = np.repeat(nd[:, :, None], nd.shape[1], axis=2)
    cols = np.repeat(nd[:, None, :], nd.shape[1], axis=1)
    p = np.asarray(pos[rows.ravel(), cols.ravel()]).ravel() - 1
    if np.any(p < 0):
        raise ValueError("block pattern lacks an element coupling")
    vals = np.zeros((colind.size, b, b))
    np.add.at(vals, p, np.transpose(K, (0, 1, 3, 2, 4)).reshape(-1, b, b))
    m = np.asarray(mask).astype(bool).reshape(n, b)
    rnode = np.repeat(np.arange(n), np.diff(rowptr))
    vals *= (~m[rnode])[:, :, None]
    vals *= (~m[colind])[:, None, :]
    diag = np.nonzero(colind == rnode)[0]
    for c in range(b):
        vals[diag[m[rnode[diag], c]], c, c] = 1.0
    return vals


def min_jacobian_det(mesh, prm, x, u, x_old, u_old):
    """The smallest det F over all Gauss points (solid cells: F of the
    condensed deformation)."""
    f = _fields(mesh, prm, *_gather(mesh, x, u, x_old, u_old))
    return float(np.linalg.det(np.eye(mesh.dim) + f["gu"][0]).min())


def condensation_residual(mesh, prm, x, u, x_old, u_old):
    """The residual of the deformation rows (eq. aletime:2, last line; eq.
    problem:2) with the solid mass matrix cancelled: at the nodes of solid
    cells u_old + k theta v + k (1 - theta) v_old - u, elsewhere 0.  Its
    Newton increment is the residual itself plus k theta times the velocity
    increment."""
    d = mesh.dim
    k, th = prm["k"], prm["theta"]
    _, v = _split(x, d)
    _, vo = _split(x_old, d)
    r = np.asarray(u_old).reshape(-1, d) + k * th * v + k * (1 - th) * vo - np.asarray(u).reshape(-1, d)
    r[~mesh.node_solid] = 0.0
    return r.ravel()


def inject(mesh_f, mesh_c, f, comps):
    """Nodal values of a fine-level field at the coarse nodes (nested Q2
    meshes: coarse node g is fine node 2g per axis)."""
    d = mesh_f.dim
    nf = [2 * c + 1 for c in mesh_f.cells]
    F = np.asarray(f).reshape(nf[::-1] + [comps])
    sl = tuple(slice(None, None, 2) for _ in range(d))
    return np.ascontiguousarray(F[sl]).reshape(-1)


def newton(mesh, prm, A_pattern, mom_mask, E, ale_mask, x, u, x_old, u_old, rtol=1e-8, atol=0.0,
           max_steps=20, gamma=0.05, max_halvings=4, jac=None):
    """One time step of the approximate Newton method (eq. newton) on the
    finest level.  A_pattern = (rowptr, colind) of the momentum matrix, E the
    ALE matrix (CSR, identity rows at interface, solid and outer-boundary
    nodes).  jac: a Jacobian (CSR) carried over from a previous time step, or
    None.  Returns (x, u, info, jac)."""
    d = mesh.dim
    k, th = prm["k"], prm["theta"]
    mmask = np.asarray(mom_mask).astype(bool)
    amask = np.asarray(ale_mask).astype(bool)
    rowptr, colind = A_pattern
    x, u = np.array(x, dtype=np.float64), np.array(u, dtype=np.float64)

    def residuals(xs, us):
        R = newton_residual(mesh, prm, xs, us, x_old, u_old, mmask)
        b5 = -(E @ us)
        b5[amask] = 0.0
        ru = condensation_residual(mesh, prm, xs, us, x_old, u_old)
        return R, b5, ru, max(np.abs(R).max(), np.abs(b5).max(), np.abs(ru).max())

    R, b5, ru, nrm = residuals(x, u)
    info = dict(res=[nrm], jacobians=0, omegas=[], status="noconv")
    nrm0, rate = nrm, None
    for _ in range(max_steps):
        if nrm <= max(rtol * nrm0, atol):
            info["status"] = "ok"
            break
        if jac is None or (rate is not None and rate > gamma):
            vals = jacobian_bsr(mesh, prm, x, u, x_old, u_old, rowptr, colind, mmask)
            jac = to_csr(type("M", (), dict(rowptr=rowptr, colind=colind, vals=vals, b=d + 1)))
            info["jacobians"] += 1
        W = spla.spsolve(jac.tocsc(), R)
        dv = W.reshape(-1, d + 1)[:, 1:]
        lift = np.zeros_like(dv)
        lift[mesh.node_solid] = k * th * dv[mesh.node_solid]
        lift += ru.reshape(-1, d)
        rhs = b5.copy()
        rhs[amask] = lift.ravel()[amask]
        du = spla.spsolve(E.tocsc(), rhs)
        omega = 1.0
        for h in range(max_halvings + 1):
            xt, ut = x + omega * W, u + omega * du
            inverted = min_jacobian_det(mesh, prm, xt, ut, x_old, u_old) <= 0.0
            Rt, b5t, rut, nt = residuals(xt, ut)
            if inverted and h == max_halvings:
                info["status"] = "inverted"
                return xt, ut, info, jac
            if not inverted and (nt < nrm or h == max_halvings):
                break
            omega *= 0.5
        info["omegas"].append(omega)
        rate = nt / nrm
        x, u, R, b5, ru, nrm = xt, ut, Rt, b5t, rut, nt
        info["res"].append(nrm)
    else:
        if nrm <= max(rtol * nrm0, atol):
            info["status"] = "ok"
    info["steps"] = len(info["res"]) - 1
    return x, u, info, jac


def force(mesh, prm, x, u, x_old, u_old, nodes):
    """Mean force of the fluid (and of anything attached) on a rigid obstacle
    over the time step, in the residual form of the benchmark's quantities of
    interest (Sec. 5): the step's operator tested with psi e_j, psi the nodal
    function that is one at the obstacle's nodes and zero at all others,
    divided by k.  The operator tested with that function equals the boundary
    integral of the traction with the fluid's outward normal; the sign is
    flipped so that the result is the force *on* the obstacle (a flow past it
    has positive drag).  Returns [d]: drag (x), lift (y) and, in 3D, z."""
    d = mesh.dim
    A = operator_value(mesh, prm, x, u, x_old, u_old).reshape(-1, d + 1)
    return -A[np.asarray(nodes), 1:].sum(axis=0) / prm["k"]


def time_step(mesh, prm, A_pattern, mom_mask, E, ale_mask, x, u, rows, vals, scale, jac=None,
              **newton_kw):
    """One time step of the benchmark: the previous state becomes the old
    level, the held velocity rows take scale * vals (inflow profile times
    the start-up factor), the Newton loop starts from the previous state.
    Returns (x, u, x_old, u_old, info, jac)."""
    x_old, u_old = np.array(x, dtype=np.float64), np.array(u, dtype=np.float64)
    x = x_old.copy()
    x[np.asarray(rows)] = scale * np.asarray(vals)
    x, u, info, jac = newton(mesh, prm, A_pattern, mom_mask, E, ale_mask, x, u_old.copy(), x_old,
                             u_old, jac=jac, **newton_kw)
    return x, u, x_old, u_old, info, jac
