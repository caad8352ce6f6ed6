"""Synthetic Newton-step systems of the condensed ALE FSI model.

Recipe (all seeded, FP64):

* mesh: [0,1]^d, tensor-product Q2 cells, graded so that every level resolves
  the faces of an axis-aligned solid box (the paper requires interface-resolving
  meshes on every multigrid level, Sec. 3.2 and Sec. 4.3 (II)).  On the coarsest
  level each axis is split at the solid faces and the coarse cells are shared
  among the three intervals in proportion to their lengths (floor, at least one,
  remainder by largest fraction, ties to the lower interval); finer levels
  bisect every cell.  A cell is solid iff its centroid lies inside the box.
* state: v_old, u_old, v_cur are sums A * sum_m c_m prod_a sin(pi m_a x_a),
  m in {1,2,3}^d, c_m ~ N(0,1)/|m|^2, drawn in the order (field, component,
  m lexicographic) from numpy's PCG64(seed); A_v = 0.1, A_u = 0.01.  The current
  deformation follows the condensation relation of Sec. 3.1 everywhere:
  u_cur = u_old + k theta v_cur + k (1-theta) v_old.
* momentum right-hand side: M xi per component, xi ~ N(0,1) per dof (drawn after
  the state), zero at identity rows, normalised to unit 2-norm.
* ALE right-hand side b5: M xi' at fluid rows (drawn next), normalised likewise.

Matrices are re-discretised on every level (the paper assembles on every
multigrid level).  Identity rows:

* momentum: velocity dofs on x=0 and on the walls (all other outer faces
  except x=1, where the do-nothing condition holds), with symmetric column
  elimination; pressure dofs at solid-interior nodes (pressure lives only in
  the fluid and on the interface, Sec. 3.2).
* ALE: every dof at outer-boundary, interface and solid nodes (no column
  elimination: those columns carry the interface data of eq. problem:3).
* deformation (mass on solid cells, eq. problem:2): every dof at fluid-only nodes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "assemble.c")
_LIB = os.path.join(_HERE, "_fsigen.so")

PARAMS_DEFAULT = dict(rho_f=1.0e3, nu_f=1.0e-3, rho_s=1.0e3, mu_s=5.0e5, lambda_s=2.0e6,
                      k=0.01, theta=0.5, alpha0=1.0)


def build_native(force: bool = False) -> str:
    """Compile the C assembly kernel (plain gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _native():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_native()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.fsigen_pattern.argtypes = [ctypes.c_int, P, P, P]
        lib.fsigen_assemble.argtypes = [ctypes.c_int, P, P, P, P, P, P, P, P, P, P, P, P, P,
                                        P, P, P, P, ctypes.c_int]
        lib.fsigen_residual.argtypes = [ctypes.c_int, P, P, P, P, P, P, P, P, P, P, P, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------- data types
@dataclass
class BSR:
    """Block-CSR matrix: row-major b x b blocks, int32 structure."""
    b: int
    rowptr: np.ndarray  # int32 [n+1]
    colind: np.ndarray  # int32 [nnzb]
    vals: np.ndarray    # float64 [nnzb, b, b]
    dirichlet: np.ndarray  # uint8 [n*b]; 1 = identity row

    @property
    def nrows(self) -> int:
        return self.rowptr.shape[0] - 1

    @property
    def nnzb(self) -> int:
        return self.colind.shape[0]


@dataclass
class Level:
    dim: int
    cells: tuple
    coords: list          # per axis node coordinates, 2*cells[a]+1 each
    cell_solid: np.ndarray  # uint8 [ncells], x fastest
    node_solid: np.ndarray  # uint8 [nnodes]: touches a solid cell
    node_fluid: np.ndarray  # uint8 [nnodes]: touches a fluid cell
    node_bdry: np.ndarray   # uint8 [nnodes]: bit a = on face x_a=0, bit a+3 = on x_a=1
    systems: dict = field(default_factory=dict)  # "mom", "ale", "mass" -> BSR
    node_rigid: np.ndarray = None  # bool [nnodes]: touches a rigid obstacle cell
    node_coords: np.ndarray = None  # [nnodes, dim] float64: isoparametric node positions
                                    # (None: the tensor grid of `coords`)

    @property
    def nnodes(self) -> int:
        return int(np.prod([2 * c + 1 for c in self.cells]))

    @property
    def ncells(self) -> int:
        return int(np.prod(self.cells))


@dataclass
class Problem:
    dim: int
    params: dict
    seed: int
    levels: list            # level 0 = finest
    v_old: np.ndarray       # finest nodal fields, node-major [nnodes, d]
    u_old: np.ndarray
    v_cur: np.ndarray
    u_cur: np.ndarray
    rhs: dict               # "mom" -> [n*(d+1)], "ale" -> [n*d]
    solid_box: tuple

    def system(self, name: str) -> list:
        return [lev.systems[name] for lev in self.levels]


# ------------------------------------------------------------------- meshes
def graded_axis(n_coarse: int, lo: float, hi: float, nlev: int) -> list:
    """Vertex coordinates per level (finest first) of a graded axis on [0,1]
    whose coarsest level has n_coarse cells with vertices at lo and hi."""
    return graded_breaks(n_coarse, [0.0, lo, hi, 1.0], nlev)


def graded_breaks(n_coarse: int, ends, nlev: int) -> list:
    """Vertex coordinates per level (finest first) of an axis from ends[0] to
    ends[-1] whose coarsest level has n_coarse cells and a vertex at every
    break in `ends`: each segment gets its share of the cells by length
    (floor, at least one, remainder by largest fraction, ties to the lower
    segment); finer levels bisect every cell."""
    ends = [float(e) for e in ends]
    lens = np.diff(np.array(ends))
    share = n_coarse * lens / (ends[-1] - ends[0])
    cnt = np.maximum(np.floor(share).astype(int), 1)
    if cnt.sum() > n_coarse:
        raise ValueError(f"{n_coarse} coarse cells cannot resolve the breaks {ends}")
    while cnt.sum() < n_coarse:
        frac = np.round(share - cnt, 9)  # exact ties must not depend on rounding
        cnt[int(np.argmax(frac))] += 1  # argmax takes the lowest index on ties
    verts = [ends[0]]
    for s in range(len(lens)):
        verts.extend(np.linspace(ends[s], ends[s + 1], cnt[s] + 1)[1:].tolist())
    v = np.array(verts)
    out = [v]
    for _ in range(nlev - 1):
        f = np.empty(2 * v.shape[0] - 1)
        f[0::2] = v
        f[1::2] = 0.5 * (v[:-1] + v[1:])
        v = f
        out.append(v)
    return out[::-1]


def _nodes_from_verts(v: np.ndarray) -> np.ndarray:
    x = np.empty(2 * v.shape[0] - 1)
    x[0::2] = v
    x[1::2] = 0.5 * (v[:-1] + v[1:])
    return x


def _tensor(vals_per_axis, dim):
    """nodal array with x fastest from per-axis 1D arrays (product)."""
    if dim == 2:
        return np.multiply.outer(vals_per_axis[1], vals_per_axis[0]).ravel()
    return np.multiply.outer(np.multiply.outer(vals_per_axis[2], vals_per_axis[1]),
                             vals_per_axis[0]).ravel()


def _grid_coords(coords, dim):
    """[nnodes, dim] physical coordinates, x fastest."""
    mesh = np.meshgrid(*coords[::-1], indexing="ij")  # z,y,x order
    return np.stack([m.ravel() for m in mesh[::-1]], axis=1)


# ---------------------------------------------------------------- the state
def _draw_state(rng, dim):
    """Coefficients of the sin series, drawn in (field, component, m) order."""
    ms = np.array(np.meshgrid(*([np.arange(1, 4)] * dim), indexing="ij")).reshape(dim, -1).T
    # lexicographic m with the first index slowest
    coef = {}
    for fld in ("v_old", "u_old", "v_cur"):
        c = np.empty((dim, ms.shape[0]))
        for comp in range(dim):
            c[comp] = rng.standard_normal(ms.shape[0]) / np.sum(ms * ms, axis=1)
        coef[fld] = c
    return ms, coef


def _eval_series(ms, c, coords, dim, amp):
    n = int(np.prod([x.shape[0] for x in coords]))
    out = np.zeros((n, dim))
    for t, m in enumerate(ms):
        basis = _tensor([np.sin(np.pi * m[a] * coords[a]) for a in range(dim)], dim)
        for comp in range(dim):
            out[:, comp] += c[comp, t] * basis
    return amp * out


# --------------------------------------------------------------- assembly
def _pattern(dim, cells):
    lib = _native()
    cells_c = np.array(list(cells) + [1] * (3 - dim), dtype=np.int32)
    n = int(np.prod([2 * c + 1 for c in cells]))
    rowptr = np.zeros(n + 1, dtype=np.int32)
    lib.fsigen_pattern(dim, _ptr(cells_c), _ptr(rowptr), None)
    colind = np.zeros(int(rowptr[-1]), dtype=np.int32)
    lib.fsigen_pattern(dim, _ptr(cells_c), _ptr(rowptr), _ptr(colind))
    return rowptr, colind


def _params_vec(p):
    return np.array([p["rho_f"], p["nu_f"], p["rho_s"], p["mu_s"], p["lambda_s"], p["k"],
                     p["theta"], p["alpha0"]], dtype=np.float64)


def _nthreads():
    return int(os.environ.get("FSIGEN_THREADS", os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))


def _coords_c(coords, dim):
    cs = [np.ascontiguousarray(c, dtype=np.float64) for c in coords]
    while len(cs) < 3:
        cs.append(np.zeros(1))
    return cs


def _row_of_block(rowptr):
    n = rowptr.shape[0] - 1
    return np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))


def _diag_blocks(rowptr, colind):
    rows = _row_of_block(rowptr)
    return np.nonzero(colind == rows)[0]


def _compress(rowptr, colind, vals):
    """drop all-zero off-diagonal blocks."""
    rows = _row_of_block(rowptr)
    keep = np.any(vals.reshape(vals.shape[0], -1) != 0.0, axis=1) | (colind == rows)
    n = rowptr.shape[0] - 1
    cnt = np.bincount(rows[keep], minlength=n)
    rp = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(cnt, out=rp[1:])
    return rp, np.ascontiguousarray(colind[keep]), np.ascontiguousarray(vals[keep])


def make_level(dim, cells, coords, solid_box, state_nodal, params, systems=("mom", "ale", "mass"),
               need_smass=False, rigid_box=None, node_coords=None):
    """Assemble the requested systems on one level.

    state_nodal: dict of nodal [nnodes, dim] arrays v_old, u_old, v_cur, u_cur.
    rigid_box: cells whose centroid lies inside it form a rigid obstacle: they
    are flagged solid and every node touching them has the velocity held
    (no-slip), so with zero velocity there they contribute nothing.
    node_coords: [nnodes, dim] positions of the nodes (isoparametric Q2
    cells); the cell and node flags still come from the tensor grid `coords`
    (the mesh's reference positions).
    """
    lib = _native()
    cells = tuple(int(c) for c in cells)
    nnode_axis = [2 * c + 1 for c in cells]
    nnodes = int(np.prod(nnode_axis))
    ncell = int(np.prod(cells))
    # cell flags
    cen = []
    for a in range(dim):
        x = coords[a]
        cen.append(0.5 * (x[0:-1:2] + x[2::2]))
    lo, hi = solid_box
    inside = [((cen[a] > lo[a]) & (cen[a] < hi[a])).astype(np.uint8) for a in range(dim)]
    cell_solid = _tensor(inside, dim).astype(np.uint8)
    if rigid_box is not None:
        rin = [((cen[a] > rigid_box[0][a]) & (cen[a] < rigid_box[1][a])).astype(np.uint8)
               for a in range(dim)]
        cell_rigid = _tensor(rin, dim).astype(bool)
        cell_solid[cell_rigid] = 1
    else:
        cell_rigid = np.zeros(cell_solid.shape, dtype=bool)
    # node flags: a node touches the cells e with 2e <= g <= 2e+2 per axis
    cs = cell_solid.reshape([cells[a] for a in range(dim)][::-1])
    touch_s = np.zeros([nnode_axis[a] for a in range(dim)][::-1], dtype=bool)
    touch_f = np.zeros_like(touch_s)
    for off in np.ndindex(*([3] * dim)):
        sl = tuple(slice(off[a], off[a] + 2 * cells[::-1][a], 2) for a in range(dim))
        touch_s[sl] |= cs.astype(bool)
        touch_f[sl] |= ~cs.astype(bool)
    node_solid = touch_s.ravel().astype(np.uint8)
    touch_r = np.zeros_like(touch_s)
    cr = cell_rigid.reshape(cs.shape)
    for off in np.ndindex(*([3] * dim)):
        sl = tuple(slice(off[a], off[a] + 2 * cells[::-1][a], 2) for a in range(dim))
        touch_r[sl] |= cr
    node_rigid = touch_r.ravel()
    node_fluid = touch_f.ravel().astype(np.uint8)
    node_bdry = np.zeros(nnodes, dtype=np.uint8)
    for a in range(dim):
        per_axis = [np.ones(nnode_axis[c], dtype=np.int64) for c in range(dim)]
        e = np.zeros(nnode_axis[a], dtype=np.int64)
        e[0] |= 1 << a
        e[-1] |= 1 << (a + 3)
        per_axis[a] = e
        node_bdry |= _tensor(per_axis, dim).astype(np.uint8)
    xyz = None if node_coords is None else np.ascontiguousarray(node_coords, dtype=np.float64)
    if xyz is not None and xyz.shape != (nnodes, dim):
        raise ValueError("node_coords must be [nnodes, dim]")
    lev = Level(dim=dim, cells=cells, coords=[np.asarray(c) for c in coords], cell_solid=cell_solid,
                node_solid=node_solid, node_fluid=node_fluid, node_bdry=node_bdry,
                node_rigid=node_rigid, node_coords=xyz)

    rowptr, colind = _pattern(dim, cells)
    nnzb = colind.shape[0]
    cells_c = np.array(list(cells) + [1] * (3 - dim), dtype=np.int32)
    cx, cy, cz = _coords_c(coords, dim)
    st = {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in state_nodal.items()}
    pv = _params_vec(params)
    bm = dim + 1
    vm = np.zeros((nnzb, bm, bm)) if "mom" in systems else None
    va = np.zeros((nnzb, dim, dim)) if "ale" in systems else None
    vs = np.zeros((nnzb, dim, dim)) if "mass" in systems else None
    vsm = np.zeros(nnzb) if need_smass else None
    rc = lib.fsigen_assemble(dim, _ptr(cells_c), _ptr(cx), _ptr(cy), _ptr(cz), _ptr(xyz), _ptr(cell_solid),
                             _ptr(st["v_old"]), _ptr(st["u_old"]), _ptr(st["v_cur"]),
                             _ptr(st["u_cur"]), _ptr(pv), _ptr(rowptr), _ptr(colind), _ptr(vm),
                             _ptr(va), _ptr(vs), _ptr(vsm), _nthreads())
    if rc != 0:
        raise ValueError("det F <= 0 (state amplitude too large) or det(dx/dxi) <= 0 (a mapped "
                         "cell inverted) at a Gauss point")
    rows = _row_of_block(rowptr)
    diag = np.nonzero(colind == rows)[0]
    walls = np.zeros(nnodes, dtype=bool)
    # velocity Dirichlet: x=0 (inflow) and every face of the other axes
    walls |= (node_bdry & 1).astype(bool)
    for a in range(1, dim):
        walls |= (node_bdry & ((1 << a) | (1 << (a + 3)))).astype(bool)
    walls |= node_rigid
    if vm is not None:
        mask = np.zeros((nnodes, bm), dtype=np.uint8)
        mask[walls, 1:] = 1
        mask[(node_solid == 1) & (node_fluid == 0), 0] = 1
        keep_row = (1.0 - mask[rows].astype(np.float64))
        vm *= keep_row[:, :, None]
        del keep_row
        keep_col = (1.0 - mask[colind].astype(np.float64))
        vm *= keep_col[:, None, :]
        del keep_col
        dm = mask[rows[diag]].astype(bool)  # [nnodes, bm] in row order
        for c in range(bm):
            vm[diag[dm[:, c]], c, c] = 1.0
        lev.systems["mom"] = BSR(bm, rowptr, colind, vm, mask.ravel())
    if va is not None:
        ident = (node_bdry != 0) | (node_solid == 1)
        mask = np.repeat(ident[:, None], dim, axis=1).astype(np.uint8)
        va[ident[rows]] = 0.0
        for c in range(dim):
            va[diag[ident], c, c] = 1.0
        rp, ci, vv = _compress(rowptr, colind, va)
        del va
        lev.systems["ale"] = BSR(dim, rp, ci, vv, mask.ravel())
    if vs is not None:
        ident = node_solid == 0
        mask = np.repeat(ident[:, None], dim, axis=1).astype(np.uint8)
        vs[ident[rows]] = 0.0
        for c in range(dim):
            vs[diag[ident], c, c] = 1.0
        rp, ci, vv = _compress(rowptr, colind, vs)
        del vs
        lev.systems["mass"] = BSR(dim, rp, ci, vv, mask.ravel())
    if vsm is not None:
        lev.systems["smass"] = BSR(1, rowptr, colind, vsm.reshape(-1, 1, 1),
                                   np.zeros(nnodes, dtype=np.uint8))
    return lev


def _bsr_apply_scalar(m: BSR, x: np.ndarray) -> np.ndarray:
    """y = M x for a b=1 matrix and x [n, c] (component-wise)."""
    import scipy.sparse as sp
    n = m.nrows
    A = sp.csr_matrix((m.vals.reshape(-1), m.colind, m.rowptr), shape=(n, n))
    return A @ x


def make_problem(dim: int, n_fine: int, nlev: int, solid_box, seed: int = 0, params=None,
                 systems=("mom", "ale", "mass"), extra_rhs: int = 0) -> Problem:
    """Seeded synthetic Newton-step problem on [0,1]^dim with n_fine cells per
    axis on the finest of nlev levels (level 0 = finest).  extra_rhs further
    momentum right-hand sides (same recipe, drawn after the others) go to
    rhs["mom_more"]."""
    p = dict(PARAMS_DEFAULT)
    if params:
        p.update(params)
    lo, hi = solid_box
    n_coarse = n_fine >> (nlev - 1)
    if n_coarse << (nlev - 1) != n_fine:
        raise ValueError("n_fine must be divisible by 2^(nlev-1)")
    verts = [graded_axis(n_coarse, lo[a], hi[a], nlev) for a in range(dim)]
    rng = np.random.Generator(np.random.PCG64(seed))
    ms, coef = _draw_state(rng, dim)
    levels = []
    fine_state = None
    kth, k1 = p["k"] * p["theta"], p["k"] * (1.0 - p["theta"])
    for l in range(nlev):
        coords = [_nodes_from_verts(verts[a][l]) for a in range(dim)]
        v_old = _eval_series(ms, coef["v_old"], coords, dim, 0.1)
        u_old = _eval_series(ms, coef["u_old"], coords, dim, 0.01)
        v_cur = _eval_series(ms, coef["v_cur"], coords, dim, 0.1)
        u_cur = u_old + kth * v_cur + k1 * v_old
        st = dict(v_old=v_old, u_old=u_old, v_cur=v_cur, u_cur=u_cur)
        cells = tuple(len(verts[a][l]) - 1 for a in range(dim))
        lev = make_level(dim, cells, coords, solid_box, st, p, systems=systems, need_smass=(l == 0))
        levels.append(lev)
        if l == 0:
            fine_state = st
    fine = levels[0]
    nn = fine.nnodes
    sm = fine.systems.pop("smass")
    rhs = {}
    if "mom" in systems:
        xi = rng.standard_normal((nn, dim + 1))
        b = _bsr_apply_scalar(sm, xi).ravel()
        b[fine.systems["mom"].dirichlet.astype(bool)] = 0.0
        rhs["mom"] = b / np.linalg.norm(b)
    if "ale" in systems:
        xi = rng.standard_normal((nn, dim))
        b = _bsr_apply_scalar(sm, xi).ravel()
        b[fine.systems["ale"].dirichlet.astype(bool)] = 0.0
        rhs["ale"] = b / np.linalg.norm(b)
    if extra_rhs and "mom" in systems:
        rhs["mom_more"] = []
        for _ in range(extra_rhs):
            xi = rng.standard_normal((nn, dim + 1))
            b = _bsr_apply_scalar(sm, xi).ravel()
            b[fine.systems["mom"].dirichlet.astype(bool)] = 0.0
            rhs["mom_more"].append(b / np.linalg.norm(b))
    return Problem(dim=dim, params=p, seed=seed, levels=levels, rhs=rhs, solid_box=solid_box,
                   **fine_state)


def residual_momentum(lev: Level, params, v_old, u_old, u_frz, v, pres):
    """Nonlinear condensed momentum residual (rows (p, v) per node, no boundary
    handling); only used to check the assembled Jacobian."""
    lib = _native()
    dim = lev.dim
    cells_c = np.array(list(lev.cells) + [1] * (3 - dim), dtype=np.int32)
    cx, cy, cz = _coords_c(lev.coords, dim)
    res = np.zeros((lev.nnodes, dim + 1))
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (v_old, u_old, u_frz, v, pres)]
    lib.fsigen_residual(dim, _ptr(cells_c), _ptr(cx), _ptr(cy), _ptr(cz), _ptr(lev.node_coords),
                        _ptr(lev.cell_solid),
                        *[_ptr(a) for a in arrs], _ptr(_params_vec(params)), _ptr(res))
    return res.ravel()


# -------------------------------------------------------- named workloads
SOLID_2D = ((0.3, 0.45), (0.7, 0.55))
SOLID_3D = ((0.3, 0.4, 0.4), (0.7, 0.6, 0.6))


def batch_instance(index: int, base_seed: int = 1000, sizes=(16, 20, 24, 32, 40),
                   systems=("mom",)) -> Problem:
    """Instance `index` of the batched workload: 3D, N ~ U(sizes) cells per
    axis (3 levels for N = 4c or 5c with c = 4, 4 levels otherwise, so the
    coarsest level keeps 3..5 cells), solid block centred at (1/2, 1/2, 1/2)
    with half-widths x ~ U[0.1, 0.25], y, z ~ U[0.05, 0.15],
    mu_s ~ logU[1e4, 1e6], lambda_s = 4 mu_s; seeded by base_seed + index."""
    rng = np.random.Generator(np.random.PCG64(base_seed + index))
    n = int(rng.choice(np.asarray(sizes)))
    hw = (rng.uniform(0.1, 0.25), rng.uniform(0.05, 0.15), rng.uniform(0.05, 0.15))
    mu = float(np.exp(rng.uniform(np.log(1e4), np.log(1e6))))
    coarse = n
    nlev = 1
    while coarse % 2 == 0 and coarse // 2 >= 3:
        coarse //= 2
        nlev += 1
    nlev = min(nlev, 4)
    box = (tuple(0.5 - h for h in hw), tuple(0.5 + h for h in hw))
    return make_problem(3, n, nlev, box, seed=base_seed + index,
                        params={"mu_s": mu, "lambda_s": 4.0 * mu}, systems=systems)


def serve_instance(dim: int, n: int, seed: int = 0) -> Problem:
    """One simulation of the serving workload: the 2D or 3D box configuration
    with n cells per axis, coarsened while the coarsest level keeps at least
    3 cells per axis (4 in 2D), momentum and ALE systems."""
    return make_problem(dim, n, _serve_levels(dim, n), SOLID_2D if dim == 2 else SOLID_3D,
                        seed=seed, systems=("mom", "ale"))


def _serve_levels(dim: int, n: int) -> int:
    coarse, nlev = n, 1
    lim = 4 if dim == 2 else 3
    while coarse % 2 == 0 and coarse // 2 >= lim:
        coarse //= 2
        nlev += 1
    return nlev


def serve_request(dim: int, n: int, seed: int = 0, n_states: int = 2, n_rhs: int = 3):
    """A serving request's data: the simulation of serve_instance (state 0,
    momentum + ALE, first momentum right-hand side), n_states - 1 further
    seeded states on the same mesh (momentum only: the Jacobian of later time
    steps) and n_rhs - 1 further momentum right-hand sides (later Newton
    steps).  Returns (problem, [state problems], [right-hand sides])."""
    nlev = _serve_levels(dim, n)
    box = SOLID_2D if dim == 2 else SOLID_3D
    P = make_problem(dim, n, nlev, box, seed=seed, systems=("mom", "ale"), extra_rhs=n_rhs - 1)
    states = [make_problem(dim, n, nlev, box, seed=seed + 7919 * s, systems=("mom",))
              for s in range(1, n_states)]
    return P, states, list(P.rhs.get("mom_more", []))


# ------------------------------------------------- the benchmark channel
# The 3D benchmark of Sec. 5 (Fig. config3d): channel (0, 2.8) x (0, 0.41)^2,
# an obstacle around the axis x = 0.5, y = 0.2 spanning the channel in z,
# an elastic beam 0.5 < x < 0.9, 0.19 < y < 0.21, 0.1 < z < 0.3 behind it.
# On the rectilinear Q2 mesh the cylinder of radius 0.05 is read as the square
# prism 0.45 < x < 0.55, 0.15 < y < 0.25 (so the beam starts at x = 0.55 and is
# 0.35 long); the 2D channel is the cut z = const of the same geometry.
CHANNEL_ENDS = ([0.0, 0.45, 0.55, 0.9, 2.8], [0.0, 0.15, 0.19, 0.21, 0.25, 0.41],
                [0.0, 0.1, 0.3, 0.41])
CHANNEL_COARSE = (7, 5, 3)
CHANNEL_OBSTACLE = ((0.45, 0.15, -1.0), (0.55, 0.25, 1.0))
CHANNEL_BEAM = ((0.55, 0.19, 0.1), (0.9, 0.21, 0.3))
CHANNEL_HEIGHT = 0.41
# material and inflow of the benchmark table (Sec. 5): mean inflow 2 (2D) and
# 1.75 (3D) m/s; time step k = 0.002 s with theta = 0.5 + 2k
CHANNEL_PARAMS = dict(rho_f=1.0e3, nu_f=1.0e-3, rho_s=1.0e3, mu_s=2.0e6, lambda_s=8.0e6,
                      k=0.002, theta=0.504, alpha0=1.0)
CHANNEL_VBAR = {2: 2.0, 3: 1.75}


@dataclass
class Channel:
    """The benchmark channel: the problem (levels with momentum and ALE
    systems, rest state), the inflow rows of the Newton vector x with the
    unscaled inflow profile there, the nodes of the obstacle (the drag / lift
    test function is one on them), the beam's cross-section where it meets
    the obstacle (area in 3D, length in 2D) and the node at the point where
    the paper reads the beam's displacement (Sec. 5: B = (0.9, 0.2, 0.3) on
    the beam's back face; (0.9, 0.2) in 2D)."""
    problem: Problem
    inflow_rows: np.ndarray   # int64 indices into x (node * (d + 1) + 1)
    inflow_vals: np.ndarray   # float64 profile at those rows (ramp factor 1)
    force_nodes: np.ndarray   # int64 nodes touching obstacle cells
    root_area: float
    vbar: float
    probe_node: int           # the node at the beam's probe point (0.9, 0.2[, 0.3])


def inflow_profile(dim, y, z=None, vbar=1.0):
    """Inflow x-velocity of the benchmark (Sec. 5): bi-parabolic
    36 vbar y (H - y) z (H - z) / H^4 in 3D, and its 2D analog
    6 vbar y (H - y) / H^2; both have the mean vbar over the inflow face."""
    H = CHANNEL_HEIGHT
    if dim == 2:
        return 6.0 * vbar * y * (H - y) / H ** 2
    return 36.0 * vbar * y * (H - y) * z * (H - z) / H ** 4


def inflow_ramp(t):
    """Start-up factor of the inflow (Sec. 5): (1 - cos(pi t)) / 2 on [0, 1),
    then 1."""
    return 0.5 - 0.5 * np.cos(np.pi * t) if t < 1.0 else 1.0


# The curved channel (isoparametric Q2 cells): the cylinder of radius 0.05
# around (0.5, 0.2) and, away from obstacle and beam, rows of even height.
CYL_CENTER = (0.5, 0.2)
CYL_RADIUS = 0.05
CYL_RING = 0.1          # the map blends back to the identity at this L-inf distance
RELAX_Y = ([0.0, 0.15, 0.19, 0.21, 0.25, 0.41], [0.0, 0.082, 0.164, 0.246, 0.328, 0.41])
RELAX_X = (0.2, 0.35, 1.05, 1.4)  # weight 1 | ramp | 0 (obstacle and beam) | ramp | 1


def channel_map(X: np.ndarray) -> np.ndarray:
    """Node positions of the curved channel from the rectilinear ones
    [n, dim] (z, if present, unchanged).

    1. Rows of even height away from obstacle and beam: y' = y + w(x) (g(y) -
       y), g piecewise linear from the row breaks 0, 0.15, 0.19, 0.21, 0.25,
       0.41 to five rows of height 0.082, w = 1 for x <= 0.2 and x >= 1.4, 0
       for 0.35 <= x <= 1.05, linear between (for every x, y' is increasing
       in y).
    2. The square obstacle onto the cylinder: with r the offset from the
       centre (0.5, 0.2) and s = |r|_inf, a point moves to centre + r (beta
       s / |r|_2 + 1 - beta), beta = 1 for s <= 0.05 (the square of L-inf
       radius s onto the circle of radius s), falling linearly to 0 at s = 0.1
       (identity beyond).  Along every ray from the centre the new distance
       grows with the old one, so the map is one to one; the beam's root face
       x = 0.55 lands on the circle."""
    X = np.array(X, dtype=np.float64)
    x, y = X[:, 0].copy(), X[:, 1].copy()
    a0, a1, a2, a3 = RELAX_X
    w = np.maximum(np.clip((a1 - x) / (a1 - a0), 0.0, 1.0), np.clip((x - a2) / (a3 - a2), 0.0, 1.0))
    y = y + w * (np.interp(y, *RELAX_Y) - y)
    rx, ry = x - CYL_CENTER[0], y - CYL_CENTER[1]
    sinf = np.maximum(np.abs(rx), np.abs(ry))
    r2 = np.hypot(rx, ry)
    beta = np.clip((CYL_RING - sinf) / (CYL_RING - CYL_RADIUS), 0.0, 1.0)
    scale = np.where(r2 > 0, beta * sinf / np.where(r2 > 0, r2, 1.0) + 1.0 - beta, 1.0)
    X[:, 0] = CYL_CENTER[0] + rx * scale
    X[:, 1] = CYL_CENTER[1] + ry * scale
    return X


def make_channel(dim: int, nlev: int, params=None, coarse=None, curved: bool = False) -> Channel:
    """The benchmark channel with nlev levels (coarsest: CHANNEL_COARSE cells
    per axis, graded so that every level resolves the obstacle and beam
    faces), at rest (v = u = 0): momentum and ALE systems assembled at that
    state, no right-hand sides.  curved: isoparametric Q2 cells whose nodes
    channel_map moves (the cylinder of radius 0.05, rows of even height away
    from obstacle and beam); the mesh topology, flags and levels are those of
    the rectilinear channel."""
    p = dict(CHANNEL_PARAMS)
    if params:
        p.update(params)
    coarse = coarse or CHANNEL_COARSE[:dim]
    verts = [graded_breaks(coarse[a], CHANNEL_ENDS[a], nlev) for a in range(dim)]
    beam = (CHANNEL_BEAM[0][:dim], CHANNEL_BEAM[1][:dim])
    obst = (CHANNEL_OBSTACLE[0][:dim], CHANNEL_OBSTACLE[1][:dim])
    levels = []
    for l in range(nlev):
        coords = [_nodes_from_verts(verts[a][l]) for a in range(dim)]
        n = int(np.prod([c.shape[0] for c in coords]))
        zero = np.zeros((n, dim))
        st = dict(v_old=zero, u_old=zero, v_cur=zero, u_cur=zero)
        cells = tuple(len(verts[a][l]) - 1 for a in range(dim))
        xyz = channel_map(_grid_coords(coords, dim)) if curved else None
        levels.append(make_level(dim, cells, coords, beam, st, p, systems=("mom", "ale"),
                                 rigid_box=obst, node_coords=xyz))
    fine = levels[0]
    nn = fine.nnodes
    zero = np.zeros((nn, dim))
    P = Problem(dim=dim, params=p, seed=0, levels=levels, v_old=zero, u_old=zero.copy(),
                v_cur=zero.copy(), u_cur=zero.copy(), rhs={}, solid_box=beam)
    X = fine.node_coords if curved else _grid_coords(fine.coords, dim)
    node = np.nonzero(fine.node_bdry & 1)[0]           # the face x = 0
    vbar = CHANNEL_VBAR[dim]
    vals = inflow_profile(dim, X[node, 1], X[node, 2] if dim == 3 else None, vbar)
    rows = node.astype(np.int64) * (dim + 1) + 1
    force = np.nonzero(fine.node_rigid)[0].astype(np.int64)
    b = CHANNEL_BEAM
    area = (b[1][1] - b[0][1]) * ((b[1][2] - b[0][2]) if dim == 3 else 1.0)
    probe = np.array([0.9, 0.2, 0.3][:dim])
    dist = np.abs(X - probe).max(axis=1)
    pn = int(np.argmin(dist))
    if dist[pn] > 1e-12:
        raise ValueError("the probe point is not a mesh node")
    return Channel(problem=P, inflow_rows=rows, inflow_vals=vals, force_nodes=force,
                   root_area=area, vbar=vbar, probe_node=pn)


def config_problem(name: str, seed: int = 0, **kw) -> Problem:
    """Named workloads: 'c1' (2D 32^2, 3 levels), 'c2' (3D 32^3, 4 levels),
    'c3' (3D 64^3, 5 levels) and small test cases 't2' (2D 8^2, 2 levels),
    't3' (3D 4^3, 2 levels)."""
    table = {
        "c1": (2, 32, 3, SOLID_2D),
        "c2": (3, 32, 4, SOLID_3D),
        "c3": (3, 64, 5, SOLID_3D),
        "t2": (2, 16, 2, SOLID_2D),
        "t3": (3, 8, 2, SOLID_3D),
    }
    dim, n, nlev, box = table[name]
    return make_problem(dim, n, nlev, box, seed=seed, **kw)
