"""Pin of the oracle's V-cycle composition against its closed-form error operator.

The multigrid preconditioner of Sec. 4.3 (II) is a linear map B_l on level l.
With the smoother written as x <- x + S (r - A x), S = D W D the masked
additive Vanka operator of eq. (vanka) (W = omega diag(1/multiplicity)
sum_i R_i^T A_i^-1 R_i, D zeroes the identity-row dofs), and the coarse-grid
correction x <- x + D P B_{l+1} P^T D (r - A x), every right-hand side
r = A e gives e - B_l A e = E_l e with

    E_l = (I - S A)^nu_post (I - D P B_{l+1} P^T D A) (I - S A)^nu_pre,
    B_{l+1} = (I - E_{l+1}) A_{l+1}^-1,   B_coarsest = D A^-1 D.

The operators here are written from these definitions alone: patches
enumerated per element, local inverses of dense submatrices of A, the
prolongation from the quadratic Lagrange basis evaluated at the fine node
coordinates, sparse LU for A^-1.  Nothing is taken from the oracle's own
patch tables, local matrices, transfer matrices or coarse factorisation, so
a mistake in how the oracle composes the cycle (a dropped smoothing pass, a
stale residual, a missing mask, a transposed transfer) fails here even though
FGMRES would still converge with it.  The negative cases plant such mistakes
in a copy of the oracle's cycle and check that the identity then fails."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from fsigen import make_problem
from fsigen.problem import SOLID_2D, SOLID_3D
from oracle import Hierarchy, to_csr, vcycle
from oracle import mg as oracle_mg

OMEGA, NU_PRE, NU_POST = 0.8, 2, 2


def _lagrange_1d(xf, xc):
    """[len(xf), len(xc)] values of the coarse quadratic Lagrange basis
    functions (one per coarse node) at the fine node coordinates: a fine node
    inside coarse cell [xc[2c], xc[2c+2]] takes the three basis functions of
    that cell, evaluated from the cell's own node positions."""
    P = np.zeros((xf.shape[0], xc.shape[0]))
    ncell = (xc.shape[0] - 1) // 2
    for i, x in enumerate(xf):
        c = min(int(np.searchsorted(xc[0::2], x, side="right")) - 1, ncell - 1)
        nodes = xc[2 * c:2 * c + 3]
        for j in range(3):
            others = [nodes[k] for k in range(3) if k != j]
            P[i, 2 * c + j] = (x - others[0]) * (x - others[1]) / (
                (nodes[j] - others[0]) * (nodes[j] - others[1]))
    P[np.abs(P) < 1e-15] = 0.0
    return P


def _prolong(fine_coords, coarse_coords, b):
    """Tensor product of the 1D interpolations (x fastest), component-wise."""
    P = sp.csr_matrix(_lagrange_1d(fine_coords[0], coarse_coords[0]))
    for a in range(1, len(fine_coords)):
        P = sp.kron(sp.csr_matrix(_lagrange_1d(fine_coords[a], coarse_coords[a])), P)
    return sp.kron(P, sp.identity(b)).tocsr()


def _element_dofs(cells, b):
    """Dof lists of the one-element patches, written out per element."""
    nn = [2 * c + 1 for c in cells]
    dim = len(cells)
    out = []
    for e in np.ndindex(*cells[::-1]):
        e = e[::-1]                                  # (ex, ey[, ez]), x fastest
        dofs = []
        for loc in np.ndindex(*([3] * dim)):
            loc = loc[::-1]
            node, stride = 0, 1
            for a in range(dim):
                node += stride * (2 * e[a] + loc[a])
                stride *= nn[a]
            dofs.extend(node * b + c for c in range(b))
        out.append(dofs)
    return np.array(out)


class ClosedForm:
    """E_l and B_l of the hierarchy built from the problem's level matrices."""

    def __init__(self, prob, name, nu_pre=NU_PRE, nu_post=NU_POST, mask_after_prolong=True,
                 masked_residual=True):
        self.nu_pre, self.nu_post = nu_pre, nu_post
        self.mask_after_prolong = mask_after_prolong
        self.masked_residual = masked_residual
        self.A, self.D, self.S, self.P, self.lu = [], [], [], [], []
        mats = prob.system(name)
        L = len(mats)
        for l, m in enumerate(mats):
            A = to_csr(m)
            free = 1.0 - m.dirichlet.astype(np.float64)
            self.A.append(A)
            self.D.append(free)
            self.lu.append(spla.splu(A.tocsc()))
            if l == L - 1:
                continue
            cells = prob.levels[l].cells
            dofs = _element_dofs(cells, m.b)
            Ad = A.toarray() if A.shape[0] <= 4000 else None
            n = A.shape[0]
            mult = np.bincount(dofs.ravel(), minlength=n).astype(np.float64)
            rows, cols, vals = [], [], []
            for I in dofs:
                Ai = Ad[np.ix_(I, I)] if Ad is not None else A[I][:, I].toarray()
                inv = np.linalg.inv(Ai)
                rows.append(np.repeat(I, I.shape[0]))
                cols.append(np.tile(I, I.shape[0]))
                vals.append(inv.ravel())
            W = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                              shape=(n, n))                 # duplicates are summed
            W = sp.diags(OMEGA / mult) @ W
            Dm = sp.diags(free)
            self.S.append((Dm @ W @ Dm).tocsr())
            self.P.append(_prolong(prob.levels[l].coords, prob.levels[l + 1].coords, m.b))

    def B(self, l, r):
        """The level-l cycle applied to r, from its error operator."""
        if l == len(self.A) - 1:
            return self.D[l] * self.lu[l].solve(self.D[l] * r)
        e = self.lu[l].solve(r)
        return e - self.E(l, e)

    def E(self, l, e):
        A, S = self.A[l], self.S[l]
        if l == len(self.A) - 1:
            return e - self.B(l, A @ e)
        for _ in range(self.nu_pre):
            e = e - S @ (A @ e)
        res = A @ e
        if self.masked_residual:
            res = self.D[l] * res
        corr = self.P[l] @ self.B(l + 1, self.P[l].T @ res)
        if self.mask_after_prolong:
            corr = self.D[l] * corr
        e = e - corr
        for _ in range(self.nu_post):
            e = e - S @ (A @ e)
        return e


def _check(prob, name, H, cf, n_vec=3, vcyc=vcycle):
    """max over random e of |(e - B A e) - E e| / |e|, B the oracle's cycle."""
    rng = np.random.default_rng(11)
    A = cf.A[0]
    worst = 0.0
    for _ in range(n_vec):
        e = rng.standard_normal(A.shape[0])
        got = e - vcyc(H, A @ e)
        ref = cf.E(0, e)
        worst = max(worst, np.abs(got - ref).max() / np.abs(e).max())
    return worst


CASES = [(2, 8, 2), (2, 16, 3), (3, 6, 2)]
# The momentum matrices are ill-conditioned (condition numbers 1e11 to 2e12 on
# these meshes: pressure and velocity rows of very different scale), so the
# oracle's dense-LU coarse solve and the sparse LU here agree only to about
# 1e-7 relative; the ALE Laplacians to rounding.  Every planted mistake below
# moves the result by more than 1e2.
TOL = {"mom": 1e-5, "ale": 1e-11}


@pytest.mark.parametrize("dim,n,nlev", CASES)
@pytest.mark.parametrize("name", ["mom", "ale"])
def test_vcycle_equals_closed_form_error_operator(dim, n, nlev, name):
    prob = make_problem(dim, n, nlev, SOLID_2D if dim == 2 else SOLID_3D, seed=3)
    H = Hierarchy(prob.system(name), [lv.cells for lv in prob.levels], omega=OMEGA,
                  nu_pre=NU_PRE, nu_post=NU_POST, weighting="mult")
    cf = ClosedForm(prob, name)
    assert _check(prob, name, H, cf) < TOL[name]


def test_vcycle_full_operator_two_grid_2d():
    """On 2D 8^2 (two levels) the whole map: columns B e_j of the oracle's
    cycle, then I - B A = E as matrices."""
    prob = make_problem(2, 8, 2, SOLID_2D, seed=3)
    H = Hierarchy(prob.system("mom"), [lv.cells for lv in prob.levels], omega=OMEGA,
                  nu_pre=NU_PRE, nu_post=NU_POST, weighting="mult")
    cf = ClosedForm(prob, "mom")
    n = cf.A[0].shape[0]
    Bm = np.stack([vcycle(H, np.eye(n)[:, j]) for j in range(n)], axis=1)
    Em = np.stack([cf.E(0, np.eye(n)[:, j]) for j in range(n)], axis=1)
    lhs = np.eye(n) - Bm @ cf.A[0].toarray()
    assert np.abs(lhs - Em).max() < TOL["mom"] * max(1.0, np.abs(Em).max())
    # on the free dofs the two-grid cycle contracts (identity-row dofs keep
    # their data: E is the identity there)
    free = cf.D[0] > 0
    np.testing.assert_array_equal(Em[np.ix_(~free, ~free)], np.eye(int((~free).sum())))
    assert np.abs(np.linalg.eigvals(Em[np.ix_(free, free)])).max() < 0.5


def _planted(kind):
    """A copy of the oracle's cycle with one plausible mistake planted."""
    def cyc(H, r, l=0):
        lev = H.levels[l]
        r = r.copy()
        r[lev.mask] = 0.0
        if l == len(H.levels) - 1:
            return H.coarse_solve(r)
        x = np.zeros_like(r)
        for s in range(H.nu_pre - (kind == "one_pre_step")):
            stale = kind == "stale_residual"
            x = oracle_mg.smooth(H, lev, r, x, d=r if (s == 0 or stale) else None)
        d = r - lev.A @ x
        d[lev.mask] = 0.0
        xc = cyc(H, lev.P.T @ d, l + 1)
        x = x + lev.P @ xc
        if kind != "no_prolong_mask":
            x[lev.mask] = 0.0
        for _ in range(0 if kind == "no_post" else H.nu_post):
            x = oracle_mg.smooth(H, lev, r, x)
        return x
    return cyc


@pytest.mark.parametrize("kind", ["no_post", "one_pre_step", "stale_residual", "no_prolong_mask"])
def test_planted_cycle_mistakes_break_the_identity(kind):
    """Each mistake, planted in a copy of the cycle, moves e - B A e away from
    E e by far more than the tolerance of the positive test."""
    prob = make_problem(2, 8, 2, SOLID_2D, seed=3)
    H = Hierarchy(prob.system("mom"), [lv.cells for lv in prob.levels], omega=OMEGA,
                  nu_pre=NU_PRE, nu_post=NU_POST, weighting="mult")
    cf = ClosedForm(prob, "mom")
    assert _check(prob, "mom", H, cf, vcyc=_planted("none")) < TOL["mom"]   # the copy is faithful
    assert _check(prob, "mom", H, cf, vcyc=_planted(kind)) > 1e5 * TOL["mom"]


@pytest.mark.parametrize("variant", [dict(nu_post=0), dict(mask_after_prolong=False),
                                     dict(masked_residual=False)])
def test_closed_form_variants_differ_from_the_oracle(variant):
    """The other direction: the closed form with a term dropped no longer
    describes the oracle's cycle, so every term of E is exercised.  (The
    masked residual is implied in the oracle by its identity rows: r and x
    vanish at those dofs, so A x does too; in E the mask is what zeroes the
    error's identity-row part.)"""
    prob = make_problem(2, 8, 2, SOLID_2D, seed=3)
    H = Hierarchy(prob.system("mom"), [lv.cells for lv in prob.levels], omega=OMEGA,
                  nu_pre=NU_PRE, nu_post=NU_POST, weighting="mult")
    cf = ClosedForm(prob, "mom", **variant)
    assert _check(prob, "mom", H, cf) > 1e5 * TOL["mom"]
