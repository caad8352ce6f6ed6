"""Block ILU(0) smoother (TEST INFRASTRUCTURE ONLY).

The paper compares its Vanka-smoothed multigrid with an ILU-smoothed one on
the same momentum system (Sec. 5.5, Fig. memoryconsumtion and the timing
tables: assembly includes computing the ILU) without defining the ILU.
Reading taken here: incomplete LU without fill-in on the block sparsity
pattern of the (p, v) matrix -- one b x b block per pair of coupled nodes,
the matrix's own node order (lexicographic) -- and the smoothing step

    x <- x + omega (L U)^{-1} (b - A x),   identity (Dirichlet) rows kept,

with L block unit-lower and U block upper triangular on the pattern.

The factorisation is the textbook row-oriented (IKJ) elimination restricted
to the pattern: for every block row i, for its lower blocks k < i in
ascending order,
    L_ik = A_ik U_kk^{-1},
    A_ij -= L_ik U_kj   for the blocks j > k of row k that row i also has,
so that (L U)_ij = A_ij on every block of the pattern.
"""
import numpy as np


class BlockILU:
    """ILU(0) factors of a block-CSR system (fsigen.BSRSystem-like: rowptr,
    colind sorted, vals row-major b x b, diagonal block present)."""

    def __init__(self, m):
        b = m.b
        rp = np.asarray(m.rowptr, dtype=np.int64)
        ci = np.asarray(m.colind, dtype=np.int64)
        n = rp.shape[0] - 1
        F = np.asarray(m.vals, dtype=np.float64).reshape(-1, b, b).copy()
        diag = np.empty(n, dtype=np.int64)
        for i in range(n):
            d = np.nonzero(ci[rp[i]:rp[i + 1]] == i)[0]
            assert d.size == 1, "diagonal block missing"
            diag[i] = rp[i] + d[0]
        for i in range(n):
            row = ci[rp[i]:rp[i + 1]]
            for p in range(rp[i], diag[i]):             # lower blocks, ascending k
                k = ci[p]
                F[p] = F[p] @ np.linalg.inv(F[diag[k]])  # L_ik = A_ik U_kk^{-1}
                q = np.arange(diag[k] + 1, rp[k + 1])    # blocks j > k of row k
                if q.size == 0:
                    continue
                j = ci[q]
                at = np.searchsorted(row, j)
                hit = (at < row.size) & (row[np.minimum(at, row.size - 1)] == j)
                if np.any(hit):
                    F[rp[i] + at[hit]] -= np.matmul(F[p][None, :, :], F[q[hit]])
        self.F, self.diag, self.rp, self.ci, self.n, self.b = F, diag, rp, ci, n, b

    def solve(self, d: np.ndarray) -> np.ndarray:
        """(L U)^{-1} d: forward substitution with the unit-lower blocks, then
        backward substitution with the upper blocks."""
        F, diag, rp, ci, n, b = self.F, self.diag, self.rp, self.ci, self.n, self.b
        y = np.asarray(d, dtype=np.float64).reshape(n, b).copy()
        for i in range(n):
            p = np.arange(rp[i], diag[i])
            if p.size:
                y[i] -= np.einsum("pab,pb->a", F[p], y[ci[p]])
        z = np.zeros_like(y)
        for i in range(n - 1, -1, -1):
            p = np.arange(diag[i] + 1, rp[i + 1])
            s = y[i] - (np.einsum("pab,pb->a", F[p], z[ci[p]]) if p.size else 0.0)
            z[i] = np.linalg.solve(F[diag[i]], s)
        return z.reshape(-1)

    def lower_upper_dense(self):
        """The factors as dense matrices (small cases): L (unit block
        diagonal) and U."""
        nb = self.n * self.b
        L = np.eye(nb)
        U = np.zeros((nb, nb))
        b = self.b
        for i in range(self.n):
            for p in range(self.rp[i], self.rp[i + 1]):
                k = self.ci[p]
                blk = (slice(i * b, i * b + b), slice(k * b, k * b + b))
                if k < i:
                    L[blk] = self.F[p]
                else:
                    U[blk] = self.F[p]
        return L, U


def ilu_sweep(A, b: np.ndarray, x: np.ndarray, ilu: BlockILU, mask: np.ndarray,
              omega: float = 1.0, d: np.ndarray = None) -> np.ndarray:
    """One ILU smoothing step; returns the new x (identity rows keep their
    value).  ``d`` may pass a residual b - A x that is already known."""
    if d is None:
        d = b - A @ x
    d = d.copy()
    d[mask] = 0.0
    xn = x + omega * ilu.solve(d)
    xn[mask] = x[mask]
    return xn
