"""Block-matrix products of the block linear-algebra layer (Sec. 4.3: block
vectors and matrices with n_c x n_c blocks).  Plain SciPy."""
import numpy as np
import scipy.sparse as sp


def to_csr(m) -> sp.csr_matrix:
    """Block-CSR (row-major b x b blocks) -> scalar CSR, FP64."""
    n = m.rowptr.shape[0] - 1
    b = m.b
    A = sp.bsr_matrix((np.asarray(m.vals, dtype=np.float64).reshape(-1, b, b), m.colind, m.rowptr),
                      shape=(n * b, n * b))
    return A.tocsr()


def matvec(A: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    """y = A x."""
    return A @ x


def masked_residual(A: sp.csr_matrix, b: np.ndarray, x: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """r = b - A x, with r = 0 at identity (Dirichlet) rows: at those dofs the
    solution is the value carried in by x (inhomogeneous data live in x)."""
    r = b - A @ x
    r[mask] = 0.0
    return r
