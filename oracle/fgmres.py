"""Outer Krylov iteration (Sec. 4.3 (I)): GMRES preconditioned by the
multigrid V-cycle.  The flexible, right-preconditioned form is used (Saad,
Iterative Methods for Sparse Linear Systems, 2nd ed., Alg. 9.6: the
preconditioned directions z_j are stored and the update is x0 + Z y), with
modified Gram-Schmidt Arnoldi, Givens rotations and restart length m.

Identity rows: the residual is taken as zero there (the solution keeps the
value that x carries in), so every Krylov vector vanishes at those dofs.

Stop test: ||r||_2 <= rtol * ||r_0||_2, confirmed with the true residual."""
import numpy as np


def fgmres(A, b, x0, precond, mask, rtol=1e-8, restart=20, maxiter=500, callback=None,
           return_basis=False):
    """Returns (x, info) with info = dict(iters, restarts, res_hist, converged, rel_res)
    (plus the last cycle's Arnoldi basis under "V" when return_basis)."""
    x = np.array(x0, dtype=np.float64, copy=True)

    def resid(xx):
        r = b - A @ xx
        r[mask] = 0.0
        return r

    r = resid(x)
    beta0 = np.linalg.norm(r)
    hist = [beta0]
    info = dict(iters=0, restarts=0, res_hist=hist, converged=True, rel_res=0.0)
    if beta0 == 0.0:
        return x, info
    tol = rtol * beta0
    it = 0
    while it < maxiter:
        beta = np.linalg.norm(r)
        m = restart
        n = b.shape[0]
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        Hm = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            z = precond(V[j])
            z[mask] = 0.0
            Z[j] = z
            w = A @ z
            w[mask] = 0.0
            for i in range(j + 1):  # modified Gram-Schmidt
                Hm[i, j] = w @ V[i]
                w = w - Hm[i, j] * V[i]
            Hm[j + 1, j] = np.linalg.norm(w)
            for i in range(j):  # previous rotations
                t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -sn[i] * Hm[i, j] + cs[i] * Hm[i + 1, j]
                Hm[i, j] = t
            den = np.hypot(Hm[j, j], Hm[j + 1, j])
            cs[j], sn[j] = Hm[j, j] / den, Hm[j + 1, j] / den
            hnext = Hm[j + 1, j]
            Hm[j, j] = den
            Hm[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            hist.append(abs(g[j + 1]))
            if callback:
                callback(it, abs(g[j + 1]))
            if abs(g[j + 1]) <= tol or it >= maxiter or hnext == 0.0:
                break
            V[j + 1] = w / hnext
        if return_basis:  # v_1..v_k and the next direction w / h_{k+1,k}
            info["V"] = np.vstack([V[:k], (w / hnext)[None, :]]) if hnext != 0.0 else V[:k].copy()
        y = np.linalg.solve(np.triu(Hm[:k, :k]), g[:k])
        x = x + Z[:k].T @ y
        r = resid(x)
        rn = np.linalg.norm(r)
        info["restarts"] += 1
        if rn <= tol:
            break
    info["iters"] = it
    info["rel_res"] = float(np.linalg.norm(r) / beta0)
    info["converged"] = bool(info["rel_res"] <= rtol)
    return x, info
