"""Krylov outer iteration preconditioned by one p-multigrid cycle (Sec. 4.4).

Oracle (test infrastructure only).

The paper preconditions GMRES (Saad and Schultz) with a single V-cycle per preconditioner
application and gives no restart length, side, orthogonalisation or stopping norm. The oracle uses
right-preconditioned flexible GMRES (the preconditioner may change between iterations), modified
Gram-Schmidt, Givens rotations, restart length ``restart``, stopping when the true relative residual
||b - A x||_2 / ||b||_2 is at most ``rtol`` (checked after every restart cycle).
"""
import numpy as np


def fgmres(apply_A, b, precond=None, x0=None, rtol=1e-10, restart=30, maxit=500):
    """Solve A x = b. Returns (x, info) with info = dict(iters, relres, history, converged)."""
    b = np.asarray(b)
    shape = b.shape
    bv = b.ravel()
    nb = np.linalg.norm(bv)
    x = np.zeros_like(bv) if x0 is None else np.asarray(x0, dtype=bv.dtype).ravel().copy()
    if precond is None:
        precond = lambda v: v
    A = lambda v: apply_A(v.reshape(shape)).ravel()
    Mi = lambda v: np.asarray(precond(v.reshape(shape))).ravel()
    hist = []
    if nb == 0.0:
        return np.zeros(shape), dict(iters=0, relres=0.0, history=hist, converged=True)
    iters = 0
    r = bv - A(x)
    beta = np.linalg.norm(r)
    hist.append(beta / nb)
    while beta / nb > rtol and iters < maxit:
        m = min(restart, maxit - iters)
        V = np.zeros((m + 1, bv.size), dtype=bv.dtype)
        Z = np.zeros((m, bv.size), dtype=bv.dtype)
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = Mi(V[j])
            w = A(Z[j])
            for i in range(j + 1):
                H[i, j] = np.dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            iters += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) / nb <= rtol or H[j, j] == 0.0:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + y @ Z[:k]
        r = bv - A(x)
        beta = np.linalg.norm(r)
    rel = beta / nb
    return x.reshape(shape), dict(iters=iters, relres=float(rel), history=hist,
                                  converged=bool(rel <= rtol))
