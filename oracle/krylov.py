"""Restarted flexible GMRES with right preconditioning.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Paper passage followed: Sec. 5.1 uses one multigrid V-cycle as the preconditioner of
FGMRES, zero initial guess, stopping on the relative residual.  The algorithm is Saad's
flexible GMRES (right preconditioned, the preconditioned directions z_j are stored), with
modified Gram-Schmidt and Givens rotations; after each cycle the true residual b - A x is
recomputed and used for the stopping test and the restart.
"""
import numpy as np


def fgmres(A, b, precond, tol=1e-8, restart=30, maxit=500, x0=None):
    """Return (x, info) with info = dict(iters, converged, rel_res_true, history)."""
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.copy()
    bnorm = np.linalg.norm(b)
    hist = []
    if bnorm == 0.0:
        return np.zeros(n), dict(iters=0, converged=True, rel_res_true=0.0, history=[0.0])
    it = 0
    r = b - A @ x
    beta = np.linalg.norm(r)
    hist.append(beta / bnorm)
    while True:
        if beta <= tol * bnorm:
            return x, dict(iters=it, converged=True, rel_res_true=beta / bnorm, history=hist)
        if it >= maxit:
            return x, dict(iters=it, converged=False, rel_res_true=beta / bnorm, history=hist)
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = A @ Z[j]
            for i in range(j + 1):                  # modified Gram-Schmidt
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                      # previous rotations
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
            it += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or it >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + Z[:k].T @ y
        r = b - A @ x
        beta = np.linalg.norm(r)
        hist[-1] = beta / bnorm


def fgmres_fixed(A, b, precond, iters):
    """Exactly `iters` FGMRES steps from x = 0 (no restart), for same-algorithm parity."""
    n = b.shape[0]
    bnorm = np.linalg.norm(b)
    m = iters
    V = np.zeros((m + 1, n))
    Z = np.zeros((m, n))
    H = np.zeros((m + 1, m))
    V[0] = b / bnorm
    for j in range(m):
        Z[j] = precond(V[j])
        w = A @ Z[j]
        for i in range(j + 1):
            H[i, j] = np.dot(w, V[i])
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V[j + 1] = w / H[j + 1, j]
    e1 = np.zeros(m + 1)
    e1[0] = bnorm
    y, *_ = np.linalg.lstsq(H, e1, rcond=None)
    return Z.T @ y


def gmres_left(A, b, precond, tol=1e-8, restart=30, maxit=500):
    """Restarted GMRES on the left-preconditioned system M^{-1} A x = M^{-1} b, x0 = 0, stopping
    when the preconditioned residual ||M^{-1}(b - A x)||_2 <= tol ||M^{-1} b||_2 (the relative
    residual of the system GMRES actually solves).  Modified Gram-Schmidt, Givens rotations; the
    preconditioner must be a fixed linear operator (one V-cycle from a zero initial guess is).
    Return (x, info) with info = dict(iters, converged, rel_res_prec, rel_res_true, history)."""
    n = b.shape[0]
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, dict(iters=0, converged=True, rel_res_prec=0.0, rel_res_true=0.0, history=[0.0])
    z = precond(b)
    znorm = np.linalg.norm(z)
    beta = znorm
    hist = [1.0]
    it = 0
    while True:
        if beta <= tol * znorm or it >= maxit:
            r = b - A @ x
            return x, dict(iters=it, converged=bool(beta <= tol * znorm), rel_res_prec=beta / znorm,
                           rel_res_true=np.linalg.norm(r) / bnorm, history=hist)
        m = restart
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = z / beta
        k = 0
        for j in range(m):
            w = precond(A @ V[j])
            for i in range(j + 1):                  # modified Gram-Schmidt
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                      # previous rotations
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
            it += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / znorm)
            if abs(g[j + 1]) <= tol * znorm or it >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + V[:k].T @ y
        z = precond(b - A @ x)
        beta = np.linalg.norm(z)
        hist[-1] = beta / znorm
