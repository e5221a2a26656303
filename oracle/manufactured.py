"""Steady-state manufactured problem of the paper's numerical results (Sec. 5.1).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

The exact solution is u = curl phi with phi = [x y (1 - x)(1 - y)]^2, p = 1, w = 0, one
backward-Euler step with tau = 1.  Right-hand side of (discrete1)-(discrete3):
  * displacement: (rho g, v) with rho g = -div(2 mu eps(u)) - lambda grad(div u) + alpha grad p
    from (Biot-eq1); here div u = 0 and p is constant, so rho g = -mu Lap(u);
  * Darcy: tau (rho_f g, r) with rho_f g = K^{-1} mu_f w + grad p = 0 from (Biot-eq2);
  * mass balance: -(f_hat, q) with f_hat = tau f + (1/M) p^{m-1} + alpha div u^{m-1}.  The
    solution does not depend on time, so with the previous step at the exact solution (or,
    equivalently, a zero previous step and f = p / (M tau)) f_hat = 1/M.

The load is integrated with a collapsed (Duffy) Gauss-Legendre rule on each triangle, exact for
polynomials up to total degree 2 k - 2; the integrands here have degree at most 7.

Error norms of a discrete solution: the H^1 seminorm of u - u_h and the L^2 norm of p - p_h,
by the same rule.
"""
import numpy as np

from .mesh import Mesh
from .fem import ElementData, _u_full_dofs


def triangle_rule(k=6):
    """Barycentric points (m, 3) and weights (m,) on a triangle, weights summing to 1 (multiply
    by |T|): Gauss-Legendre in s and t, point (1 - s, s (1 - t), s t), Jacobian 2 s."""
    x, w = np.polynomial.legendre.leggauss(k)
    s = 0.5 * (x + 1.0)
    ws = 0.5 * w
    pts, wts = [], []
    for a in range(k):
        for b in range(k):
            l1 = s[a] * (1.0 - s[b])
            l2 = s[a] * s[b]
            pts.append((1.0 - l1 - l2, l1, l2))
            wts.append(2.0 * ws[a] * ws[b] * s[a])
    return np.array(pts), np.array(wts)


def _ab(x):
    """a(x) = x^2 (1 - x)^2 and its first three derivatives."""
    return (x * x * (1 - x) ** 2, 2 * x - 6 * x * x + 4 * x ** 3, 2 - 12 * x + 12 * x * x, -12 + 24 * x)


def exact_u(x, y):
    """u = curl phi = (d_y phi, -d_x phi) with phi = a(x) a(y)."""
    ax, ay = _ab(x), _ab(y)
    return np.stack([ax[0] * ay[1], -ax[1] * ay[0]], axis=-1)


def exact_grad_u(x, y):
    """[component, derivative] of u = curl phi."""
    ax, ay = _ab(x), _ab(y)
    g = np.zeros(np.shape(x) + (2, 2))
    g[..., 0, 0] = ax[1] * ay[1]
    g[..., 0, 1] = ax[0] * ay[2]
    g[..., 1, 0] = -ax[2] * ay[0]
    g[..., 1, 1] = -ax[1] * ay[1]
    return g


def body_force(x, y, mu):
    """rho g = -mu Lap(u), with Lap(curl phi) = curl Lap(phi) = (d_y Lap phi, -d_x Lap phi)."""
    ax, ay = _ab(x), _ab(y)
    dy_lap = ax[2] * ay[1] + ax[0] * ay[3]
    dx_lap = ax[3] * ay[0] + ax[1] * ay[2]
    return -mu * np.stack([dy_lap, -dx_lap], axis=-1)


def _u_values(ed, beta):
    """Displacement basis values at barycentric point beta: (nT, 9, 2)."""
    nT = ed.X.shape[0]
    out = np.zeros((nT, 9, 2))
    for a in range(3):
        out[:, a, 0] = beta[a]
        out[:, 3 + a, 1] = beta[a]
    for k in range(3):
        p, q = (k + 1) % 3, (k + 2) % 3
        out[:, 6 + k] = 4.0 * beta[p] * beta[q] * ed.nglob[:, k]
    return out


def rhs(n, params, k=6):
    """Right-hand side of the manufactured problem in the canonical free-DoF order."""
    mesh = Mesh(n)
    ed = ElementData(mesh)
    pts, wts = triangle_rule(k)
    bfull = np.zeros(mesh.n_full)
    ud = _u_full_dofs(mesh)
    loc = np.zeros((mesh.n_tri, 9))
    for beta, wq in zip(pts, wts):
        xy = np.einsum("a,tai->ti", beta, ed.X)
        f = body_force(xy[:, 0], xy[:, 1], params.mu)          # (nT, 2)
        phi = _u_values(ed, beta)                               # (nT, 9, 2)
        loc += (wq * ed.area)[:, None] * np.einsum("ti,tji->tj", f, phi)
    np.add.at(bfull, ud.ravel(), loc.ravel())
    bfull[mesh.off_p:] = -ed.area * params.inv_M               # -(f_hat, q_T), f_hat = 1/M
    return bfull[mesh.free_full]


def errors(n, params, x, k=6):
    """(|u - u_h|_{H^1}, ||p - p_h||_{L^2}, ||p - p_h||_{L^2} with the means of p_h and p
    matched) for a discrete solution x in the canonical free-DoF order."""
    mesh = Mesh(n)
    ed = ElementData(mesh)
    pts, wts = triangle_rule(k)
    xf = np.zeros(mesh.n_full)
    xf[mesh.free_full] = x
    cu = xf[_u_full_dofs(mesh)]                                 # (nT, 9)
    e1 = 0.0
    for beta, wq in zip(pts, wts):
        xy = np.einsum("a,tai->ti", beta, ed.X)
        gh = np.einsum("tj,tjab->tab", cu, ed._u_grads(beta))
        d = exact_grad_u(xy[:, 0], xy[:, 1]) - gh
        e1 += float(np.sum(wq * ed.area * np.einsum("tab,tab->t", d, d)))
    ph = xf[mesh.off_p:]
    e_p = float(np.sqrt(np.sum(ed.area * (ph - 1.0) ** 2)))
    pm = np.sum(ed.area * ph) / np.sum(ed.area)
    e_p0 = float(np.sqrt(np.sum(ed.area * (ph - pm) ** 2)))
    return float(np.sqrt(e1)), e_p, e_p0
