"""Time-dependent smooth manufactured problem of the paper's numerical results (Sec. 5, the
smooth test problem; Table 5 and its convergence study).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Exact solution, with E(t) = e^{-t} and s = 1 / (lambda + mu):
  u = E ( sin(pi y) (-cos(pi x) + s sin(pi x)),  sin(pi x) (cos(pi y) + s sin(pi y)) ),
  p = E sin(pi x) sin(pi y),   w = -(k / mu_f) grad p   (K = k I).
Forcing from (Biot-eq1)-(Biot-eq3):
  div u = s pi E sin(pi (x + y)),   Lap u = -2 pi^2 u,
  rho g   = -mu Lap u - (lambda + mu) grad div u + alpha grad p
          = 2 mu pi^2 u - pi^2 E cos(pi (x + y)) (1, 1) + alpha grad p,
  rho_f g = K^{-1} mu_f w + grad p = 0,
  f       = d/dt (p / M + alpha div u) + div w = -(p / M + alpha div u) + 2 pi^2 (k / mu_f) p.

Every field is E(t) times its value at t = 0, so loads and boundary data are computed once.

Boundary conditions (a reading): the paper prescribes displacement and pressure on the whole
boundary.  The discretization here keeps u and w.n as essential conditions on the whole boundary
(the library's unknowns are the free DoFs of that setting).  Both take the exact solution's
values there and are lifted into the right-hand side: u at the boundary vertices, the bubble and
RT0 DoFs of the boundary edges from the exact edge fluxes.  The free-DoF system then has the
library's structure and the exact solution satisfies every equation, so the discrete solution
converges to it at the rate of the discretization.

Backward Euler step m (t_m = m tau), right-hand side of (discrete1)-(discrete3) in the full
numbering, then restricted to the free DoFs with the boundary values lifted:
  b_u = (rho g(t_m), v),   b_w = tau (rho_f g, r) = 0,
  b_p = -(f_hat, q) = -tau (f(t_m), q) - (1/M)(p^{m-1}, q) - alpha (div u^{m-1}, q)
      = -tau F - (1/M) M_p p^{m-1} + alpha B_u u^{m-1}        (B_u <-> -(div u, q)).
The initial state is the interpolant at t = 0 (vertex values and edge fluxes for u, cell means
for p, edge fluxes for w).
"""
import numpy as np

from .fem import Assembly, ElementData, _u_full_dofs
from .manufactured import triangle_rule, _u_values
from .mesh import Mesh

PI = np.pi


def exact_u(x, y, t, lam, mu):
    s = 1.0 / (lam + mu)
    e = np.exp(-t)
    return np.stack([e * np.sin(PI * y) * (-np.cos(PI * x) + s * np.sin(PI * x)),
                     e * np.sin(PI * x) * (np.cos(PI * y) + s * np.sin(PI * y))], axis=-1)


def exact_grad_u(x, y, t, lam, mu):
    """[component, derivative]."""
    s = 1.0 / (lam + mu)
    e = np.exp(-t)
    sx, cx, sy, cy = np.sin(PI * x), np.cos(PI * x), np.sin(PI * y), np.cos(PI * y)
    g = np.zeros(np.shape(x) + (2, 2))
    g[..., 0, 0] = e * sy * PI * (sx + s * cx)
    g[..., 0, 1] = e * PI * cy * (-cx + s * sx)
    g[..., 1, 0] = e * PI * cx * (cy + s * sy)
    g[..., 1, 1] = e * sx * PI * (-sy + s * cy)
    return g


def exact_p(x, y, t):
    return np.exp(-t) * np.sin(PI * x) * np.sin(PI * y)


def exact_grad_p(x, y, t):
    e = np.exp(-t)
    return np.stack([e * PI * np.cos(PI * x) * np.sin(PI * y), e * PI * np.sin(PI * x) * np.cos(PI * y)], axis=-1)


def exact_w(x, y, t, k, mu_f=1.0):
    return -(k / mu_f) * exact_grad_p(x, y, t)


def body_force(x, y, t, lam, mu, alpha):
    """rho g = 2 mu pi^2 u - pi^2 E cos(pi (x + y)) (1, 1) + alpha grad p."""
    c = PI * PI * np.exp(-t) * np.cos(PI * (x + y))
    return (2.0 * mu * PI * PI * exact_u(x, y, t, lam, mu) - np.stack([c, c], axis=-1)
            + alpha * exact_grad_p(x, y, t))


def mass_source(x, y, t, lam, mu, alpha, inv_M, k, mu_f=1.0):
    """f = -(p / M + alpha div u) + 2 pi^2 (k / mu_f) p."""
    s = 1.0 / (lam + mu)
    p = exact_p(x, y, t)
    div_u = s * PI * np.exp(-t) * np.sin(PI * (x + y))
    return -(inv_M * p + alpha * div_u) + 2.0 * PI * PI * (k / mu_f) * p


def _edge_flux(mesh, fn, k=6):
    """Integral over each edge of fn(x, y) . n_e (Gauss-Legendre with k points)."""
    xg, wg = np.polynomial.legendre.leggauss(k)
    s = 0.5 * (xg + 1.0)
    a = mesh.vert_xy[mesh.edge_ends[:, 0]]
    b = mesh.vert_xy[mesh.edge_ends[:, 1]]
    length = np.linalg.norm(b - a, axis=1)
    out = np.zeros(mesh.n_edge)
    for sq, wq in zip(s, wg):
        xy = a + sq * (b - a)
        out += 0.5 * wq * np.einsum("ei,ei->e", fn(xy[:, 0], xy[:, 1]), mesh.edge_normal)
    return out * length, length


def interpolant(n, params, k, t=0.0):
    """Full DoF vector of the interpolant at time t: u vertex values, bubble coefficients that
    make each edge's normal flux exact, P0 cell means of p, RT0 edge fluxes of w."""
    mesh = Mesh(n)
    P = params
    x = np.zeros(mesh.n_full)
    uv = exact_u(mesh.vert_xy[:, 0], mesh.vert_xy[:, 1], t, P.lam, P.mu)
    x[mesh.off_ux:mesh.off_ux + mesh.n_vert] = uv[:, 0]
    x[mesh.off_uy:mesh.off_uy + mesh.n_vert] = uv[:, 1]
    flux_u, length = _edge_flux(mesh, lambda xx, yy: exact_u(xx, yy, t, P.lam, P.mu))
    ua, ub = uv[mesh.edge_ends[:, 0]], uv[mesh.edge_ends[:, 1]]
    flux_p1 = 0.5 * length * np.einsum("ei,ei->e", ua + ub, mesh.edge_normal)
    x[mesh.off_b:mesh.off_b + mesh.n_edge] = (flux_u - flux_p1) / (2.0 / 3.0 * length)
    flux_w, _ = _edge_flux(mesh, lambda xx, yy: exact_w(xx, yy, t, k, P.mu_f))
    x[mesh.off_w:mesh.off_w + mesh.n_edge] = flux_w / length
    ed = ElementData(mesh)
    pts, wts = triangle_rule(6)
    pm = np.zeros(mesh.n_tri)
    for beta, wq in zip(pts, wts):
        xy = np.einsum("a,tai->ti", beta, ed.X)
        pm += wq * exact_p(xy[:, 0], xy[:, 1], t)
    x[mesh.off_p:] = pm
    return x


class SmoothProblem:
    """Backward-Euler stepping of the smooth problem on the n x n mesh with K = k I; the step
    length is params.tau."""

    def __init__(self, n, params, k):
        self.n, self.P, self.k = n, params, k
        self.mesh = Mesh(n)
        self.asm = Assembly(self.mesh, params, k)
        m = self.mesh
        P = params
        ed = ElementData(m)
        pts, wts = triangle_rule(6)
        fu = np.zeros(m.n_full)
        loc = np.zeros((m.n_tri, 9))
        fp = np.zeros(m.n_tri)
        for beta, wq in zip(pts, wts):
            xy = np.einsum("a,tai->ti", beta, ed.X)
            g = body_force(xy[:, 0], xy[:, 1], 0.0, P.lam, P.mu, P.alpha)
            loc += (wq * ed.area)[:, None] * np.einsum("ti,tji->tj", g, _u_values(ed, beta))
            fp += wq * ed.area * mass_source(xy[:, 0], xy[:, 1], 0.0, P.lam, P.mu, P.alpha, P.inv_M, k, P.mu_f)
        np.add.at(fu, _u_full_dofs(m).ravel(), loc.ravel())
        self.load_u0 = fu                      # (rho g(0), v) over every u DoF
        self.load_p0 = fp                      # (f(0), q_T)
        x0 = interpolant(n, params, k, 0.0)
        self.x0 = x0
        free = np.zeros(m.n_full, dtype=bool)
        free[m.free_full] = True
        self.bnd = np.nonzero(~free)[0]
        self.bnd0 = x0[self.bnd]              # boundary values at t = 0 (scaled by e^{-t})
        A = self.asm.A_full.tocsr()
        self.A_fb = A[m.free_full][:, self.bnd].tocsr()

    def rhs(self, t, x_prev):
        """Free-DoF right-hand side of the step ending at t from the full previous state (the
        step length is the tau of the parameters, which also scales the Darcy block)."""
        m, P = self.mesh, self.P
        tau = P.tau
        e = np.exp(-t)
        b = np.zeros(m.n_full)
        b[: m.off_w] = e * self.load_u0[: m.off_w]
        b[m.off_p:] = (-tau * e * self.load_p0 - P.inv_M * (self.asm.Mp_full @ x_prev)[m.off_p:]
                       + P.alpha * (self.asm.Bu_full @ x_prev)[m.off_p:])
        return b[m.free_full] - self.A_fb @ (e * self.bnd0)

    def full(self, x_free, t):
        """Full state from the free solution and the boundary values at t."""
        x = np.zeros(self.mesh.n_full)
        x[self.mesh.free_full] = x_free
        x[self.bnd] = np.exp(-t) * self.bnd0
        return x

    def errors(self, x_full, t, k=6):
        """(|u - u_h|_{H^1}, ||p - p_h||_{L^2}, ||p - p_h||_{L^2} with the means of p and p_h
        matched) at time t."""
        m, P = self.mesh, self.P
        ed = ElementData(m)
        pts, wts = triangle_rule(k)
        cu = x_full[_u_full_dofs(m)]
        ph = x_full[m.off_p:]
        area = np.sum(ed.area)
        e1 = 0.0
        pe = []
        for beta, wq in zip(pts, wts):
            xy = np.einsum("a,tai->ti", beta, ed.X)
            gh = np.einsum("tj,tjab->tab", cu, ed._u_grads(beta))
            d = exact_grad_u(xy[:, 0], xy[:, 1], t, P.lam, P.mu) - gh
            e1 += float(np.sum(wq * ed.area * np.einsum("tab,tab->t", d, d)))
            pe.append((wq, exact_p(xy[:, 0], xy[:, 1], t) - ph))
        mean = sum(float(np.sum(wq * ed.area * d)) for wq, d in pe) / area
        ep = sum(float(np.sum(wq * ed.area * d * d)) for wq, d in pe)
        ep0 = sum(float(np.sum(wq * ed.area * (d - mean) ** 2)) for wq, d in pe)
        return float(np.sqrt(e1)), float(np.sqrt(ep)), float(np.sqrt(ep0))

    def run(self, steps, solve, warm=False):
        """Step from the interpolant at t = 0; solve(b_free, m) returns the free solution of step m.
        With warm=True it is called as solve(b_free, m, guess), guess being the free values of the
        previous state (the interpolant's at step 1): the iterative solve of a time step starts
        from the last step's solution, the reading under which Table 5's counts come out.
        Returns the full state at t = steps * tau."""
        x = self.x0.copy()
        for m_ in range(1, steps + 1):
            t = m_ * self.P.tau
            b = self.rhs(t, x)
            xf = solve(b, m_, x[self.mesh.free_full].copy()) if warm else solve(b, m_)
            x = self.full(xf, t)
        return x
