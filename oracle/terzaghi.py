"""Terzaghi's consolidation problem (Sec. 5, Terzaghi's problem; Table 6).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Setup (Sec. 5): Omega = [0, 1]^2 with the column's axis along x; alpha = 1, mu_f = 1,
E = 3e4, M = infinity (no pressure mass), K = k I, a load p0 = 1 on the face x = 0.  Boundary
conditions (Mesh(bc="terzaghi")): loaded and drained on x = 0 (traction (p0, 0), p = 0, both
natural), fixed and impermeable on x = 1, rollers on y = 0 and y = 1.  Time scale
tau_hat = 1 / (0.25 pi^2 k (lambda + 2 mu)); steps of tau = tau_hat / 100 from t = 0 to
tau_hat / 10.  Initial state u = 0; with M = infinity the initial pressure p0 enters only as the
undrained response of the first step.  With 1/M = 0 the pressure block of the matrix vanishes
and the Vanka patches add 1e-8 to their diagonal (AdditiveVanka(shift=1e-8)).

Series solution, with c = k (lambda + 2 mu) / mu_f and a_i = (2 i + 1) pi / 2:
  u_x = p0 / (lambda + 2 mu) [1 - x - sum_i 2 / a_i^2 e^{-a_i^2 c t} cos(a_i x)],   u_y = 0,
  p   = p0 sum_i 2 / a_i e^{-a_i^2 c t} sin(a_i x),                 w = -(k / mu_f) grad p.
Reading: the printed pressure series has cos(a_i x); the pressure that vanishes on the drained
face x = 0, has no flux through x = 1 and equals p0 at t = 0+ is the sine series, and only with
it does sigma_xx = (lambda + 2 mu) d_x u_x - alpha p equal the load -p0 everywhere.

Backward Euler step m (Sec. 2.1, eq. block_form with 1/M = 0), right-hand side in the full
numbering, then restricted to the free DoFs:
  b_u = int_{x=0} (p0, 0) . v ds:  p0 h at each face vertex's u_x (p0 h / 2 at the two ends),
        p0 int_e 4 lambda_a lambda_b ds = (2/3) p0 h at the bubble of each face edge (normal +x),
  b_w = 0,
  b_p = alpha B_u u^{m-1}          (B_u <-> -(div u, q); the smooth problem's form with 1/M = 0).
"""
import numpy as np

from .fem import Assembly, BiotParams, ElementData, _u_full_dofs, lame_from_E_nu
from .manufactured import triangle_rule
from .mesh import Mesh

PI = np.pi
E_TERZAGHI = 3.0e4
P0 = 1.0


def tau_hat(k, lam, mu):
    """Time scale of the analytical solution's slowest mode: 1 / (0.25 pi^2 k (lambda + 2 mu))."""
    return 1.0 / (0.25 * PI ** 2 * k * (lam + 2.0 * mu))


def _modes(terms):
    i = np.arange(terms)
    return (2 * i + 1) * PI / 2.0


def exact_p(x, t, k, lam, mu, terms=2000, p0=P0):
    a = _modes(terms)
    c = k * (lam + 2.0 * mu)
    x = np.asarray(x, dtype=float)
    e = np.exp(-np.multiply.outer(np.ones_like(x), a ** 2) * c * t)
    return p0 * np.sum(2.0 / a * e * np.sin(np.multiply.outer(x, a)), axis=-1)


def exact_ux(x, t, k, lam, mu, terms=2000, p0=P0):
    a = _modes(terms)
    c = k * (lam + 2.0 * mu)
    x = np.asarray(x, dtype=float)
    e = np.exp(-np.multiply.outer(np.ones_like(x), a ** 2) * c * t)
    s = np.sum(2.0 / a ** 2 * e * np.cos(np.multiply.outer(x, a)), axis=-1)
    return p0 / (lam + 2.0 * mu) * (1.0 - x - s)


def exact_dux_dx(x, t, k, lam, mu, terms=2000, p0=P0):
    """d_x u_x from the series term by term: (p - p0) / (lambda + 2 mu)."""
    a = _modes(terms)
    c = k * (lam + 2.0 * mu)
    x = np.asarray(x, dtype=float)
    e = np.exp(-np.multiply.outer(np.ones_like(x), a ** 2) * c * t)
    s = np.sum(2.0 / a * e * np.sin(np.multiply.outer(x, a)), axis=-1)
    return p0 / (lam + 2.0 * mu) * (-1.0 + s)


class Terzaghi:
    """The discrete problem on the n x n mesh for Poisson ratio nu and permeability k, with
    steps of length tau (default tau_hat / 100)."""

    def __init__(self, n, nu, k, tau=None, E=E_TERZAGHI, p0=P0):
        lam, mu = lame_from_E_nu(E, nu)
        self.lam, self.mu, self.k, self.p0 = lam, mu, float(k), float(p0)
        self.tau_hat = tau_hat(k, lam, mu)
        self.tau = self.tau_hat / 100.0 if tau is None else float(tau)
        self.params = BiotParams(lam, mu, alpha=1.0, M=np.inf, mu_f=1.0, tau=self.tau)
        self.mesh = Mesh(n, "terzaghi")
        self.asm = Assembly(self.mesh, self.params, self.k)
        m = self.mesh
        h = 1.0 / n
        load = np.zeros(m.n_full)
        for j in range(n + 1):
            load[m.off_ux + m.vid(0, j)] = p0 * (h / 2.0 if j in (0, n) else h)
        for j in range(n):
            load[m.off_b + m.vedge(0, j)] = p0 * 2.0 * h / 3.0
        self.load_u = load

    @property
    def A(self):
        return self.asm.A

    def rhs(self, x_prev_full):
        m = self.mesh
        b = self.load_u.copy()
        b[m.off_p:] = self.params.alpha * (self.asm.Bu_full @ x_prev_full)[m.off_p:]
        return b[m.free_full]

    def full(self, x_free):
        x = np.zeros(self.mesh.n_full)
        x[self.mesh.free_full] = x_free
        return x

    def run(self, steps, solve):
        """Step from u = 0; solve(b_free, m) returns the free solution of step m.  Returns the
        full state after `steps` steps (t = steps * tau)."""
        x = np.zeros(self.mesh.n_full)
        for m_ in range(1, steps + 1):
            x = self.full(solve(self.rhs(x), m_))
        return x

    def errors(self, x_full, t, k=6, terms=2000):
        """(|u - u_h|_{H^1}, ||p - p_h||_{L^2}) at time t against the series."""
        m = self.mesh
        ed = ElementData(m)
        pts, wts = triangle_rule(k)
        cu = x_full[_u_full_dofs(m)]
        ph = x_full[m.off_p:]
        e1 = ep = 0.0
        for beta, wq in zip(pts, wts):
            xy = np.einsum("a,tai->ti", beta, ed.X)
            gh = np.einsum("tj,tjab->tab", cu, ed._u_grads(beta))
            d = -gh
            d[:, 0, 0] += exact_dux_dx(xy[:, 0], t, self.k, self.lam, self.mu, terms, self.p0)
            e1 += float(np.sum(wq * ed.area * np.einsum("tab,tab->t", d, d)))
            dp = exact_p(xy[:, 0], t, self.k, self.lam, self.mu, terms, self.p0) - ph
            ep += float(np.sum(wq * ed.area * dp * dp))
        return float(np.sqrt(e1)), float(np.sqrt(ep))
