"""Pins of the time-dependent smooth manufactured problem (oracle/manufactured_time.py; the
paper's smooth test problem, Sec. 5, Table 5 and its convergence study).

* The closed forms agree with central differences of the exact solution: grad u, the body force
  -mu Lap u - (lambda + mu) grad div u + alpha grad p, and the mass source
  d/dt (p/M + alpha div u) + div w with w = -k grad p (time derivative by differences too).
* The RT0 interpolant reproduces the exact normal flux of w across every edge when its basis
  function is integrated along the edge (flux = DoF x |e|), and the P0 interpolant's cell sums
  give the integral of p.
* Backward-Euler stepping with direct solves (plus refinement steps: the systems are very
  ill-conditioned at nu = 0.499, k = 1e-6, M = 1e6) converges with tau = h: first order in the
  H^1 seminorm of u and at least first order in L^2 for p, as the paper reports O(h + tau)
  (measured ~2 for p, with a large constant at nu = 0.4 from the 1/M-weighted pressure).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import manufactured_time as mt
from oracle.fem import BiotParams, ElementData
from oracle.manufactured import triangle_rule
from oracle.mesh import Mesh

LAM, MU, ALPHA, INV_M, K = 5.0, 2.0, 0.7, 1e-3, 0.3


def test_closed_forms_by_differences():
    rng = np.random.default_rng(3)
    x, y, t = rng.uniform(0.05, 0.95, 30), rng.uniform(0.05, 0.95, 30), 0.37
    h = 1e-3
    u = lambda a, b, tt=t: mt.exact_u(a, b, tt, LAM, MU)
    g = mt.exact_grad_u(x, y, t, LAM, MU)
    du_dx = (u(x + h, y) - u(x - h, y)) / (2 * h)
    du_dy = (u(x, y + h) - u(x, y - h)) / (2 * h)
    scale = np.abs(g).max()
    assert np.abs(g[..., :, 0] - du_dx).max() < 1e-5 * scale
    assert np.abs(g[..., :, 1] - du_dy).max() < 1e-5 * scale

    def div_u(a, b, tt=t):
        return ((u(a + h, b, tt)[..., 0] - u(a - h, b, tt)[..., 0]) + (u(a, b + h, tt)[..., 1] - u(a, b - h, tt)[..., 1])) / (2 * h)

    lap = (u(x + h, y) + u(x - h, y) + u(x, y + h) + u(x, y - h) - 4 * u(x, y)) / h ** 2
    H = 1e-2
    grad_div = np.stack([(div_u(x + H, y) - div_u(x - H, y)) / (2 * H),
                         (div_u(x, y + H) - div_u(x, y - H)) / (2 * H)], axis=-1)
    p = lambda a, b, tt=t: mt.exact_p(a, b, tt)
    grad_p = np.stack([(p(x + h, y) - p(x - h, y)) / (2 * h), (p(x, y + h) - p(x, y - h)) / (2 * h)], axis=-1)
    f = mt.body_force(x, y, t, LAM, MU, ALPHA)
    ref = -MU * lap - (LAM + MU) * grad_div + ALPHA * grad_p
    assert np.abs(f - ref).max() < 1e-3 * np.abs(f).max()
    # mass source: d/dt (p/M + alpha div u) + div w, w = -K grad p
    dt = 1e-4
    storage = lambda tt: INV_M * p(x, y, tt) + ALPHA * div_u(x, y, tt)
    w = lambda a, b: mt.exact_w(a, b, t, K)
    div_w = ((w(x + h, y)[..., 0] - w(x - h, y)[..., 0]) + (w(x, y + h)[..., 1] - w(x, y - h)[..., 1])) / (2 * h)
    src = (storage(t + dt) - storage(t - dt)) / (2 * dt) + div_w
    s = mt.mass_source(x, y, t, LAM, MU, ALPHA, INV_M, K)
    assert np.abs(s - src).max() < 1e-5 * np.abs(s).max()


def test_interpolant_fluxes_and_means():
    n = 6
    mesh = Mesh(n)
    P = BiotParams(LAM, MU, alpha=ALPHA, M=1.0 / INV_M, mu_f=1.0, tau=0.5)
    t = 0.2
    x = mt.interpolant(n, P, K, t)
    # RT0: DoF x |e| against the exact flux by a 2-point rule per half edge (another rule)
    a = mesh.vert_xy[mesh.edge_ends[:, 0]]
    b = mesh.vert_xy[mesh.edge_ends[:, 1]]
    length = np.linalg.norm(b - a, axis=1)
    xg, wg = np.polynomial.legendre.leggauss(8)
    flux = np.zeros(mesh.n_edge)
    for half in (0, 1):
        for sq, wq in zip(0.25 * (xg + 1.0) + 0.5 * half, 0.25 * wg):
            xy = a + sq * (b - a)
            flux += wq * np.einsum("ei,ei->e", mt.exact_w(xy[:, 0], xy[:, 1], t, K), mesh.edge_normal)
    flux *= length
    assert np.allclose(x[mesh.off_w:mesh.off_w + mesh.n_edge] * length, flux, rtol=0, atol=1e-13)
    # P0: sum of |T| p_T equals the integral of p over the square (closed form)
    ed = ElementData(mesh)
    total = float(np.sum(ed.area * x[mesh.off_p:]))
    assert abs(total - np.exp(-t) * 4.0 / np.pi ** 2) < 1e-12


@pytest.mark.parametrize("nu", [0.4, 0.499])
def test_backward_euler_rates(nu):
    errs = []
    for n in (8, 16, 32):
        tau = 1.0 / n
        P = BiotParams.from_E_nu(3e4, nu, alpha=1.0, M=1e6, mu_f=1.0, tau=tau)
        prob = mt.SmoothProblem(n, P, 1e-6)
        A = prob.asm.A.tocsc()
        lu = spla.splu(A)

        def solve(b, m):
            x = lu.solve(b)
            for _ in range(3):
                x = x + lu.solve(b - A @ x)
            return x

        x = prob.run(int(round(0.5 / tau)), solve)
        errs.append(prob.errors(x, 0.5))
    e = np.array(errs)
    r_u = np.log2(e[:-1, 0] / e[1:, 0])
    r_p = np.log2(e[:-1, 1] / e[1:, 1])
    print("nu %.3f  H1(u) %s rates %s   L2(p) %s rates %s" % (nu, e[:, 0], np.round(r_u, 3), e[:, 1], np.round(r_p, 3)))
    assert np.all(np.abs(r_u - 1.0) < 0.1)
    assert np.all(r_p > 1.0)
