"""Pins of the steady-state manufactured problem of Sec. 5.1 (oracle/manufactured.py).

* The triangle rule integrates every monomial l1^a l2^b with a + b <= 10 to its closed form
  a! b! / (a + b + 2)! (times 2 on the unit-area normalisation).
* The exact displacement is divergence-free and the body force equals -mu Lap(u), both checked
  by central differences of the closed forms (not by the derivative formulas themselves).
* The load vector of a constant force integrates the basis exactly: |T|/3 per P1 hat and per
  bubble (normal value 1 at the midpoint) per triangle.
* The discrete solution converges at the rates the paper reports for this problem (Sec. 5.1,
  convergence study at k = 1e-6, tau = 1): first order in the H^1 seminorm for u and second
  order in L^2 for p (superconvergence of P0 on the uniform mesh), for nu = 0.4 and 0.499.
"""
from math import factorial

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import manufactured as mf
from oracle.fem import Assembly, BiotParams, ElementData, _u_full_dofs
from oracle.mesh import Mesh


def _params(nu):
    return BiotParams.from_E_nu(3e4, nu, alpha=1.0, M=1e6, mu_f=1.0, tau=1.0)


def test_triangle_rule_is_exact_to_degree_ten():
    pts, w = mf.triangle_rule(6)
    assert abs(w.sum() - 1.0) < 1e-14
    for a in range(11):
        for b in range(11 - a):
            exact = 2.0 * factorial(a) * factorial(b) / factorial(a + b + 2)
            q = float(np.sum(w * pts[:, 1] ** a * pts[:, 2] ** b))
            assert abs(q - exact) <= 1e-13 * exact, (a, b)


def test_exact_solution_derivatives_by_differences():
    rng = np.random.default_rng(0)
    x, y = rng.uniform(0.05, 0.95, 40), rng.uniform(0.05, 0.95, 40)
    h = 1e-3
    u = mf.exact_u
    du_dx = (u(x + h, y) - u(x - h, y)) / (2 * h)
    du_dy = (u(x, y + h) - u(x, y - h)) / (2 * h)
    g = mf.exact_grad_u(x, y)
    scale = np.abs(g).max()
    assert np.abs(g[..., :, 0] - du_dx).max() < 1e-5 * scale
    assert np.abs(g[..., :, 1] - du_dy).max() < 1e-5 * scale
    assert np.abs(du_dx[:, 0] + du_dy[:, 1]).max() < 1e-5 * scale          # div u = 0
    # -mu Lap(u) by the five-point difference of u
    lap = (u(x + h, y) + u(x - h, y) + u(x, y + h) + u(x, y - h) - 4 * u(x, y)) / h ** 2
    mu = 7.0
    f = mf.body_force(x, y, mu)
    assert np.abs(f + mu * lap).max() < 1e-4 * np.abs(f).max()


def test_constant_load_integrates_the_basis():
    """With rho g = (c, 0) the displacement load is c |T|/3 per hat and c n_x |T|/3 per bubble,
    summed over the triangles of each DoF's support."""
    n = 4
    mesh = Mesh(n)
    ed = ElementData(mesh)
    pts, wts = mf.triangle_rule(6)
    loc = np.zeros((mesh.n_tri, 9))
    for beta, wq in zip(pts, wts):
        phi = mf._u_values(ed, beta)
        loc += (wq * ed.area)[:, None] * phi[:, :, 0]
    expect = np.zeros((mesh.n_tri, 9))
    expect[:, 0:3] = ed.area[:, None] / 3.0
    expect[:, 6:9] = ed.area[:, None] / 3.0 * ed.nglob[:, :, 0]
    assert np.abs(loc - expect).max() < 1e-15
    # and the assembled right-hand side uses the same element integrals
    P = _params(0.3)
    b = mf.rhs(n, P)
    assert b.shape == (mesh.n_free,)
    nT = mesh.n_tri
    assert np.allclose(b[-nT:], -ed.area / P.M, rtol=0, atol=1e-22)


@pytest.mark.parametrize("nu", [0.4, 0.499])
def test_discretization_rates(nu):
    P = _params(nu)
    errs = []
    for n in (8, 16, 32):
        A = Assembly(Mesh(n), P, 1e-6).A
        x = spla.spsolve(A.tocsc(), mf.rhs(n, P))
        errs.append(mf.errors(n, P, x))
    e = np.array(errs)
    r_u = np.log2(e[:-1, 0] / e[1:, 0])
    r_p = np.log2(e[:-1, 1] / e[1:, 1])
    print("nu %.3f  H1(u) rates %s  L2(p) rates %s" % (nu, np.round(r_u, 3), np.round(r_p, 3)))
    assert np.all(np.abs(r_u - 1.0) < 0.15)
    assert np.all(r_p > 1.8)
