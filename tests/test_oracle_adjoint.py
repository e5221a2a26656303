"""Pins of the oracle's adjoint gradient (test infrastructure) against brute-force central
finite differences of the directly solved loss: dL/dtheta_T for theta_T = ln K_T, with
L = 0.5 ||p(theta) - p_obs||^2 and x(theta) = A(theta)^{-1} b (Sec. 2.1: K enters only
through the Darcy block tau M_w(K))."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle.mesh import Mesh
from oracle.fem import Assembly, BiotParams
from oracle import adjoint


def _problem(n, seed):
    rng = np.random.default_rng(seed)
    p = BiotParams(1.3, 0.7, alpha=0.9, M=40.0, mu_f=1.5, tau=0.8)
    theta = rng.uniform(-1.5, 1.5, 2 * n * n)
    nf = Mesh(n).n_free
    b = rng.uniform(-1, 1, nf)
    p_obs = rng.uniform(-1, 1, 2 * n * n)
    return p, theta, b, p_obs


def _loss(n, p, theta, b, p_obs):
    asm = Assembly(Mesh(n), p, np.exp(theta))
    x = spla.spsolve(asm.A.tocsc(), b)
    return adjoint.pressure_loss(asm, x, p_obs)


def test_adjoint_every_triangle_against_fd():
    """n = 4: each of the 32 gradient components against a central difference, h = 1e-5."""
    n = 4
    p, theta, b, p_obs = _problem(n, 0)
    L, g, _, _ = adjoint.loss_and_grad(n, p, theta, b, p_obs)
    h = 1e-5
    fd = np.zeros_like(g)
    for T in range(theta.size):
        e = np.zeros_like(theta)
        e[T] = h
        fd[T] = (_loss(n, p, theta + e, b, p_obs) - _loss(n, p, theta - e, b, p_obs)) / (2 * h)
    assert np.abs(g).max() > 1e-6
    assert np.abs(fd - g).max() <= 1e-6 * np.abs(g).max()


def test_adjoint_directional_fd():
    """n = 8: directional derivatives g . d in 5 random directions.  The random right-hand
    side excites the nearly singular constant-pressure mode, so the loss is large (~5e6) and
    the step is h = 1e-4 (cancellation ~ eps L / h stays below the tolerance)."""
    n = 8
    p, theta, b, p_obs = _problem(n, 1)
    _, g, _, _ = adjoint.loss_and_grad(n, p, theta, b, p_obs)
    rng = np.random.default_rng(2)
    h = 1e-4
    for _ in range(5):
        d = rng.standard_normal(theta.size)
        fd = (_loss(n, p, theta + h * d, b, p_obs) - _loss(n, p, theta - h * d, b, p_obs)) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * abs(fd)


def test_grad_terms_vanish_without_flux():
    """With w = 0 (or lam_w = 0) every gradient term is zero; the terms are bilinear."""
    n = 4
    p, theta, b, _ = _problem(n, 3)
    asm = Assembly(Mesh(n), p, np.exp(theta))
    rng = np.random.default_rng(4)
    x = rng.standard_normal(asm.n_free)
    lam = rng.standard_normal(asm.n_free)
    _, sw, _ = asm.slices()
    x0 = x.copy()
    x0[sw] = 0
    assert np.all(adjoint.grad_terms(asm, x0, lam) == 0)
    g1 = adjoint.grad_terms(asm, x, lam)
    g2 = adjoint.grad_terms(asm, 2 * x, 3 * lam)
    assert np.allclose(g2, 6 * g1, rtol=1e-14, atol=0)
