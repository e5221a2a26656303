"""Adjoint gradient with respect to the per-triangle log-permeability theta_T = ln K_T.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Paper passages followed:
  * Sec. 2.1: K enters the system only through the Darcy term (K^{-1} mu_f w, r), i.e. the
    block tau M_w(K) of (block_form) / (block_form_rq), with M_w(K) = sum_T (mu_f / K_T) M_w^T
    and M_w^T the RT0 mass matrix of triangle T for K = mu_f = 1;
  * (block_form_rq) is symmetric, so the adjoint system uses the same matrix.

For x(theta) = A(theta)^{-1} b and a loss L(x):
    dA/dtheta_T = -tau mu_f e^{-theta_T} M_w^T        (at the three RT0 DoFs of T)
    A lam = dL/dx
    dL/dtheta_T = -lam^T (dA/dtheta_T) x = tau mu_f e^{-theta_T} lam_w|_T^T M_w^T w|_T.
The test loss is L = 0.5 ||p(theta) - p_obs||^2, so dL/dx = (0, 0, p - p_obs).
"""
import numpy as np
import scipy.sparse.linalg as spla

from .mesh import Mesh
from .fem import Assembly


def _full(asm, v):
    out = np.zeros(asm.mesh.n_full)
    out[asm.mesh.free_full] = v
    return out


def grad_terms(asm, x, lam):
    """g_T = tau mu_f / K_T * lam_w|_T^T M_w^T w|_T for every triangle (free vectors in)."""
    m = asm.mesh
    wd = m.off_w + m.tri_edge                  # (nT, 3) full indices of the RT0 DoFs of T
    xw = _full(asm, x)[wd]
    lw = _full(asm, lam)[wd]
    P = asm.params
    return P.tau * P.mu_f / asm.K_tri * np.einsum("tk,tkl,tl->t", lw, asm.ed.Mw_unit, xw)


def pressure_loss(asm, x, p_obs):
    _, _, sp_ = asm.slices()
    d = x[sp_] - p_obs
    return 0.5 * float(d @ d)


def loss_and_grad(n, params, theta, b, p_obs):
    """Loss 0.5 ||p - p_obs||^2 of the direct solution and its adjoint gradient in theta."""
    asm = Assembly(Mesh(n), params, np.exp(theta))
    A = asm.A.tocsc()
    x = spla.spsolve(A, b)
    _, _, sp_ = asm.slices()
    g_x = np.zeros_like(b)
    g_x[sp_] = x[sp_] - p_obs
    lam = spla.spsolve(A, g_x)
    return pressure_loss(asm, x, p_obs), grad_terms(asm, x, lam), x, lam
