"""Shared parameter sets and helpers of the GPU parity tests (no solver arithmetic)."""
import numpy as np

from paper_2107_04060_amd import inputs
from oracle.fem import BiotParams

TOL = 1e-10
EPS = np.finfo(float).eps


def tol_from_conds(conds):
    """max(1e-10, 4 eps kappa): the oracle's LU solves carry a forward error up to
    cond * eps, the library's elimination is exact in exact arithmetic."""
    kap = max(conds)
    return max(TOL, 4.0 * EPS * kap), kap


def case(name):
    """(lam, mu, alpha, M, mu_f, tau) of the parity cases."""
    if name == "small":                      # the 16 x 16 workload's physics
        lam, mu = 1.0, 1.0
        return lam, mu, 1.0, inputs.biot_modulus(inputs.young_from_lame(lam, mu)), 1.0, 1.0
    if name == "stiff":                      # nearly incompressible
        lam, mu = inputs.lame(1.0, 0.49)
        return lam, mu, 1.0, inputs.biot_modulus(1.0), 1.0, 1.0
    if name == "block":                      # the 2048 x 2048 block-contrast workload's physics
        lam, mu = inputs.lame(1.0, 0.4999)
        return lam, mu, 1.0, inputs.biot_modulus(1.0), 1.0, 1.0
    if name == "scaled":                     # tau and mu_f away from 1
        lam, mu = inputs.lame(1.0, 0.3)
        return lam, mu, 0.8, inputs.biot_modulus(1.0, 0.8), 2.5, 1e-2
    raise KeyError(name)


def perm(n, kind, seed=11):
    if kind == "const":
        return 1.0
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(0.2), np.log(5.0), 2 * n * n))


def params(name):
    lam, mu, al, M, mf, tau = case(name)
    return BiotParams(lam, mu, alpha=al, M=M, mu_f=mf, tau=tau)


def solver(binding, torch, n, name, Kk, levels=None, smoother="vanka", nu=2, omega=0.8, omega_J=1.0,
           precision="fp64"):
    lam, mu, al, M, mf, tau = case(name)
    K = Kk if np.isscalar(Kk) else torch.tensor(Kk, dtype=torch.float64, device="cuda")
    s = binding.BiotSolver(n, lam, mu, alpha=al, M=M, mu_f=mf, tau=tau, K=K)
    if levels:
        s.setup(levels=levels, smoother=smoother, nu1=nu, nu2=nu, omega=omega, omega_J=omega_J,
                precision=precision)
    return s


def rel(a, b):
    """The larger of the relative 2-norm difference and the largest entrywise difference
    relative to the largest reference entry: an error confined to a few entries (a tile seam, a
    boundary class) cannot hide in the 2-norm."""
    a = np.asarray(a)
    b = np.asarray(b)
    two = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
    inf = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300) if b.size else 0.0
    return max(two, inf)


def block_perm(n, seed=3, values=(1.0, 1e-6)):
    """The 2048 x 2048 block-contrast permeability at a smaller mesh: K in `values` on tiles of
    n / 32 cells (1/32 of the side, as 64 cells are at 2048), Bernoulli(1/2), per triangle."""
    rng = np.random.default_rng(seed)
    return inputs.squares_to_triangles(inputs.block_contrast_squares(n, max(1, n // 32), rng, values))
