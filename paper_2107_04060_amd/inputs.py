"""Seeded synthetic inputs: right-hand sides, permeability fields and the workload
definitions.  Holds none of the solver's arithmetic; both the GPU path's tests/bench and
the CPU reference use exactly these arrays.

Workloads (synthetic stand-ins; the paper's own experiments use manufactured solutions):
  * small      16 x 16,   3 levels, lambda = mu = 1, K = 1, tau = 1, Vanka V(1,1), seed 0
  * sweep256  256 x 256,  7 levels, E = 1, nu in {0.2, 0.49, 0.4999}, K in {1, 1e-3, 1e-6},
              Vanka V(2,2) and inexact BSR V(1,1), seed 1
  * grf1024  1024 x 1024, 9 levels, log10 K = -3 + GRF(corr 0.1), nu = 0.49, tau = 1e-2,
              FP32 smoother, seed 2
  * block2048 2048 x 2048, 10 levels, K in {1, 1e-6} on 64 x 64-cell blocks, nu = 0.4999,
              16 right-hand sides, seed 3
  * adjoint512 512 x 512, 8 levels, ln K = GRF(corr 0.05), 8 samples from seed 4;
              p_obs = p(theta_obs), theta_obs = GRF(corr 0.05) from seed 5; right-hand side
              from seed 4; loss 0.5 ||p(theta) - p_obs||^2

Biot modulus: the workloads do not state M.  The method depends on the parameters only
through nu and the groups E / (alpha^2 M) and E tau K / (alpha^2 mu_f) (a constant
rescaling of u, w and p maps one system onto another and leaves Vanka, BSR, the transfers
and the rediscretized coarse operators invariant).  The paper fixes E = 3e4, M = 1e6,
i.e. E / (alpha^2 M) = 0.03; the workloads keep that ratio: M = E / (0.03 alpha^2).
"""
import numpy as np

PAPER_STORAGE_RATIO = 3.0e4 / 1.0e6      # E / (alpha^2 M) in all of the paper's tests


def lame(E, nu):
    mu = E / (2.0 + 2.0 * nu)
    lam = E * nu / ((1.0 - 2.0 * nu) * (1.0 + nu))
    return lam, mu


def young_from_lame(lam, mu):
    return mu * (3.0 * lam + 2.0 * mu) / (lam + mu)


def biot_modulus(E, alpha=1.0):
    """M with E / (alpha^2 M) equal to the paper's 0.03."""
    return E / (PAPER_STORAGE_RATIO * alpha * alpha)


def n_free(n):
    return 10 * n * n - 8 * n + 2


def n_free_terzaghi(n):
    """Free DoFs of the n x n mesh under Terzaghi's boundary conditions: 10 n^2 - 2 n."""
    return 10 * n * n - 2 * n


# Terzaghi's column (Sec. 5, Terzaghi's problem): E = 3e4, alpha = mu_f = 1, M = infinity,
# k = 1e-6, a unit load on the face x = 0; steps of tau_hat / 100, ten of them, on the 64 x 64 mesh
TERZAGHI = dict(E=3.0e4, k=1e-6, p0=1.0, n=64, steps=10, levels=4, nu=(0.4, 0.45, 0.49, 0.499))


def terzaghi_tau_hat(k, lam, mu):
    """The time scale of the column's slowest mode, 1 / (0.25 pi^2 k (lambda + 2 mu))."""
    return 1.0 / (0.25 * np.pi ** 2 * k * (lam + 2.0 * mu))


def terzaghi_load(n, p0=1.0):
    """The displacement part of the right-hand side of Terzaghi's column, in the canonical free
    order of the mixed boundary conditions: the traction (p0, 0) on the face x = 0 integrated
    against the basis, p0 h at the u_x of each face vertex (p0 h / 2 at the two corners) and
    (2/3) p0 h at the bubble of each face edge (the vertical edges V(0, j), normal +x, whose
    bubble integrates to 2/3 of the edge length).  The blocks before b_V: u_x (n (n + 1)), u_y,
    b_H (n (n - 1) each); u_x of vertex (0, j) is entry j n, b_V of edge V(0, j) entry j n of its
    block."""
    h = 1.0 / n
    b = np.zeros(n_free_terzaghi(n))
    for j in range(n + 1):
        b[j * n] = p0 * (h / 2.0 if j in (0, n) else h)
    off_bv = n * (n + 1) + 2 * n * (n - 1)
    for j in range(n):
        b[off_bv + j * n] = p0 * 2.0 * h / 3.0
    return b


def rhs_uniform(n, seed, count=1):
    """Right-hand side(s) iid uniform[-1, 1] in the canonical free-DoF order."""
    rng = np.random.default_rng(seed)
    out = rng.uniform(-1.0, 1.0, (count, n_free(n)))
    return out[0] if count == 1 else out


def grf_squares(n, corr_len, rng):
    """Gaussian random field on the n x n squares of the unit square, standardized to
    sample mean 0 and std 1: white noise on a zero-padded 2n x 2n periodic grid filtered
    in Fourier space by the transform of exp(-r^2 / (2 l^2)), cropped to n x n.
    Row-major [j, i]."""
    m = 2 * n
    noise = rng.standard_normal((m, m))
    k = np.fft.fftfreq(m, d=1.0 / n)            # cycles per unit length
    kx, ky = np.meshgrid(k, k, indexing="xy")
    filt = np.exp(-0.5 * (2.0 * np.pi) ** 2 * corr_len ** 2 * (kx ** 2 + ky ** 2) / 2.0)
    f = np.real(np.fft.ifft2(np.fft.fft2(noise) * filt))[:n, :n]
    f = (f - f.mean()) / f.std()
    return f


def squares_to_triangles(f_sq):
    """Per-square field [j, i] -> per-triangle array [L(j n + i) ..., U(j n + i) ...]."""
    v = np.asarray(f_sq, dtype=np.float64).ravel()
    return np.concatenate([v, v])


def block_contrast_squares(n, block, rng, values=(1.0, 1e-6)):
    """Piecewise-constant field on block x block cell tiles, each tile value drawn with
    probability 1/2 from `values`."""
    nb = max(1, n // block)
    pick = rng.integers(0, 2, (nb, nb))
    tiles = np.where(pick == 0, values[0], values[1])
    return np.kron(tiles, np.ones((block, block)))[:n, :n]


def workload(name):
    """Definition dictionary of a named workload (params, mesh, smoother settings)."""
    if name == "small":
        lam, mu = 1.0, 1.0
        E = young_from_lame(lam, mu)
        return dict(name=name, n=16, levels=3, cases=[dict(lam=lam, mu=mu, K=1.0)],
                    alpha=1.0, M=biot_modulus(E), mu_f=1.0, tau=1.0, seed=0,
                    smoothers=["vanka"], nu12={"vanka": 2, "bsr": 1})
    if name == "sweep256":
        cases = []
        for nu in (0.2, 0.49, 0.4999):
            for K in (1.0, 1e-3, 1e-6):
                lam, mu = lame(1.0, nu)
                cases.append(dict(lam=lam, mu=mu, K=K, nu=nu))
        return dict(name=name, n=256, levels=7, cases=cases, alpha=1.0, M=biot_modulus(1.0),
                    mu_f=1.0, tau=1.0, seed=1, smoothers=["vanka", "bsr"],
                    nu12={"vanka": 2, "bsr": 1})
    if name == "grf1024":
        lam, mu = lame(1.0, 0.49)
        return dict(name=name, n=1024, levels=9, cases=[dict(lam=lam, mu=mu, nu=0.49)],
                    alpha=1.0, M=biot_modulus(1.0), mu_f=1.0, tau=1e-2, seed=2,
                    smoothers=["vanka"], nu12={"vanka": 2, "bsr": 1}, corr_len=0.1,
                    log10K_mean=-3.0, log10K_std=1.0)
    if name == "block2048":
        lam, mu = lame(1.0, 0.4999)
        return dict(name=name, n=2048, levels=10, cases=[dict(lam=lam, mu=mu, nu=0.4999)],
                    alpha=1.0, M=biot_modulus(1.0), mu_f=1.0, tau=1.0, seed=3,
                    smoothers=["vanka"], nu12={"vanka": 2, "bsr": 1}, block=64, n_rhs=16)
    if name == "adjoint512":
        lam, mu = lame(1.0, 0.3)
        return dict(name=name, n=512, levels=8, cases=[dict(lam=lam, mu=mu, nu=0.3)],
                    alpha=1.0, M=biot_modulus(1.0), mu_f=1.0, tau=1.0, seed=4, obs_seed=5,
                    smoothers=["vanka"], nu12={"vanka": 2, "bsr": 1}, corr_len=0.05, batch=8)
    raise KeyError(name)


def adjoint_fields(n, count=1):
    """Log-permeability fields of the adjoint workload: `count` samples theta = ln K, drawn
    in sequence from its seed, and theta_obs from the observation seed (standardized Gaussian
    random fields, correlation length 0.05).  The observed pressures are those of the
    solution for theta_obs with the same right-hand side."""
    w = workload("adjoint512")
    rng = np.random.default_rng(w["seed"])
    thetas = [squares_to_triangles(grf_squares(n, w["corr_len"], rng)) for _ in range(count)]
    obs = squares_to_triangles(grf_squares(n, w["corr_len"], np.random.default_rng(w["obs_seed"])))
    return thetas, obs


def permeability_triangles(name, n=None):
    """Per-triangle permeability of a workload (array) or a scalar."""
    w = workload(name)
    n = w["n"] if n is None else n
    if name == "grf1024":
        rng = np.random.default_rng(w["seed"])
        f = grf_squares(n, w["corr_len"], rng)
        return squares_to_triangles(10.0 ** (w["log10K_mean"] + w["log10K_std"] * f))
    if name == "block2048":
        rng = np.random.default_rng(w["seed"])
        return squares_to_triangles(block_contrast_squares(n, w["block"], rng))
    if name == "adjoint512":
        return np.exp(adjoint_fields(n, 1)[0][0])
    return None


# Relaxation weights: the two-grid LFA optimum of every parameter set (Sec. 4), computed by the
# CPU reference's local Fourier analysis at the workload's own cell size and parameters and
# stored in relaxation_weights.json (heterogeneous permeabilities use the geometric mean of
# their range as the representative constant K).
_WEIGHTS = None


def _weights_table():
    global _WEIGHTS
    if _WEIGHTS is None:
        import json
        import os
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "relaxation_weights.json")) as f:
            _WEIGHTS = json.load(f)
    return _WEIGHTS


def relaxation_weights(smoother, nu=None, K=None, workload="sweep256"):
    """(omega, omega_J) of a smoother for a workload (for sweep256: of its set (nu, K))."""
    tab = _weights_table()[workload]
    if workload == "sweep256":
        tab = tab["%g/%g" % (nu, K)]
    e = tab[smoother]
    return e["omega"], e["omega_J"]
