"""Terzaghi's column on the GPU (Sec. 5, Terzaghi's problem; Table 6): the general-boundary
path of the library (bc = BIOT_BC_TERZAGHI, compressed-row operators and explicit patch
inverses) against the oracle (oracle/terzaghi.py, oracle/multigrid.py with bc = "terzaghi").

* Numbering: the block sizes of the free DoFs under the mixed boundary conditions.
* Operators on every level (M = infinity, constant and heterogeneous K), restriction and
  prolongation: entry by entry against the oracle's sparse matrices.
* One additive Vanka step with the 1e-8 shift (read as a compressibility: + on u, w, - on p),
  V- and W-cycles: entry by entry against the oracle.
* The time step's right-hand side formed on the GPU (load plus alpha B_u u^{m-1}, the pressure
  rows of A applied to the previous displacement) equals the oracle's.
* Table 6 on the GPU: every step's left-preconditioned GMRES iteration count within one of the
  oracle's (tests/golden/terzaghi_table6_oracle.json, written by the committed script beside it
  from the oracle only), the average within 2 of the paper's, and the errors against the series
  at t = tau_hat / 10 equal to the oracle's.
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.fem import Assembly, BiotParams, lame_from_E_nu          # noqa: E402
from oracle.krylov import gmres_left                                   # noqa: E402
from oracle.mesh import Mesh, canonical_block_sizes                    # noqa: E402
from oracle.multigrid import Hierarchy                                 # noqa: E402
from oracle.smoothers import AdditiveVanka, patch_table                # noqa: E402
from oracle.terzaghi import Terzaghi, tau_hat                          # noqa: E402
from tests.gpu_cases import rel                                        # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "terzaghi_table6_oracle.json")
TABLE6 = {0.4: 7.3, 0.45: 7.6, 0.49: 8.7, 0.499: 14.5}   # Table 6, average iterations
K_TZ = 1e-6
SHIFT = 1e-8


def _binding():
    from paper_2107_04060_amd import binding
    binding.load()
    return binding


def _gpu(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _params(nu, n, tau=None):
    lam, mu = lame_from_E_nu(3e4, nu)
    t = tau_hat(K_TZ, lam, mu) / 100.0 if tau is None else tau
    return lam, mu, BiotParams(lam, mu, alpha=1.0, M=np.inf, mu_f=1.0, tau=t)


def _solver(n, nu, K=K_TZ, levels=None, omega=0.8, nu_s=2, gamma=1, shift=SHIFT):
    b = _binding()
    lam, mu, P = _params(nu, n)
    Kg = _gpu(K) if not np.isscalar(K) else K
    s = b.BiotSolver(n, lam, mu, alpha=1.0, M=float("inf"), mu_f=1.0, tau=P.tau, K=Kg, bc="terzaghi")
    if levels:
        s.setup(levels=levels, nu1=nu_s, nu2=nu_s, omega=omega, gamma=gamma, vanka_shift=shift)
    return s, P


@pytest.mark.parametrize("n", [4, 8, 32])
def test_free_dof_counts(n):
    s, _ = _solver(n, 0.4)
    lay = s.export_layout(patches=False)
    m = Mesh(n, "terzaghi")
    assert lay["n_free"] == m.n_free == 10 * n * n - 2 * n == s.nf()
    # blocks: the full counts minus the eliminated entities of each type
    full = canonical_block_sizes(n)
    assert sum(lay["blocks"]) == m.n_free
    assert lay["blocks"][0] == n * (n + 1) and lay["blocks"][1] == n * (n - 1)      # u_x, u_y
    assert lay["blocks"][2] == n * (n - 1) == lay["blocks"][5]                      # H edges
    assert lay["blocks"][3] == n * n == lay["blocks"][6]                            # V edges
    assert lay["blocks"][4] == n * n == lay["blocks"][7] == full[4]                 # D edges
    assert lay["blocks"][8] == lay["blocks"][9] == n * n


@pytest.mark.parametrize("nu,kind", [(0.45, "const"), (0.499, "hetero")])
def test_operators_and_transfers_match_the_oracle(nu, kind):
    n, levels = 32, 3
    K = K_TZ if kind == "const" else K_TZ * np.exp(np.random.default_rng(21).uniform(-2, 2, 2 * n * n))
    s, P = _solver(n, nu, K=K, levels=levels)
    H = Hierarchy(n, P, K_tri=K, smoother="vanka", omega=0.8, nu1=2, nu2=2, levels=levels, bc="terzaghi",
                  vanka_shift=SHIFT)
    rng = np.random.default_rng(5)
    for l, lev in enumerate(H.levels):
        x = rng.standard_normal(lev.A.shape[0])
        y = _cpu(s.apply(_gpu(x), level=l))
        assert rel(y, lev.A @ x) < 1e-13, l
    for l in range(levels - 1):
        Pm = H.levels[l].P
        rf = rng.standard_normal(Pm.shape[0])
        assert rel(_cpu(s.restrict(_gpu(rf), level=l)), Pm.T @ rf) < 1e-14
        xc = rng.standard_normal(Pm.shape[1])
        xf = rng.standard_normal(Pm.shape[0])
        assert rel(_cpu(s.prolong_add(_gpu(xc), _gpu(xf), level=l)), xf + Pm @ xc) < 1e-14


@pytest.mark.parametrize("nu", [0.4, 0.499])
def test_vanka_step_matches_the_oracle(nu):
    """One shifted additive Vanka step from a random iterate.  Both sides invert the same
    shifted 20 x 20 patch matrices (LU with partial pivoting against Gauss-Jordan with partial
    pivoting).  The shifted patches are badly conditioned (up to 1e15: the star-constant
    pressure is held only by the 1e-8 shift), so cond times the rounding unit bounds nothing
    useful; the two sides meet at the rounding level (5e-16 measured), and the bar 1e-12 sits far
    below the O(1) error of a wrong index, sign or shift."""
    n = 16
    s, P = _solver(n, nu, levels=2)
    m = Mesh(n, "terzaghi")
    A = Assembly(m, P, K_TZ).A
    _, slots = patch_table(m, "full")
    sm = AdditiveVanka(A, slots, 0.8, shift=SHIFT, p_start=m.n_u + m.n_w)
    rng = np.random.default_rng(8)
    x = rng.standard_normal(m.n_free)
    b = rng.standard_normal(m.n_free)
    got = _cpu(s.smooth(_gpu(x), _gpu(b), level=0))
    ref = sm.smooth(x, b)
    conds = [np.linalg.cond(B) for _, G in sm.groups for B in G[:50]]
    print("nu %g: rel diff %.2e, max patch cond %.1e" % (nu, rel(got, ref), max(conds)))
    assert rel(got, ref) < 1e-12


@pytest.mark.parametrize("gamma", [1, 2])
def test_cycle_matches_the_oracle(gamma):
    n, levels = 32, 3
    s, P = _solver(n, 0.49, levels=levels, gamma=gamma)
    H = Hierarchy(n, P, K_tri=K_TZ, smoother="vanka", omega=0.8, nu1=2, nu2=2, levels=levels, bc="terzaghi",
                  vanka_shift=SHIFT, gamma=gamma)
    rng = np.random.default_rng(13)
    b = rng.standard_normal(H.A.shape[0])
    got = _cpu(s.vcycle(_gpu(b)))
    ref = H.vcycle(b)
    print("gamma %d: rel diff %.2e" % (gamma, rel(got, ref)))
    assert rel(got, ref) < 1e-8


def test_time_step_rhs_from_the_operator():
    """b^m = load + (0, 0, alpha B_u u^{m-1}): the pressure rows of A applied to the previous
    displacement alone, formed on the GPU, equal the oracle's right-hand side."""
    n = 16
    T = Terzaghi(n, 0.45, K_TZ)
    s, _ = _solver(n, 0.45)
    m = T.mesh
    rng = np.random.default_rng(17)
    x_prev = T.full(rng.standard_normal(m.n_free))
    ref = T.rhs(x_prev)
    got = _gpu_rhs(s, T, x_prev[m.free_full])
    assert rel(got, ref) < 1e-14


def _gpu_rhs(s, T, x_prev_free):
    m = T.mesh
    xu = np.zeros(m.n_free)
    xu[:m.n_u] = x_prev_free[:m.n_u]
    y = _cpu(s.apply(_gpu(xu)))
    b = T.load_u[m.free_full].copy()
    b[m.n_u + m.n_w:] = y[m.n_u + m.n_w:]
    return b


def test_first_step_matches_the_oracle():
    """The first step of the nu = 0.4 run (left-preconditioned GMRES(30) to 1e-6): the same
    iteration count, and the same iterate to within the solves' common tolerance."""
    n = 64
    T = Terzaghi(n, 0.4, K_TZ)
    s, P = _solver(n, 0.4, levels=4)
    b = T.rhs(np.zeros(T.mesh.n_full))
    H = Hierarchy(n, T.params, K_tri=K_TZ, smoother="vanka", omega=0.8, nu1=2, nu2=2, levels=4, bc="terzaghi",
                  vanka_shift=SHIFT)
    xr, ir = gmres_left(H.A, b, H.vcycle, tol=1e-6, restart=30, maxit=60)
    xg, ig = s.solve(_gpu(b), tol=1e-6, restart=30, maxit=60, side="left")
    assert ig["converged"] and ir["converged"]
    assert ig["iters"] == ir["iters"]
    d = rel(_cpu(xg), xr)
    print("first step: %d iterations, rel diff %.2e" % (ig["iters"], d))
    assert d < 1e-8


def _gpu_run(nu, golden):
    n = golden["n"]
    T = Terzaghi(n, nu, K_TZ)
    s, _ = _solver(n, nu, levels=golden["levels"], omega=golden["omega"], nu_s=golden["nu1"], shift=golden["shift"])
    x = np.zeros(T.mesh.n_free)
    its = []
    for _ in range(golden["steps"]):
        b = _gpu_rhs(s, T, x)
        xg, info = s.solve(_gpu(b), tol=golden["tol"], restart=golden["restart"], maxit=60, side="left")
        assert info["converged"]
        its.append(info["iters"])
        x = _cpu(xg)
    eu, ep = T.errors(T.full(x), golden["steps"] * T.tau)
    return its, eu, ep


@pytest.mark.parametrize("nu", [0.4, 0.45, 0.49, 0.499])
def test_table6_on_the_gpu(nu):
    golden = json.load(open(GOLDEN))
    ref = golden["runs"][repr(nu)]
    its, eu, ep = _gpu_run(nu, golden)
    print("nu %g: GPU %s (avg %.1f), oracle %s (avg %.1f), paper %.1f; errors u %.3e p %.3e (oracle %.3e %.3e)"
          % (nu, its, np.mean(its), ref["iters"], np.mean(ref["iters"]), TABLE6[nu], eu, ep, ref["err_u_H1"],
             ref["err_p_L2"]))
    assert all(abs(a - b) <= 1 for a, b in zip(its, ref["iters"]))
    assert abs(np.mean(its) - TABLE6[nu]) <= 2.0
    assert abs(ep - ref["err_p_L2"]) <= 1e-3 * ref["err_p_L2"]
    assert abs(eu - ref["err_u_H1"]) <= 1e-2 * ref["err_u_H1"]


def test_unavailable_calls_and_singular_patches_are_refused():
    b = _binding()
    s, _ = _solver(8, 0.4)
    with pytest.raises(b.BiotError) as e:
        s.setup(levels=2, nu1=1, nu2=1, omega=0.8, vanka_shift=0.0)
    assert e.value.code == b.BIOT_ERR_ARG and b"vanka_shift" in str(e.value).encode()
    with pytest.raises(b.BiotError):
        s.setup(levels=2, smoother="bsr", vanka_shift=SHIFT)
    with pytest.raises(b.BiotError):
        s.setup(levels=2, precision="fp32", vanka_shift=SHIFT)
    s.setup(levels=2, nu1=1, nu2=1, omega=0.8, vanka_shift=SHIFT)
    x = _gpu(np.zeros(s.nf()))
    with pytest.raises(b.BiotError):
        s.solve_noalloc(x, torch.empty_like(x))
    with pytest.raises(b.BiotError):
        s.grad_logK(x, x)
    with pytest.raises(b.BiotError):
        s.timing_start()
    with pytest.raises(b.BiotError):
        s.export_layout(patches=True)
    # the Dirichlet path refuses a patch shift
    lam, mu, P = _params(0.4, 8)
    d = b.BiotSolver(8, lam, mu, alpha=1.0, M=1e6, mu_f=1.0, tau=P.tau, K=K_TZ)
    with pytest.raises(b.BiotError):
        d.setup(levels=2, vanka_shift=SHIFT)


def test_update_K_reassembles_every_level():
    n, levels = 16, 3
    s, P = _solver(n, 0.45, levels=levels)
    K = K_TZ * np.exp(np.random.default_rng(23).uniform(-1, 1, 2 * n * n))
    s.update_K(_gpu(K))
    H = Hierarchy(n, P, K_tri=K, smoother="vanka", omega=0.8, nu1=2, nu2=2, levels=levels, bc="terzaghi",
                  vanka_shift=SHIFT)
    rng = np.random.default_rng(29)
    for l, lev in enumerate(H.levels):
        x = rng.standard_normal(lev.A.shape[0])
        assert rel(_cpu(s.apply(_gpu(x), level=l)), lev.A @ x) < 1e-13
    b = rng.standard_normal(H.A.shape[0])
    assert rel(_cpu(s.vcycle(_gpu(b))), H.vcycle(b)) < 1e-8


def test_update_logK_on_the_general_path():
    """biot_update_logK on the general-boundary path: 1/K = exp(-theta) formed on the device, every
    level re-assembled; the operators match the oracle's for K = exp(theta)."""
    n, levels = 16, 3
    s, P = _solver(n, 0.49, levels=levels)
    theta = np.log(K_TZ) + np.random.default_rng(37).uniform(-1.5, 1.5, 2 * n * n)
    s.update_logK(_gpu(theta))
    K = np.exp(theta)
    H = Hierarchy(n, P, K_tri=K, smoother="vanka", omega=0.8, nu1=2, nu2=2, levels=levels, bc="terzaghi",
                  vanka_shift=SHIFT)
    rng = np.random.default_rng(41)
    for l, lev in enumerate(H.levels):
        x = rng.standard_normal(lev.A.shape[0])
        assert rel(_cpu(s.apply(_gpu(x), level=l)), lev.A @ x) < 1e-13, l
    b = rng.standard_normal(H.A.shape[0])
    assert rel(_cpu(s.vcycle(_gpu(b))), H.vcycle(b)) < 1e-8
