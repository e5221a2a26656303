"""Pins of the BSR Schur-complement sweeps (oracle/smoothers.py, InexactBSR with
schur_sweeps > 1: k weighted-Jacobi sweeps on the approximate Schur complement of Sec. 3.2.2
and Appendix D instead of the paper's single step).

* S_hat applied by the smoother equals c_u M_p + A_pw (tau D_w)^{-1} A_pw^T assembled as a
  sparse matrix from the operator blocks, and its diagonal is the smoother's diag(S_hat).
* Many sweeps converge to the exact solve of S_hat (sparse LU).
* Two sweeps with weight w from zero give w s/d + w (s - S_hat w s/d)/d, written out.
* On the paper's steady problem (Sec. 5.1) at nu = 0.45, k = 1e-8, where the single step fails
  (the paper needs 452 iterations), two sweeps converge in about 20 FGMRES iterations.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import manufactured as mf
from oracle.fem import Assembly, BiotParams
from oracle.krylov import fgmres
from oracle.mesh import Mesh
from oracle.multigrid import Hierarchy
from oracle.smoothers import InexactBSR


def _smoother(n=8, k=1e-3, sweeps=1, w=1.0):
    P = BiotParams.from_E_nu(1.0, 0.3, alpha=1.0, M=50.0, mu_f=1.0, tau=0.5)
    K = np.exp(np.random.default_rng(1).uniform(-2, 2, 2 * n * n)) * k
    asm = Assembly(Mesh(n), P, K)
    return asm, P, InexactBSR(asm, 0.8, 1.1, sweeps, w)


def test_schur_operator_and_diagonal():
    asm, P, sm = _smoother()
    su, sw, sp_ = asm.slices()
    A = asm.A.tocsr()
    Apw = A[sp_, sw]
    Dww = A[sw, sw].diagonal()
    Mp = asm.free(asm.Mp_full)[sp_, sp_].diagonal()
    c_u = P.inv_M + P.alpha ** 2 / (P.lam + P.mu)
    S = sp.diags(c_u * Mp) + Apw @ sp.diags(1.0 / Dww) @ Apw.T
    v = np.random.default_rng(2).standard_normal(S.shape[0])
    assert np.allclose(sm.schur_apply(v), S @ v, rtol=1e-13, atol=0)
    assert np.allclose(sm.diagS, S.diagonal(), rtol=1e-13, atol=0)


def test_many_sweeps_reach_the_exact_solve():
    asm, P, sm = _smoother(sweeps=400, w=1.0)
    su, sw, sp_ = asm.slices()
    s = np.random.default_rng(3).standard_normal(sp_.stop - sp_.start)
    S = sp.diags(sm.cMp) + sm.Apw @ sp.diags(1.0 / sm.Dww) @ sm.Apw.T
    exact = spla.spsolve(S.tocsc(), s)
    assert np.linalg.norm(sm.schur_solve(s) - exact) <= 1e-8 * np.linalg.norm(exact)


def test_two_sweeps_written_out():
    asm, P, sm = _smoother(sweeps=2, w=0.7)
    s = np.random.default_rng(4).standard_normal(sm.diagS.size)
    d1 = 0.7 * s / sm.diagS
    d2 = d1 + 0.7 * (s - sm.schur_apply(d1)) / sm.diagS
    assert np.allclose(sm.schur_solve(s), d2, rtol=1e-14, atol=0)
    one = InexactBSR(asm, 0.8, 1.1)
    assert np.allclose(one.schur_solve(s), 1.1 * s / one.diagS, rtol=1e-15, atol=0)


def test_two_sweeps_rescue_the_failing_cell():
    P = BiotParams.from_E_nu(3e4, 0.45, alpha=1.0, M=1e6, mu_f=1.0, tau=1.0)
    b = mf.rhs(64, P)
    H = Hierarchy(64, P, K_tri=1e-8, smoother="bsr", omega=0.74, omega_J=1.26, nu1=1, nu2=1, levels=4,
                  schur_sweeps=2, omega_S=1.0)
    _, info = fgmres(H.A, b, H.vcycle, tol=1e-6, restart=30, maxit=100)
    print("nu 0.45 k 1e-8, two Schur sweeps: %d iterations" % info["iters"])
    assert info["converged"] and info["iters"] <= 30


def _cg_smoother(k, n=8):
    P = BiotParams.from_E_nu(1.0, 0.3, alpha=1.0, M=50.0, mu_f=1.0, tau=0.5)
    K = np.exp(np.random.default_rng(1).uniform(-2, 2, 2 * n * n)) * 1e-3
    asm = Assembly(Mesh(n), P, K)
    return asm, InexactBSR(asm, 0.8, 1.1, schur_cg=k)


def _schur_matrix(sm):
    return (sp.diags(sm.cMp) + sm.Apw @ sp.diags(1.0 / sm.Dww) @ sm.Apw.T).tocsc()


def test_cg_steps_minimize_the_energy_error_over_the_krylov_space():
    """k steps of diag(S_hat)-preconditioned CG from zero return the vector of the Krylov space
    span{D^-1 s, (D^-1 S) D^-1 s, ...} (k vectors, D = diag(S_hat)) closest to S^-1 s in the S-norm:
    checked against that Galerkin projection built from an explicit orthonormal basis."""
    for k in (1, 3, 6):
        asm, sm = _cg_smoother(k)
        S = _schur_matrix(sm).toarray()
        s = np.random.default_rng(7).standard_normal(S.shape[0])
        D = sm.diagS
        vecs = [s / D]
        for _ in range(k - 1):
            vecs.append((S @ vecs[-1]) / D)
        Q, _ = np.linalg.qr(np.column_stack(vecs))
        ref = Q @ np.linalg.solve(Q.T @ S @ Q, Q.T @ s)
        got = sm.schur_solve(s)
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref), k


def test_one_cg_step_written_out():
    asm, sm = _cg_smoother(1)
    s = np.random.default_rng(8).standard_normal(sm.diagS.size)
    z = s / sm.diagS
    ref = (s @ z) / (z @ sm.schur_apply(z)) * z
    assert np.allclose(sm.schur_solve(s), ref, rtol=1e-14, atol=0)


def test_many_cg_steps_give_exact_bsr():
    """With enough CG steps the pressure correction is the exact solve of S_hat (sparse LU), and
    the whole BSR correction equals the one with that exact solve in its place (exact BSR on the
    approximate Schur complement, Sec. 3.2.2)."""
    asm, sm = _cg_smoother(200)
    S = _schur_matrix(sm)
    lu = spla.splu(S)
    s = np.random.default_rng(9).standard_normal(S.shape[0])
    exact = lu.solve(s)
    assert np.linalg.norm(sm.schur_solve(s) - exact) <= 1e-10 * np.linalg.norm(exact)
    r = np.random.default_rng(10).standard_normal(asm.n_free)
    got = sm.step_correction(r)
    sm_exact = InexactBSR(asm, 0.8, 1.1)
    sm_exact.schur_solve = lu.solve
    ref = sm_exact.step_correction(r)
    assert np.linalg.norm(got - ref) <= 1e-9 * np.linalg.norm(ref)


def test_cg_rescues_the_failing_cell():
    P = BiotParams.from_E_nu(3e4, 0.45, alpha=1.0, M=1e6, mu_f=1.0, tau=1.0)
    b = mf.rhs(64, P)
    H = Hierarchy(64, P, K_tri=1e-8, smoother="bsr", omega=0.74, omega_J=1.26, nu1=1, nu2=1, levels=4,
                  schur_cg=4)
    _, info = fgmres(H.A, b, H.vcycle, tol=1e-6, restart=30, maxit=100)
    print("nu 0.45 k 1e-8, four Schur CG steps: %d iterations" % info["iters"])
    assert info["converged"] and info["iters"] <= 30
