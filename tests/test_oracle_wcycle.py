"""Pins of the cycle index gamma of oracle/multigrid.py (the W-cycle, gamma = 2).

* gamma = 1 is the V-cycle, and with two levels every gamma gives the same cycle (the coarsest
  level is solved exactly and not revisited).
* Revisiting a level gamma times makes its correction converge to the exact coarse solve: with
  three levels and a large gamma, one cycle equals the two-level cycle whose coarse problem (the
  middle mesh) is solved by sparse LU, to the contraction of the middle level's own cycle raised
  to gamma.
* On the paper's steady problem the W-cycle makes BSR converge where the V-cycle stalls
  (nu = 0.45, k = 1e-8 and nu = 0.4, k = 1e-4, Table 4).
"""
import os

import numpy as np
import pytest

from oracle import manufactured as mf
from oracle.fem import BiotParams
from oracle.krylov import fgmres
from oracle.multigrid import Hierarchy
from paper_2107_04060_amd import inputs


def _P():
    return BiotParams.from_E_nu(1.0, 0.3, alpha=1.0, M=50.0, mu_f=1.0, tau=0.5)


@pytest.mark.parametrize("smoother", ["vanka", "bsr"])
def test_gamma_one_and_two_levels(smoother):
    n = 16
    b = inputs.rhs_uniform(n, 3)
    kw = dict(K_tri=1e-2, smoother=smoother, omega=0.8, omega_J=1.0, nu1=1, nu2=1)
    v = Hierarchy(n, _P(), levels=3, **kw).vcycle(b)
    v1 = Hierarchy(n, _P(), levels=3, gamma=1, **kw).vcycle(b)
    assert np.array_equal(v, v1)
    t1 = Hierarchy(n, _P(), levels=2, gamma=1, **kw).vcycle(b)
    t3 = Hierarchy(n, _P(), levels=2, gamma=3, **kw).vcycle(b)
    assert np.array_equal(t1, t3)


@pytest.mark.parametrize("smoother", ["vanka", "bsr"])
def test_many_visits_reach_the_two_level_cycle(smoother):
    n = 16
    b = inputs.rhs_uniform(n, 4)
    kw = dict(K_tri=1e-2, smoother=smoother, omega=0.8, omega_J=1.0, nu1=2, nu2=2)
    tg = Hierarchy(n, _P(), levels=2, **kw).vcycle(b)          # middle mesh (8 x 8) by LU
    w = Hierarchy(n, _P(), levels=3, gamma=40, **kw).vcycle(b)
    assert np.linalg.norm(w - tg) <= 1e-10 * np.linalg.norm(tg)
    w2 = Hierarchy(n, _P(), levels=3, gamma=2, **kw).vcycle(b)
    assert np.linalg.norm(w2 - tg) > 1e-6 * np.linalg.norm(tg)   # two visits are not yet exact


def _bsr_weights(nu, k):
    """(omega, omega_J) of Table 3 (tests/golden/table3_bsr.txt)."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "table3_bsr.txt")) as f:
        for l in f:
            r = l.split()
            if r and not l.startswith("#") and float(r[0]) == nu and float(r[1]) == k:
                return float(r[3]), float(r[2])
    raise KeyError((nu, k))


@pytest.mark.parametrize("nu,k", [(0.45, 1e-8), (0.4, 1e-4)])
def test_wcycle_converges_where_the_vcycle_stalls(nu, k):
    omega, omega_J = _bsr_weights(nu, k)
    P = BiotParams.from_E_nu(3e4, nu, alpha=1.0, M=1e6, mu_f=1.0, tau=1.0)
    b = mf.rhs(64, P)
    H = Hierarchy(64, P, K_tri=k, smoother="bsr", omega=omega, omega_J=omega_J, nu1=1, nu2=1, levels=4, gamma=2)
    _, info = fgmres(H.A, b, H.vcycle, tol=1e-6, restart=30, maxit=100)
    print("nu %g k %g BSR W(1,1): %d iterations" % (nu, k, info["iters"]))
    assert info["converged"] and info["iters"] <= 60


def test_gamma_from_keeps_the_fine_levels_to_one_correction():
    """gamma_from = 1 on four levels: the finest level takes one coarse correction, which is the
    W-cycle of the three coarser levels, composed here by hand from the full W-cycle hierarchy's
    own level-1 cycle; gamma_from = levels - 2 repeats nothing and is the V-cycle."""
    n = 32
    b = inputs.rhs_uniform(n, 5)
    kw = dict(K_tri=1e-2, smoother="vanka", omega=0.8, nu1=2, nu2=2, levels=4)
    Hw = Hierarchy(n, _P(), gamma=2, **kw)
    Hf = Hierarchy(n, _P(), gamma=2, gamma_from=1, **kw)
    lev = Hw.levels[0]
    x = np.zeros_like(b)
    for _ in range(2):
        x = lev.smoother.smooth(x, b)
    xc = Hw.vcycle(lev.P.T @ (b - lev.A @ x), level=1)
    x = x + lev.P @ xc
    for _ in range(2):
        x = lev.smoother.smooth(x, b)
    got = Hf.vcycle(b)
    assert np.linalg.norm(got - x) <= 1e-13 * np.linalg.norm(x)
    assert np.linalg.norm(got - Hw.vcycle(b)) > 1e-6 * np.linalg.norm(x)
    v = Hierarchy(n, _P(), **kw).vcycle(b)
    assert np.array_equal(Hierarchy(n, _P(), gamma=2, gamma_from=2, **kw).vcycle(b), v)
