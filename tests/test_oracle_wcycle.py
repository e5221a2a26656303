"""Pins of the cycle index gamma of oracle/multigrid.py (the W-cycle, gamma = 2).

* gamma = 1 is the V-cycle, and with two levels every gamma gives the same cycle (the coarsest
  level is solved exactly and not revisited).
* Revisiting a level gamma times makes its correction converge to the exact coarse solve: with
  three levels and a large gamma, one cycle equals the two-level cycle whose coarse problem (the
  middle mesh) is solved by sparse LU, to the contraction of the middle level's own cycle raised
  to gamma.
* On the paper's steady problem the W-cycle makes BSR converge where the V-cycle stalls
  (nu = 0.45, k = 1e-8 and nu = 0.4, k = 1e-4, Table 4).
* The F-cycle (fcycle: the further coarse corrections are V-cycles): on three levels it is the
  W-cycle; on four its top level is the F-cycle of the three coarser levels followed by a
  V-cycle of them, composed here by hand; counted smoother calls give m + 1 visits of level m
  (W-cycle: 2^m); with gamma = 1 it is the V-cycle.
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


def _count_visits(H, b):
    """Smoothing calls per level of one cycle, divided by nu1 + nu2 (visits)."""
    counts = [0] * (len(H.levels) - 1)
    for l, lev in enumerate(H.levels[:-1]):
        f = lev.smoother.smooth

        def wrapped(x, bb, _f=f, _l=l):
            counts[_l] += 1
            return _f(x, bb)
        lev.smoother.smooth = wrapped
    H.vcycle(b)
    return [c // (H.nu1 + H.nu2) for c in counts]


def test_fcycle_pins():
    n = 32
    b = inputs.rhs_uniform(n, 6)
    kw = dict(K_tri=1e-2, smoother="vanka", omega=0.8, nu1=1, nu2=1)
    # three levels: the F-cycle is the W-cycle
    assert np.array_equal(Hierarchy(n, _P(), levels=3, gamma=2, fcycle=True, **kw).vcycle(b),
                          Hierarchy(n, _P(), levels=3, gamma=2, **kw).vcycle(b))
    # gamma = 1: the V-cycle
    assert np.array_equal(Hierarchy(n, _P(), levels=4, gamma=1, fcycle=True, **kw).vcycle(b),
                          Hierarchy(n, _P(), levels=4, **kw).vcycle(b))
    # four levels, composed by hand from the level-1 cycles of the F and V hierarchies
    Hf = Hierarchy(n, _P(), levels=4, gamma=2, fcycle=True, **kw)
    Hv = Hierarchy(n, _P(), levels=4, **kw)
    lev = Hf.levels[0]
    x = lev.smoother.smooth(np.zeros_like(b), b)
    bc = lev.P.T @ (b - lev.A @ x)
    xc = Hf.vcycle(bc, level=1)
    xc = xc + Hv.vcycle(bc - Hf.levels[1].A @ xc, level=1)
    x = lev.smoother.smooth(x + lev.P @ xc, b)
    got = Hf.vcycle(b)
    assert np.linalg.norm(got - x) <= 1e-13 * np.linalg.norm(x)
    Hw = Hierarchy(n, _P(), levels=4, gamma=2, **kw)
    assert np.linalg.norm(got - Hw.vcycle(b)) > 1e-6 * np.linalg.norm(x)


def test_fcycle_and_wcycle_visit_counts():
    n = 64
    b = inputs.rhs_uniform(n, 7)
    kw = dict(K_tri=1e-2, smoother="vanka", omega=0.8, nu1=1, nu2=1, levels=5)
    assert _count_visits(Hierarchy(n, _P(), gamma=2, fcycle=True, **kw), b) == [1, 2, 3, 4]
    assert _count_visits(Hierarchy(n, _P(), gamma=2, **kw), b) == [1, 2, 4, 8]
    assert _count_visits(Hierarchy(n, _P(), gamma=2, gamma_from=1, fcycle=True, **kw), b) == [1, 1, 2, 3]
    assert _count_visits(Hierarchy(n, _P(), **kw), b) == [1, 1, 1, 1]


def test_gamma_to_stops_the_repetition():
    """gamma_to = k: only levels gamma_from <= l < k repeat their coarse correction, so the levels
    below k are visited as often as level k; gamma_to = gamma_from is the V-cycle."""
    n = 64
    b = inputs.rhs_uniform(n, 9)
    kw = dict(K_tri=1e-2, smoother="vanka", omega=0.8, nu1=1, nu2=1, levels=6)
    assert _count_visits(Hierarchy(n, _P(), gamma=2, gamma_from=1, **kw), b) == [1, 1, 2, 4, 8]
    assert _count_visits(Hierarchy(n, _P(), gamma=2, gamma_from=1, gamma_to=3, **kw), b) == [1, 1, 2, 4, 4]
    assert _count_visits(Hierarchy(n, _P(), gamma=2, gamma_from=0, gamma_to=2, **kw), b) == [1, 2, 4, 4, 4]
    v = Hierarchy(n, _P(), **kw).vcycle(b)
    assert np.array_equal(Hierarchy(n, _P(), gamma=2, gamma_from=2, gamma_to=2, **kw).vcycle(b), v)


def test_additive_levels_pins():
    """additive_levels = 0 is the multiplicative hierarchy; additive_levels = levels - 1 (every
    smoothing level additive, with omega_additive) is the additive hierarchy of that weight; one
    additive level is neither (the finest level's smoother is additive, the rest coloured)."""
    n = 32
    b = inputs.rhs_uniform(n, 11)
    kw = dict(K_tri=1e-2, smoother="vanka", nu1=1, nu2=1, levels=4, gamma=2, gamma_from=1)
    m = Hierarchy(n, _P(), omega=1.1, vanka_colors=3, **kw).vcycle(b)
    assert np.array_equal(Hierarchy(n, _P(), omega=1.1, vanka_colors=3, additive_levels=0, **kw).vcycle(b), m)
    a = Hierarchy(n, _P(), omega=0.7, **kw).vcycle(b)
    assert np.array_equal(Hierarchy(n, _P(), omega=1.1, vanka_colors=3, additive_levels=3, omega_additive=0.7,
                                    **kw).vcycle(b), a)
    h = Hierarchy(n, _P(), omega=1.1, vanka_colors=3, additive_levels=1, omega_additive=0.7, **kw).vcycle(b)
    assert np.linalg.norm(h - m) > 1e-6 * np.linalg.norm(m) and np.linalg.norm(h - a) > 1e-6 * np.linalg.norm(a)
