"""The oracle against Table 4 (Sec. 5.1) under the left-preconditioned reading of its stopping
test: GMRES on M^{-1} A x = M^{-1} b with one V(2,2) Vanka cycle as M (the paper's Table 2
weights, h = 1/64, four levels, direct solve at h = 1/8), stopping when the preconditioned
residual falls below 1e-6 of its initial value.  The paper states only a relative-residual
tolerance; with the true residual of right-preconditioned FGMRES the oracle takes 1.2 to 1.4
times the printed counts in every cell, with this reading it takes the printed counts to +-2
(all 36 Vanka cells were run; three are checked here, the GPU test checks all 36).  The same reading does
not reproduce the BSR row (tabulated in the design notes)."""
import os

import pytest

from paper_2107_04060_amd import inputs
from oracle import manufactured as mf
from oracle.fem import BiotParams
from oracle.krylov import gmres_left
from oracle.multigrid import Hierarchy

GOLD = os.path.join(os.path.dirname(__file__), "golden")
KS = [1.0, 1e-2, 1e-4, 1e-6, 1e-8, 1e-10]


def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        return [l.split() for l in f if l.strip() and not l.startswith("#")]


def _paper(sm, nu, k):
    for r in _rows("table4_iterations.txt"):
        if r[0] == sm and float(r[1]) == nu:
            return int(r[2 + KS.index(k)])
    raise KeyError((sm, nu, k))


def _omega(nu, k):
    for r in _rows("table2_vanka.txt"):
        if float(r[0]) == nu and float(r[1]) == k:
            return float(r[2])
    raise KeyError((nu, k))


@pytest.mark.slow
@pytest.mark.parametrize("nu,k", [(0.0, 1e-4), (0.4, 1.0), (0.499, 1e-10)])
def test_vanka_counts_under_the_left_preconditioned_reading(nu, k):
    lam, mu = inputs.lame(3e4, nu)
    P = BiotParams(lam, mu, alpha=1.0, M=1e6, mu_f=1.0, tau=1.0)
    H = Hierarchy(64, P, K_tri=k, smoother="vanka", omega=_omega(nu, k), nu1=2, nu2=2, levels=4)
    _, info = gmres_left(H.A, mf.rhs(64, P), H.vcycle, tol=1e-6, restart=30, maxit=100)
    print("vanka nu %g k %g: %d iterations (paper %d)" % (nu, k, info["iters"], _paper("vanka", nu, k)))
    assert info["converged"]
    assert abs(info["iters"] - _paper("vanka", nu, k)) <= 2
