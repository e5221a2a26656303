"""Pins of the oracle's two-grid local Fourier analysis (Sec. 4) against the paper's
printed LFA predictions: Table 2 (additive Vanka V(2,2)) and Table 3 (inexact BSR V(1,1)),
h = 1/64, E = 3e4, M = 1e6, alpha = mu_f = tau = 1, K = k I
(tests/golden/table2_vanka.txt, table3_bsr.txt).

Every cell's rho_LFA at the printed weights must agree to within 1e-3 (the print has three
decimals).  The search must also return the printed Vanka omega_opt, and the printed BSR
weights must be a local minimum on the 0.01 grid.  These pins exercise the whole
discretization at once: operator symbols (App. A), restriction symbols including the
divergence-preserving P_u (App. B), and the Vanka and BSR symbols (App. C-D)."""
import os

import numpy as np
import pytest

from oracle.fem import BiotParams, lame_from_E_nu
from oracle.lfa import TwoGridLFA, Stencil, scaled_matrix, theta_samples
from oracle.symbols import operator_symbol

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _table(name):
    with open(os.path.join(GOLD, name)) as f:
        return [[float(v) for v in l.split()] for l in f if l.strip() and not l.startswith("#")]


def _params(nu):
    lam, mu = lame_from_E_nu(3e4, nu)
    return BiotParams(lam, mu, alpha=1.0, M=1e6, mu_f=1.0, tau=1.0)


def test_stencil_symbol_matches_row_symbol():
    """The vectorized symbol of the extracted stencil equals the row-by-row symbol."""
    P = _params(0.3)
    asm, A = scaled_matrix(P, 1 / 64, 1e-3)
    st = Stencil(A, asm.mesh)
    th = theta_samples(4)[:5]
    S = st.symbol(th)
    for k in range(th.shape[0]):
        assert np.allclose(S[k], operator_symbol(A, asm.mesh, th[k], ref=(4, 4)), rtol=0, atol=1e-12)


def test_table2_vanka_rho_lfa_every_cell():
    worst = 0.0
    for nu, k, w, rho_lfa, _ in _table("table2_vanka.txt"):
        rho = TwoGridLFA(_params(nu), 1 / 64, K=k, smoother="vanka", nu=4).rho(w)
        worst = max(worst, abs(rho - rho_lfa))
        assert abs(rho - rho_lfa) < 1e-3, (nu, k, rho, rho_lfa)
    print("worst deviation %.1e" % worst)


def test_table3_bsr_rho_lfa_every_cell():
    for nu, k, wj, w, rho_lfa, _ in _table("table3_bsr.txt"):
        rho = TwoGridLFA(_params(nu), 1 / 64, K=k, smoother="bsr", nu=2).rho(w, wj)
        assert abs(rho - rho_lfa) < 1e-3, (nu, k, rho, rho_lfa)


@pytest.mark.parametrize("nu,k", [(0.0, 1.0), (0.4, 1.0), (0.499, 1e-6)])
def test_table2_vanka_omega_opt(nu, k):
    row = [r for r in _table("table2_vanka.txt") if r[0] == nu and r[1] == k][0]
    w, rho = TwoGridLFA(_params(nu), 1 / 64, K=k, smoother="vanka", nu=4).optimize_vanka(0.6, 1.0, 0.02)
    assert abs(w - row[2]) < 0.021 and abs(rho - row[3]) < 1e-3, (w, rho, row)


@pytest.mark.parametrize("nu,k", [(0.4, 1.0), (0.49, 1.0)])
def test_table3_bsr_weights_are_local_minimum(nu, k):
    row = [r for r in _table("table3_bsr.txt") if r[0] == nu and r[1] == k][0]
    L = TwoGridLFA(_params(nu), 1 / 64, K=k, smoother="bsr", nu=2)
    at = L.rho(row[3], row[2])
    for da in (-0.01, 0.0, 0.01):
        for db in (-0.01, 0.0, 0.01):
            assert L.rho(row[3] + db, row[2] + da) >= at - 2e-3


def test_stored_workload_weights_are_the_lfa_optimum():
    """The weights table the workloads use (written by oracle/relaxation_weights.py) holds
    the LFA optimum: recompute one Vanka entry and one BSR rho."""
    from paper_2107_04060_amd import inputs
    from oracle.relaxation_weights import vanka_weight
    lam, mu = inputs.lame(1.0, 0.49)
    P = BiotParams(lam, mu, alpha=1.0, M=inputs.biot_modulus(1.0), mu_f=1.0, tau=1.0)
    w = vanka_weight(P, 1 / 256, 1e-3, 2)
    assert inputs.relaxation_weights("vanka", 0.49, 1e-3) == (w["omega"], 1.0)
    om, omj = inputs.relaxation_weights("bsr", 0.49, 1e-3)
    rho = TwoGridLFA(P, 1 / 256, K=1e-3, smoother="bsr", nu=2).rho(om, omj)
    stored = inputs._weights_table()["sweep256"]["0.49/0.001"]["bsr"]["rho_lfa"]
    assert abs(rho - stored) < 1e-3


def test_table4_ridge_weights_are_as_good_as_the_papers():
    """tests/golden/table4_bsr_lfa_weights.txt (written by oracle/relaxation_weights.py --table4)
    holds one BSR weight pair per cell of Table 4.  In sampled cells (the paper's two failures,
    the cell where the paper's weights need 341 iterations here, and one plain cell) the stored
    two-grid factor is reproduced and is no worse than that of the paper's Table 3 weights
    (within the search's 1e-3 flatness tolerance); in the two failing cells the two factors agree
    to 0.02 while omega_J differs by more than 0.2: both pairs lie on the same flat ridge."""
    paper = {(r[0], r[1]): (r[3], r[2]) for r in _table("table3_bsr.txt")}
    rows = _table("table4_bsr_lfa_weights.txt")
    assert len(rows) == 36
    for nu, k, wj, w, rho_lfa in rows:
        if (nu, k) not in ((0.45, 1e-8), (0.49, 1e-8), (0.4, 1e-4), (0.0, 1.0)):
            continue
        L = TwoGridLFA(_params(nu), 1 / 64, K=k, smoother="bsr", nu=2)
        rho = L.rho(w, wj)
        pw, pwj = paper[(nu, k)]
        rho_paper = L.rho(pw, pwj)
        assert abs(rho - rho_lfa) < 1e-3, (nu, k, rho, rho_lfa)
        assert rho <= rho_paper + 1.5e-3, (nu, k, rho, rho_paper)
        if k == 1e-8 and nu in (0.45, 0.49):
            assert abs(rho - rho_paper) < 0.02 and abs(wj - pwj) > 0.2, (nu, k, rho, rho_paper, wj, pwj)
