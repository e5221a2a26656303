"""Pins of the oracle's grid transfers: Appendix B restriction symbols, divergence
preservation (Sec. 3.1), exactness of the canonical RT0 and P0 interpolants."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.mesh import Mesh
from oracle.fem import Assembly, BiotParams
from oracle.transfer import prolongation
from oracle.symbols import restriction_symbol

S2 = np.sqrt(2.0)


@pytest.fixture(scope="module")
def P16():
    mf, mc = Mesh(16), Mesh(8)
    return mf, mc, prolongation(mf, mc)[1]


def _cc(a):
    return np.exp(1j * a) + np.exp(-1j * a)


ALPHAS = [(0, 0), (1, 0), (0, 1), (1, 1)]


@pytest.mark.parametrize("alpha", ALPHAS)
def test_appendixB_Ru_symbol(P16, alpha):
    """Appendix B, R_u: bubble block, P1 block, P1->bubble block and d1..d6.

    Reading: the bubble block's off-diagonal D/(V,H) factors come out as 5 sqrt2/8 in the
    coarse-D row and sqrt2/8 in the coarse-(V,H) rows, i.e. the printed matrix has these two
    factors in swapped positions; the flux reading of Sec. 3.1 (tested for exact divergence
    preservation below) fixes them this way."""
    mf, mc, P = P16
    th0 = np.random.default_rng(hash(alpha) % 2 ** 31).uniform(-np.pi / 2, np.pi / 2, 2)
    t1, t2 = th0 + np.pi * np.array(alpha)
    e1, e2 = (-1) ** alpha[0], (-1) ** alpha[1]
    E = lambda a: np.exp(1j * a)
    R = restriction_symbol(P, mf, mc, (t1, t2), alpha,
                           row_types=["bD", "bV", "bH"], col_types=["bD", "bV", "bH"])
    ref = np.array([
        [0.25 * _cc((t1 - t2) / 2) * e1 * e2, 5 * S2 / 8 * _cc(t2 / 2) * e1 * e2, 5 * S2 / 8 * _cc(t1 / 2) * e1 * e2],
        [S2 / 8 * _cc((t1 - t2) / 2) * e2, 0.25 * _cc(t2 / 2) * e2, -_cc(t1 / 2) * e2],
        [S2 / 8 * _cc((t1 - t2) / 2) * e1, -_cc(t2 / 2) * e1, 0.25 * _cc(t1 / 2) * e1]])
    assert np.abs(R - ref).max() < 1e-13
    R = restriction_symbol(P, mf, mc, (t1, t2), alpha, row_types=["ux", "uy"], col_types=["ux", "uy"])
    dg = 1 + 0.5 * (_cc(t1) + _cc(t2) + (E(t1 - t2) + E(t2 - t1)))
    assert np.abs(R - dg * np.eye(2)).max() < 1e-13
    R = restriction_symbol(P, mf, mc, (t1, t2), alpha, row_types=["bD", "bV", "bH"], col_types=["ux", "uy"])
    ref = np.array([[S2 / 2 * e1 * e2, S2 / 2 * e1 * e2], [e2, 0], [0, e1]])
    assert np.abs(R - ref).max() < 1e-13
    R = restriction_symbol(P, mf, mc, (t1, t2), alpha, row_types=["ux", "uy"], col_types=["bD", "bV", "bH"])
    a = 3 * S2 / 16
    b = 3 / 8
    d1 = a * _cc((t1 + t2) / 2) - a * (E((3 * t1 - t2) / 2) + E((-3 * t1 + t2) / 2))
    d2 = -b * _cc((2 * t1 + t2) / 2) + b * (E((-2 * t1 + t2) / 2) + E((2 * t1 - t2) / 2))
    d3 = -b * _cc((t1 + 2 * t2) / 2) + b * (E((3 * t1 - 2 * t2) / 2) + E((-3 * t1 + 2 * t2) / 2))
    d4 = a * _cc((t1 + t2) / 2) - a * (E((t1 - 3 * t2) / 2) + E((-t1 + 3 * t2) / 2))
    d5 = -b * _cc((2 * t1 + t2) / 2) + b * (E((-2 * t1 + 3 * t2) / 2) + E((2 * t1 - 3 * t2) / 2))
    d6 = -b * _cc((t1 + 2 * t2) / 2) + b * (E((t1 - 2 * t2) / 2) + E((-t1 + 2 * t2) / 2))
    assert np.abs(R - np.array([[d1, d2, d3], [d4, d5, d6]])).max() < 1e-13


@pytest.mark.parametrize("alpha", ALPHAS)
def test_appendixB_Rw_Rp_symbols(P16, alpha):
    mf, mc, P = P16
    th0 = np.random.default_rng(17 + 3 * alpha[0] + alpha[1]).uniform(-np.pi / 2, np.pi / 2, 2)
    t1, t2 = th0 + np.pi * np.array(alpha)
    e1, e2 = (-1) ** alpha[0], (-1) ** alpha[1]
    c1, c2 = np.cos(t1 / 2), np.cos(t2 / 2)
    c3, c4 = np.cos((t1 - t2) / 2), np.cos((t1 + t2) / 2)
    c5, c6 = np.cos((2 * t1 - t2) / 2), np.cos((t1 - 2 * t2) / 2)
    R = restriction_symbol(P, mf, mc, (t1, t2), alpha,
                           row_types=["wD", "wV", "wH"], col_types=["wD", "wV", "wH"])
    ref = np.array([[(2 * c3 + c4) * e1 * e2, S2 * c2 * e1 * e2, S2 * c1 * e1 * e2],
                    [S2 / 2 * c3 * e2, (2 * c2 + c5) * e2, -c1 * e2],
                    [S2 / 2 * c3 * e1, -c2 * e1, (2 * c1 + c6) * e1]])
    assert np.abs(R - ref).max() < 1e-13
    R = restriction_symbol(P, mf, mc, (t1, t2), alpha, row_types=["pL", "pU"], col_types=["pL", "pU"])
    em, ep = np.exp(-0.5j * (t1 + t2)), np.exp(0.5j * (t1 + t2))
    ref = e1 * e2 * np.array([[em + 2 * c3, em], [ep, ep + 2 * c3]])
    assert np.abs(R - ref).max() < 1e-13


@pytest.mark.parametrize("nc", [2, 4])
def test_divergence_preserving_prolongation(nc):
    """Sec. 3.1, eq. (divfreefine): P_u maps the RQ-divergence-free coarse space into the
    RQ-divergence-free fine space; corner children get zero flux, the interior child the
    coarse triangle's flux."""
    mf, mc = Mesh(2 * nc), Mesh(nc)
    _, P = prolongation(mf, mc)
    af, ac = Assembly(mf, BiotParams(1, 1)), Assembly(mc, BiotParams(1, 1))
    Buf = af.free(af.Bu_full)[mf.n_u + mf.n_w:, :mf.n_u]
    Buc = ac.free(ac.Bu_full)[mc.n_u + mc.n_w:, :mc.n_u]
    Pu = P[:mf.n_u, :mc.n_u]
    Z = sla.null_space(Buc.toarray())
    assert Z.shape[1] == 3 * (nc - 1) ** 2
    assert np.abs(Buf @ (Pu @ Z)).max() < 1e-13
    # arbitrary coarse field: fine fluxes are 0 on corner children, coarse flux on the
    # interior child (fine triangles listed per coarse parent)
    u = np.random.default_rng(nc).standard_normal(mc.n_u)
    fc = Buc @ u
    ff = Buf @ (Pu @ u)
    for J in range(nc):
        for I in range(nc):
            L, U = mc.dof_p(False, I, J) - mc.n_u - mc.n_w, mc.dof_p(True, I, J) - mc.n_u - mc.n_w
            off = mf.n_u + mf.n_w
            kidsL = [mf.dof_p(False, 2 * I, 2 * J), mf.dof_p(False, 2 * I + 1, 2 * J), mf.dof_p(False, 2 * I, 2 * J + 1)]
            kidsU = [mf.dof_p(True, 2 * I + 1, 2 * J + 1), mf.dof_p(True, 2 * I + 1, 2 * J), mf.dof_p(True, 2 * I, 2 * J + 1)]
            for k in kidsL + kidsU:
                assert abs(ff[k - off]) < 1e-13
            assert abs(ff[mf.dof_p(True, 2 * I, 2 * J) - off] - fc[L]) < 1e-13
            assert abs(ff[mf.dof_p(False, 2 * I + 1, 2 * J + 1) - off] - fc[U]) < 1e-13


def _rt0_eval(m, coef_w, pts):
    """Evaluate an RT0 field (free coefficients) at points, triangle by triangle."""
    full = np.zeros(m.n_full)
    full[m.free_full[m.n_u:m.n_u + m.n_w]] = coef_w
    wv = full[m.off_w:m.off_w + m.n_edge]
    out = np.zeros((pts.shape[0], 2))
    h = m.h
    for k, x in enumerate(pts):
        I, J = int(x[0] // h), int(x[1] // h)
        up = (x[0] - I * h) + (x[1] - J * h) > h
        t = m.uid(I, J) if up else m.lid(I, J)
        X = m.vert_xy[m.tri_vert[t]]
        area = 0.5 * h * h
        for kk in range(3):
            e = m.tri_edge[t, kk]
            a, b = X[(kk + 1) % 3], X[(kk + 2) % 3]
            sig = np.sign(np.dot(m.edge_normal[e], 0.5 * (a + b) - X[kk]))
            out[k] += wv[e] * sig * np.linalg.norm(b - a) / (2 * area) * (x - X[kk])
    return out


def test_Pw_reproduces_coarse_rt0_fields_and_Pp_injects():
    """Sec. 3: P_w and P_p are the canonical interpolants; an RT0 field on the coarse mesh
    is an RT0 field on the fine mesh, so P_w reproduces it pointwise, and P0 injection
    copies each parent's value to its four children."""
    mf, mc = Mesh(8), Mesh(4)
    _, P = prolongation(mf, mc)
    rng = np.random.default_rng(3)
    wc = rng.standard_normal(mc.n_w)
    wf = P[mf.n_u:mf.n_u + mf.n_w, mc.n_u:mc.n_u + mc.n_w] @ wc
    pts = rng.uniform(0.01, 0.99, (200, 2))
    assert np.abs(_rt0_eval(mf, wf, pts) - _rt0_eval(mc, wc, pts)).max() < 1e-12
    pc = rng.standard_normal(mc.n_p)
    pf = P[mf.n_u + mf.n_w:, mc.n_u + mc.n_w:] @ pc
    cen = mf.vert_xy[mf.tri_vert].mean(axis=1)
    for t in range(mf.n_tri):
        x = cen[t]
        I, J = int(x[0] // mc.h), int(x[1] // mc.h)
        up = (x[0] - I * mc.h) + (x[1] - J * mc.h) > mc.h
        assert pf[mf.full_to_free[mf.off_p + t] - mf.n_u - mf.n_w] == pc[mc.dof_p(up, I, J) - mc.n_u - mc.n_w]
    # the blocks couple no fields
    assert abs(P[:mf.n_u, mc.n_u:]).max() == 0 and abs(P[mf.n_u:mf.n_u + mf.n_w, :mc.n_u]).max() == 0
