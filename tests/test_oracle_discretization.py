"""Pins of the oracle's discretization against what the paper prints and what the
mathematics fixes: DoF counts, the Appendix A stencils and symbols, symmetry, inertia,
the rank of B_u (Sec. 2.3) and the reduced-quadrature identity."""
import os

import numpy as np
import pytest

from oracle.mesh import Mesh, canonical_block_sizes
from oracle.fem import Assembly, BiotParams, ElementData
from oracle.symbols import operator_symbol, dof_at

GOLD = os.path.join(os.path.dirname(__file__), "golden")
S2 = np.sqrt(2.0)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16])
def test_free_dof_count(n):
    m = Mesh(n)
    assert m.n_free == 10 * n * n - 8 * n + 2
    assert sum(canonical_block_sizes(n)) == m.n_free
    # the canonical order is block by block, row-major inside every block
    sizes = canonical_block_sizes(n)
    starts = np.cumsum([0] + sizes)
    assert m.dof_ux(1, 1) == starts[0] if n > 1 else True
    assert m.dof_p(False, 0, 0) == starts[8]
    assert m.dof_p(True, n - 1, n - 1) == m.n_free - 1


def _fixture_rows():
    rows = []
    with open(os.path.join(GOLD, "appendixA_stencils.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            p = line.split()
            if p[2] == "all":
                rows.append((p[0], p[1], None, None, 0.0))
            else:
                val = eval(p[4], {"sqrt": np.sqrt})
                rows.append((p[0], p[1], int(p[2]), int(p[3]), float(val)))
    return rows


def test_appendixA_stencils_of_2mu_Aeps():
    """Appendix A: every printed interior stencil value of 2 mu A_eps (mu = 1)."""
    n, i0, j0 = 8, 4, 4
    m = Mesh(n)
    asm = Assembly(m, BiotParams(lam=0.0, mu=1.0))
    A = (2.0 * asm.free(asm.A_eps_full)).tocsr()
    rows = _fixture_rows()
    pairs = {}
    for (rt, ct, di, dj, v) in rows:
        pairs.setdefault((rt, ct), {})
        if di is not None:
            pairs[(rt, ct)][(di, dj)] = v
    for (rt, ct), ent in pairs.items():
        r = dof_at(m, rt, i0, j0)
        assert r >= 0
        # all nonzeros of row r within column type ct
        got = {}
        for dj in range(-3, 4):
            for di in range(-3, 4):
                c = dof_at(m, ct, i0 + di, j0 + dj)
                if c >= 0 and A[r, c] != 0.0:
                    got[(di, dj)] = A[r, c]
        for k in set(got) | set(ent):
            assert abs(got.get(k, 0.0) - ent.get(k, 0.0)) < 1e-12, (rt, ct, k, got.get(k), ent.get(k))


def _rand_theta(seed):
    return np.random.default_rng(seed).uniform(-np.pi, np.pi, 2)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_appendixA_symbols(seed):
    """Appendix A symbols of 2 mu A_eps, M_w, M_p, B_u, B_w at a random frequency.

    Reading: the printed second/third bubble positions are the x-normal edge (offset
    (0, h/2)) and the y-normal edge (offset (h/2, 0)), as the B_u / B_w symbols imply; the
    last entry of the printed B_w symbol is read as -exp(i theta_2 / 2)."""
    n, h = 8, 1.0 / 8
    m = Mesh(n)
    k, mu = 0.37, 1.0
    asm = Assembly(m, BiotParams(lam=0.0, mu=mu, mu_f=1.0), K_tri=k)
    t1, t2 = th = _rand_theta(seed)
    E = lambda a: np.exp(1j * a)
    c = np.cos
    # --- 2 mu A_eps: bubble-bubble (D, V, H), P1-P1, bubble->P1 -----------------------
    Aeps = 2.0 * asm.free(asm.A_eps_full)
    S = operator_symbol(Aeps, m, th, row_types=["bD", "bV", "bH"], col_types=["bD", "bV", "bH"])
    ref = mu * np.array([[28 / 3, -10 * S2 / 3 * c(t1 / 2), -10 * S2 / 3 * c(t2 / 2)],
                         [-10 * S2 / 3 * c(t1 / 2), 8, 4 / 3 * c((t1 - t2) / 2)],
                         [-10 * S2 / 3 * c(t2 / 2), 4 / 3 * c((t1 - t2) / 2), 8]])
    assert np.abs(S - ref).max() < 1e-12
    S = operator_symbol(Aeps, m, th, row_types=["ux", "uy"], col_types=["ux", "uy"])
    off = 1 - c(t1) - c(t2) + c(t1 - t2)
    ref = mu * np.array([[6 - 4 * c(t1) - 2 * c(t2), off], [off, 6 - 4 * c(t2) - 2 * c(t1)]])
    assert np.abs(S - ref).max() < 1e-12
    S = operator_symbol(Aeps, m, th, row_types=["ux", "uy"], col_types=["bD", "bV", "bH"])
    dd = S2 * (c((t1 - t2) / 2) - c((t1 + t2) / 2))
    ref = 8 * mu / 3 * np.array([[dd, c(t2 / 2) - c(t1 - t2 / 2), 0.0],
                                 [dd, 0.0, c(t1 / 2) - c(t2 - t1 / 2)]])
    assert np.abs(S - ref).max() < 1e-12
    # --- M_w (order D, V, H) -------------------------------------------------------------
    Mw = asm.free(asm.Mw_full)
    S = operator_symbol(Mw, m, th, row_types=["wD", "wV", "wH"], col_types=["wD", "wV", "wH"])
    ref = h * h / (3 * k) * np.array([[2, 0, 0], [0, 2, -c((t1 - t2) / 2)], [0, -c((t1 - t2) / 2), 2]])
    assert np.abs(S - ref).max() < 1e-14
    # --- M_p -----------------------------------------------------------------------------
    Mp = asm.free(asm.Mp_full)
    S = operator_symbol(Mp, m, th, row_types=["pL", "pU"], col_types=["pL", "pU"])
    assert np.abs(S - h * h / 2 * np.eye(2)).max() < 1e-15
    # --- B_u (rows pL, pU; columns bD, bV, bH, ux, uy) -------------------------------
    Bu = asm.free(asm.Bu_full)
    S = operator_symbol(Bu, m, th, row_types=["pL", "pU"], col_types=["bD", "bV", "bH", "ux", "uy"])
    d1 = E(t1 / 2) - E(-t1 / 2)
    d2 = E(t2 / 2) - E(-t2 / 2)
    ref = h * np.array([
        [-2 * S2 / 3, 2 / 3 * E(-t1 / 2), 2 / 3 * E(-t2 / 2), -0.5 * d1 * E(-t2 / 2), -0.5 * d2 * E(-t1 / 2)],
        [2 * S2 / 3, -2 / 3 * E(t1 / 2), -2 / 3 * E(t2 / 2), -0.5 * d1 * E(t2 / 2), -0.5 * d2 * E(t1 / 2)]])
    assert np.abs(S - ref).max() < 1e-14
    # --- B_w (rows pL, pU; columns wD, wV, wH) ------------------------------------------
    Bw = asm.free(asm.Bw_full)
    S = operator_symbol(Bw, m, th, row_types=["pL", "pU"], col_types=["wD", "wV", "wH"])
    ref = h * np.array([[-S2, E(-t1 / 2), E(-t2 / 2)], [S2, -E(t1 / 2), -E(t2 / 2)]])
    assert np.abs(S - ref).max() < 1e-14


@pytest.mark.parametrize("n", [2, 4])
def test_symmetry_and_saddle_point_inertia(n):
    """Sec. 2.1: the scaling makes the system symmetric; the u and w blocks are SPD and the
    pressure Schur complement is negative definite, so the inertia is (n_u + n_w, 0, n_p)."""
    m = Mesh(n)
    p = BiotParams.from_E_nu(1.0, 0.3, alpha=0.8, M=50.0, mu_f=1.3, tau=0.7)
    K = np.random.default_rng(n).uniform(0.2, 3.0, m.n_tri)
    A = Assembly(m, p, K).A
    assert abs(A - A.T).max() == 0.0
    ev = np.linalg.eigvalsh(A.toarray())
    assert np.sum(ev > 0) == m.n_u + m.n_w
    assert np.sum(ev < 0) == m.n_p


@pytest.mark.parametrize("n", [4, 8])
def test_rank_of_Bu_and_divergence_free_count(n):
    """Sec. 2.3: with reduced quadrature the divergence constraint has N_T - 1 independent
    rows (Dirichlet data), leaving 3 divergence-free functions per interior vertex."""
    m = Mesh(n)
    asm = Assembly(m, BiotParams(1.0, 1.0))
    su, sw, sp_ = asm.slices()
    Bu = asm.free(asm.Bu_full)[sp_, su].toarray()
    s = np.linalg.svd(Bu, compute_uv=False)
    rank = int(np.sum(s > 1e-10 * s[0]))
    assert rank == m.n_tri - 1
    assert m.n_u - rank == 3 * (n - 1) ** 2


def _edge_flux(m, ed, coef_u):
    """int_{dT} u . n_out for every triangle, from field values at the edge end points and
    midpoint (Simpson's rule, exact for the quadratic field along an edge)."""
    ux = np.zeros(m.n_vert)
    uy = np.zeros(m.n_vert)
    bb = np.zeros(m.n_edge)
    full = np.zeros(m.n_full)
    full[m.free_full[: m.n_u]] = coef_u
    ux[:] = full[m.off_ux:m.off_ux + m.n_vert]
    uy[:] = full[m.off_uy:m.off_uy + m.n_vert]
    bb[:] = full[m.off_b:m.off_b + m.n_edge]
    flux = np.zeros(m.n_tri)
    for t in range(m.n_tri):
        vs = m.tri_vert[t]
        cen = m.vert_xy[vs].mean(axis=0)
        for k in range(3):
            a, b = vs[(k + 1) % 3], vs[(k + 2) % 3]
            e = m.tri_edge[t, k]
            xa, xb = m.vert_xy[a], m.vert_xy[b]
            L = np.linalg.norm(xb - xa)
            nrm = np.array([xb[1] - xa[1], xa[0] - xb[0]]) / L
            if np.dot(nrm, 0.5 * (xa + xb) - cen) < 0:
                nrm = -nrm
            va = np.array([ux[a], uy[a]])
            vb = np.array([ux[b], uy[b]])
            vm = 0.5 * (va + vb) + bb[e] * m.edge_normal[e]   # bubble value 1 at midpoint
            flux[t] += L / 6.0 * np.dot(va + 4 * vm + vb, nrm)
    return flux


def test_reduced_quadrature_term_from_boundary_fluxes():
    """Sec. 2.3: lambda (P_Q div u, P_Q div v) = lambda sum_T (int_T div u)(int_T div v)/|T|,
    computed here from boundary fluxes (divergence theorem), independently of the
    element divergence integrals used in the assembly."""
    n = 4
    m = Mesh(n)
    lam = 2.5
    asm = Assembly(m, BiotParams(lam=lam, mu=0.0))
    su, _, _ = asm.slices()
    Arq = asm.A[su, su]
    rng = np.random.default_rng(7)
    u = rng.standard_normal(m.n_u)
    v = rng.standard_normal(m.n_u)
    ed = ElementData(m)
    fu = _edge_flux(m, ed, u)
    fv = _edge_flux(m, ed, v)
    ref = lam * np.sum(fu * fv / ed.area)
    assert abs(u @ (Arq @ v) - ref) < 1e-12 * max(1.0, abs(ref))
