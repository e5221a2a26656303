"""Fourier symbols of the assembled operators on the ten DoF types (Sec. 4, App. A-B).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Paper passages followed:
  * Sec. 4.1, Def. (formulation-symbol-classical): the symbol of a stencil operator is
    sum_kappa s_kappa exp(i theta . kappa).
  * Appendix A: for the staggered DoF types the stencil offsets kappa are the differences of
    DoF positions; bubble/RT0 DoFs sit at their edge midpoints, P1 DoFs at the vertices.
    The P0 DoFs of both triangles of a square are placed at the square centre, which is
    what the printed B_u and B_w symbols imply.
  * Appendix B, Def. (def-R-symbol-G): restriction symbol
        R~(theta^alpha) = (sum_kappa r_kappa exp(i kappa . theta^alpha)) exp(i pi alpha . x / h)
    with x the coarse DoF position on the fine grid.

Positions are in units of the level's own h, relative to the lower-left vertex (i, j).
"""
import numpy as np

from .mesh import Mesh

TYPES = ["ux", "uy", "bH", "bV", "bD", "wH", "wV", "wD", "pL", "pU"]
OFFSET = {"ux": (0.0, 0.0), "uy": (0.0, 0.0), "bH": (0.5, 0.0), "bV": (0.0, 0.5),
          "bD": (0.5, 0.5), "wH": (0.5, 0.0), "wV": (0.0, 0.5), "wD": (0.5, 0.5),
          "pL": (0.5, 0.5), "pU": (0.5, 0.5)}


def dof_at(mesh: Mesh, t, i, j):
    """Canonical free index of the DoF of type t anchored at (i, j), or -1."""
    if t == "ux":
        return mesh.dof_ux(i, j)
    if t == "uy":
        return mesh.dof_uy(i, j)
    k = {"H": 0, "V": 1, "D": 2}
    if t[0] == "b":
        return mesh.dof_b(k[t[1]], i, j)
    if t[0] == "w":
        return mesh.dof_w(k[t[1]], i, j)
    return mesh.dof_p(t == "pU", i, j)


def dof_types_positions(mesh: Mesh):
    """(type index, position (x, y) in units of h) of every canonical free DoF."""
    typ = -np.ones(mesh.n_free, dtype=np.int64)
    pos = np.zeros((mesh.n_free, 2))
    n = mesh.n
    for ti, t in enumerate(TYPES):
        ox, oy = OFFSET[t]
        for j in range(n + 1):
            for i in range(n + 1):
                d = dof_at(mesh, t, i, j)
                if d >= 0:
                    typ[d] = ti
                    pos[d] = (i + ox, j + oy)
    assert np.all(typ >= 0)
    return typ, pos


def operator_symbol(A, mesh: Mesh, theta, ref=None, row_types=TYPES, col_types=TYPES):
    """Block symbol of a free-DoF matrix A read off the rows anchored at cell `ref`."""
    if ref is None:
        ref = (mesh.n // 2, mesh.n // 2)
    typ, pos = dof_types_positions(mesh)
    A = A.tocsr()
    th = np.asarray(theta, dtype=float)
    S = np.zeros((len(row_types), len(col_types)), dtype=complex)
    cidx = {TYPES.index(t): k for k, t in enumerate(col_types)}
    for a, t in enumerate(row_types):
        r = dof_at(mesh, t, *ref)
        assert r >= 0, "reference cell must be interior"
        lo, hi = A.indptr[r], A.indptr[r + 1]
        for c, v in zip(A.indices[lo:hi], A.data[lo:hi]):
            ct = int(typ[c])
            if ct in cidx:
                S[a, cidx[ct]] += v * np.exp(1j * np.dot(th, pos[c] - pos[r]))
    return S


def restriction_symbol(P, mf: Mesh, mc: Mesh, theta_a, alpha, ref=None,
                       row_types=TYPES, col_types=TYPES):
    """Restriction symbol block R~(theta^alpha) of R = P^T (rows coarse types, cols fine)."""
    if ref is None:
        ref = (mc.n // 2, mc.n // 2)
    typ_f, pos_f = dof_types_positions(mf)
    R = P.T.tocsr()
    th = np.asarray(theta_a, dtype=float)
    al = np.asarray(alpha, dtype=float)
    S = np.zeros((len(row_types), len(col_types)), dtype=complex)
    cidx = {TYPES.index(t): k for k, t in enumerate(col_types)}
    for a, t in enumerate(row_types):
        rc = dof_at(mc, t, *ref)
        assert rc >= 0
        ox, oy = OFFSET[t]
        X = 2.0 * np.array([ref[0] + ox, ref[1] + oy])      # coarse position, fine units
        lo, hi = R.indptr[rc], R.indptr[rc + 1]
        for f, v in zip(R.indices[lo:hi], R.data[lo:hi]):
            ft = int(typ_f[f])
            if ft in cidx:
                S[a, cidx[ft]] += v * np.exp(1j * np.dot(th, pos_f[f] - X))
        S[a] *= np.exp(1j * np.pi * np.dot(al, X))
    return S
