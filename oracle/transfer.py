"""Block prolongation P = diag(P_u, P_w, P_p) between nested uniform meshes n/2 -> n.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Paper passages followed:
  * Sec. 3, eq. (eq:block_interp): P is block diagonal; P_w and P_p are the canonical
    finite-element interpolants for RT0 and P0; restriction R = P^T; coarse operators by
    rediscretization.
  * Sec. 3.1 (divergence-preserving interpolation, Fig. div_free_interp): P_u starts from
    the standard finite-element interpolant of each coarse basis function; then, on every
    coarse triangle, the bubble DoFs of the three fine edges interior to it are replaced so
    that the interpolated function has zero net normal flux out of each fine triangle it is
    asked for (eq. divfreefine).  Reading used here: each of the three *corner* children has
    exactly one interior edge, and that edge's bubble is set so that the corner child's net
    flux vanishes; the interior child then carries the whole flux of the coarse triangle,
    so an RQ-divergence-free coarse field maps to an RQ-divergence-free fine field.
  * Sec. 2.1: the bubble DoF interpolates the integrated normal displacement across the
    edge; with the bubble normalised to normal value 1 at the midpoint its coefficient on a
    fine edge e is  (int_e (u_H - I_1 u_H).n_e) / (int_e b_e.n_e).

Everything is evaluated geometrically from barycentric coordinates; no stencil constant is
typed in by hand.
"""
import numpy as np
import scipy.sparse as sp

from .mesh import Mesh


def _bary(Xtri, x):
    """Barycentric coordinates of points x (m, 2) in triangles Xtri (m, 3, 2)."""
    a, b, c = Xtri[:, 0], Xtri[:, 1], Xtri[:, 2]
    det = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    l1 = ((x[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (x[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])) / det
    l2 = ((b[:, 0] - a[:, 0]) * (x[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (x[:, 0] - a[:, 0])) / det
    return np.stack([1.0 - l1 - l2, l1, l2], axis=1)


def _coarse_u_values(mc: Mesh, T, beta):
    """Values (m, 9, 2) of the 9 local displacement basis functions of coarse triangles T
    at barycentric points beta (m, 3); local order [ux(v0..2), uy(v0..2), b(e0..2)]."""
    m = T.size
    out = np.zeros((m, 9, 2))
    for a in range(3):
        out[:, a, 0] = beta[:, a]
        out[:, 3 + a, 1] = beta[:, a]
    nrm = mc.edge_normal[mc.tri_edge[T]]          # (m, 3, 2)
    for k in range(3):
        p, q = (k + 1) % 3, (k + 2) % 3
        out[:, 6 + k] = 4.0 * (beta[:, p] * beta[:, q])[:, None] * nrm[:, k]
    return out


def _coarse_u_dofs(mc: Mesh, T):
    tv = mc.tri_vert[T]
    te = mc.tri_edge[T]
    return np.concatenate([mc.off_ux + tv, mc.off_uy + tv, mc.off_b + te], axis=1)


class _Setter:
    """Sparse matrix builder with 'set' semantics: repeated writes must agree."""

    def __init__(self, shape):
        self.shape = shape
        self.d = {}

    def set(self, r, c, v, tol=1e-12):
        for ri, ci, vi in zip(np.ravel(r), np.ravel(c), np.ravel(v)):
            key = (int(ri), int(ci))
            if key in self.d:
                if abs(self.d[key] - vi) > tol * max(1.0, abs(vi)):
                    raise AssertionError("inconsistent prolongation entry %s: %g vs %g" % (key, self.d[key], vi))
            else:
                self.d[key] = float(vi)

    def csr(self):
        if not self.d:
            return sp.csr_matrix(self.shape)
        keys = np.array(list(self.d.keys()), dtype=np.int64)
        vals = np.array(list(self.d.values()))
        M = sp.coo_matrix((vals, (keys[:, 0], keys[:, 1])), shape=self.shape).tocsr()
        M.eliminate_zeros()
        return M


def _fine_edge_lookup(mf: Mesh):
    return {tuple(sorted(map(int, e))): k for k, e in enumerate(mf.edge_ends)}


def _vertex_id_at(mf: Mesh, x):
    ij = np.rint(x / mf.h).astype(np.int64)
    return ij[..., 1] * (mf.n + 1) + ij[..., 0]


def prolongation(mf: Mesh, mc: Mesh):
    """Return (P_full, P_free): fine-full x coarse-full and fine-free x coarse-free."""
    assert mf.n == 2 * mc.n
    Nf, Nc = mf.n_full, mc.n_full
    S = _Setter((Nf, Nc))
    elook = _fine_edge_lookup(mf)
    Tc = np.arange(mc.n_tri)
    Xc = mc.vert_xy[mc.tri_vert]                     # (nTc, 3, 2)
    cdofs = _coarse_u_dofs(mc, Tc)                   # (nTc, 9)
    # ---- P_u, canonical step: fine vertex values --------------------------------------
    # fine vertices inside coarse triangle T: its corners and edge midpoints
    bpts = [np.array(b, dtype=float) for b in
            ([1, 0, 0], [0, 1, 0], [0, 0, 1], [0, .5, .5], [.5, 0, .5], [.5, .5, 0])]
    for b in bpts:
        beta = np.repeat(b[None, :], Tc.size, axis=0)
        x = np.einsum("ta,tai->ti", beta, Xc)
        vf = _vertex_id_at(mf, x)
        vals = _coarse_u_values(mc, Tc, beta)         # (nTc, 9, 2)
        for comp, off in ((0, mf.off_ux), (1, mf.off_uy)):
            rows = np.repeat((off + vf)[:, None], 9, axis=1)
            S.set(rows, cdofs, vals[:, :, comp])
    # ---- P_u, canonical step: bubbles of fine edges on and inside T -------------------
    # the 9 fine edges of a coarse triangle, as pairs of barycentric points
    corner = [np.eye(3)[k] for k in range(3)]
    mid = {}
    for k in range(3):
        p, q = (k + 1) % 3, (k + 2) % 3
        mv = np.zeros(3)
        mv[p] = mv[q] = 0.5
        mid[(min(p, q), max(p, q))] = mv
    def M(a, b):
        return mid[(min(a, b), max(a, b))]
    half_edges = []
    for k in range(3):
        p, q = (k + 1) % 3, (k + 2) % 3
        half_edges.append((corner[p], M(p, q)))
        half_edges.append((M(p, q), corner[q]))
    # corner child at local vertex k: (corner k, mid(k,k+1), mid(k,k+2)); interior edge
    # joins the two midpoints
    children = []
    for k in range(3):
        a, b = (k + 1) % 3, (k + 2) % 3
        children.append((corner[k], M(k, a), M(k, b)))

    def fine_edge(xa, xb):
        va = _vertex_id_at(mf, xa)
        vb = _vertex_id_at(mf, xb)
        return np.array([elook[tuple(sorted((int(s), int(t))))] for s, t in zip(va, vb)])

    def pts(b):
        beta = np.repeat(b[None, :], Tc.size, axis=0)
        return beta, np.einsum("ta,tai->ti", beta, Xc)

    def bubble_coef(ba, bb):
        """Canonical bubble coefficient on fine edge [ba, bb]: (u(m) - (u(a)+u(b))/2).n_e."""
        beta_a, xa = pts(ba)
        beta_b, xb = pts(bb)
        beta_m, xm = pts(0.5 * (ba + bb))
        ua = _coarse_u_values(mc, Tc, beta_a)
        ub = _coarse_u_values(mc, Tc, beta_b)
        um = _coarse_u_values(mc, Tc, beta_m)
        e = fine_edge(xa, xb)
        n_e = mf.edge_normal[e]                       # (nTc, 2)
        c = np.einsum("tfi,ti->tf", um - 0.5 * (ua + ub), n_e)
        return e, c

    for (ba, bb) in half_edges:
        e, c = bubble_coef(ba, bb)
        rows = np.repeat((mf.off_b + e)[:, None], 9, axis=1)
        S.set(rows, cdofs, c)
    # ---- P_u, correction: zero net flux out of every corner child ---------------------
    for (b0, b1, b2) in children:
        verts = [b0, b1, b2]
        flux = np.zeros((Tc.size, 9))
        xs = [pts(b)[1] for b in verts]
        cen = (xs[0] + xs[1] + xs[2]) / 3.0
        e_int = None
        sig_int = None
        len_int = None
        for (ka, kb) in ((0, 1), (1, 2), (2, 0)):
            ba, bb = verts[ka], verts[kb]
            beta_a, xa = pts(ba)
            beta_b, xb = pts(bb)
            e = fine_edge(xa, xb)
            d = xb - xa
            L = np.linalg.norm(d, axis=1)
            n_e = mf.edge_normal[e]
            out = 0.5 * (xa + xb) - cen
            sig = np.sign(np.einsum("ti,ti->t", n_e, out))
            # outward unit normal of the child on this edge
            n_out = sig[:, None] * n_e
            # P1 part: int_e (linear interpolant) . n_out = |e| (u(a) + u(b))/2 . n_out
            ua = _coarse_u_values(mc, Tc, beta_a)
            ub = _coarse_u_values(mc, Tc, beta_b)
            flux += L[:, None] * np.einsum("tfi,ti->tf", 0.5 * (ua + ub), n_out)
            interior = not (np.any(np.isclose(ba, 1.0)) or np.any(np.isclose(bb, 1.0)))
            if interior:
                e_int, sig_int, len_int = e, sig, L
            else:
                _, c = bubble_coef(ba, bb)
                flux += (sig * (2.0 / 3.0) * L)[:, None] * c
        c_int = -flux / (sig_int * (2.0 / 3.0) * len_int)[:, None]
        rows = np.repeat((mf.off_b + e_int)[:, None], 9, axis=1)
        S.set(rows, cdofs, c_int)
    # ---- P_w: normal component of the coarse RT0 field on each fine edge --------------
    te_c = mc.tri_edge
    sig_c = np.zeros((mc.n_tri, 3))
    len_c = np.zeros((mc.n_tri, 3))
    area_c = 0.5 * np.abs((Xc[:, 1, 0] - Xc[:, 0, 0]) * (Xc[:, 2, 1] - Xc[:, 0, 1])
                          - (Xc[:, 1, 1] - Xc[:, 0, 1]) * (Xc[:, 2, 0] - Xc[:, 0, 0]))
    for k in range(3):
        a, b = Xc[:, (k + 1) % 3], Xc[:, (k + 2) % 3]
        len_c[:, k] = np.linalg.norm(b - a, axis=1)
        out = 0.5 * (a + b) - Xc[:, k]
        sig_c[:, k] = np.sign(np.einsum("ti,ti->t", mc.edge_normal[te_c[:, k]], out))
    fine_edges_of_T = half_edges + [(M(0, 1), M(1, 2)), (M(1, 2), M(2, 0)), (M(2, 0), M(0, 1))]
    for (ba, bb) in fine_edges_of_T:
        beta_m, xm = pts(0.5 * (ba + bb))
        _, xa = pts(ba)
        _, xb = pts(bb)
        e = fine_edge(xa, xb)
        n_e = mf.edge_normal[e]
        for k in range(3):
            psi = (sig_c[:, k] * len_c[:, k] / (2.0 * area_c))[:, None] * (xm - Xc[:, k])
            val = np.einsum("ti,ti->t", psi, n_e)
            S.set(mf.off_w + e, mc.off_w + te_c[:, k], val)
    # ---- P_p: injection (fine triangle takes its parent's value) -----------------------
    cen_f = mf.vert_xy[mf.tri_vert].mean(axis=1)
    H = mc.h
    I = np.floor(cen_f[:, 0] / H).astype(np.int64)
    J = np.floor(cen_f[:, 1] / H).astype(np.int64)
    upper = (cen_f[:, 0] - I * H) + (cen_f[:, 1] - J * H) > H
    parent = np.where(upper, mc.n * mc.n, 0) + J * mc.n + I
    S.set(mf.off_p + np.arange(mf.n_tri), mc.off_p + parent, np.ones(mf.n_tri))
    P_full = S.csr()
    P_free = P_full[mf.free_full][:, mc.free_full].tocsr()
    return P_full, P_free
