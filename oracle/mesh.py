"""Structured triangulation of the unit square and the canonical numbering of the
bubble-enriched P1 / RT0 / P0 degrees of freedom.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Paper passages followed:
  * Sec. 2.1: displacement in P1 enriched with one face-normal bubble per edge,
    Darcy velocity in lowest-order Raviart-Thomas (RT0), pressure in P0.
  * Appendix A (opening paragraph): the mesh of the unit square is a grid of squares,
    each cut once along the diagonal from its top-left to its bottom-right corner.
  * Sec. 4.2, Fig. DoF_structure2: per square, 2 P1 components, 3 edge bubbles,
    3 RT0 fluxes and 2 P0 values (lower-left and upper-right triangle).

Conventions (the paper does not fix them; they are the readings listed in the design
notes and are pinned by the Appendix A stencils in the tests):
  * n cells per side, h = 1/n; vertex (i, j) sits at (i h, j h), 0 <= i, j <= n.
  * H(i, j): edge (i, j)-(i+1, j), unit normal +y.   0 <= i < n, 0 <= j <= n
    V(i, j): edge (i, j)-(i, j+1), unit normal +x.   0 <= i <= n, 0 <= j < n
    D(i, j): edge (i, j+1)-(i+1, j), normal (1,1)/sqrt2.  0 <= i, j < n
  * L(i, j) = {(i,j), (i+1,j), (i,j+1)},  U(i, j) = {(i+1,j), (i+1,j+1), (i,j+1)}.
    Local edge k of a triangle is the edge opposite local vertex k.
  * Boundary conditions (bc):
      "dirichlet" (the default, Sec. 5.1): u = 0 and w.n = 0 on the whole boundary: the P1 DoFs
        of boundary vertices and the bubble / RT0 DoFs of boundary edges are eliminated.
      "terzaghi" (Sec. 5, Terzaghi's problem): the column is loaded and drained on x = 0
        (traction and p = 0, both natural: u and w.n free there), fixed and impermeable on
        x = 1 (u = 0, w.n = 0), and on rollers, impermeable, on y = 0 and y = 1 (u.n = u_y = 0,
        w.n = 0; u_x free).  Eliminated: u_x, u_y at x = 1; u_y at y = 0, 1; bubble and RT0 on
        the edges of x = 1, y = 0 and y = 1.
  * Canonical free-DoF order, each block row-major in (j, i):
      [u_x(interior vertices), u_y(interior vertices), b_H, b_V, b_D (interior edges),
       w_H, w_V, w_D (interior edges), p_L, p_U]
"""
import numpy as np

SQRT2 = np.sqrt(2.0)


class Mesh:
    """Uniform n x n triangulated square with the full and the free DoF numbering."""

    BCS = ("dirichlet", "terzaghi")

    def __init__(self, n, bc="dirichlet"):
        n = int(n)
        if n < 1:
            raise ValueError("n must be >= 1")
        if bc not in self.BCS:
            raise ValueError("bc: one of %s" % (self.BCS,))
        self.n = n
        self.bc = bc
        self.h = 1.0 / n
        nv1 = n + 1
        # ---- entity counts and ids ------------------------------------------------
        self.n_vert = nv1 * nv1
        self.n_H = n * nv1
        self.n_V = nv1 * n
        self.n_D = n * n
        self.n_edge = self.n_H + self.n_V + self.n_D
        self.n_tri = 2 * n * n
        # ---- vertex coordinates -----------------------------------------------------
        jj, ii = np.meshgrid(np.arange(nv1), np.arange(nv1), indexing="ij")
        self.vert_ij = np.stack([ii.ravel(), jj.ravel()], axis=1)  # id = j*(n+1)+i
        self.vert_xy = self.vert_ij * self.h
        # ---- edges: endpoints and global unit normal -------------------------------
        ends = np.zeros((self.n_edge, 2), dtype=np.int64)
        normal = np.zeros((self.n_edge, 2))
        kind = np.zeros(self.n_edge, dtype=np.int64)  # 0 = H, 1 = V, 2 = D
        e_ij = np.zeros((self.n_edge, 2), dtype=np.int64)
        e = 0
        for j in range(nv1):
            for i in range(n):
                ends[e] = (self.vid(i, j), self.vid(i + 1, j))
                normal[e] = (0.0, 1.0)
                kind[e] = 0
                e_ij[e] = (i, j)
                e += 1
        for j in range(n):
            for i in range(nv1):
                ends[e] = (self.vid(i, j), self.vid(i, j + 1))
                normal[e] = (1.0, 0.0)
                kind[e] = 1
                e_ij[e] = (i, j)
                e += 1
        for j in range(n):
            for i in range(n):
                ends[e] = (self.vid(i, j + 1), self.vid(i + 1, j))
                normal[e] = (1.0 / SQRT2, 1.0 / SQRT2)
                kind[e] = 2
                e_ij[e] = (i, j)
                e += 1
        self.edge_ends = ends
        self.edge_normal = normal
        self.edge_kind = kind
        self.edge_ij = e_ij
        # ---- triangles: vertices (counter-clockwise) and opposite edges -------------
        tv = np.zeros((self.n_tri, 3), dtype=np.int64)
        te = np.zeros((self.n_tri, 3), dtype=np.int64)
        t = 0
        for j in range(n):
            for i in range(n):  # L(i, j)
                tv[t] = (self.vid(i, j), self.vid(i + 1, j), self.vid(i, j + 1))
                te[t] = (self.did(i, j), self.vedge(i, j), self.hid(i, j))
                t += 1
        for j in range(n):
            for i in range(n):  # U(i, j)
                tv[t] = (self.vid(i + 1, j), self.vid(i + 1, j + 1), self.vid(i, j + 1))
                te[t] = (self.hid(i, j + 1), self.did(i, j), self.vedge(i + 1, j))
                t += 1
        self.tri_vert = tv
        self.tri_edge = te
        # ---- boundary flags ----------------------------------------------------------
        vi, vj = self.vert_ij[:, 0], self.vert_ij[:, 1]
        self.vert_interior = (vi > 0) & (vi < n) & (vj > 0) & (vj < n)
        ei, ej = e_ij[:, 0], e_ij[:, 1]
        self.edge_interior = np.where(
            kind == 0, (ej > 0) & (ej < n), np.where(kind == 1, (ei > 0) & (ei < n), True)
        )
        # ---- full DoF numbering --------------------------------------------------------
        self.off_ux = 0
        self.off_uy = self.n_vert
        self.off_b = 2 * self.n_vert
        self.off_w = self.off_b + self.n_edge
        self.off_p = self.off_w + self.n_edge
        self.n_full = self.off_p + self.n_tri
        if bc == "dirichlet":
            ux_free = uy_free = self.vert_interior
            e_free = self.edge_interior
        else:
            ux_free = vi < n
            uy_free = (vi < n) & (vj > 0) & (vj < n)
            e_free = np.where(kind == 0, (ej > 0) & (ej < n), np.where(kind == 1, ei < n, True))
        free = np.zeros(self.n_full, dtype=bool)
        free[self.off_ux:self.off_ux + self.n_vert] = ux_free
        free[self.off_uy:self.off_uy + self.n_vert] = uy_free
        free[self.off_b:self.off_b + self.n_edge] = e_free
        free[self.off_w:self.off_w + self.n_edge] = e_free
        free[self.off_p:] = True
        self.free_mask = free
        self.free_full = np.nonzero(free)[0]          # canonical index -> full index
        self.full_to_free = -np.ones(self.n_full, dtype=np.int64)
        self.full_to_free[self.free_full] = np.arange(self.free_full.size)
        self.n_free = int(self.free_full.size)
        # number of free DoFs of each field in canonical order
        nu = int(ux_free.sum()) + int(uy_free.sum()) + int(e_free.sum())
        nw = int(e_free.sum())
        self.n_u, self.n_w, self.n_p = nu, nw, self.n_tri

    # ---- entity id helpers -------------------------------------------------------------
    def vid(self, i, j):
        return j * (self.n + 1) + i

    def hid(self, i, j):
        return j * self.n + i

    def vedge(self, i, j):
        return self.n_H + j * (self.n + 1) + i

    def did(self, i, j):
        return self.n_H + self.n_V + j * self.n + i

    def lid(self, i, j):
        return j * self.n + i

    def uid(self, i, j):
        return self.n * self.n + j * self.n + i

    # ---- DoF helpers (canonical free index, or -1 when the DoF is eliminated / absent) --
    def _free(self, full):
        return int(self.full_to_free[full])

    def dof_ux(self, i, j):
        if 0 <= i <= self.n and 0 <= j <= self.n:
            return self._free(self.off_ux + self.vid(i, j))
        return -1

    def dof_uy(self, i, j):
        if 0 <= i <= self.n and 0 <= j <= self.n:
            return self._free(self.off_uy + self.vid(i, j))
        return -1

    def _edge_ok(self, kind, i, j):
        n = self.n
        if kind == 0:
            return 0 <= i < n and 0 <= j <= n
        if kind == 1:
            return 0 <= i <= n and 0 <= j < n
        return 0 <= i < n and 0 <= j < n

    def _edge_id(self, kind, i, j):
        return (self.hid, self.vedge, self.did)[kind](i, j)

    def dof_b(self, kind, i, j):
        if not self._edge_ok(kind, i, j):
            return -1
        return self._free(self.off_b + self._edge_id(kind, i, j))

    def dof_w(self, kind, i, j):
        if not self._edge_ok(kind, i, j):
            return -1
        return self._free(self.off_w + self._edge_id(kind, i, j))

    def dof_p(self, upper, i, j):
        if not (0 <= i < self.n and 0 <= j < self.n):
            return -1
        t = self.uid(i, j) if upper else self.lid(i, j)
        return self._free(self.off_p + t)

    def free_count_formula(self):
        """10 n^2 - 8 n + 2 free DoFs under full Dirichlet data."""
        n = self.n
        return 10 * n * n - 8 * n + 2


def canonical_block_sizes(n):
    """Sizes of the ten canonical blocks [ux, uy, bH, bV, bD, wH, wV, wD, pL, pU]."""
    nv = (n - 1) * (n - 1)
    ne_h = n * (n - 1)
    ne_v = n * (n - 1)
    nd = n * n
    return [nv, nv, ne_h, ne_v, nd, ne_h, ne_v, nd, n * n, n * n]
