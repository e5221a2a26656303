"""Vertex patches, additive Vanka and inexact Braess-Sarazin relaxation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Paper passages followed:
  * Sec. 3.2.1 (Vanka): for blocks l with restriction V_l, solve
    V_l A V_l^T xhat_l = V_l r and update x <- x + omega sum_l V_l^T D_l xhat_l, with the
    "natural weights" D_l = 1 / (number of patches containing the DoF).
  * Sec. 3.2.1, Fig. patches: vertex patches; the full-system patch holds the two P1 DoFs
    of the vertex, the bubble and RT0 DoFs of its six edges and the P0 DoFs of its six
    triangles (20 DoFs); the displacement patch holds the P1 and bubble DoFs (8 DoFs).
  * Sec. 3.2.2 and Appendix D (inexact BSR): M = [[F, B^T], [B, -C_2]] with
    F = diag(A_{V,u}, tau D_w), D_w = diag(M_w), A_{V,u}^{-1} one additive Vanka sweep on
    the displacement block with the 8-DoF patches, and C_2 chosen so that the Schur
    complement of M is (1/omega_J) diag(S),
        S = (1/M + alpha^2 / (lambda + 2 mu / d)) M_p + tau B_w D_w^{-1} B_w^T,  d = 2.

Readings where the paper is silent (listed in the design notes):
  * a patch is built for every vertex whose patch holds at least one free displacement or
    Darcy DoF (full patch), resp. at least one free displacement DoF (displacement patch);
    only the two corners (0,0) and (n,n) drop out, since their patches hold pressure only;
  * the inner Vanka weight inside BSR and the Jacobi weight on D_w are 1.

Patch slot order (20 slots; absent or eliminated DoFs are -1):
    [ux(v), uy(v),
     b on H(i-1,j), H(i,j), V(i,j-1), V(i,j), D(i-1,j), D(i,j-1),
     w on the same six edges,
     p on L(i,j), L(i-1,j), L(i,j-1), U(i-1,j-1), U(i-1,j), U(i,j-1)]
"""
import numpy as np

from .mesh import Mesh

EDGES_OF_VERTEX = [(0, -1, 0), (0, 0, 0), (1, 0, -1), (1, 0, 0), (2, -1, 0), (2, 0, -1)]
TRIS_OF_VERTEX = [(0, 0, 0), (0, -1, 0), (0, 0, -1), (1, -1, -1), (1, -1, 0), (1, 0, -1)]


def vertex_patch_slots(mesh: Mesh, i, j):
    """The 20 slot entries (canonical free index or -1) of the patch of vertex (i, j)."""
    s = [mesh.dof_ux(i, j), mesh.dof_uy(i, j)]
    s += [mesh.dof_b(k, i + di, j + dj) for (k, di, dj) in EDGES_OF_VERTEX]
    s += [mesh.dof_w(k, i + di, j + dj) for (k, di, dj) in EDGES_OF_VERTEX]
    s += [mesh.dof_p(up, i + di, j + dj) for (up, di, dj) in TRIS_OF_VERTEX]
    return np.array(s, dtype=np.int64)


def patch_table(mesh: Mesh, kind="full"):
    """Return (vertex ids, slots) of all kept patches, vertices in row-major (j, i) order.

    kind = "full": 20 slots; kind = "u": the first 8 slots (displacement patch).
    """
    verts, rows = [], []
    for j in range(mesh.n + 1):
        for i in range(mesh.n + 1):
            s = vertex_patch_slots(mesh, i, j)
            if kind == "u":
                s = s[:8]
                keep = np.any(s >= 0)
            else:
                keep = np.any(s[:14] >= 0)
            if keep:
                verts.append(mesh.vid(i, j))
                rows.append(s)
    return np.array(verts, dtype=np.int64), np.array(rows, dtype=np.int64)


def _dense_blocks(A, idx):
    """Dense V_l A V_l^T for index sets idx (P, s) of one common size."""
    P, s = idx.shape
    r = np.repeat(idx, s, axis=1).ravel()
    c = np.tile(idx, (1, s)).ravel()
    vals = np.asarray(A[r, c]).ravel()
    return vals.reshape(P, s, s)


class AdditiveVanka:
    """x <- x + omega * sum_l V_l^T D_l (V_l A V_l^T + shift S)^{-1} V_l (b - A x).

    shift: Sec. 5 (Terzaghi's problem) adds a weight 1e-8 to the diagonal of the Vanka blocks
    when M = infinity, where the pressure block -(1/M) M_p of A vanishes and an interior patch
    matrix is singular (the constant pressure on its star).  Reading: the weight enlarges each
    diagonal block of the patch taken in its definite form, A_u + shift, tau M_w + shift and
    (1/M) M_p + shift, like a small compressibility; in the symmetric saddle-point numbering
    used here S is +1 on the displacement and Darcy entries and -1 on the pressure entries
    (canonical indices >= p_start).  The other sign on the pressures (+shift, a negative
    compressibility) leaves the nearly incompressible Terzaghi cases of Table 6 unconverged."""

    def __init__(self, A, slots, omega=1.0, shift=0.0, p_start=None):
        self.A = A.tocsr()
        self.omega = float(omega)
        self.shift = float(shift)
        if self.shift != 0.0 and p_start is None:
            raise ValueError("a patch shift needs p_start, the first pressure index")
        n = A.shape[0]
        mult = np.zeros(n)
        self.groups = []   # (index array (P, s), patch matrices (P, s, s))
        sets = [np.array(sorted(r[r >= 0])) for r in slots]
        sizes = sorted(set(len(t) for t in sets))
        for s in sizes:
            idx = np.array([t for t in sets if len(t) == s], dtype=np.int64)
            if s == 0:
                continue
            blocks = _dense_blocks(self.A, idx)
            if self.shift != 0.0:
                sgn = np.where(idx >= p_start, -1.0, 1.0)
                blocks = blocks + self.shift * sgn[:, :, None] * np.eye(s)[None]
            self.groups.append((idx, blocks))
            np.add.at(mult, idx.ravel(), 1.0)
        if np.any(mult == 0):
            raise ValueError("some DoF lies in no patch")
        self.weight = 1.0 / mult
        self.n_patches = len(sets)

    def correction(self, r):
        """sum_l V_l^T D_l (V_l A V_l^T)^{-1} V_l r (LAPACK gesv per patch)."""
        out = np.zeros_like(r)
        for idx, Al in self.groups:
            xl = np.linalg.solve(Al, r[idx][:, :, None])[:, :, 0]
            np.add.at(out, idx.ravel(), (self.weight[idx] * xl).ravel())
        return out

    def smooth(self, x, b):
        return x + self.omega * self.correction(b - self.A @ x)


class MulticolorVanka:
    """Multiplicative Vanka in colours (Sec. 3.2.1 describes additive and multiplicative forms).
    Two vertex patches share a DoF only when their vertices are joined by a mesh edge (the patch
    of a vertex holds the DoFs of its incident edges and star triangles), so any colouring of
    the vertex graph makes the patches of one colour disjoint.  Four colours: (i mod 2) +
    2 (j mod 2) (edge neighbours differ in a parity).  Three colours: (i + 2 j) mod 3, the
    smallest count for this triangulation (its H, V and D edge neighbours (i +- 1, j),
    (i, j +- 1), (i +- 1, j -+ 1) shift i + 2 j by +-1, +-2, -+1).  One step runs the colours in
    turn: r = b - A x, then x <- x + omega sum over the colour's patches of
    V_l^T (V_l A V_l^T)^{-1} V_l r (no weights: each DoF lies in at most one patch of a colour)."""

    def __init__(self, A, mesh, omega=1.0, ncolors=4):
        self.A = A.tocsr()
        self.omega = float(omega)
        if ncolors not in (3, 4):
            raise ValueError("ncolors: 3 or 4")
        self.ncolors = int(ncolors)
        verts, slots = patch_table(mesh, "full")
        ij = mesh.vert_ij[verts]
        if self.ncolors == 4:
            col = (ij[:, 0] % 2) + 2 * (ij[:, 1] % 2)
        else:
            col = (ij[:, 0] + 2 * ij[:, 1]) % 3
        self.colors = []
        for c in range(self.ncolors):
            sets = [np.array(sorted(slots[k][slots[k] >= 0])) for k in np.nonzero(col == c)[0]]
            groups = []
            for sz in sorted(set(len(t) for t in sets)):
                if sz == 0:
                    continue
                idx = np.array([t for t in sets if len(t) == sz], dtype=np.int64)
                groups.append((idx, _dense_blocks(self.A, idx)))
            self.colors.append(groups)

    def color_correction(self, c, r):
        out = np.zeros_like(r)
        for idx, Al in self.colors[c]:
            xl = np.linalg.solve(Al, r[idx][:, :, None])[:, :, 0]
            np.add.at(out, idx.ravel(), xl.ravel())
        return out

    def smooth(self, x, b):
        for c in range(self.ncolors):
            x = x + self.omega * self.color_correction(c, b - self.A @ x)
        return x


class InexactBSR:
    """One inexact Braess-Sarazin step (Sec. 3.2.2, Appendix D).

    The pressure correction solves the approximate Schur complement system
    S_hat dp = s, S_hat = c_u M_p + A_pw (tau D_w)^{-1} A_pw^T.  schur_sweeps = 1 is the paper's
    form: one weighted-Jacobi step dp = omega_J s / diag(S_hat).  schur_sweeps = k > 1 runs k
    Jacobi sweeps with weight omega_S from dp = 0 instead, a short inner iteration on S_hat
    (exact BSR as k grows).  schur_cg = k > 0 runs k steps of conjugate gradients on S_hat
    (symmetric positive definite) preconditioned by diag(S_hat), from dp = 0: exact BSR (the
    exact solve of the approximate Schur complement, Sec. 3.2.2) as k grows."""

    def __init__(self, asm, omega, omega_J, schur_sweeps=1, omega_S=1.0, schur_cg=0):
        mesh = asm.mesh
        P = asm.params
        A = asm.A.tocsr()
        self.A = A
        su, sw, sp_ = asm.slices()
        self.su, self.sw, self.sp = su, sw, sp_
        self.omega = float(omega)
        self.omega_J = float(omega_J)
        Auu = A[su, su].tocsr()
        self.Aup = A[su, sp_].tocsr()
        self.Awp = A[sw, sp_].tocsr()
        self.Apu = A[sp_, su].tocsr()
        self.Apw = A[sp_, sw].tocsr()
        self.Dww = A[sw, sw].diagonal()                         # tau D_w
        _, uslots = patch_table(mesh, "u")
        self.fu = AdditiveVanka(Auu, uslots, omega=1.0)        # A_{V,u}^{-1}
        Mp = asm.free(asm.Mp_full)[sp_, sp_].diagonal()
        d = 2.0
        c_u = P.inv_M + P.alpha ** 2 / (P.lam + 2.0 * P.mu / d)
        # tau B_w D_w^{-1} B_w^T = A_pw (tau D_w)^{-1} A_pw^T; its diagonal:
        wdiag = np.asarray(self.Apw.multiply(self.Apw) @ (1.0 / self.Dww)).ravel()
        self.diagS = c_u * Mp + wdiag
        self.cMp = c_u * Mp
        self.schur_sweeps = int(schur_sweeps)
        self.omega_S = float(omega_S)
        self.schur_cg = int(schur_cg)
        if self.schur_sweeps < 1 or self.schur_cg < 0:
            raise ValueError("schur_sweeps >= 1, schur_cg >= 0")

    def schur_apply(self, dp):
        """S_hat dp = c_u M_p dp + A_pw (tau D_w)^{-1} A_pw^T dp."""
        return self.cMp * dp + self.Apw @ ((self.Apw.T @ dp) / self.Dww)

    def schur_cg_solve(self, s):
        """k steps of diag(S_hat)-preconditioned conjugate gradients on S_hat dp = s, dp0 = 0
        (Hestenes-Stiefel with the preconditioned residual z = r / diag(S_hat))."""
        dp = np.zeros_like(s)
        r = s.copy()
        z = r / self.diagS
        p = z.copy()
        rho = r @ z
        for _ in range(self.schur_cg):
            if rho == 0.0:
                break
            q = self.schur_apply(p)
            alpha = rho / (p @ q)
            dp = dp + alpha * p
            r = r - alpha * q
            z = r / self.diagS
            rho_new = r @ z
            p = z + (rho_new / rho) * p
            rho = rho_new
        return dp

    def schur_solve(self, s):
        if self.schur_cg > 0:
            return self.schur_cg_solve(s)
        if self.schur_sweeps == 1:
            return self.omega_J * s / self.diagS
        dp = np.zeros_like(s)
        for _ in range(self.schur_sweeps):
            dp = dp + self.omega_S * (s - self.schur_apply(dp)) / self.diagS
        return dp

    def step_correction(self, r):
        ru, rw, rp = r[self.su], r[self.sw], r[self.sp]
        zu = self.fu.correction(ru)
        zw = rw / self.Dww
        s = self.Apu @ zu + self.Apw @ zw - rp
        dp = self.schur_solve(s)
        du = self.fu.correction(ru - self.Aup @ dp)
        dw = (rw - self.Awp @ dp) / self.Dww
        return np.concatenate([du, dw, dp])

    def smooth(self, x, b):
        return x + self.omega * self.step_correction(b - self.A @ x)
