"""Element matrices and global assembly of the reduced-quadrature (RQ) Biot system.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Paper passages followed:
  * Sec. 2.1, eqs. (discrete1)-(discrete3) and (block_form): one backward-Euler step,
    Darcy row scaled by tau and mass-balance row by -1, giving the symmetric system
        [[A_u, 0, alpha B_u^T], [0, tau M_w, tau B_w^T], [alpha B_u, tau B_w, -(1/M) M_p]]
    with B_u <- -(div u, q), B_w <- -(div w, q), M_w <- (K^{-1} mu_f w, r), M_p <- (p, q).
  * Sec. 2.3, eq. (block_form_rq): A_u is replaced by A_u^RQ from
        a^RQ(u, v) = 2 mu (eps(u), eps(v)) + lambda (P_Q div u, P_Q div v),
    and Appendix A: A_u^RQ = 2 mu A_eps + lambda B_u^T M_p^{-1} B_u.
  * Sec. 2 (after Biot-eq3): mu = E / (2 + 2 nu), lambda = E nu / ((1 - 2 nu)(1 + nu)).

Basis normalisation (pinned by the Appendix A stencils in the tests):
  * P1 hats phi_a e_x, phi_a e_y;
  * face bubble on edge e with end points p, q: 4 lambda_p lambda_q n_e (normal value 1 at
    the edge midpoint);
  * RT0 function of edge e: normal component 1 on e.
Every integrand below is at most quadratic on a triangle, so the three-point edge-midpoint
rule (weights |T|/3) integrates it exactly.
"""
import numpy as np
import scipy.sparse as sp

from .mesh import Mesh

# barycentric coordinates of the three edge midpoints (quadrature points)
_QB = np.array([[0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])


def lame_from_E_nu(E, nu):
    """Sec. 2: mu = E/(2+2nu), lambda = E nu/((1-2nu)(1+nu))."""
    mu = E / (2.0 + 2.0 * nu)
    lam = E * nu / ((1.0 - 2.0 * nu) * (1.0 + nu))
    return lam, mu


class BiotParams:
    """Physical parameters of one time step.  M = inf means 1/M = 0."""

    def __init__(self, lam, mu, alpha=1.0, M=1.0e6, mu_f=1.0, tau=1.0):
        self.lam = float(lam)
        self.mu = float(mu)
        self.alpha = float(alpha)
        self.M = float(M)
        self.mu_f = float(mu_f)
        self.tau = float(tau)

    @property
    def inv_M(self):
        return 0.0 if np.isinf(self.M) else 1.0 / self.M

    @classmethod
    def from_E_nu(cls, E, nu, **kw):
        lam, mu = lame_from_E_nu(E, nu)
        return cls(lam, mu, **kw)


class ElementData:
    """Per-triangle local matrices, vectorised over all triangles of a mesh.

    Local displacement DoFs: [ux(v0), ux(v1), ux(v2), uy(v0), uy(v1), uy(v2), b(e0), b(e1), b(e2)],
    local edge k opposite local vertex k.
    """

    def __init__(self, mesh: Mesh):
        X = mesh.vert_xy[mesh.tri_vert]                      # (nT, 3, 2)
        self.X = X
        d1 = X[:, 1] - X[:, 0]
        d2 = X[:, 2] - X[:, 0]
        det = d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0]      # 2 |T| (ccw > 0)
        self.area = 0.5 * det
        # gradients of barycentric coordinates: for a counter-clockwise triangle, grad l_k is
        # the opposite edge vector x_{k+2} - x_{k+1} turned by +90 degrees, over 2|T|
        G = np.zeros((X.shape[0], 3, 2))
        for k in range(3):
            a = X[:, (k + 1) % 3]
            b = X[:, (k + 2) % 3]
            e = b - a
            G[:, k, 0] = -e[:, 1] / det
            G[:, k, 1] = e[:, 0] / det
        self.grad_l = G
        # edges: length, global normal, outward normal sign
        nT = X.shape[0]
        elen = np.zeros((nT, 3))
        sigma = np.zeros((nT, 3))
        nglob = mesh.edge_normal[mesh.tri_edge]              # (nT, 3, 2)
        for k in range(3):
            a = X[:, (k + 1) % 3]
            b = X[:, (k + 2) % 3]
            elen[:, k] = np.linalg.norm(b - a, axis=1)
            # outward normal points away from the opposite vertex k
            mid = 0.5 * (a + b)
            out = mid - X[:, k]
            s = np.einsum("ti,ti->t", nglob[:, k], out)
            sigma[:, k] = np.sign(s)
        self.elen = elen
        self.sigma = sigma
        self.nglob = nglob
        self._build()

    # -- displacement basis gradients at barycentric point beta: (nT, 9, 2, 2) [comp, deriv]
    def _u_grads(self, beta):
        G = self.grad_l
        nT = G.shape[0]
        out = np.zeros((nT, 9, 2, 2))
        for a in range(3):
            out[:, a, 0, :] = G[:, a]          # ux(v_a)
            out[:, 3 + a, 1, :] = G[:, a]      # uy(v_a)
        for k in range(3):
            p, q = (k + 1) % 3, (k + 2) % 3
            # grad(4 l_p l_q) = 4 (l_q grad l_p + l_p grad l_q)
            gs = 4.0 * (beta[q] * G[:, p] + beta[p] * G[:, q])   # (nT, 2)
            nrm = self.nglob[:, k]                               # (nT, 2)
            out[:, 6 + k] = nrm[:, :, None] * gs[:, None, :]
        return out

    def _rt0(self, beta):
        """RT0 basis values at barycentric point beta: (nT, 3, 2)."""
        X = self.X
        x = np.einsum("a,tai->ti", beta, X)
        out = np.zeros((X.shape[0], 3, 2))
        for k in range(3):
            coef = self.sigma[:, k] * self.elen[:, k] / (2.0 * self.area)
            out[:, k] = coef[:, None] * (x - X[:, k])
        return out

    def _build(self):
        nT = self.X.shape[0]
        w = self.area / 3.0
        Keps = np.zeros((nT, 9, 9))
        g = np.zeros((nT, 9))
        Mw = np.zeros((nT, 3, 3))
        divw = np.zeros((nT, 3))
        for qp in range(3):
            beta = _QB[qp]
            Gu = self._u_grads(beta)
            eps = 0.5 * (Gu + np.swapaxes(Gu, 2, 3))
            Keps += w[:, None, None] * np.einsum("tiab,tjab->tij", eps, eps)
            g += w[:, None] * np.einsum("tiaa->ti", Gu)
            psi = self._rt0(beta)
            Mw += w[:, None, None] * np.einsum("tki,tli->tkl", psi, psi)
            # div psi_k = sigma_k |e_k| / |T|  (div (x - x_k) = 2)
            divw += w[:, None] * (self.sigma * self.elen / self.area[:, None])
        self.K_eps = Keps          # int eps(phi_i) : eps(phi_j)
        self.g_div = g             # int_T div phi_i
        self.Mw_unit = Mw          # int psi_k . psi_l  (K = mu_f = 1)
        self.Bw_loc = -divw        # -(div psi_k, 1_T)
        self.Bu_loc = -g           # -(div phi_i, 1_T)


def _u_full_dofs(mesh: Mesh):
    """Full-space indices of the 9 local displacement DoFs per triangle."""
    tv = mesh.tri_vert
    te = mesh.tri_edge
    return np.concatenate(
        [mesh.off_ux + tv, mesh.off_uy + tv, mesh.off_b + te], axis=1
    )


class Assembly:
    """Global RQ Biot matrix on the free DoFs, plus its building blocks.

    K_tri: permeability per triangle, ordered [L(0..n^2-1), U(0..n^2-1)] (row-major (j, i)),
    or a scalar.
    """

    def __init__(self, mesh: Mesh, params: BiotParams, K_tri=1.0):
        self.mesh = mesh
        self.params = params
        ed = ElementData(mesh)
        self.ed = ed
        nT = mesh.n_tri
        K = np.broadcast_to(np.asarray(K_tri, dtype=np.float64), (nT,)).copy()
        if np.any(K <= 0):
            raise ValueError("permeability must be positive")
        self.K_tri = K
        N = mesh.n_full
        ud = _u_full_dofs(mesh)
        wd = mesh.off_w + mesh.tri_edge
        pd = mesh.off_p + np.arange(nT)
        P = params

        def coo(rows, cols, vals):
            return sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(N, N)).tocsr()

        r9 = np.repeat(ud[:, :, None], 9, axis=2)
        c9 = np.repeat(ud[:, None, :], 9, axis=1)
        self.A_eps_full = coo(r9, c9, ed.K_eps)                               # A_eps
        rq = ed.g_div[:, :, None] * ed.g_div[:, None, :] / ed.area[:, None, None]
        self.RQ_full = coo(r9, c9, rq)                                        # B_u^T M_p^-1 B_u
        r3 = np.repeat(wd[:, :, None], 3, axis=2)
        c3 = np.repeat(wd[:, None, :], 3, axis=1)
        mw = ed.Mw_unit * (P.mu_f / K)[:, None, None]
        self.Mw_full = coo(r3, c3, mw)                                        # M_w
        self.Bu_full = coo(np.repeat(pd[:, None], 9, axis=1), ud, ed.Bu_loc)  # B_u (p rows)
        self.Bw_full = coo(np.repeat(pd[:, None], 3, axis=1), wd, ed.Bw_loc)  # B_w (p rows)
        self.Mp_full = sp.csr_matrix((ed.area, (pd, pd)), shape=(N, N))      # M_p
        Au = 2.0 * P.mu * self.A_eps_full + P.lam * self.RQ_full
        A = (
            Au
            + P.tau * self.Mw_full
            + P.alpha * (self.Bu_full + self.Bu_full.T)
            + P.tau * (self.Bw_full + self.Bw_full.T)
            - P.inv_M * self.Mp_full
        )
        f = mesh.free_full
        self.A_full = A.tocsr()
        self.A = self.A_full[f][:, f].tocsr()
        self.A.sort_indices()
        self.n_free = mesh.n_free

    def free(self, Mfull):
        f = self.mesh.free_full
        return Mfull.tocsr()[f][:, f].tocsr()

    # ---- field slices of the canonical free vector --------------------------------
    def slices(self):
        m = self.mesh
        return (slice(0, m.n_u), slice(m.n_u, m.n_u + m.n_w), slice(m.n_u + m.n_w, m.n_free))


def coarsen_inverse_K(n, Kinv_tri):
    """Coarse-level 1/K per triangle: the mean of 1/K over the four child triangles.

    The paper uses a constant permeability and is silent on coarsening a heterogeneous
    one; this harmonic mean of K over the children is the reading documented in the
    design notes (it is exact for the RT0 mass of fields that are constant on the parent).
    Triangle order: [L(j*n+i), U(j*n+i)].
    """
    nc = n // 2
    L = Kinv_tri[: n * n].reshape(n, n)   # [j, i]
    U = Kinv_tri[n * n:].reshape(n, n)
    Lc = np.zeros((nc, nc))
    Uc = np.zeros((nc, nc))
    for J in range(nc):
        for I in range(nc):
            i0, j0 = 2 * I, 2 * J
            # children of coarse L(I,J): L(2I,2J), L(2I+1,2J), L(2I,2J+1), U(2I,2J)
            Lc[J, I] = 0.25 * (L[j0, i0] + L[j0, i0 + 1] + L[j0 + 1, i0] + U[j0, i0])
            # children of coarse U(I,J): U(2I+1,2J+1), U(2I+1,2J), U(2I,2J+1), L(2I+1,2J+1)
            Uc[J, I] = 0.25 * (U[j0 + 1, i0 + 1] + U[j0, i0 + 1] + U[j0 + 1, i0] + L[j0 + 1, i0 + 1])
    return np.concatenate([Lc.ravel(), Uc.ravel()])
