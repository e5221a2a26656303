"""Two-grid local Fourier analysis of the monolithic multigrid method and the choice of the
relaxation weights.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Paper passages followed:
  * Sec. 4.1: Fourier modes exp(i theta . x / h); low frequencies T_low = [-pi/2, pi/2)^2;
    harmonics theta^alpha = theta + pi alpha, alpha in {00, 10, 01, 11}; the two-grid symbol
        E_TG(theta) = E_s^{nu2} (I - P~ L~_2h(2 theta)^{-1} R~ L~_h) E_s^{nu1}    (real-TGM)
    on the 4 x 10 harmonic space; rho_LFA = sup over T_low of its spectral radius, taken
    over a discrete sample of T_low.
  * Sec. 4.2 and Appendix A: a 10 x 10 block symbol with one block per DoF type; the
    off-diagonal symbols use the offsets between DoF positions (P1 at vertices, bubble and
    RT0 DoFs at edge midpoints, both P0 DoFs at the square centre).
  * Sec. 4.2 and Appendix B: restriction symbols R~(theta^alpha); interpolation by the
    scaled transpose: with R = P^T, P~ = R~^H / 4 (four fine points per coarse point).
  * Sec. 4.2 and Appendix C: the additive Vanka symbol V(theta)^H D A_l^{-1} V(theta), the
    patch residual being the restriction of a Fourier mode to a patch and the correction
    its weighted prolongation.
  * Appendix D: the inexact BSR symbol, composed of the displacement-patch Vanka symbol,
    (tau D_w)^{-1}, and one weighted-Jacobi step on the approximate Schur complement.
  * Sec. 5 (LFA validation): 32 evenly spaced samples per direction, offset so that the
    origin is not sampled; brute-force search of the weights (step 0.02).

Readings (listed in the design notes): the samples are the midpoints
theta_k = -pi/2 + (k + 1/2) pi / 32; the BSR weights are searched on a 0.01 grid (the
printed values such as 1.15 and 0.71 are not on a 0.02 grid).

Implementation notes: the stencils are read off an interior cell of an 8 x 8 assembly;
every block of the RQ system is homogeneous in the cell size (A_eps and the RQ term h^0,
B_u and B_w h^1, M_w and M_p h^2), so scaling the blocks gives the rediscretized operator at
any h.  rho(E_s^{nu2} K E_s^{nu1}) = rho(K E_s^{nu1 + nu2}) (eigenvalues of AB and BA
coincide), so only the sum nu1 + nu2 enters.
"""
import numpy as np

from .mesh import Mesh
from .fem import Assembly
from .transfer import prolongation
from .symbols import TYPES, OFFSET, dof_at, dof_types_positions
from .smoothers import vertex_patch_slots

N_REF = 8                      # reference mesh of the stencils (interior cell (4, 4))
REF = (4, 4)
TU = [0, 1, 2, 3, 4]           # displacement types in TYPES order
TW = [5, 6, 7]
TP = [8, 9]
ALPHAS = [(0, 0), (1, 0), (0, 1), (1, 1)]


def theta_samples(m=32):
    """m x m midpoint samples of T_low = [-pi/2, pi/2)^2 (origin not sampled)."""
    t = -0.5 * np.pi + (np.arange(m) + 0.5) * np.pi / m
    T1, T2 = np.meshgrid(t, t, indexing="ij")
    return np.stack([T1.ravel(), T2.ravel()], axis=1)


def scaled_matrix(params, h, K=1.0):
    """Free-DoF RQ matrix of the 8 x 8 reference mesh with its blocks rescaled to cell size h."""
    asm = Assembly(Mesh(N_REF), params, K)
    s = h * N_REF
    P = params
    A = (2.0 * P.mu * asm.A_eps_full + P.lam * asm.RQ_full
         + P.tau * s * s * asm.Mw_full
         + P.alpha * s * (asm.Bu_full + asm.Bu_full.T)
         + P.tau * s * (asm.Bw_full + asm.Bw_full.T)
         - P.inv_M * s * s * asm.Mp_full)
    return asm, asm.free(A)


class Stencil:
    """Interior rows of a free-DoF matrix: (row type, column type, position offset, value)."""

    def __init__(self, A, mesh):
        typ, pos = dof_types_positions(mesh)
        A = A.tocsr()
        rows, cols, offs, vals = [], [], [], []
        for a in range(len(TYPES)):
            r = dof_at(mesh, TYPES[a], *REF)
            for k in range(A.indptr[r], A.indptr[r + 1]):
                c = A.indices[k]
                rows.append(a)
                cols.append(int(typ[c]))
                offs.append(pos[c] - pos[r])
                vals.append(A.data[k])
        self.rows = np.array(rows)
        self.cols = np.array(cols)
        self.offs = np.array(offs)
        self.vals = np.array(vals)

    def symbol(self, theta):
        """10 x 10 symbols at the frequencies theta (N, 2): sum_kappa s_kappa e^{i theta.kappa}."""
        th = np.atleast_2d(theta)
        ph = np.exp(1j * th @ self.offs.T) * self.vals          # (N, entries)
        S = np.zeros((th.shape[0], len(TYPES), len(TYPES)), dtype=complex)
        np.add.at(S, (slice(None), self.rows, self.cols), ph)
        return S


class RestrictionStencil:
    """Rows of R = P^T at an interior coarse cell; R~(theta^alpha) as in Appendix B."""

    def __init__(self):
        mf, mc = Mesh(N_REF), Mesh(N_REF // 2)
        _, P = prolongation(mf, mc)
        R = P.T.tocsr()
        typ_f, pos_f = dof_types_positions(mf)
        ref = (N_REF // 4, N_REF // 4)
        rows, cols, offs, vals, X = [], [], [], [], []
        for a, t in enumerate(TYPES):
            rc = dof_at(mc, t, *ref)
            ox, oy = OFFSET[t]
            Xa = 2.0 * np.array([ref[0] + ox, ref[1] + oy])   # coarse DoF position, fine units
            X.append(Xa)
            for k in range(R.indptr[rc], R.indptr[rc + 1]):
                f = R.indices[k]
                rows.append(a)
                cols.append(int(typ_f[f]))
                offs.append(pos_f[f] - Xa)
                vals.append(R.data[k])
        self.rows = np.array(rows)
        self.cols = np.array(cols)
        self.offs = np.array(offs)
        self.vals = np.array(vals)
        self.X = np.array(X)

    def symbol(self, theta, alpha):
        th = np.atleast_2d(theta) + np.pi * np.asarray(alpha, dtype=float)
        ph = np.exp(1j * th @ self.offs.T) * self.vals
        S = np.zeros((th.shape[0], len(TYPES), len(TYPES)), dtype=complex)
        np.add.at(S, (slice(None), self.rows, self.cols), ph)
        S *= np.exp(1j * np.pi * (self.X @ np.asarray(alpha, dtype=float)))[None, :, None]
        return S


def _patch_symbol(A, mesh, slots, weights, theta, types):
    """V(theta)^H D A_l^{-1} V(theta) on the DoF types `types` for the patch `slots` of the
    vertex REF (Sec. 3.2.1 / Appendix C)."""
    typ, pos = dof_types_positions(mesh)
    slots = np.asarray(slots)
    keep = slots >= 0
    idx = slots[keep]
    w = np.asarray(weights, dtype=float)[keep]
    Al = A.tocsr()[idx][:, idx].toarray()
    Ainv = np.linalg.inv(Al)
    vpos = np.array(REF, dtype=float)
    delta = pos[idx] - vpos
    col = {TYPES.index(t): k for k, t in enumerate(types)}
    th = np.atleast_2d(theta)
    V = np.zeros((th.shape[0], idx.size, len(types)), dtype=complex)
    ph = np.exp(1j * th @ delta.T)                              # (N, s)
    for s in range(idx.size):
        V[:, s, col[int(typ[idx[s]])]] = ph[:, s]
    inner = (w[:, None] * Ainv)[None, :, :] @ V                 # D A^-1 V
    return np.conj(np.swapaxes(V, 1, 2)) @ inner


VANKA_WEIGHTS = [1.0, 1.0] + [0.5] * 12 + [1.0 / 3.0] * 6       # interior patch (Sec. 3.2.1)


class TwoGridLFA:
    """Two-grid LFA of the RQ Biot multigrid at cell size h with Vanka or inexact BSR."""

    def __init__(self, params, h, K=1.0, smoother="vanka", nu=4, samples=32):
        self.params = params
        self.h = float(h)
        self.smoother = smoother
        self.nu = int(nu)                                       # nu1 + nu2
        asm, A = scaled_matrix(params, h, K)
        _, A2 = scaled_matrix(params, 2.0 * h, K)
        self.mesh = asm.mesh
        self.A = A
        Lh = Stencil(A, asm.mesh)
        L2h = Stencil(A2, asm.mesh)
        R = RestrictionStencil()
        th = theta_samples(samples)
        th = th[th[:, 1] > 0]                 # theta and -theta give conjugate symbols
        self.theta = th
        N = th.shape[0]
        self.Lh = [Lh.symbol(th + np.pi * np.array(a)) for a in ALPHAS]   # 4 x (N, 10, 10)
        Rt = np.concatenate([R.symbol(th, a) for a in ALPHAS], axis=2)     # (N, 10, 40)
        Pt = np.conj(np.swapaxes(Rt, 1, 2)) / 4.0                            # (N, 40, 10)
        L2 = L2h.symbol(2.0 * th)
        Lbig = np.zeros((N, 40, 40), dtype=complex)
        for k in range(4):
            Lbig[:, 10 * k:10 * k + 10, 10 * k:10 * k + 10] = self.Lh[k]
        self.K = np.eye(40)[None] - Pt @ np.linalg.solve(L2, Rt @ Lbig)
        self._patch_data()

    def _patch_data(self):
        m, A = self.mesh, self.A
        slots = vertex_patch_slots(m, *REF)
        if self.smoother == "vanka":
            self.Minv = [_patch_symbol(A, m, slots, VANKA_WEIGHTS, self.theta + np.pi * np.array(a), TYPES)
                         for a in ALPHAS]
            return
        # inexact BSR pieces (Appendix D)
        uw = [1.0, 1.0] + [0.5] * 6
        self.Fu = [_patch_symbol(A, m, slots[:8], uw, self.theta + np.pi * np.array(a), TYPES[:5])
                   for a in ALPHAS]
        Ad = A.tocsr()
        self.Dw = np.array([Ad[dof_at(m, TYPES[t], *REF), dof_at(m, TYPES[t], *REF)] for t in TW])
        P = self.params
        cu = P.inv_M + P.alpha ** 2 / (P.lam + P.mu)
        area = 0.5 * self.h * self.h
        dS = []
        for t in TP:
            r = dof_at(m, TYPES[t], *REF)
            row = Ad[r]
            s = cu * area
            typ, _ = dof_types_positions(m)
            for c, v in zip(row.indices, row.data):
                ct = int(typ[c])
                if ct in TW:
                    s += v * v / self.Dw[TW.index(ct)]
            dS.append(s)
        self.dS = np.array(dS)

    def _bsr_minv(self, k, omega_J):
        """10 x 10 symbol of the inexact BSR correction r -> (du, dw, dp) at harmonic k."""
        L = self.Lh[k]
        Fu = self.Fu[k]
        N = L.shape[0]
        Apu, Apw = L[:, TP][:, :, TU], L[:, TP][:, :, TW]
        Aup, Awp = L[:, TU][:, :, TP], L[:, TW][:, :, TP]
        Dwi = np.diag(1.0 / self.Dw)[None]
        Si = np.diag(omega_J / self.dS)[None]
        # dp = omega_J S^-1 (Apu Fu r_u + Apw Dw^-1 r_w - r_p)
        Gp = np.zeros((N, 2, 10), dtype=complex)
        Gp[:, :, TU] = Si @ Apu @ Fu
        Gp[:, :, TW] = Si @ Apw @ Dwi
        Gp[:, :, TP] = -Si
        M = np.zeros((N, 10, 10), dtype=complex)
        # du = Fu (r_u - Aup dp), dw = Dw^-1 (r_w - Awp dp)
        Eu = np.zeros((N, 5, 10), dtype=complex)
        Eu[:, :, TU] = np.eye(5)[None]
        M[:, TU, :] = Fu @ (Eu - Aup @ Gp)
        Ew = np.zeros((N, 3, 10), dtype=complex)
        Ew[:, :, TW] = np.eye(3)[None]
        M[:, TW, :] = Dwi @ (Ew - Awp @ Gp)
        M[:, TP, :] = Gp
        return M

    def smoother_symbols(self, omega_J=1.0):
        """Q_k = M~^{-1} L~_h at the four harmonics."""
        if self.smoother == "vanka":
            return [self.Minv[k] @ self.Lh[k] for k in range(4)]
        return [self._bsr_minv(k, omega_J) @ self.Lh[k] for k in range(4)]

    def rho(self, omega, omega_J=1.0, Q=None):
        """rho_LFA: the largest spectral radius of E_TG(theta) over the samples."""
        if Q is None:
            Q = self.smoother_symbols(omega_J)
        N = self.theta.shape[0]
        E = np.zeros((N, 40, 40), dtype=complex)
        for k in range(4):
            Es = np.eye(10)[None] - omega * Q[k]
            Ek = np.broadcast_to(np.eye(10), Es.shape).copy()
            for _ in range(self.nu):
                Ek = Es @ Ek
            E[:, 10 * k:10 * k + 10, 10 * k:10 * k + 10] = Ek
        ev = np.linalg.eigvals(self.K @ E)
        return float(np.abs(ev).max())

    def optimize_vanka(self, lo=0.5, hi=1.1, step=0.02):
        """Brute-force omega on the grid lo, lo + step, ... (Sec. 5): (omega_opt, rho_LFA)."""
        Q = self.smoother_symbols()
        grid = np.round(np.arange(lo, hi + 1e-9, step), 10)
        vals = [self.rho(w, Q=Q) for w in grid]
        k = int(np.argmin(vals))
        return float(grid[k]), float(vals[k])

    def optimize_bsr(self, wj=(0.6, 1.6), w=(0.4, 1.3), coarse=0.05, fine=0.01):
        """Brute-force (omega_J, omega): a coarse grid, then the fine grid around its best point."""
        def search(wjs, ws):
            best = (np.inf, None, None)
            for a in wjs:
                Q = self.smoother_symbols(a)
                for b in ws:
                    r = self.rho(b, Q=Q)
                    if r < best[0]:
                        best = (r, a, b)
            return best
        g1 = np.round(np.arange(wj[0], wj[1] + 1e-9, coarse), 10)
        g2 = np.round(np.arange(w[0], w[1] + 1e-9, coarse), 10)
        r, a, b = search(g1, g2)
        f1 = np.round(np.arange(a - coarse, a + coarse + 1e-9, fine), 10)
        f2 = np.round(np.arange(b - coarse, b + coarse + 1e-9, fine), 10)
        r, a, b = search(f1, f2)
        return float(a), float(b), float(r)
