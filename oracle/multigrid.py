"""Monolithic geometric multigrid hierarchy and V-cycle.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Paper passages followed:
  * Sec. 3, eq. (TG-Operator-Biot): E_TG = E_s^{nu2} E_CGC E_s^{nu1}, E_s = I - omega M^{-1} A,
    E_CGC = I - P A_H^{-1} R A, R = P^T, coarse operators by rediscretization; the
    multilevel cycle replaces A_H^{-1} by the same cycle on the coarser level.
  * Sec. 5.1: direct solve on the coarsest mesh.
Readings: coarsest mesh 4 x 4 unless told otherwise; one omega on every level; the
heterogeneous permeability is coarsened by averaging 1/K over the four children; every level
takes the boundary conditions of the finest (bc), and the Vanka patch shift (vanka_shift,
Sec. 5, Terzaghi's problem) applies on every level.
"""
import numpy as np
import scipy.linalg as sla

from .mesh import Mesh
from .fem import Assembly, coarsen_inverse_K
from .transfer import prolongation
from .smoothers import MulticolorVanka, AdditiveVanka, InexactBSR, patch_table


class Level:
    def __init__(self, n, params, K_tri, bc="dirichlet"):
        self.mesh = Mesh(n, bc)
        self.asm = Assembly(self.mesh, params, K_tri)
        self.A = self.asm.A
        self.P = None          # prolongation from the next coarser level
        self.smoother = None


class Hierarchy:
    """Levels 0 (finest, n) .. L-1 (coarsest, n_coarse)."""

    def __init__(self, n, params, K_tri=1.0, smoother="vanka", omega=1.0, omega_J=1.0,
                 nu1=1, nu2=1, n_coarse=4, levels=None, schur_sweeps=1, omega_S=1.0, gamma=1,
                 vanka_colors=0, schur_cg=0, gamma_from=0, fcycle=False, bc="dirichlet", vanka_shift=0.0,
                 gamma_to=0, additive_levels=0, omega_additive=0.0):
        if levels is not None:
            n_coarse = n >> (levels - 1)
        self.params = params
        self.nu1, self.nu2 = int(nu1), int(nu2)
        self.gamma = int(gamma)                 # coarse corrections per level: 1 V-cycle, 2 W-cycle
        self.gamma_from = int(gamma_from)       # levels finer than this take one coarse correction
        self.fcycle = bool(fcycle)              # further coarse corrections are V-cycles (F-cycle)
        self.gamma_to = int(gamma_to)           # > 0: levels from this one down take one correction
        if self.gamma < 1:
            raise ValueError("gamma >= 1")
        self.levels = []
        Kinv = 1.0 / np.broadcast_to(np.asarray(K_tri, dtype=np.float64), (2 * n * n,))
        nn = n
        while True:
            lev = Level(nn, params, 1.0 / Kinv, bc)
            self.levels.append(lev)
            if nn <= n_coarse:
                break
            Kinv = coarsen_inverse_K(nn, Kinv)
            nn //= 2
        for l in range(len(self.levels) - 1):
            _, self.levels[l].P = prolongation(self.levels[l].mesh, self.levels[l + 1].mesh)
        # additive_levels: with vanka_colors, the finest levels take the additive step (weight
        # omega_additive, or omega when 0) and the coarser ones the colours
        for l, lev in enumerate(self.levels[:-1]):
            if smoother == "vanka" and vanka_colors and l < additive_levels:
                _, slots = patch_table(lev.mesh, "full")
                lev.smoother = AdditiveVanka(lev.A, slots, omega_additive if omega_additive > 0 else omega,
                                             vanka_shift, lev.mesh.n_u + lev.mesh.n_w)
            elif smoother == "vanka" and vanka_colors:
                if vanka_colors not in (3, 4):
                    raise ValueError("vanka_colors: 0 (additive), 3 or 4")
                lev.smoother = MulticolorVanka(lev.A, lev.mesh, omega, vanka_colors)
            elif smoother == "vanka":
                _, slots = patch_table(lev.mesh, "full")
                lev.smoother = AdditiveVanka(lev.A, slots, omega, vanka_shift, lev.mesh.n_u + lev.mesh.n_w)
            elif smoother == "bsr":
                lev.smoother = InexactBSR(lev.asm, omega, omega_J, schur_sweeps, omega_S, schur_cg)
            else:
                raise ValueError(smoother)
        self.coarse_lu = sla.lu_factor(self.levels[-1].A.toarray())

    @property
    def A(self):
        return self.levels[0].A

    def vcycle(self, b, level=0, vonly=False):
        """One V(nu1, nu2) cycle for A_level x = b from x = 0; with gamma > 1 the coarse
        correction is gamma cycles of the next level (a W-cycle for gamma = 2), each further one
        on the residual left by the previous ones, except at the coarsest level, whose direct
        solve is exact, and on levels finer than gamma_from or (gamma_to > 0) from gamma_to down,
        which take one.

        fcycle: the first coarse cycle is of the same kind, the further ones are V-cycles (for
        gamma = 2 the F-cycle, which visits level m below the first repeating level m + 1
        times rather than 2^m).  vonly: this cycle and every one below it is a V-cycle."""
        lev = self.levels[level]
        if level == len(self.levels) - 1:
            return sla.lu_solve(self.coarse_lu, b)
        x = np.zeros_like(b)
        for _ in range(self.nu1):
            x = lev.smoother.smooth(x, b)
        r = b - lev.A @ x
        bc = lev.P.T @ r
        xc = self.vcycle(bc, level + 1, vonly)
        repeat = level >= self.gamma_from and (self.gamma_to <= 0 or level < self.gamma_to)
        if not vonly and level + 1 < len(self.levels) - 1 and repeat:
            for _ in range(self.gamma - 1):
                xc = xc + self.vcycle(bc - self.levels[level + 1].A @ xc, level + 1, self.fcycle)
        x = x + lev.P @ xc
        for _ in range(self.nu2):
            x = lev.smoother.smooth(x, b)
        return x

    def error_propagation(self, e):
        """Error propagation of one cycle used as a stationary iteration: e - V(A e).

        With two levels this is the two-grid operator E_TG of Sec. 3 (exact coarse solve)."""
        return e - self.vcycle(self.levels[0].A @ e)
