"""Pins of the multiplicative Vanka smoother (oracle/smoothers.py, MulticolorVanka), in four
colours (i mod 2) + 2 (j mod 2) and in three colours (i + 2 j) mod 3.

* The patches of one colour share no DoF, and the colours together cover every free DoF.
* Patches share DoFs exactly when their vertices are joined by a mesh edge: the checkerboard
  (i + j) mod 2 puts the two ends of every D edge in one colour and fails, so three colours are
  the fewest.
* One colour's correction equals a sparse direct solve (SuperLU) of A restricted to the union
  of that colour's patches with the couplings between different patches removed.
* One step is the four colour updates in turn, each on the residual left by the previous one.
* On the paper's steady problem (Sec. 5.1, nu = 0.499, k = 1e-6) FGMRES with a multiplicative
  V(1,1) cycle converges in fewer iterations than with the additive V(2,2) cycle.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import manufactured as mf
from oracle.fem import Assembly, BiotParams
from oracle.krylov import fgmres
from oracle.mesh import Mesh
from oracle.multigrid import Hierarchy
from oracle.smoothers import MulticolorVanka
from paper_2107_04060_amd import inputs


import pytest

from oracle.smoothers import patch_table


def _setup(n=8, ncolors=4):
    P = BiotParams.from_E_nu(1.0, 0.3, alpha=1.0, M=50.0, mu_f=1.0, tau=0.5)
    K = np.exp(np.random.default_rng(5).uniform(-1, 1, 2 * n * n)) * 1e-2
    asm = Assembly(Mesh(n), P, K)
    return asm, MulticolorVanka(asm.A, asm.mesh, 0.9, ncolors)


@pytest.mark.parametrize("ncolors", [3, 4])
def test_colours_do_not_overlap_and_cover(ncolors):
    asm, sm = _setup(ncolors=ncolors)
    assert len(sm.colors) == ncolors
    cover = np.zeros(asm.A.shape[0], dtype=int)
    for groups in sm.colors:
        seen = np.concatenate([idx.ravel() for idx, _ in groups])
        assert len(np.unique(seen)) == len(seen)
        cover[seen] += 1
    assert np.all(cover >= 1)


def test_patches_share_dofs_exactly_across_mesh_edges():
    mesh = Mesh(6)
    verts, slots = patch_table(mesh, "full")
    ij = mesh.vert_ij[verts]
    sets = [set(slots[k][slots[k] >= 0].tolist()) for k in range(len(verts))]
    edges = {tuple(sorted(e)) for e in mesh.edge_ends.tolist()}
    for a in range(len(verts)):
        for b in range(a + 1, len(verts)):
            if not sets[a] or not sets[b]:
                continue
            joined = tuple(sorted((int(verts[a]), int(verts[b])))) in edges
            assert bool(sets[a] & sets[b]) == joined, (ij[a], ij[b])
    # the checkerboard: the ends (i, j + 1), (i + 1, j) of a D edge have one colour
    d = mesh.edge_ends[mesh.edge_kind == 2][0]
    (i1, j1), (i2, j2) = mesh.vert_ij[d[0]], mesh.vert_ij[d[1]]
    assert (i1 + j1) % 2 == (i2 + j2) % 2
    assert (i1 + 2 * j1) % 3 != (i2 + 2 * j2) % 3


@pytest.mark.parametrize("ncolors", [3, 4])
def test_colour_correction_is_a_block_solve(ncolors):
    asm, sm = _setup(ncolors=ncolors)
    A = asm.A.tocsr()
    r = np.random.default_rng(6).standard_normal(A.shape[0])
    for c in range(ncolors):
        pid = -np.ones(A.shape[0], dtype=int)
        k = 0
        for idx, _ in sm.colors[c]:
            for row in idx:
                pid[row] = k
                k += 1
        U = np.nonzero(pid >= 0)[0]
        B = A[U][:, U].tocoo()
        keep = pid[U][B.row] == pid[U][B.col]
        Bm = sp.csc_matrix((B.data[keep], (B.row[keep], B.col[keep])), shape=B.shape)
        x = np.zeros_like(r)
        x[U] = spla.spsolve(Bm, r[U])
        assert np.allclose(sm.color_correction(c, r), x, rtol=0, atol=1e-12 * np.abs(x).max())


@pytest.mark.parametrize("ncolors", [3, 4])
def test_step_is_the_colours_in_turn(ncolors):
    asm, sm = _setup(ncolors=ncolors)
    A = asm.A.tocsr()
    rng = np.random.default_rng(7)
    x0, b = rng.standard_normal(A.shape[0]), rng.standard_normal(A.shape[0])
    x = x0.copy()
    for c in range(ncolors):
        x = x + 0.9 * sm.color_correction(c, b - A @ x)
    assert np.allclose(sm.smooth(x0, b), x, rtol=1e-14, atol=0)


def test_multiplicative_cycle_needs_fewer_iterations():
    lam, mu = inputs.lame(3e4, 0.499)
    P = BiotParams(lam, mu, alpha=1.0, M=1e6, mu_f=1.0, tau=1.0)
    b = mf.rhs(64, P)
    add = Hierarchy(64, P, K_tri=1e-6, smoother="vanka", omega=0.72, nu1=2, nu2=2, levels=4)
    mul = Hierarchy(64, P, K_tri=1e-6, smoother="vanka", omega=0.9, nu1=1, nu2=1, levels=4, vanka_colors=4)
    _, ia = fgmres(add.A, b, add.vcycle, tol=1e-6, restart=30, maxit=200)
    _, im = fgmres(mul.A, b, mul.vcycle, tol=1e-6, restart=30, maxit=200)
    print("additive V(2,2) %d iterations, multiplicative V(1,1) %d" % (ia["iters"], im["iters"]))
    assert ia["converged"] and im["converged"] and im["iters"] < ia["iters"]


@pytest.mark.slow
def test_stored_multiplicative_weight_reproduces():
    """The multiplicative-Vanka weight stored for the sweep256 set nu = 0.2, K = 1
    (paper_2107_04060_amd/relaxation_weights.json, written by python -m oracle.relaxation_weights
    --multiplicative) is 0.6: the oracle's FGMRES counts on the 64 x 64 mesh at omega 0.6 and 0.9
    are those stored, and 0.9, the weight used before the search, takes three times as many."""
    import json
    import os
    from oracle.krylov import fgmres
    from oracle.relaxation_weights import lame
    path = os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_2107_04060_amd", "relaxation_weights.json")
    e = json.load(open(path))["sweep256"]["0.2/1"]["vanka_mult"]
    assert e["omega"] == 0.6
    lam, mu = lame(1.0, 0.2)
    P = BiotParams(lam, mu, alpha=1.0, M=1.0 / 0.03, mu_f=1.0, tau=1.0)
    b = np.random.default_rng(1).uniform(-1.0, 1.0, 10 * 64 * 64 - 8 * 64 + 2)
    for om in (0.6, 0.9):
        H = Hierarchy(64, P, K_tri=1.0, smoother="vanka", omega=om, nu1=1, nu2=1, levels=5, vanka_colors=4)
        _, info = fgmres(H.A, b, H.vcycle, tol=1e-8, restart=30, maxit=150)
        assert info["converged"] and info["iters"] == e["counts_64"]["%.1f" % om]
    assert e["counts_64"]["0.9"] >= 3 * e["counts_64"]["0.6"]
