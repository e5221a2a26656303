"""CPU reference ("oracle") for the reduced-quadrature Biot multigrid solver.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
baseline may import it; the product path (the HIP library and its binding) never does,
and this package imports nothing from the product path.  Plain FP64 NumPy/SciPy code
written from the paper, arXiv:2107.04060 (Adler, He, Hu, MacLachlan, Ohm):

  mesh.py        structured mesh, canonical DoF numbering            (Sec. 2.1, App. A)
  fem.py         element matrices, RQ assembly, K coarsening          (Sec. 2.1, 2.3)
  transfer.py    P = diag(P_u, P_w, P_p), divergence preserving P_u   (Sec. 3, 3.1)
  smoothers.py   vertex patches, additive Vanka, inexact BSR          (Sec. 3.2, App. D)
  multigrid.py   rediscretized hierarchy, V-cycle, two-grid operator  (Sec. 3, 5.1)
  krylov.py      restarted flexible GMRES                             (Sec. 5.1)
  symbols.py     Fourier symbols of assembled operators               (Sec. 4, App. A-B)

Every function is pinned by tests under tests/test_oracle_*.py against values the
paper prints (Appendix A/B stencils and symbols, Tables 2-3) or against brute-force
dense constructions.
"""
