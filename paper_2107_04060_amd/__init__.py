"""MI355X-native monolithic multigrid (FGMRES + V-cycle with Vanka / Braess-Sarazin
relaxation) for the reduced-quadrature three-field Biot system.

The compute path lives in the HIP library built from ``csrc/`` and is reached through
``paper_2107_04060_amd.binding`` (loaded on first use, never at package import, so the
seeded input generators in ``paper_2107_04060_amd.inputs`` stay importable anywhere).
"""
__all__ = ["inputs", "binding"]
