"""FGMRES with a restart length above the fused Gram-Schmidt bound (GS_FUSED = 32 basis vectors,
beyond which the library takes the unfused two-pass path) against the oracle's FGMRES with the
same restart, on the nearly incompressible 32 x 32 BSR case that needs about 50 iterations.
Both precision forms must reach 1e-8 in the true residual, recomputed on the CPU."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2107_04060_amd import inputs  # noqa: E402
from oracle.multigrid import Hierarchy  # noqa: E402
from oracle.krylov import fgmres  # noqa: E402
from gpu_cases import params, solver  # noqa: E402

N, LEVELS, K, OM, OMJ = 32, 4, 1e-3, 0.69, 1.23


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_04060_amd import binding as b
    b.load()
    return b


@pytest.fixture(scope="module")
def reference():
    H = Hierarchy(N, params("stiff"), K_tri=K, smoother="bsr", omega=OM, omega_J=OMJ, nu1=1, nu2=1, levels=LEVELS)
    b = inputs.rhs_uniform(N, 1)
    _, io = fgmres(H.A, b, H.vcycle, tol=1e-8, restart=60, maxit=300)
    return H.A, b, io


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_restart_beyond_fused_bound(binding, reference, precision):
    A, b, io = reference
    s = solver(binding, torch, N, "stiff", K, levels=LEVELS, smoother="bsr", nu=1, omega=OM, omega_J=OMJ,
               precision=precision)
    x, info = s.solve(torch.tensor(b, dtype=torch.float64, device="cuda"), tol=1e-8, restart=60, maxit=300)
    s.close()
    x = x.cpu().numpy()
    print("  %s restart 60: gpu %d iterations, oracle %d" % (precision, info["iters"], io["iters"]), flush=True)
    assert io["iters"] > 40                      # the cycle runs past 32 basis vectors
    assert info["converged"] and np.all(np.isfinite(x))
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b) * (1 + 1e-6)
    if precision == "fp64":
        assert abs(info["iters"] - io["iters"]) <= 1
    else:
        assert info["iters"] <= io["iters"] + 3


@pytest.mark.parametrize("reorth", [1.0, 1e-12])
@pytest.mark.parametrize("restart", [30, 60])
def test_gram_schmidt_threshold(binding, reference, reorth, restart):
    """The second Gram-Schmidt pass always (reorth = 1: |w_1| <= |w_0| always holds) and never
    (1e-12), on the fused (restart 30) and the unfused (60) paths: both converge in the oracle's
    iteration count (+-1) for the oracle's restart, and the true residual is recomputed here."""
    A, b, io = reference
    if restart == 30:
        H = Hierarchy(N, params("stiff"), K_tri=K, smoother="bsr", omega=OM, omega_J=OMJ, nu1=1, nu2=1,
                      levels=LEVELS)
        _, io = fgmres(H.A, b, H.vcycle, tol=1e-8, restart=30, maxit=300)
    s = solver(binding, torch, N, "stiff", K, levels=LEVELS, smoother="bsr", nu=1, omega=OM, omega_J=OMJ)
    x, info = s.solve(torch.tensor(b, dtype=torch.float64, device="cuda"), tol=1e-8, restart=restart, maxit=300,
                      reorth=reorth)
    s.close()
    x = x.cpu().numpy()
    print("  reorth %g restart %d: gpu %d iterations, oracle %d" % (reorth, restart, info["iters"], io["iters"]),
          flush=True)
    assert info["converged"]
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b) * (1 + 1e-6)
    assert abs(info["iters"] - io["iters"]) <= 1
