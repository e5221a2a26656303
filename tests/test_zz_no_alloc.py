"""biot_solve_noalloc, the solve for callers that cannot allocate device memory, against
biot_solve through the C ABI: two calls in a row on one GPU, the second on a smaller mesh (the
shared workspace array still holds the first call's vectors), each compared with biot_solve on
the same context; device memory does not change across a no-allocation call (biot_solve's first
call on the same context allocates its workspace, which the same measurement sees); requests
beyond the fixed workspace are rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2107_04060_amd import inputs  # noqa: E402


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_04060_amd import binding as b
    b.load()
    return b


def _solver(binding, n, levels):
    lam, mu = 1.0, 1.0
    M = inputs.biot_modulus(inputs.young_from_lame(lam, mu))
    s = binding.BiotSolver(n, lam, mu, alpha=1.0, M=M, mu_f=1.0, tau=1.0, K=1.0)
    s.setup(levels=levels, smoother="vanka", nu1=2, nu2=2, omega=0.9)
    return s


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_noalloc_solve_matches_solve_twice_second_smaller(binding):
    warm = _solver(binding, 16, 3)        # loads the kernels before memory is measured
    bw = torch.tensor(inputs.rhs_uniform(16, 5), dtype=torch.float64, device="cuda")
    warm.solve(bw, tol=1e-8, restart=8, maxit=100)
    out = []
    for n, levels, seed, restart in ((64, 5, 0, 30), (16, 3, 1, 12)):
        s = _solver(binding, n, levels)
        b = torch.tensor(inputs.rhs_uniform(n, seed), dtype=torch.float64, device="cuda")
        x_na = torch.empty_like(b)
        f0 = _free()
        x_na, i_na = s.solve_noalloc(b, x_na, tol=1e-8, restart=restart, maxit=300)
        f1 = _free()
        x_ref, i_ref = s.solve(b, tol=1e-8, restart=restart, maxit=300)
        f2 = _free()
        a, r = x_na.cpu().numpy(), x_ref.cpu().numpy()
        d = np.abs(a - r).max() / np.abs(r).max()
        print("  n %d restart %d: noalloc %d iters (%.2e), solve %d iters (%.2e), max|diff|/max|x| %.1e; "
              "free memory change %d B (noalloc), %d B (first solve)"
              % (n, restart, i_na["iters"], i_na["rel_res_true"], i_ref["iters"], i_ref["rel_res_true"], d,
                 f1 - f0, f2 - f1), flush=True)
        out.append((n, i_na, i_ref, d, f0 - f1, f1 - f2))
        s.close()
    warm.close()
    for n, i_na, i_ref, d, used_na, used_ref in out:
        assert i_na["converged"] and i_ref["converged"], n
        assert i_na["iters"] == i_ref["iters"], n
        assert i_na["rel_res_true"] <= 1e-8 and abs(i_na["rel_res_true"] - i_ref["rel_res_true"]) <= 1e-12, n
        assert d <= 1e-12, (n, d)
        assert used_na <= 2 << 20, (n, used_na)          # no allocation (2 MiB slack for the runtime)
    # the measurement sees an allocation: biot_solve's workspace at n = 64, restart 30 is ~27 MB
    assert out[0][5] >= 16 << 20, out[0][5]


def test_noalloc_with_csr_small_levels(binding):
    """The same with the small levels on CSR (csr_below) and the multiplicative W-cycle of the
    block workload: their buffers are set up with the hierarchy, so the no-allocation solve still
    allocates nothing and matches biot_solve."""
    from gpu_cases import block_perm, case
    n, levels = 64, 5
    lam, mu, al, M, mf_, tau = case("block")
    K = torch.tensor(block_perm(n), dtype=torch.float64, device="cuda")
    s = binding.BiotSolver(n, lam, mu, alpha=al, M=M, mu_f=mf_, tau=tau, K=K)
    s.setup(levels=levels, smoother="vanka", nu1=1, nu2=1, omega=1.1, vanka_colors=3, gamma=2, gamma_from=1,
            csr_below=16)
    b = torch.tensor(inputs.rhs_uniform(n, 4), dtype=torch.float64, device="cuda")
    s.solve(b, tol=1e-8, restart=30, maxit=300)                   # workspace of biot_solve, kernels loaded
    x_na = torch.empty_like(b)
    f0 = _free()
    x_na, i_na = s.solve_noalloc(b, x_na, tol=1e-8, restart=30, maxit=300)
    f1 = _free()
    x_ref, i_ref = s.solve(b, tol=1e-8, restart=30, maxit=300)
    s.close()
    d = (x_na - x_ref).abs().max().item() / x_ref.abs().max().item()
    print("  csr_below 16: noalloc %d iters, solve %d iters, max|diff|/max|x| %.1e, free memory change %d B"
          % (i_na["iters"], i_ref["iters"], d, f1 - f0), flush=True)
    assert i_na["converged"] and i_na["iters"] == i_ref["iters"]
    assert d <= 1e-12
    assert f0 - f1 <= 2 << 20


def test_noalloc_rejects_requests_beyond_its_workspace(binding):
    s = _solver(binding, 128, 6)
    b = torch.zeros(s.nf(), dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    with pytest.raises(binding.BiotError) as e:
        s.solve_noalloc(b, x, restart=30)
    assert e.value.code == binding.BIOT_ERR_ARG and "64 MiB" in str(e.value)
    with pytest.raises(binding.BiotError) as e:
        s.solve_noalloc(b, x, restart=33)
    assert e.value.code == binding.BIOT_ERR_ARG
    # n = 128 fits with restart 19
    b = torch.tensor(inputs.rhs_uniform(128, 2), dtype=torch.float64, device="cuda")
    x, info = s.solve_noalloc(b, x, tol=1e-8, restart=19, maxit=400)
    x_ref, i_ref = s.solve(b, tol=1e-8, restart=19, maxit=400)
    s.close()
    assert info["converged"] and info["iters"] == i_ref["iters"]
    d = (x - x_ref).abs().max().item() / x_ref.abs().max().item()
    assert d <= 1e-12, d
