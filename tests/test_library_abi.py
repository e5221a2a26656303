"""Host-side checks of the C ABI: the library builds, loads on a machine without a GPU and
exports every function declared in include/biot_mg.h (no compute calls here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "biot_mg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(biot_[a-z_A-Z0-9]+)\s*\(", src)))


def _lib():
    from paper_2107_04060_amd import build as b
    if not os.path.exists(b.LIB):
        b.build(verbose=False)
    return ctypes.CDLL(b.LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("biot_assemble", "biot_setup_hierarchy", "biot_vcycle", "biot_solve",
                     "biot_update_K", "biot_grad_logK", "biot_export_layout", "biot_destroy",
                     "biot_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_last_error_is_empty_string_initially():
    lib = _lib()
    lib.biot_last_error.restype = ctypes.c_char_p
    assert lib.biot_last_error() == b""


def test_invalid_arguments_are_rejected_without_touching_the_device():
    """Argument validation happens before any HIP call: a bad mesh size returns -1."""
    from paper_2107_04060_amd import binding
    lib = binding.load()
    prob = binding.Problem()
    prob.n = 6                       # not a power of two
    prob.lambda_, prob.mu, prob.alpha = 1.0, 1.0, 1.0
    prob.inv_M, prob.mu_f, prob.tau, prob.K_scalar = 0.03, 1.0, 1.0, 1.0
    ctx = ctypes.c_void_p()
    code = lib.biot_assemble(ctypes.byref(prob), None, ctypes.byref(ctx))
    assert code == binding.BIOT_ERR_ARG
    assert b"power of two" in lib.biot_last_error()
    assert not ctx.value
    code = lib.biot_solve(None, None, None, None, None)
    assert code == binding.BIOT_ERR_ARG


def test_boundary_condition_arguments_are_validated_on_the_host():
    """bc outside {Dirichlet, Terzaghi}, Terzaghi above n = 256 and 1/M = 0 with Dirichlet data
    are rejected before any HIP call; 1/M = 0 passes validation only with Terzaghi's bc."""
    from paper_2107_04060_amd import binding
    lib = binding.load()

    def try_assemble(n, bc, inv_M):
        prob = binding.Problem()
        prob.n, prob.bc = n, bc
        prob.lambda_, prob.mu, prob.alpha = 1.0, 1.0, 1.0
        prob.inv_M, prob.mu_f, prob.tau, prob.K_scalar = inv_M, 1.0, 1.0, 1.0
        ctx = ctypes.c_void_p()
        code = lib.biot_assemble(ctypes.byref(prob), None, ctypes.byref(ctx))
        assert not ctx.value
        return code, lib.biot_last_error()

    code, msg = try_assemble(16, 2, 0.03)
    assert code == binding.BIOT_ERR_ARG and b"bc" in msg
    code, msg = try_assemble(512, binding.BCS["terzaghi"], 0.0)
    assert code == binding.BIOT_ERR_ARG and b"256" in msg
    code, msg = try_assemble(16, binding.BCS["dirichlet"], 0.0)
    assert code == binding.BIOT_ERR_ARG and b"1/M" in msg
    code, msg = try_assemble(16, binding.BCS["terzaghi"], -1.0)
    assert code == binding.BIOT_ERR_ARG and b"1/M" in msg


def test_free_counts_of_the_binding():
    from paper_2107_04060_amd import binding
    from oracle.mesh import Mesh
    for n in (4, 8, 16):
        assert binding.n_free(n) == Mesh(n).n_free
        assert binding.n_free(n, "terzaghi") == Mesh(n, "terzaghi").n_free
