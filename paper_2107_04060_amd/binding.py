"""ctypes binding of libbiot_mg.so (the C ABI declared in include/biot_mg.h).

Argument marshalling only: every numerical step runs in the HIP library.  Vectors are
torch CUDA (ROCm) float64 tensors in the canonical free-DoF order; the stream is torch's
current stream.  Loading fails loudly when the library has not been built.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbiot_mg.so")

BIOT_OK = 0
BIOT_NOT_CONVERGED = 1
BIOT_ERR_ARG = -1
BIOT_ERR_HIP = -2
BIOT_ERR_OOM = -3
BIOT_ERR_SINGULAR = -4
BIOT_ERR_NAN = -5
SMOOTHERS = {"vanka": 0, "bsr": 1}
PRECISIONS = {"fp64": 0, "fp32": 1, "fp32_patch": 2}
SIDES = {"right": 0, "left": 1}
BCS = {"dirichlet": 0, "terzaghi": 1}

_lib = None


class BiotError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("biot error %d: %s" % (code, msg))
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("lambda_", ctypes.c_double), ("mu", ctypes.c_double),
                ("alpha", ctypes.c_double), ("inv_M", ctypes.c_double), ("mu_f", ctypes.c_double),
                ("tau", ctypes.c_double), ("K_scalar", ctypes.c_double), ("K_tri", ctypes.c_void_p),
                ("bc", ctypes.c_int)]


class MGOpts(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("smoother", ctypes.c_int), ("nu1", ctypes.c_int),
                ("nu2", ctypes.c_int), ("omega", ctypes.c_double), ("omega_J", ctypes.c_double),
                ("precision", ctypes.c_int), ("schur_sweeps", ctypes.c_int), ("omega_S", ctypes.c_double),
                ("gamma", ctypes.c_int), ("vanka_colors", ctypes.c_int), ("schur_cg", ctypes.c_int),
                ("gamma_from", ctypes.c_int), ("fcycle", ctypes.c_int), ("gamma_to", ctypes.c_int),
                ("vanka_shift", ctypes.c_double), ("csr_below", ctypes.c_int), ("additive_levels", ctypes.c_int),
                ("omega_additive", ctypes.c_double)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("maxit", ctypes.c_int),
                ("iters", ctypes.c_int), ("converged", ctypes.c_int), ("rel_res_true", ctypes.c_double),
                ("side", ctypes.c_int), ("rel_res_prec", ctypes.c_double), ("reorth", ctypes.c_double),
                ("x0", ctypes.c_int)]


def load():
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libbiot_mg.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    lib.biot_assemble.argtypes = [ctypes.POINTER(Problem), P, ctypes.POINTER(P)]
    lib.biot_setup_hierarchy.argtypes = [P, ctypes.POINTER(MGOpts), P]
    lib.biot_vcycle.argtypes = [P, P, P, P]
    lib.biot_solve.argtypes = [P, P, P, ctypes.POINTER(SolveInfo), P]
    lib.biot_solve_noalloc.argtypes = [P, P, P, ctypes.POINTER(SolveInfo), P]
    lib.biot_apply_operator.argtypes = [P, I, P, P, P]
    lib.biot_smooth.argtypes = [P, I, P, P, P]
    lib.biot_restrict.argtypes = [P, I, P, P, P]
    lib.biot_prolong_add.argtypes = [P, I, P, P, P]
    lib.biot_update_K.argtypes = [P, P, P]
    lib.biot_update_logK.argtypes = [P, P, P]
    lib.biot_grad_logK.argtypes = [P, P, P, P, P]
    lib.biot_export_layout.argtypes = [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), P]
    lib.biot_kernel_timing.argtypes = [P, I, I, ctypes.POINTER(ctypes.c_double), P]
    lib.biot_destroy.argtypes = [P]
    lib.biot_destroy.restype = None
    lib.biot_last_error.restype = ctypes.c_char_p
    for name in ("biot_assemble", "biot_setup_hierarchy", "biot_vcycle", "biot_solve", "biot_solve_noalloc",
                 "biot_apply_operator", "biot_smooth", "biot_restrict", "biot_prolong_add",
                 "biot_update_K", "biot_update_logK", "biot_grad_logK", "biot_export_layout",
                 "biot_kernel_timing"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(code, allow=(BIOT_OK,)):
    if code not in allow:
        raise BiotError(code, load().biot_last_error().decode())
    return code


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, n=None, name="vector"):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("%s must be a contiguous float64 CUDA tensor" % name)
    if n is not None and t.numel() != n:
        raise ValueError("%s has %d entries, expected %d" % (name, t.numel(), n))
    return ctypes.c_void_p(t.data_ptr())


def n_free(n, bc="dirichlet"):
    """Free DoFs of the n x n mesh: 10 n^2 - 8 n + 2 (Dirichlet), 10 n^2 - 2 n (Terzaghi)."""
    return 10 * n * n - 8 * n + 2 if bc == "dirichlet" else 10 * n * n - 2 * n


class BiotSolver:
    """One assembled RQ Biot system with its multigrid hierarchy on the current device."""

    def __init__(self, n, lam, mu, alpha=1.0, M=1e6, mu_f=1.0, tau=1.0, K=1.0, bc="dirichlet"):
        """bc: "dirichlet" (u = 0, w.n = 0 on the whole boundary) or "terzaghi" (the column of
        Sec. 5; M = float("inf") allowed)."""
        lib = load()
        self.n = int(n)
        self.bc = bc
        prob = Problem()
        prob.n = self.n
        prob.bc = BCS[bc]
        prob.lambda_ = float(lam)
        prob.mu = float(mu)
        prob.alpha = float(alpha)
        prob.inv_M = 1.0 / float(M)
        prob.mu_f = float(mu_f)
        prob.tau = float(tau)
        self._K = None
        if isinstance(K, torch.Tensor):
            self._K = K.to(device="cuda", dtype=torch.float64).contiguous()
            _dev(self._K, 2 * self.n * self.n, "K")
            prob.K_tri = self._K.data_ptr()
            prob.K_scalar = 0.0
        else:
            prob.K_tri = None
            prob.K_scalar = float(K)
        ctx = ctypes.c_void_p()
        _check(lib.biot_assemble(ctypes.byref(prob), _stream(), ctypes.byref(ctx)))
        self._ctx = ctx
        self.levels = 0

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            load().biot_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def nf(self, level=0):
        return n_free(self.n >> level, self.bc)

    def setup(self, levels, smoother="vanka", nu1=2, nu2=2, omega=0.8, omega_J=1.0, precision="fp64",
              schur_sweeps=1, omega_S=1.0, gamma=1, vanka_colors=0, schur_cg=0, gamma_from=0, fcycle=False,
              gamma_to=0, vanka_shift=0.0, csr_below=0, additive_levels=0, omega_additive=0.0):
        """csr_below: levels below the finest with at most this many cells per side smooth on
        CSR operators and explicit patch inverses (FP64 Vanka; the same cycle up to rounding).
        additive_levels, omega_additive: with vanka_colors, the finest additive_levels levels take
        the additive step with weight omega_additive (0: omega)."""
        o = MGOpts(int(levels), SMOOTHERS[smoother], int(nu1), int(nu2), float(omega), float(omega_J),
                   PRECISIONS[precision], int(schur_sweeps), float(omega_S), int(gamma), int(vanka_colors),
                   int(schur_cg), int(gamma_from), int(bool(fcycle)), int(gamma_to), float(vanka_shift),
                   int(csr_below), int(additive_levels), float(omega_additive))
        _check(load().biot_setup_hierarchy(self._ctx, ctypes.byref(o), _stream()))
        self.levels = int(levels)
        return self

    def vcycle(self, r):
        z = torch.empty_like(r)
        _check(load().biot_vcycle(self._ctx, _dev(r, self.nf(), "r"), _dev(z), _stream()))
        return z

    def solve(self, b, tol=1e-8, restart=30, maxit=500, out=None, side="right", reorth=0.0, x0=None):
        """side "right": flexible GMRES stopping on the true residual; "left": GMRES on the
        left-preconditioned system stopping on the preconditioned residual.  reorth: the DGKS
        threshold of the second Gram-Schmidt pass (0: 1/sqrt(2)).  x0: initial guess (device FP64,
        canonical order; copied into the output first), else zero."""
        x = torch.empty_like(b) if out is None else out
        if x0 is not None:
            _dev(x0, self.nf(), "x0")
            x.copy_(x0.reshape(x.shape))
        info = SolveInfo(float(tol), int(restart), int(maxit), 0, 0, 0.0, SIDES[side], 0.0, float(reorth),
                         0 if x0 is None else 1)
        code = _check(load().biot_solve(self._ctx, _dev(b, self.nf(), "b"), _dev(x, self.nf(), "x"),
                                        ctypes.byref(info), _stream()), allow=(BIOT_OK, BIOT_NOT_CONVERGED))
        return x, dict(iters=info.iters, converged=bool(info.converged), rel_res_true=info.rel_res_true,
                       rel_res_prec=info.rel_res_prec, code=code)

    def solve_noalloc(self, b, out, tol=1e-8, restart=30, maxit=500, side="right", reorth=0.0, warm=False):
        """solve() through biot_solve_noalloc: no device allocation in the library; the caller
        passes the output tensor (with warm=True it holds the initial guess on entry)."""
        info = SolveInfo(float(tol), int(restart), int(maxit), 0, 0, 0.0, SIDES[side], 0.0, float(reorth),
                         1 if warm else 0)
        code = _check(load().biot_solve_noalloc(self._ctx, _dev(b, self.nf(), "b"), _dev(out, self.nf(), "x"),
                                                ctypes.byref(info), _stream()),
                      allow=(BIOT_OK, BIOT_NOT_CONVERGED))
        return out, dict(iters=info.iters, converged=bool(info.converged), rel_res_true=info.rel_res_true,
                         rel_res_prec=info.rel_res_prec, code=code)

    def apply(self, x, level=0):
        y = torch.empty_like(x)
        _check(load().biot_apply_operator(self._ctx, int(level), _dev(x, self.nf(level), "x"), _dev(y),
                                          _stream()))
        return y

    def smooth(self, x, b, level=0):
        x = x.clone()
        _check(load().biot_smooth(self._ctx, int(level), _dev(x, self.nf(level), "x"),
                                  _dev(b, self.nf(level), "b"), _stream()))
        return x

    def restrict(self, r, level=0):
        rc = torch.empty(self.nf(level + 1), dtype=torch.float64, device=r.device)
        _check(load().biot_restrict(self._ctx, int(level), _dev(r, self.nf(level), "r"), _dev(rc), _stream()))
        return rc

    def prolong_add(self, xc, xf, level=0):
        xf = xf.clone()
        _check(load().biot_prolong_add(self._ctx, int(level), _dev(xc, self.nf(level + 1), "x_c"),
                                       _dev(xf, self.nf(level), "x_f"), _stream()))
        return xf

    def update_K(self, K):
        self._K = K.to(device="cuda", dtype=torch.float64).contiguous()
        _check(load().biot_update_K(self._ctx, _dev(self._K, 2 * self.n * self.n, "K"), _stream()))

    def update_logK(self, theta):
        """Re-assemble for the per-triangle log-permeability theta = ln K (1/K = exp(-theta)
        is formed in the library)."""
        self._K = theta.to(device="cuda", dtype=torch.float64).contiguous()
        _check(load().biot_update_logK(self._ctx, _dev(self._K, 2 * self.n * self.n, "theta"), _stream()))

    def grad_logK(self, x, lam):
        g = torch.empty(2 * self.n * self.n, dtype=torch.float64, device=x.device)
        _check(load().biot_grad_logK(self._ctx, _dev(x, self.nf(), "x"), _dev(lam, self.nf(), "lam"),
                                     _dev(g), _stream()))
        return g

    def timing_start(self, level=0):
        _check(load().biot_kernel_timing(self._ctx, 1, int(level), None, _stream()))

    def timing_stop(self, level=0):
        out = (ctypes.c_double * 4)()
        _check(load().biot_kernel_timing(self._ctx, 0, int(level), out, _stream()))
        return dict(vanka_ms=out[0], vanka_launches=int(out[1]), resid_ms=out[2], resid_launches=int(out[3]))

    def export_layout(self, patches=True):
        counts = (ctypes.c_int * 12)()
        rows = (self.n + 1) ** 2 - 2
        table = (ctypes.c_int * (rows * 20))() if patches else None
        _check(load().biot_export_layout(self._ctx, counts, table, _stream()))
        out = dict(n=counts[0], n_free=counts[1], blocks=list(counts[2:12]))
        if patches:
            import numpy as np
            out["patches"] = np.frombuffer(table, dtype=np.int32).reshape(rows, 20).copy()
        return out


class SolveFn(torch.autograd.Function):
    """x = A(theta)^{-1} b with theta = ln K per triangle.  Backward: adjoint solve with the
    same hierarchy (A is symmetric) and the per-triangle gradient kernel."""

    @staticmethod
    def forward(ctx, theta, b, solver, tol, restart, maxit, adj_tol):
        solver.update_logK(theta.detach())
        token = object()
        solver._k_token = token
        x, info = solver.solve(b.detach().contiguous(), tol=tol, restart=restart, maxit=maxit)
        if not info["converged"]:
            raise BiotError(BIOT_NOT_CONVERGED, "forward solve did not converge")
        ctx.solver = solver
        ctx.token = token
        ctx.opts = (adj_tol, restart, maxit)
        ctx.save_for_backward(x, theta.detach())
        return x

    @staticmethod
    def backward(ctx, gx):
        x, theta = ctx.saved_tensors
        tol, restart, maxit = ctx.opts
        if getattr(ctx.solver, "_k_token", None) is not ctx.token:
            # the solver was re-assembled for another theta since this forward pass
            ctx.solver.update_logK(theta)
            ctx.solver._k_token = ctx.token
        lam, info = ctx.solver.solve(gx.contiguous(), tol=tol, restart=restart, maxit=maxit)
        if not info["converged"]:
            raise BiotError(BIOT_NOT_CONVERGED, "adjoint solve did not converge")
        g_theta = ctx.solver.grad_logK(x, lam)
        return g_theta, lam, None, None, None, None, None


def solve(theta, b, solver, tol=1e-10, restart=30, maxit=500, adj_tol=None):
    """x = A(theta)^{-1} b, differentiable in theta (per-triangle ln K) and b.  The adjoint
    solve of the backward pass runs to adj_tol (default: tol)."""
    return SolveFn.apply(theta, b, solver, tol, restart, maxit, tol if adj_tol is None else adj_tol)
