#!/usr/bin/env python
"""Throughput benchmark: FGMRES + monolithic multigrid V-cycle solves to relative residual
1e-8 (true FP64 residual), MDOF/s, FP32-smoother form against plain FP64.

Default workload (block2048): the 2048 x 2048 mesh (41,926,658 free DoFs, 10 levels), K = 1 or
1e-6 on 64 x 64-cell blocks (Bernoulli 1/2, seed 3), nu = 0.4999, E = 1, tau = 1, Vanka V(2,2)
with its LFA weight; its 16 right-hand sides (uniform[-1, 1] from the seed-3 stream, as time
steps) are solved in sequence with the hierarchy reused.  One step = one right-hand-side
solve from x = 0; the warm-up steps take the first right-hand sides, the timed steps the next
ones.  Every right-hand side is resident in device memory before the timed region.  The FP64
form gives `value`; the FP32-smoother form is timed the same way in the same run.  Prints one
JSON line.

--workload sweep256 (also small, grf1024) runs the 256 x 256 sweep instead: one step = the 18
solves of its 9 parameter sets x {Vanka V(2,2), BSR V(1,1)}, concurrently on --streams streams.

--workload terzaghi runs Terzaghi's column (Sec. 5, Table 6: h = 1/64, M = infinity, k = 1e-6,
tau = tau_hat / 100, additive Vanka V(2,2) with the 1e-8 patch shift, left-preconditioned
GMRES(30) to 1e-6) on the general-boundary path: one step = one backward-Euler time step (its
right-hand side formed on the device, then the solve), ten per Poisson ratio.  The default run
appends the same measurement to its line ("terzaghi_table6"; --no-terzaghi skips it).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BLOCK_RESTART = 100          # FGMRES restart of the block-contrast workload
BLOCK_REORTH = 0.01          # its Gram-Schmidt threshold: a second pass after two digits of cancellation
# the cycle of the block-contrast workload: the fastest to 1e-8 among the V-, W- and partial
# W-cycles with additive and multiplicative Vanka and 8 to 10 levels measured on it (the
# V(2,2) cycle with the LFA weight on 10 levels takes 178 iterations, 3.6 s per solve); the levels
# of 64 x 64 cells and below smooth on CSR operators with explicit patch inverses (468 -> 395 ms
# per solve with the fused colour step; 128: 395, 256: 428)
BLOCK_CYCLE = dict(nu12=1, omega=1.1, colors=3, gamma=2, gamma_from=1, levels=8, fcycle=0, csr_below=64)
CSRC = os.path.join(ROOT, "paper_2107_04060_amd", "csrc")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_vanka_step_sweep256_fp64.md")
BLOCK_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_vanka_step_block2048_fp64.md")


# sources that define the finest-level Vanka step (its traffic summary is valid while they are
# unchanged)
VANKA_SOURCES = ["vanka.hip", "tile.h", "patch_solve.h", "structure.h", "common.h", "kernels.h"]


def kernel_source_hash():
    """sha256 over the sources of the Vanka step kernel (file names and contents, in order)."""
    import hashlib
    h = hashlib.sha256()
    for name in VANKA_SOURCES:
        h.update(name.encode())
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(path=None):
    """HBM bytes per finest-level Vanka launch from a committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the Vanka step's sources changed
    since the counters were taken (or no summary exists)."""
    try:
        with open(path or TRAFFIC_PROFILE) as f:
            text = f.read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return int(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 8 right-hand sides for block2048, 3 sweeps for sweep256)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="block2048",
                    choices=["block2048", "sweep256", "small", "grf1024", "terzaghi"], help="the timed workload")
    ap.add_argument("--no-terzaghi", action="store_true",
                    help="block2048: skip the Terzaghi (Table 6) runs appended to the line")
    ap.add_argument("--terzaghi-n", type=int, default=64, help="terzaghi: cells per side (<= 256)")
    ap.add_argument("--forms", default="fp64,fp32",
                    help="block2048: the precision forms timed in turn (the first one gives value)")
    ap.add_argument("--nu12", type=int, default=BLOCK_CYCLE["nu12"],
                    help="block2048: pre- and post-smoothing steps")
    ap.add_argument("--omega", type=float, default=BLOCK_CYCLE["omega"], help="block2048: relaxation weight")
    ap.add_argument("--colors", type=int, default=BLOCK_CYCLE["colors"],
                    help="block2048: 0 additive Vanka, 3 or 4 multiplicative (three or four colours)")
    ap.add_argument("--gamma", type=int, default=BLOCK_CYCLE["gamma"], help="block2048: cycle index")
    ap.add_argument("--gamma-from", type=int, default=BLOCK_CYCLE["gamma_from"],
                    help="block2048: levels from this one down repeat their coarse correction gamma times")
    ap.add_argument("--fcycle", type=int, default=BLOCK_CYCLE["fcycle"], choices=[0, 1],
                    help="block2048: 1 = the repeated coarse corrections are V-cycles (F-cycle), 0 = W-cycle")
    ap.add_argument("--restart", type=int, default=BLOCK_RESTART, help="block2048: FGMRES restart")
    ap.add_argument("--additive-levels", type=int, default=0,
                    help="block2048: the finest levels taking the additive step instead of the colours")
    ap.add_argument("--omega-additive", type=float, default=0.0, help="block2048: their weight (0: --omega)")
    ap.add_argument("--csr-below", type=int, default=BLOCK_CYCLE["csr_below"],
                    help="block2048: levels below the finest with at most this many cells per side smooth on CSR "
                         "operators and explicit patch inverses, in FP64 (0: off)")
    ap.add_argument("--reorth", type=float, default=BLOCK_REORTH,
                    help="block2048: Gram-Schmidt second pass when |w1| < reorth |w0| (0: 1/sqrt(2))")
    ap.add_argument("--levels", type=int, default=BLOCK_CYCLE["levels"],
                    help="block2048: mesh levels (8: direct solve on the 16 x 16 mesh)")
    ap.add_argument("--reference", type=int, default=1,
                    help="block2048: also solve the first timed right-hand side to 1e-10 in FP64 (restart 100) "
                         "as the reference of the per-field errors")
    ap.add_argument("--smoothers", default="vanka,bsr")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "fp32_patch"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--streams", type=int, default=8,
                    help="the independent solves of a step run concurrently on this many streams (one host "
                         "thread each)")
    ap.add_argument("--extras", action="store_true",
                    help="sweep256: also run the precision-form, adjoint, Schur-sweep and multiplicative-Vanka "
                         "comparisons (several minutes)")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="before the warm-up, copy a device buffer of this many MiB once (the plain "
                         "copy kernel that scales the HBM byte counters)")
    return ap.parse_args()


def weights(smoother, nu, K):
    """LFA-optimized relaxation weights of the workload's parameter sets."""
    from paper_2107_04060_amd import inputs
    return inputs.relaxation_weights(smoother, nu, K)


def poisson(case):
    """Poisson ratio of a parameter set given by its Lame parameters."""
    return round(case["lam"] / (2.0 * (case["lam"] + case["mu"])), 6)


def cpu_baseline(case, b, iters, nu12, omega, omega_J, smoother, n, levels):
    """Oracle (plain FP64 NumPy/SciPy, single thread) on a bounded sample of the workload:
    the time of one FGMRES iteration (one V-cycle, one matvec, Gram-Schmidt) of one
    parameter set on the full 256 x 256 mesh, scaled by the GPU's iteration count."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.fem import BiotParams
    from oracle.multigrid import Hierarchy
    from oracle.krylov import fgmres
    from paper_2107_04060_amd import inputs
    with threadpool_limits(limits=1):
        p = BiotParams(case["lam"], case["mu"], alpha=1.0, M=inputs.biot_modulus(1.0), mu_f=1.0, tau=1.0)
        H = Hierarchy(n, p, K_tri=case["K"], smoother=smoother, omega=omega, omega_J=omega_J,
                      nu1=nu12, nu2=nu12, levels=levels)
        t0 = time.perf_counter()
        fgmres(H.A, b, H.vcycle, tol=1e-30, restart=30, maxit=2)
        t_it = (time.perf_counter() - t0) / 2.0
    nf = inputs.n_free(n)
    return {"value": nf / (t_it * iters) / 1e6, "unit": "MDOF/s", "cores": 1, "kind": "oracle",
            "sample": "2 FGMRES iterations (V(%d,%d) %s cycle + matvec + MGS) of nu=%.4g K=%g on the "
                      "%dx%d mesh, single thread, %.2f s/iteration, scaled by the GPU's %d iterations"
                      % (nu12, nu12, smoother, case["nu"], case["K"], n, n, t_it, iters)}


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, (time.perf_counter() - t) * 1e3


def field_diffs(x, ref, n):
    """Per field (canonical order u, w, p) |x - ref| / |ref|; p with its mean removed, since the
    constant pressure is the near-null mode that dominates |x| for a random right-hand side."""
    import torch
    nu_, nw_ = 5 * n * n - 6 * n + 2, 3 * n * n - 2 * n
    out = {}
    for name, a, z in (("u", 0, nu_), ("w", nu_, nu_ + nw_), ("p_mean_removed", nu_ + nw_, None)):
        xa, ra = x[a:z], ref[a:z]
        if name.startswith("p"):
            xa, ra = xa - xa.mean(), ra - ra.mean()
        out[name] = float(torch.linalg.norm(xa - ra) / torch.linalg.norm(ra))
    return out


def schur_extra(binding, inputs, torch, cg=4):
    """BSR V(1,1) on the sweep256 parameter sets, one solve at a time (FP64, 1e-8): the paper's
    single weighted-Jacobi step on the approximate Schur complement against two Jacobi sweeps
    (weight 1) and `cg` conjugate-gradient steps on it, with the same outer weights; iterations
    and solve times per set."""
    w = inputs.workload("sweep256")
    n, levels = w["n"], w["levels"]
    b = torch.tensor(inputs.rhs_uniform(n, w["seed"]), dtype=torch.float64, device="cuda")
    forms = (("jacobi_step", {}), ("sweeps_2", dict(schur_sweeps=2, omega_S=1.0)),
             ("cg_%d" % cg, dict(schur_cg=cg)))
    rows = []
    tot = {f: [0, 0.0] for f, _ in forms}
    for case in w["cases"]:
        om, omj = inputs.relaxation_weights("bsr", case["nu"], case["K"])
        row = {"nu": case["nu"], "K": case["K"]}
        for f, kw in forms:
            s = binding.BiotSolver(n, case["lam"], case["mu"], alpha=w["alpha"], M=w["M"], mu_f=w["mu_f"],
                                   tau=w["tau"], K=case["K"])
            s.setup(levels=levels, smoother="bsr", nu1=1, nu2=1, omega=om, omega_J=omj, **kw)
            s.solve(b, tol=1e-8, restart=30, maxit=500)                 # warm-up
            (x, info), ms = _timed(lambda: s.solve(b, tol=1e-8, restart=30, maxit=500))
            s.close()
            row[f] = {"iters": info["iters"], "ms": round(ms, 2), "converged": bool(info["converged"])}
            tot[f][0] += info["iters"]
            tot[f][1] += ms
        rows.append(row)
    return {"workload": "sweep256 BSR V(1,1) parameter sets, one solve at a time, FP64, 1e-8", "cases": rows,
            "total": {f: {"iters": v[0], "ms": round(v[1], 1)} for f, v in tot.items()}}


def multicolor_extra(binding, inputs, torch, omega_m=None):
    """Vanka on the sweep256 parameter sets, one solve at a time (FP64, 1e-8): the paper's additive
    V(2,2) cycle against the four-colour multiplicative V(1,1) cycle (weight omega_m, or by default
    the set's weight from the oracle's search on the 64 x 64 mesh, vanka_mult).  Per unit of
    smoothing traffic: a fused Vanka launch moves the same bytes in both forms; an additive V(2,2)
    cycle makes 4 launches per level, a multiplicative V(1,1) cycle 8."""
    w = inputs.workload("sweep256")
    n, levels = w["n"], w["levels"]
    b = torch.tensor(inputs.rhs_uniform(n, w["seed"]), dtype=torch.float64, device="cuda")
    rows = []
    tot = {"additive": [0, 0.0, 0], "multiplicative": [0, 0.0, 0]}
    for case in w["cases"]:
        om, omj = inputs.relaxation_weights("vanka", case["nu"], case["K"])
        om_m = omega_m if omega_m else inputs.relaxation_weights("vanka_mult", case["nu"], case["K"])[0]
        row = {"nu": case["nu"], "K": case["K"], "omega_multiplicative": om_m}
        for form, nu12, omega, colors, per_cycle in (("additive", 2, om, 0, 4), ("multiplicative", 1, om_m, 4, 8)):
            s = binding.BiotSolver(n, case["lam"], case["mu"], alpha=w["alpha"], M=w["M"], mu_f=w["mu_f"],
                                   tau=w["tau"], K=case["K"])
            s.setup(levels=levels, smoother="vanka", nu1=nu12, nu2=nu12, omega=omega, omega_J=omj,
                    vanka_colors=colors)
            s.solve(b, tol=1e-8, restart=30, maxit=500)                 # warm-up
            (x, info), ms = _timed(lambda: s.solve(b, tol=1e-8, restart=30, maxit=500))
            s.close()
            row[form] = {"iters": info["iters"], "ms": round(ms, 2), "converged": bool(info["converged"]),
                         "fused_launches_per_level": per_cycle * info["iters"]}
            tot[form][0] += info["iters"]
            tot[form][1] += ms
            tot[form][2] += per_cycle * info["iters"]
        rows.append(row)
    return {"workload": "sweep256 Vanka parameter sets, one solve at a time, FP64, 1e-8; additive V(2,2) with the "
                        "LFA weights, multiplicative V(1,1) with %s" % (
                            "omega %.2f" % omega_m if omega_m else "the weights of the oracle's 64 x 64 search"),
            "cases": rows,
            "total": {k: {"iters": v[0], "ms": round(v[1], 1), "fused_launches_per_level": v[2]}
                      for k, v in tot.items()}}


def precision_extra(binding, inputs, torch):
    """The 1024 x 1024 heterogeneous-permeability workload solved by the plain FP64 form and by the
    two precision forms: "fp32" (FP32 vectors and residuals, FP64 patch arithmetic and Krylov) and
    "fp32_patch" (the variable-K Vanka eliminations in FP32 too); same right-hand side, tolerance
    1e-8 in the FP64 true residual; per field, the relative difference of each FP32 form's
    solution from the FP64 one."""
    import numpy as np
    w = inputs.workload("grf1024")
    c = w["cases"][0]
    n = w["n"]
    K = torch.tensor(inputs.permeability_triangles("grf1024"), dtype=torch.float64, device="cuda")
    om, omj = inputs.relaxation_weights("vanka", workload="grf1024")
    b = torch.tensor(inputs.rhs_uniform(n, w["seed"]), dtype=torch.float64, device="cuda")
    res = {}
    sol = {}
    forms = ("fp64", "fp32", "fp32_patch")
    for prec in forms:
        s = binding.BiotSolver(n, c["lam"], c["mu"], alpha=w["alpha"], M=w["M"], mu_f=w["mu_f"], tau=w["tau"], K=K)
        s.setup(levels=w["levels"], smoother="vanka", nu1=2, nu2=2, omega=om, omega_J=omj, precision=prec)
        s.solve(b, tol=1e-8, restart=30, maxit=300)                     # warm-up
        (x, info), ms = _timed(lambda: s.solve(b, tol=1e-8, restart=30, maxit=300))
        sol[prec] = x
        res[prec] = {"ms": round(ms, 3), "iters": info["iters"], "rel_res_true": info["rel_res_true"],
                     "MDOF/s": round(inputs.n_free(n) / (ms * 1e-3) / 1e6, 2)}
        s.close()
    # reference: the FP64 form at 1e-12 (the oracle's FGMRES does not finish at this size)
    s = binding.BiotSolver(n, c["lam"], c["mu"], alpha=w["alpha"], M=w["M"], mu_f=w["mu_f"], tau=w["tau"], K=K)
    s.setup(levels=w["levels"], smoother="vanka", nu1=2, nu2=2, omega=om, omega_J=omj, precision="fp64")
    xref, iref = s.solve(b, tol=1e-12, restart=30, maxit=600)
    s.close()
    res["reference"] = {"form": "fp64", "tol": 1e-12, "iters": iref["iters"], "rel_res_true": iref["rel_res_true"]}
    for prec in forms:
        res[prec]["rel_err_vs_reference"] = field_diffs(sol[prec], xref, n)
    for prec in forms[1:]:
        res[prec]["rel_diff_vs_fp64_solution"] = field_diffs(sol[prec], sol["fp64"], n)
        res[prec]["speedup_vs_fp64"] = round(res["fp64"]["ms"] / res[prec]["ms"], 3)
    res["workload"] = "grf1024 (1024x1024, log10 K = -3 + GRF(0.1), nu 0.49, tau 1e-2, Vanka V(2,2))"
    return res


def adjoint_extra(binding, inputs, torch, batch=8):
    """The 512 x 512 adjoint workload: for each of `batch` log-permeability samples, the forward
    solve alone, and forward + adjoint solve + per-triangle gradient (FP64, 1e-10)."""
    from paper_2107_04060_amd.binding import solve
    w = inputs.workload("adjoint512")
    c = w["cases"][0]
    n = w["n"]
    thetas, theta_obs = inputs.adjoint_fields(n, batch)
    om, omj = inputs.relaxation_weights("vanka", workload="adjoint512")
    s = binding.BiotSolver(n, c["lam"], c["mu"], alpha=w["alpha"], M=w["M"], mu_f=w["mu_f"], tau=w["tau"], K=1.0)
    s.setup(levels=w["levels"], smoother="vanka", nu1=2, nu2=2, omega=om, omega_J=omj)
    b = torch.tensor(inputs.rhs_uniform(n, w["seed"]), dtype=torch.float64, device="cuda")
    nu = inputs.n_free(n) - 2 * n * n
    s.update_K(torch.exp(torch.tensor(theta_obs, dtype=torch.float64, device="cuda")))
    p_obs = s.solve(b, tol=1e-12, restart=30, maxit=1000)[0][nu:].clone()
    th = [torch.tensor(t, dtype=torch.float64, device="cuda") for t in thetas]
    fwd_ms = grad_ms = 0.0
    for t in th:
        def fwd():
            with torch.no_grad():
                return solve(t, b, s, tol=1e-10, restart=30, maxit=1000)
        _, ms = _timed(fwd)
        fwd_ms += ms

        def both():
            tt = t.clone().requires_grad_(True)
            x = solve(tt, b, s, tol=1e-10, restart=30, maxit=1000)
            loss = 0.5 * ((x[nu:] - p_obs) ** 2).sum()
            loss.backward()
            return tt.grad
        _, ms = _timed(both)
        grad_ms += ms
    s.close()
    return {"workload": "adjoint512 (512x512, ln K = GRF(0.05), batch %d, tol 1e-10)" % batch,
            "forward_ms_per_sample": round(fwd_ms / batch, 3),
            "forward_adjoint_gradient_ms_per_sample": round(grad_ms / batch, 3),
            "gradient_over_forward": round(grad_ms / fwd_ms, 3)}


def large_mesh_extra(binding, inputs, torch, n=2048, cycles=4):
    """Finest-level kernel durations on a 2048 x 2048 mesh (41.9 M free DoFs, 10 levels, constant
    K, nu = 0.49): V(2,2) Vanka cycles with HIP-event kernel timing, algorithmic bytes per launch
    over the average launch time."""
    lam, mu = inputs.lame(1.0, 0.49)
    om, omj = inputs.relaxation_weights("vanka", 0.49, 1e-3)
    s = binding.BiotSolver(n, lam, mu, alpha=1.0, M=inputs.biot_modulus(1.0), mu_f=1.0, tau=1.0, K=1e-3)
    s.setup(levels=10, smoother="vanka", nu1=2, nu2=2, omega=om, omega_J=omj)
    nf = inputs.n_free(n)
    r = torch.rand(nf, dtype=torch.float64, device="cuda") * 2 - 1
    s.vcycle(r)
    torch.cuda.synchronize()
    s.timing_start(0)
    for _ in range(cycles):
        s.vcycle(r)
    t = s.timing_stop(0)
    s.close()
    vk = t["vanka_ms"] / t["vanka_launches"] * 1e-3
    rr = t["resid_ms"] / t["resid_launches"] * 1e-3
    vb = 3 * 8 * nf
    rb = 2 * 8 * nf + 8 * inputs.n_free(n // 2)
    return {"workload": "2048x2048, 10 levels, nu 0.49, K 1e-3, FP64, V(2,2) Vanka cycles",
            "k_vanka_step": {"avg_launch_us": round(vk * 1e6, 1), "algorithmic_bytes_per_launch": vb,
                             "achieved_GBs": round(vb / vk / 1e9, 1), "frac": round(vb / vk / 1e9 / HBM_PEAK_GBS, 3)},
            "k_residual_restrict": {"avg_launch_us": round(rr * 1e6, 1), "algorithmic_bytes_per_launch": rb,
                                    "achieved_GBs": round(rb / rr / 1e9, 1),
                                    "frac": round(rb / rr / 1e9 / HBM_PEAK_GBS, 3)}}




def cpu_baseline_block(n_gpu, iters_gpu, cyc, n_sample=256):
    """Oracle (plain FP64 NumPy/SciPy) on a bounded sample of the block-contrast workload: the
    same physics (K = 1 or 1e-6 on tiles of 1/32 of the side, nu = 0.4999) and the same cycle at
    n = 256 (7 levels), the time of 3 FGMRES iterations (one cycle, one matvec, MGS each) after a
    warm-up iteration, extrapolated per free DoF to the 2048 x 2048 mesh and scaled by the GPU's
    mean iteration count: an extrapolation, since the oracle cannot hold the full mesh.  The
    BLAS/LAPACK threads are set to the host's core count."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.fem import BiotParams
    from oracle.multigrid import Hierarchy
    from oracle.krylov import fgmres
    from paper_2107_04060_amd import inputs
    cores = os.cpu_count() or 1
    w = inputs.workload("block2048")
    c = w["cases"][0]
    with threadpool_limits(limits=cores):
        rng = np.random.default_rng(w["seed"])
        K = inputs.squares_to_triangles(inputs.block_contrast_squares(n_sample, n_sample // 32, rng))
        p = BiotParams(c["lam"], c["mu"], alpha=w["alpha"], M=w["M"], mu_f=w["mu_f"], tau=w["tau"])
        lv = int(np.log2(n_sample // cyc.get("n_coarse", 4))) + 1
        H = Hierarchy(n_sample, p, K_tri=K, smoother="vanka", omega=cyc["omega"], nu1=cyc["nu1"], nu2=cyc["nu2"],
                      levels=lv, gamma=cyc["gamma"], gamma_from=cyc["gamma_from"], vanka_colors=cyc["vanka_colors"],
                      fcycle=cyc["fcycle"])
        b = inputs.rhs_uniform(n_sample, w["seed"])
        fgmres(H.A, b, H.vcycle, tol=1e-30, restart=30, maxit=1)
        t0 = time.perf_counter()
        fgmres(H.A, b, H.vcycle, tol=1e-30, restart=30, maxit=3)
        t_it = (time.perf_counter() - t0) / 3.0
    nf_s, nf = inputs.n_free(n_sample), inputs.n_free(n_gpu)
    t_solve = t_it * (nf / nf_s) * iters_gpu
    return {"value": round(nf / t_solve / 1e6, 6), "unit": "MDOF/s", "cores": cores, "kind": "oracle",
            "sample": "3 FGMRES iterations (the same cycle + matvec + MGS) of the block-contrast physics on "
                      "the %dx%d mesh (%d free DoFs), %.2f s/iteration with %d BLAS threads, extrapolated per "
                      "free DoF to %dx%d and scaled by the GPU's %.1f iterations per solve (extrapolation)"
                      % (n_sample, n_sample, nf_s, t_it, cores, n_gpu, n_gpu, iters_gpu)}


TABLE6_PAPER = {0.4: 7.3, 0.45: 7.6, 0.49: 8.7, 0.499: 14.5}   # Table 6: average iterations


def terzaghi_runs(binding, inputs, torch, n=None, reps=1):
    """Terzaghi's column for each Poisson ratio of Table 6: set-up, then `steps` backward-Euler
    steps from u = 0, each a right-hand side formed on the device (the load plus the pressure rows
    of A applied to the previous displacement: alpha B_u u^{m-1}) and one left-preconditioned
    GMRES(30) solve to 1e-6.  The steps are timed together (HIP synchronization at both ends);
    `reps` repeats the ten steps, the last repetition is reported."""
    import numpy as np
    tz = inputs.TERZAGHI
    n = tz["n"] if n is None else n
    levels = max(2, int(round(np.log2(n))) - 2)          # direct solve on the 8 x 8 mesh
    load = torch.tensor(inputs.terzaghi_load(n, tz["p0"]), dtype=torch.float64, device="cuda")
    nf = inputs.n_free_terzaghi(n)
    rows = {}
    for nu in tz["nu"]:
        lam, mu = inputs.lame(tz["E"], nu)
        tau = inputs.terzaghi_tau_hat(tz["k"], lam, mu) / 100.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = binding.BiotSolver(n, lam, mu, alpha=1.0, M=float("inf"), mu_f=1.0, tau=tau, K=tz["k"], bc="terzaghi")
        s.setup(levels=levels, nu1=2, nu2=2, omega=0.8, vanka_shift=1e-8)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        blocks = s.export_layout(patches=False)["blocks"]
        n_u, n_w = sum(blocks[:5]), sum(blocks[5:8])
        for _ in range(reps):
            x = torch.zeros(nf, dtype=torch.float64, device="cuda")
            its = []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(tz["steps"]):
                xu = x.clone()
                xu[n_u:] = 0.0
                y = s.apply(xu)
                b = load.clone()
                b[n_u + n_w:] = y[n_u + n_w:]
                x, info = s.solve(b, tol=1e-6, restart=30, maxit=60, side="left")
                if not info["converged"]:
                    raise RuntimeError("Terzaghi nu %g: a step did not converge" % nu)
                its.append(info["iters"])
            torch.cuda.synchronize()
            total = time.perf_counter() - t0
        s.close()
        rows[repr(nu)] = {"iters": its, "mean_iters": round(float(np.mean(its)), 2), "paper_mean": TABLE6_PAPER[nu],
                          "ms_per_step": round(total * 1e3 / tz["steps"], 3), "setup_s": round(setup_s, 3),
                          "MDOF/s": round(tz["steps"] * nf / total / 1e6, 3)}
        print("terzaghi n %d nu %g: %s, %.2f ms per step" % (n, nu, its, total * 1e3 / tz["steps"]), file=sys.stderr,
              flush=True)
    return {"workload": "Terzaghi column (Sec. 5, Table 6): %d x %d (%d free DoFs, %d levels), E 3e4, k 1e-6, M inf, "
                        "tau tau_hat/100, %d steps, additive Vanka V(2,2) omega 0.8 with the 1e-8 shift, left GMRES(30) "
                        "to 1e-6; general-boundary path (CSR)" % (n, n, nf, levels, tz["steps"]),
            "n": n, "free_dofs": nf, "runs": rows}


def main_terzaghi(args, binding, inputs, torch):
    """--workload terzaghi: the Table 6 runs as the timed workload (value: MDOF/s over all steps)."""
    res = terzaghi_runs(binding, inputs, torch, n=args.terzaghi_n, reps=1 + args.warmup)
    runs = list(res["runs"].values())
    ms = sum(r["ms_per_step"] for r in runs) / len(runs)
    out = {"metric": "Terzaghi column backward-Euler steps (right-hand side + left GMRES(30) to 1e-6): MDOF/s",
           "value": round(res["free_dofs"] / (ms * 1e-3) / 1e6, 3), "unit": "MDOF/s", "n_gpus": 1,
           "steps": inputs.TERZAGHI["steps"] * len(runs), "warmup": args.warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "terzaghi", "n": res["n"], "free_dofs": res["free_dofs"]},
           "terzaghi_table6": res, "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def main_block2048(args, binding, inputs, torch):
    """The block-contrast workload: one step = one right-hand-side solve, hierarchy reused."""
    import numpy as np
    steps = 8 if args.steps is None else args.steps
    w = inputs.workload("block2048")
    c = w["cases"][0]
    n, levels = w["n"], args.levels
    nf = inputs.n_free(n)
    nrhs = w["n_rhs"]
    forms = [f for f in args.forms.split(",") if f]
    K = torch.tensor(inputs.permeability_triangles("block2048"), dtype=torch.float64, device="cuda")
    om, omj = args.omega, 1.0
    cyc = dict(nu1=args.nu12, nu2=args.nu12, omega=om, omega_J=omj, gamma=args.gamma, gamma_from=args.gamma_from,
               vanka_colors=args.colors, fcycle=bool(args.fcycle), additive_levels=args.additive_levels,
               omega_additive=args.omega_additive)
    restart = args.restart
    # right-hand sides k = 0 .. nrhs-1 of the seed stream (row k of rhs_uniform(n, seed, nrhs)),
    # uploaded before anything is timed; warm-up steps take the first ones, timed steps the next
    order = [(args.warmup + k) % nrhs for k in range(steps)]
    need = sorted(set(range(min(args.warmup, nrhs))) | set(order))
    rng = np.random.default_rng(w["seed"])
    rhs = {}
    for k in range(max(need) + 1):
        v = rng.uniform(-1.0, 1.0, nf)
        if k in need:
            rhs[k] = torch.tensor(v, dtype=torch.float64, device="cuda")
    del v
    x = torch.empty(nf, dtype=torch.float64, device="cuda")
    res = {}
    first = {}
    roofline = resid = None
    for fi, form in enumerate(forms):
        s = binding.BiotSolver(n, c["lam"], c["mu"], alpha=w["alpha"], M=w["M"], mu_f=w["mu_f"], tau=w["tau"], K=K)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.setup(levels=levels, smoother="vanka", precision=form, csr_below=args.csr_below, **cyc)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        if fi == 0 and args.copy_calib_mb > 0:
            # a plain device copy of known size: the scale of the HBM byte counters
            src = torch.ones(args.copy_calib_mb * 2**20 // 8, dtype=torch.float64, device="cuda")
            torch.empty_like(src).copy_(src)
            torch.cuda.synchronize()
            del src
        try:
            for k in range(args.warmup):
                _, info = s.solve(rhs[k % nrhs], tol=args.tol, restart=restart, maxit=600, out=x,
                                  reorth=args.reorth)
                print("block2048 %s warm-up rhs %d: %d iterations" % (form, k % nrhs, info["iters"]),
                      file=sys.stderr, flush=True)
        except binding.BiotError as e:
            # a form that breaks down (NaN met in the iteration) is reported, not timed
            print("block2048 %s: %s" % (form, e), file=sys.stderr, flush=True)
            res[form] = {"error": str(e)}
            s.close()
            if fi == 0:
                raise
            continue
        if fi == 0:
            s.timing_start(0)
        iters, ms, rr, conv = [], [], [], True
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in order:
            ta = time.perf_counter()
            _, info = s.solve(rhs[k], tol=args.tol, restart=restart, maxit=600, out=x, reorth=args.reorth)
            torch.cuda.synchronize()
            ms.append(round((time.perf_counter() - ta) * 1e3, 1))
            iters.append(info["iters"])
            rr.append(info["rel_res_true"])
            conv = conv and bool(info["converged"])
            if k == order[0]:
                first[form] = x.clone()
            print("block2048 %s rhs %d: %d iterations, %.0f ms" % (form, k, info["iters"], ms[-1]), file=sys.stderr,
                  flush=True)
        torch.cuda.synchronize()
        total_s = time.perf_counter() - t0
        if fi == 0:
            t = s.timing_stop(0)
            word = 8 if form == "fp64" else 4
            if t["vanka_launches"]:
                avg = t["vanka_ms"] / t["vanka_launches"] * 1e-3
                vb = 3 * word * nf + 2 * word * n * n
                roofline = {"kernel": "k_vanka_step<double, double, false, false, 4, false, 1> (fused residual + "
                                      "Vanka step on a non-zero iterate, variable K, finest level; in the "
                                      "multiplicative cycle one colour per launch)",
                            "bound": "hbm", "achieved": round(vb / avg / 1e9, 1), "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": round(vb / avg / 1e9 / HBM_PEAK_GBS, 4),
                            "traffic": measured_traffic(BLOCK_TRAFFIC_PROFILE) if form == "fp64" else None,
                            "avg_launch_us": round(avg * 1e6, 2), "launches": t["vanka_launches"],
                            "algorithmic_bytes_per_launch": vb,
                            "timed_in": "the timed steps of the first form (HIP events on the solve's stream)"}
            if t["resid_launches"]:
                avg = t["resid_ms"] / t["resid_launches"] * 1e-3
                rb = 2 * word * nf + word * inputs.n_free(n // 2)
                resid = {"kernel": "k_residual_restrict (finest level)", "avg_launch_us": round(avg * 1e6, 2),
                         "achieved_GBs": round(rb / avg / 1e9, 1), "launches": t["resid_launches"],
                         "algorithmic_bytes_per_launch": rb}
        s.close()
        res[form] = {"setup_s": round(setup_s, 2), "steps": len(order), "total_s": round(total_s, 3),
                     "ms_per_step": round(total_s * 1e3 / len(order), 1),
                     "MDOF/s": round(len(order) * nf / total_s / 1e6, 3), "iters": iters,
                     "mean_iters": round(float(np.mean(iters)), 2), "ms": ms, "rel_res_true_max": max(rr),
                     "all_converged": conv}
    for form in forms[1:]:
        if "error" in res[form]:
            continue
        res[form]["speedup_vs_" + forms[0]] = round(res[forms[0]]["total_s"] / res[form]["total_s"], 3)
        res[form]["first_rhs_rel_diff_vs_" + forms[0]] = field_diffs(first[form], first[forms[0]], n)
    if args.reference:
        s = binding.BiotSolver(n, c["lam"], c["mu"], alpha=w["alpha"], M=w["M"], mu_f=w["mu_f"], tau=w["tau"], K=K)
        s.setup(levels=levels, smoother="vanka", precision="fp64", **cyc)
        xref, iref = s.solve(rhs[order[0]], tol=1e-10, restart=restart, maxit=400)
        s.close()
        res["reference"] = {"form": "fp64", "tol": 1e-10, "rhs": order[0], "iters": iref["iters"],
                            "rel_res_true": iref["rel_res_true"],
                            "note": "the oracle cannot hold this mesh; the FP64 form to a tighter tolerance, itself "
                                    "parity-checked against the oracle on the same physics at n = 64 and 128"}
        for form in forms:
            if form in first:
                res[form]["first_rhs_rel_err_vs_reference"] = field_diffs(first[form], xref, n)
        del xref
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_block(n, res[forms[0]]["mean_iters"], dict(cyc, n_coarse=n >> (levels - 1)))
    head = res[forms[0]]
    out = {
        "metric": "FGMRES+V-cycle solve to rel.res 1e-8: MDOF/s (free DoFs 10n^2-8n+2 per right-hand-side solve)",
        "value": head["MDOF/s"], "unit": "MDOF/s", "n_gpus": 1, "steps": len(order), "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if forms[0] == "fp64" else "f32-smoother/f64-krylov", "data": "synthetic",
        "config": {"workload": "block2048", "n": n, "levels": levels, "free_dofs": nf,
                   "physics": "K 1 or 1e-6 per 64x64-cell block (seed 3), nu 0.4999, E 1, tau 1, M E/0.03",
                   "cycle": "%s Vanka, %d pre- and post-smoothing steps, omega %.2f, cycle index %d on levels >= %d "
                            "(finer levels: one coarse correction; %s), %d levels (direct solve at %d x %d)" % (
                                "multiplicative (%d colours)" % args.colors if args.colors else "additive", args.nu12, om,
                                args.gamma, args.gamma_from,
                                "the repeated corrections are V-cycles: F-cycle" if args.fcycle else "W-cycle",
                                levels, n >> (levels - 1), n >> (levels - 1)),
                   "restart": restart, "tol": args.tol, "gram_schmidt_second_pass_below": args.reorth,
                   "csr_levels_below": args.csr_below,
                   "step": "one right-hand-side solve from x = 0, hierarchy reused", "rhs_order": order,
                   "forms": forms, "all_converged": all(res[f].get("all_converged", False) for f in forms)},
        "precision_forms": res, "roofline": roofline, "residual_kernel": resid, "cpu_baseline": cpu,
    }
    if not args.no_terzaghi:
        out["terzaghi_table6"] = terzaghi_runs(binding, inputs, torch)
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the solver runs on one GPU (it has no multi-GPU path); "
              "--gpus %d is not supported" % max(args.gpus, world), file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2107_04060_amd import binding, inputs
    from paper_2107_04060_amd.build import LIB
    if not os.path.exists(LIB):
        from paper_2107_04060_amd import build as _b
        _b.build(verbose=False)
    torch.cuda.set_device(0)
    if args.workload == "block2048":
        main_block2048(args, binding, inputs, torch)
    elif args.workload == "terzaghi":
        main_terzaghi(args, binding, inputs, torch)
    else:
        if args.steps is None:
            args.steps = 3
        main_sweep(args, binding, inputs, torch)


def main_sweep(args, binding, inputs, torch):
    import numpy as np
    w = inputs.workload(args.workload)
    n, levels = w["n"], w["levels"]
    nf = inputs.n_free(n)
    smoothers = [s for s in args.smoothers.split(",") if s]
    b_np = inputs.rhs_uniform(n, w["seed"])
    b = torch.tensor(b_np, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    runs = []
    # the parameter sets of sweep256 carry a scalar K; the other workloads a per-triangle field
    if args.workload != "sweep256":
        smoothers = [sm for sm in smoothers if sm in w["smoothers"]]
    Kfield = None
    if any("K" not in case for case in w["cases"]):
        Kfield = torch.tensor(inputs.permeability_triangles(args.workload), dtype=torch.float64, device="cuda")
    for sm in smoothers:
        for case in w["cases"]:
            if args.workload == "sweep256":
                om, omj = weights(sm, case["nu"], case["K"])
            else:
                om, omj = inputs.relaxation_weights(sm, workload=args.workload)
            s = binding.BiotSolver(n, case["lam"], case["mu"], alpha=w["alpha"], M=w["M"], mu_f=w["mu_f"],
                                   tau=w["tau"], K=case.get("K", Kfield))
            nu12 = w["nu12"][sm]
            s.setup(levels=levels, smoother=sm, nu1=nu12, nu2=nu12, omega=om, omega_J=omj,
                    precision=args.precision)
            runs.append(dict(solver=s, smoother=sm, case=case, omega=om, omega_J=omj, nu12=nu12))
    torch.cuda.synchronize()

    # the solves of a step are independent systems: with --streams K, K host threads each issue
    # solves on a stream of their own (default priority), taking the next solve from a shared
    # queue, longest first by the previous step's solve times (a greedy longest-processing-time
    # schedule; the first step takes them in workload order)
    import threading
    nstreams = max(1, min(args.streams, len(runs)))
    streams = [torch.cuda.Stream() for _ in range(nstreams)] if nstreams > 1 else [torch.cuda.current_stream()]
    xs = [torch.empty_like(b) for _ in runs]
    bs = [b.clone() for _ in range(nstreams)]
    torch.cuda.synchronize()
    order = list(range(len(runs)))

    def work(k, out, queue, lock):
        with torch.cuda.stream(streams[k]):
            while True:
                with lock:
                    if not queue:
                        break
                    idx = queue.pop(0)
                t_a = time.perf_counter()
                _, info = runs[idx]["solver"].solve(bs[k], tol=args.tol, restart=30, maxit=400, out=xs[idx])
                streams[k].synchronize()
                info["solve_ms"] = (time.perf_counter() - t_a) * 1e3
                out[idx] = info
            streams[k].synchronize()

    def step(record, sequential=False):
        out = [None] * len(runs)
        queue, lock = list(order), threading.Lock()
        if nstreams == 1 or sequential:
            work(0, out, list(range(len(runs))), lock)
        else:
            th = [threading.Thread(target=work, args=(k, out, queue, lock)) for k in range(nstreams)]
            for t in th:
                t.start()
            for t in th:
                t.join()
        if not sequential:
            order[:] = sorted(range(len(runs)), key=lambda i: -out[i]["solve_ms"])
        if record is not None:
            record.extend(out)
        return out

    if args.copy_calib_mb > 0:
        src = torch.ones(args.copy_calib_mb * 2**20 // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step(None)
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(infos)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    solves_per_step = len(runs)
    value = solves_per_step * nf / (ms_per_step * 1e-3) / 1e6
    # one more step, solves one after the other on one stream (outside the timed region): the
    # per-smoother rates and per-solve times without concurrency, and the finest-level kernel
    # durations (HIP events around every launch, on the stream the kernels run on) without other
    # streams sharing the device
    for r in runs:
        r["solver"].timing_start(0)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    seq = step(None, sequential=True)
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t2) * 1e3
    vk_ms, vk_n, rs_ms, rs_n = 0.0, 0, 0.0, 0
    for r in runs:
        t = r["solver"].timing_stop(0)
        vk_ms += t["vanka_ms"]
        vk_n += t["vanka_launches"]
        rs_ms += t["resid_ms"]
        rs_n += t["resid_launches"]
    per_case = []
    for k, r in enumerate(runs):
        info = infos[k]
        per_case.append({"smoother": r["smoother"], "nu": r["case"].get("nu", poisson(r["case"])), "K": r["case"].get("K", "field"),
                         "omega": r["omega"], "omega_J": r["omega_J"], "iters": info["iters"],
                         "rel_res_true": info["rel_res_true"], "converged": info["converged"],
                         "solve_ms_sequential": round(seq[k]["solve_ms"], 3)})
    per_smoother = {}
    for sm in smoothers:
        ms_sm = [seq[k]["solve_ms"] for k, r in enumerate(runs) if r["smoother"] == sm]
        its = [seq[k]["iters"] for k, r in enumerate(runs) if r["smoother"] == sm]
        per_smoother[sm] = {"MDOF/s": round(len(ms_sm) * nf / (sum(ms_sm) * 1e-3) / 1e6, 3),
                            "solves": len(ms_sm), "iters": sum(its),
                            "ms_per_iteration": round(sum(ms_sm) / max(1, sum(its)), 4)}
    sequential = {"value": round(len(runs) * nf / (seq_ms * 1e-3) / 1e6, 3), "ms_per_step": round(seq_ms, 3),
                  "per_smoother": per_smoother}
    all_conv = all(i["converged"] for i in infos)
    word = 8 if args.precision == "fp64" else 4
    # fused step: read x_in and b, write x_out; with a permeability field also read 1/K (2 n^2)
    bytes_per_launch = 3 * word * nf + (2 * word * n * n if Kfield is not None else 0)
    roofline = None
    if vk_n > 0:
        avg_s = vk_ms / vk_n * 1e-3
        achieved = bytes_per_launch / avg_s / 1e9
        traffic = measured_traffic() if (args.workload == "sweep256" and args.precision == "fp64") else None
        roofline = {"kernel": "k_vanka_step (fused residual + additive Vanka, finest level)", "bound": "hbm",
                    "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "avg_launch_us": round(avg_s * 1e6, 2), "launches": vk_n,
                    "timed_in": "the sequential step (one stream)",
                    "algorithmic_bytes_per_launch": bytes_per_launch}
    resid = None
    if rs_n > 0:
        avg_r = rs_ms / rs_n * 1e-3
        rb = 2 * word * nf + word * inputs.n_free(n // 2)      # read x, b; write the coarse right-hand side
        resid = {"kernel": "k_residual_restrict (finest level)", "avg_launch_us": round(avg_r * 1e6, 2),
                 "achieved_GBs": round(rb / avg_r / 1e9, 1), "launches": rs_n,
                 "algorithmic_bytes_per_launch": rb}
    extras = None
    if args.extras and args.workload == "sweep256":
        extras = {"precision_form": precision_extra(binding, inputs, torch),
                  "adjoint": adjoint_extra(binding, inputs, torch),
                  "kernels_2048": large_mesh_extra(binding, inputs, torch),
                  "bsr_schur_sweeps": schur_extra(binding, inputs, torch),
                  "vanka_multiplicative": multicolor_extra(binding, inputs, torch)}
    cpu = None
    if not args.no_cpu_baseline and args.workload == "sweep256":
        r0 = runs[0]
        cpu = cpu_baseline(r0["case"], b_np, infos[0]["iters"], r0["nu12"], r0["omega"], r0["omega_J"],
                           r0["smoother"], n, levels)
    out = {
        "metric": "FGMRES+V-cycle solve to rel.res 1e-8: MDOF/s (free DoFs 10n^2-8n+2 per solve)",
        "value": round(value, 3), "unit": "MDOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32-smoother/f64-krylov",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "levels": levels, "free_dofs": nf,
                   "solves_per_step": solves_per_step, "smoothers": smoothers, "streams": nstreams,
                   "schedule": "greedy longest-first over the streams",
                   "precision": args.precision, "tol": args.tol, "all_converged": all_conv},
        "sequential": sequential, "extras": extras,
        "roofline": roofline, "residual_kernel": resid, "cpu_baseline": cpu, "cases": per_case,
    }
    print(json.dumps(out), flush=True)
    for r in runs:
        r["solver"].close()


if __name__ == "__main__":
    main()
