#!/usr/bin/env python
"""Throughput benchmark: FGMRES + monolithic multigrid V-cycle solves to relative residual
1e-8 on the 256 x 256 workload (9 parameter sets: nu in {0.2, 0.49, 0.4999} x K in
{1, 1e-3, 1e-6}, E = 1, tau = 1, right-hand side uniform[-1, 1] from seed 1, 7 levels).

One step = one full solve of every (parameter set, smoother) pair, hierarchies built
beforehand, inputs resident in device memory.  Metric: free DoFs solved per second
(MDOF/s).  Prints one JSON line.
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
CSRC = os.path.join(ROOT, "paper_2107_04060_amd", "csrc")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_vanka_uniform_sweep256_fp64.md")


def kernel_source_hash():
    """sha256 over the HIP/C++ sources of the library (file names and contents, sorted)."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per finest-level Vanka launch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the kernel sources changed
    since the counters were taken (or no summary exists)."""
    try:
        with open(TRAFFIC_PROFILE) as f:
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
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sweep256")
    ap.add_argument("--smoothers", default="vanka,bsr")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="before the warm-up, copy a device buffer of this many MiB once (the plain "
                         "copy kernel that scales the HBM byte counters)")
    return ap.parse_args()


def weights(smoother, nu, K):
    """LFA-optimized relaxation weights of the workload's parameter sets."""
    from paper_2107_04060_amd import inputs
    return inputs.relaxation_weights(smoother, nu, K)


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


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only (the solver has no multi-GPU path); "
              "--gpus %d is not supported" % max(args.gpus, world), file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2107_04060_amd import binding, inputs
    from paper_2107_04060_amd.build import LIB
    if not os.path.exists(LIB):
        from paper_2107_04060_amd import build as _b
        _b.build(verbose=False)
    torch.cuda.set_device(0)
    w = inputs.workload(args.workload)
    n, levels = w["n"], w["levels"]
    nf = inputs.n_free(n)
    smoothers = [s for s in args.smoothers.split(",") if s]
    b_np = inputs.rhs_uniform(n, w["seed"])
    b = torch.tensor(b_np, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    runs = []
    for sm in smoothers:
        for case in w["cases"]:
            om, omj = weights(sm, case["nu"], case["K"])
            s = binding.BiotSolver(n, case["lam"], case["mu"], alpha=w["alpha"], M=w["M"], mu_f=w["mu_f"],
                                   tau=w["tau"], K=case["K"])
            nu12 = w["nu12"][sm]
            s.setup(levels=levels, smoother=sm, nu1=nu12, nu2=nu12, omega=om, omega_J=omj,
                    precision=args.precision)
            runs.append(dict(solver=s, smoother=sm, case=case, omega=om, omega_J=omj, nu12=nu12))
    torch.cuda.synchronize()

    def step(record):
        for r in runs:
            _, info = r["solver"].solve(b, tol=args.tol, restart=30, maxit=400, out=x)
            if record is not None:
                record.append(info)

    if args.copy_calib_mb > 0:
        src = torch.ones(args.copy_calib_mb * 2**20 // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step(None)
    for r in runs:
        r["solver"].timing_start(0)
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(infos)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    vk_ms, vk_n, rs_ms, rs_n = 0.0, 0, 0.0, 0
    for r in runs:
        t = r["solver"].timing_stop(0)
        vk_ms += t["vanka_ms"]
        vk_n += t["vanka_launches"]
        rs_ms += t["resid_ms"]
        rs_n += t["resid_launches"]
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    solves_per_step = len(runs)
    value = solves_per_step * nf / (ms_per_step * 1e-3) / 1e6
    per_case = []
    for k, r in enumerate(runs):
        info = infos[k]
        per_case.append({"smoother": r["smoother"], "nu": r["case"]["nu"], "K": r["case"]["K"],
                         "omega": r["omega"], "omega_J": r["omega_J"], "iters": info["iters"],
                         "rel_res_true": info["rel_res_true"], "converged": info["converged"]})
    all_conv = all(i["converged"] for i in infos)
    word = 8 if args.precision == "fp64" else 4
    bytes_per_launch = 3 * word * nf + 2 * word * n * n
    roofline = None
    if vk_n > 0:
        avg_s = vk_ms / vk_n * 1e-3
        achieved = bytes_per_launch / avg_s / 1e9
        traffic = measured_traffic() if (args.workload == "sweep256" and args.precision == "fp64") else None
        roofline = {"kernel": "k_vanka_uniform (additive Vanka, finest level)", "bound": "hbm",
                    "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "avg_launch_us": round(avg_s * 1e6, 2), "launches": vk_n,
                    "algorithmic_bytes_per_launch": bytes_per_launch}
    resid = None
    if rs_n > 0:
        avg_r = rs_ms / rs_n * 1e-3
        rb = 3 * word * nf + 2 * word * n * n
        resid = {"kernel": "k_apply residual (finest level)", "avg_launch_us": round(avg_r * 1e6, 2),
                 "achieved_GBs": round(rb / avg_r / 1e9, 1), "launches": rs_n}
    cpu = None
    if not args.no_cpu_baseline:
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
                   "solves_per_step": solves_per_step, "smoothers": smoothers,
                   "precision": args.precision, "tol": args.tol, "all_converged": all_conv},
        "roofline": roofline, "residual_kernel": resid, "cpu_baseline": cpu, "cases": per_case,
    }
    print(json.dumps(out), flush=True)
    for r in runs:
        r["solver"].close()


if __name__ == "__main__":
    main()
