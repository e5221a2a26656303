"""Writes tests/golden/terzaghi_table6_oracle.json from the oracle only (oracle/terzaghi.py,
oracle/multigrid.py, oracle/krylov.py): the Table 6 runs of Sec. 5 (h = 1/64, tau = tau_hat / 100,
10 steps, k = 1e-6, additive Vanka V(2,2) with omega = 0.8 and the 1e-8 patch shift, direct
solve at h = 1/8, left-preconditioned GMRES(30) to 1e-6) for each Poisson ratio: the iteration
count of every step and the errors (|u - u_h|_{H^1}, ||p - p_h||_{L^2}) against the series at
t = tau_hat / 10.  Run: python tests/golden/make_terzaghi_oracle.py"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.krylov import gmres_left            # noqa: E402
from oracle.multigrid import Hierarchy          # noqa: E402
from oracle.terzaghi import Terzaghi            # noqa: E402

N, K, STEPS = 64, 1e-6, 10


def run(nu):
    T = Terzaghi(N, nu, K)
    H = Hierarchy(N, T.params, K_tri=K, smoother="vanka", omega=0.8, nu1=2, nu2=2, levels=4, bc="terzaghi",
                  vanka_shift=1e-8)
    its = []

    def solve(b, m):
        x, info = gmres_left(H.A, b, H.vcycle, tol=1e-6, restart=30, maxit=60)
        assert info["converged"]
        its.append(int(info["iters"]))
        return x
    x = T.run(STEPS, solve)
    eu, ep = T.errors(x, STEPS * T.tau)
    return dict(iters=its, err_u_H1=eu, err_p_L2=ep)


if __name__ == "__main__":
    out = {"n": N, "k": K, "steps": STEPS, "omega": 0.8, "nu1": 2, "nu2": 2, "levels": 4, "shift": 1e-8,
           "restart": 30, "tol": 1e-6, "runs": {}}
    for nu in (0.4, 0.45, 0.49, 0.499):
        out["runs"][repr(nu)] = run(nu)
        print(nu, out["runs"][repr(nu)], flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "terzaghi_table6_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
