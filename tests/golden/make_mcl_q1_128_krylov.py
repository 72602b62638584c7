"""Writes mcl_q1_128_krylov.json: the Krylov iterations the oracle's
GMRES(30)-Jacobi (FP64, restarted, to 1e-10 ||b||) takes for the stationary
MCL workload on Q1 128^3 (Sec. 4): the low-order solve A_low u = F from zero,
and the first fixed-point iteration from that solution.  Calls only the
oracle (one thread, a few minutes).  Run from the repository root:
    python tests/golden/make_mcl_q1_128_krylov.py
"""
import json
import os
import sys
import time

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))

from threadpoolctl import threadpool_limits  # noqa: E402

from oracle import afc_oracle as O  # noqa: E402
from paper_2110_15676_amd import inputs as I  # noqa: E402


def main(n=128):
    inst = I.config3(n)
    with threadpool_limits(1):
        P = O.problem_from_instance(inst, conv=True)
        t = time.perf_counter()
        lo = O.low_order_solution(P, inst.F, lin_rtol=1e-10)
        t_lo = time.perf_counter() - t
        t = time.perf_counter()
        _, st = O.stationary_mcl(P, inst.F, lo.x, tol=0.0, tol_mode="rel", maxit=1, lin_rtol=1e-10)
        t_fp = time.perf_counter() - t
    out = {
        "workload": "stationary MCL, Q1 %d^3 (config 3), %d nodes" % (n, inst.N),
        "solver": "oracle GMRES(30), Jacobi, FP64, relative tolerance 1e-10",
        "low_order_krylov_iters": int(lo.iters),
        "first_iteration_krylov_iters": int(sum(st.krylov_iters)),
        "oracle_seconds": [round(t_lo, 1), round(t_fp, 1)],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mcl_q1_%d_krylov.json" % n)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
