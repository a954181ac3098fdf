"""Write the oracle's outcomes on the uneven-clique workload (n = 5000,
cliques of 4-96 vertices, m = 2000) and its infeasible twin (m = 2002).

Calls only oracle/ (and the seeded generator).  Each solve runs eqs.
(Step1)-(Step3) from the initial point with eps_tol = 1e-4, at most 2000
iterations and the status checked after every iteration (Section 5's
stopping rule; the residuals and tests of readings R4-R5 in oracle/hsde.py).
Records per run: status, stop iteration, c^T x / tau, b^T y / tau and the
residuals at the stop.  Output: uneven_cliques_5000_oracle.json.

Run:  python tests/golden/make_uneven_solves.py   (about 15 minutes)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import hsde  # noqa: E402
from sdpgen import configs  # noqa: E402

OUT = os.path.join(HERE, "uneven_cliques_5000_oracle.json")


def run(inst, alpha):
    t0 = time.time()
    res = hsde.solve(inst, eps_tol=1e-4, max_iter=2000, alpha=alpha)
    r = res.res
    tau = r["tau"]
    out = {"alpha": alpha, "status": hsde.STATUS_NAMES[res.status], "iterations": res.iters,
           "eps_p": r["eps_p"], "eps_d": r["eps_d"], "eps_g": r["eps_g"], "cx": r["cx"], "by": r["by"],
           "tau": tau, "kappa": r["kappa"], "seconds": round(time.time() - t0, 1)}
    if tau > 0:
        out["obj_p"] = r["cx"] / tau
        out["obj_d"] = r["by"] / tau
    print(json.dumps(out), flush=True)
    return out


def main():
    feas = configs.uneven_cliques_5000()
    twin = configs.uneven_cliques_5000(twin=True)
    rec = {"feasible": {"plain": run(feas, 1.0), "relaxed": run(feas, 1.8)},
           "twin": {"plain": run(twin, 1.0)}}
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
