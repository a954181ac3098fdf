"""Write the oracle's dense reference gradient for instance 0 of the
differentiated block-arrow batch (n = 200, block 16, arrow 4, m = 100).

Calls only oracle/ (and the seeded generator): the forward solve is the
oracle's ADMM to eps_tol = 5e-11 (its residuals stop falling at eps_d ~2e-11,
eps_p ~2e-12 on this instance, after ~6000 iterations: the FP64 rounding
floor of step 1 here), the gradient is oracle.grad's dense
implicit differentiation of the fixed point (explicit T' from the dense
(I + Q)^-1 and the Daleckii-Krein derivative of the projection, least squares
on (I - T')^T mu = g).  Loss L = <W, X*> (Frobenius) with W from the
generator.  Output: grad_block_arrow_n200.txt, one value per line, the
nE values of dL/dc (svec over E', canonical order) then the m values of
dL/db, followed by a header line with the run's figures.

Run:  python tests/golden/make_grad_block_arrow_n200.py   (a few minutes)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import grad, hsde  # noqa: E402
from sdpgen import configs  # noqa: E402

OUT = os.path.join(HERE, "grad_block_arrow_n200.txt")
EPS = 5e-11


def loss_weights(inst, prob):
    """svec(W) over E' in canonical order."""
    wr, wc, wv = inst.meta["W"]
    key = {(int(r), int(c)): e for e, (r, c) in enumerate(zip(prob.erow, prob.ecol))}
    w = np.zeros(prob.nE)
    for r, c, x in zip(wr, wc, wv):
        w[key[(int(r), int(c))]] = x * (1.0 if r == c else np.sqrt(2.0))
    return w


def main():
    inst = configs.block_arrow_grad64(count=1)[0]
    prob = hsde.build_problem(inst)
    w = loss_weights(inst, prob)
    t0 = time.time()
    L, res = grad.objective_weight_loss(inst, w, eps_tol=EPS, max_iter=400000)
    t1 = time.time()
    gc, gb = grad.adjoint_gradient_dense(res, w)
    t2 = time.time()
    head = dict(instance="block_arrow_grad64[0]", n=inst.n, m=inst.m, nE=prob.nE, eps_tol=EPS,
                forward_iterations=res.iters, loss=L, forward_s=round(t1 - t0, 1),
                gradient_s=round(t2 - t1, 1))
    with open(OUT, "w") as f:
        f.write("# " + json.dumps(head) + "\n")
        for v in np.concatenate([gc, gb]):
            f.write(f"{v:.17e}\n")
    print(json.dumps(head))


if __name__ == "__main__":
    main()
