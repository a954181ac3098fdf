"""Write the oracle's dense reference gradient for a block-arrow instance
whose cliques have 70 and 24 vertices (n = 90, block 66, arrow 4, m = 40):
the larger clique is above the 64-vertex Jacobi size, so the GPU adjoint
takes its eigen-cache of up to 96 vertices there.  Instance 87 is strictly
complementary at the solution with some margin: the smallest |eigenvalue| of
the clique blocks of u* - v~* is 8e-4 (70 vertices) and 9e-3 (24) of the
largest.  The gradient's sensitivity to the forward solve grows as that
margin shrinks (DPi has a kink at a zero eigenvalue); of the block-arrow
instances screened, several have an eigenvalue of ~1e-10 at the solution,
where the gradient is not defined, and others a margin of ~2e-5, where a
solve to 1e-11 fixes it to only ~1e-3.

Calls only oracle/ (and the seeded generator): the forward solve is the
oracle's ADMM to eps_tol = 1e-11, the gradient is oracle.grad's dense
implicit differentiation of the fixed point (explicit T' from the dense
(I + Q)^-1 and the Daleckii-Krein derivative of the projection, least squares
on (I - T')^T mu = g).  Loss L = w^T x / tau with w ~ N(0, 1) over E'
(seed 4).  Output: grad_block_arrow_k70.txt, a header line with the run's
figures, then the nE values of dL/dc (svec over E', canonical order) and the
m values of dL/db, one per line.

Run:  python tests/golden/make_grad_block_arrow_k70.py   (several minutes)
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

OUT = os.path.join(HERE, "grad_block_arrow_k70.txt")
EPS = 1e-11
SHAPE = dict(n=90, block=66, arrow=4, m=40)
INSTANCE = 87


def instance():
    return configs.small_block_arrow(INSTANCE, **SHAPE)


def weights(prob):
    return np.random.default_rng(4).standard_normal(prob.nE)


def main():
    inst = instance()
    prob = hsde.build_problem(inst)
    w = weights(prob)
    t0 = time.time()
    L, res = grad.objective_weight_loss(inst, w, eps_tol=EPS, max_iter=400000)
    t1 = time.time()
    print(f"forward: {res.iters} iterations, {t1 - t0:.1f}s", flush=True)
    gc, gb = grad.adjoint_gradient_dense(res, w)
    t2 = time.time()
    head = dict(instance=f"small_block_arrow({INSTANCE}, {SHAPE})", cliques=[len(c) for c in inst.cliques],
                nE=prob.nE, eps_tol=EPS, forward_iterations=res.iters, loss=L,
                forward_s=round(t1 - t0, 1), gradient_s=round(t2 - t1, 1))
    with open(OUT, "w") as f:
        f.write("# " + json.dumps(head) + "\n")
        for v in np.concatenate([gc, gb]):
            f.write(f"{v:.17e}\n")
    print(json.dumps(head))


if __name__ == "__main__":
    main()
