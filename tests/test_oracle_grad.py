"""Pin of the oracle's implicit gradient: central finite differences of
L(C, b) = <W, X*> on tightly solved instances."""
import numpy as np
import pytest

from oracle import grad, hsde
from sdpgen import configs


def _with_data(inst, prob, dc, db):
    sc = np.where(prob.erow == prob.ecol, 1.0, np.sqrt(2.0))
    key = {(int(r), int(c)): e for e, (r, c) in enumerate(zip(prob.erow, prob.ecol))}
    Cv = np.zeros(prob.nE)
    for r, c, v in zip(*inst.C):
        Cv[key[(int(r), int(c))]] += v
    Cv = Cv + dc / sc
    return configs.SDPInstance(inst.n, inst.m, (prob.erow.astype(np.int32), prob.ecol.astype(np.int32), Cv),
                               inst.A, inst.b + db, inst.cliques, inst.parent)


@pytest.mark.parametrize("seed", [11, 12])
def test_adjoint_gradient_matches_central_differences(seed):
    inst = configs.small_block_arrow(seed, n=10, block=3, arrow=2, m=4)
    prob = hsde.build_problem(inst)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(prob.nE)
    L0, res = grad.objective_weight_loss(inst, w, eps_tol=1e-11)
    gc, gb = grad.adjoint_gradient_dense(res, w)
    h = 1e-5
    for _ in range(3):
        dc = rng.standard_normal(prob.nE)
        db = rng.standard_normal(prob.m)
        Lp = grad.objective_weight_loss(_with_data(inst, prob, h * dc, h * db), w, eps_tol=1e-11)[0]
        Lm = grad.objective_weight_loss(_with_data(inst, prob, -h * dc, -h * db), w, eps_tol=1e-11)[0]
        fd = (Lp - Lm) / (2 * h)
        an = float(gc @ dc + gb @ db)
        # FD error ~ (solve accuracy)/h + h^2 L''' ; scale by the directional norm
        assert abs(fd - an) <= 1e-4 * (abs(an) + np.linalg.norm(gc) + np.linalg.norm(gb)), (fd, an)


def test_adjoint_iteration_reaches_the_dense_adjoint():
    """The fixed-point form mu <- mu - q + DPi(2q - mu) + g (what the GPU
    iterates) converges to a solution of the dense adjoint system."""
    inst = configs.small_block_arrow(13, n=10, block=3, arrow=2, m=4)
    prob = hsde.build_problem(inst)
    w = np.random.default_rng(3).standard_normal(prob.nE)
    _, res = grad.objective_weight_loss(inst, w, eps_tol=1e-11)
    gc, gb = grad.adjoint_gradient_dense(res, w)
    u = grad.flat(res.u)
    z = u - grad.flat(res.vt)
    ts = grad.TransposeSolver(prob)
    _, gu = grad.loss_and_du(prob, res.u, w)
    g = grad.dproj_apply(prob, z, gu)
    mu = g.copy()
    for _ in range(20000):
        new = grad.adjoint_step(prob, ts, z, mu, g)
        if np.linalg.norm(new - mu) <= 1e-13 * np.linalg.norm(new):
            mu = new
            break
        mu = new
    nu = ts.solve_transpose(mu)
    off = grad.offsets(prob)
    tau = u[off[4]]
    dc = -(tau * nu[off[0]:off[1]] - nu[off[4]] * u[off[0]:off[1]])
    db = tau * nu[off[2]:off[3]] - nu[off[4]] * u[off[2]:off[3]]
    assert np.linalg.norm(dc - gc) <= 1e-7 * np.linalg.norm(gc)
    assert np.linalg.norm(db - gb) <= 1e-7 * max(np.linalg.norm(gb), 1e-12)
