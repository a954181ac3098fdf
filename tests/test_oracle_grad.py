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


# ----------------------------------------------------------------------------
# the Daleckii-Krein derivative of the PSD projection on its own
# ----------------------------------------------------------------------------

def _sym(rng, K):
    G = rng.standard_normal((K, K))
    return (G + G.T) / 2


@pytest.mark.parametrize("K", [2, 3, 5, 8, 13, 20])
def test_dproj_block_matches_central_differences_of_the_projection(K):
    """dproj_block(Y, dY) against (Pi(Y + h dY) - Pi(Y - h dY)) / 2h, with Pi
    the projection by eigendecomposition.  Random Y has no eigenvalue near 0
    (where Pi is not differentiable): the truncation error is O(h^2) and the
    rounding error O(eps / h)."""
    rng = np.random.default_rng(100 + K)
    for _ in range(5):
        Y = _sym(rng, K)
        lam = np.linalg.eigvalsh(Y)
        assert np.min(np.abs(lam)) > 1e-3
        dY = _sym(rng, K)
        h = 1e-5
        fd = (hsde.proj_psd(Y + h * dY) - hsde.proj_psd(Y - h * dY)) / (2 * h)
        an = grad.dproj_block(Y, dY)
        assert np.linalg.norm(an - fd) <= 1e-8 * np.linalg.norm(fd), np.linalg.norm(an - fd)


def test_dproj_block_special_cases():
    """Positive definite Y: the projection is the identity near Y, so DPi = I.
    Negative definite: DPi = 0.  A 2x2 diagonal Y = diag(a, -c): the
    off-diagonal entry of dY is scaled by a / (a + c) (the divided difference
    of max(., 0) between a and -c), the diagonal keeps only the (1,1) entry."""
    rng = np.random.default_rng(7)
    G = rng.standard_normal((6, 6))
    P = G @ G.T + 0.1 * np.eye(6)
    dY = _sym(rng, 6)
    assert np.allclose(grad.dproj_block(P, dY), dY, rtol=0, atol=1e-13)
    assert np.allclose(grad.dproj_block(-P, dY), 0.0, rtol=0, atol=1e-13)
    a, c = 3.0, 1.0
    Y = np.diag([a, -c])
    dY = np.array([[0.7, 0.4], [0.4, -0.2]])
    want = np.array([[0.7, 0.4 * a / (a + c)], [0.4 * a / (a + c), 0.0]])
    assert np.allclose(grad.dproj_block(Y, dY), want, rtol=0, atol=1e-15)


def test_dproj_block_is_self_adjoint_and_a_contraction():
    """DPi at Y is symmetric in the trace inner product with eigenvalues in
    [0, 1] (the projection is firmly nonexpansive)."""
    rng = np.random.default_rng(8)
    K = 7
    Y = _sym(rng, K)
    A, B = _sym(rng, K), _sym(rng, K)
    lhs = np.sum(grad.dproj_block(Y, A) * B)
    rhs = np.sum(A * grad.dproj_block(Y, B))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))
    nA = np.sum(A * A)
    q = np.sum(A * grad.dproj_block(Y, A))
    assert -1e-13 <= q <= nA * (1 + 1e-13)


def test_adjoint_solution_route_does_not_change_the_gradient(monkeypatch):
    """The dense adjoint takes the minimum-norm least-squares solution of its
    singular system; when the divide-and-conquer SVD does not converge it
    falls back to the QR-iteration SVD, which gives the same solution (a
    basic solution instead differs along the near-null directions by ~1e-5
    of the gradient on this instance)."""
    inst = configs.small_block_arrow(14, n=12, block=4, arrow=2, m=5)
    prob = hsde.build_problem(inst)
    w = np.random.default_rng(5).standard_normal(prob.nE)
    _, res = grad.objective_weight_loss(inst, w, eps_tol=1e-11)
    gc, gb = grad.adjoint_gradient_dense(res, w)

    def refuse(*args, **kw):
        raise np.linalg.LinAlgError("SVD did not converge")

    monkeypatch.setattr(np.linalg, "lstsq", refuse)
    gc2, gb2 = grad.adjoint_gradient_dense(res, w)
    assert np.linalg.norm(gc2 - gc) <= 1e-8 * np.linalg.norm(gc)
    assert np.linalg.norm(gb2 - gb) <= 1e-8 * max(np.linalg.norm(gb), 1e-12)
