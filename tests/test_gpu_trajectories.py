"""Iterate parity over the first 50 iterations on the two large single-SDP
workloads, with a bar on every block of the state as well as on the whole.

The GPU (through the C ABI) and the oracle step side by side from the
initial point, plain (eqs. Step1-Step3) and over-relaxed (alpha = 1.8).
After each iteration:
  * whole state:  ||(u,v~)_gpu - (u,v~)_orc|| <= t ||(u,v~)_orc|| + 1e-12 ||S||
    with t = 1e-10 (3e-10 for the relaxed form: with alpha = 1.8 every step
    extrapolates the step-1 point by 1.8 and the rounding differences that
    its cancellation leaves grow faster) and S the vector of the block
    scales S_b below: the sum of the per-block allowances, so the whole
    state gets the same cancellation allowance as its blocks.  For scale:
    two FP64 oracles that differ only in rounding order (K factorised in
    reversed row order, LAPACK's syevr in place of syevd) drift 3.3e-11
    apart over the 50 iterations of the uneven-clique workload; the GPU
    path (a sparse factor of K in another order, tridiagonal or Jacobi
    eigensolvers) ~1e-10.
  * every block b of u = (x, s, y, v, tau) and v~ = (h, z, r, w, kappa):
        ||b_gpu - b_orc|| <= 1e-10 ||b_orc|| + 1e-12 S_b
    where S_b is the size of the terms the block is the difference of.
    Step 1 forms x+ = p_x - gamma zt_x and y+ = p_y - gamma zt_y (eq.
    MatrixInverseResult, zt = M^-1 zeta): on these workloads |gamma| ~ tau +
    kappa and ||zt_x|| ~ 100, so at iteration 1 of the max-cut x+ (norm
    0.009) is the difference of two vectors of norm 198, and any FP64
    evaluation of it (the oracle's as much as the GPU's) carries ~1e-12
    absolute error, ~1e-10 of its own norm.  So S_x = |gamma| ||zt_x||,
    S_y = |gamma| ||zt_y||, S_s = S_v = S_z = |gamma| ||zt_s|| (they take
    H x+ / 2), S_tau = S_kappa = tau + kappa + |gamma| (den - 1) (u_tau adds
    c^T x+ - b^T y+, whose terms cancel the same way; den - 1 = c^T zt_x -
    b^T zt_y), S_h = S_r = S_w = 0 (exactly zero on both sides), with gamma
    and tau + kappa of the oracle's step (times alpha when relaxed: steps 2-3
    then take alpha u_hat + (1 - alpha) u).  1e-12 S_b is ~5000 units of
    rounding of those terms; any error of the method itself is of the size
    of the block and fails.  The figures logged are the largest
    ||b_gpu - b_orc|| / ||b_orc|| per block (own-norm relative).
The max-cut workload (cliques up to 673 vertices) exercises the two-stage
and blocked tridiagonalisation paths, the uneven-clique one (cliques of 4-96
vertices, sparse factor of K) the Jacobi buckets up to 32 vertices beside the
LDS-tail path (the default routing), and with jacobi_max = 64 the 64-vertex
Jacobi bucket as well.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import hsde  # noqa: E402
from sdpgen import configs  # noqa: E402

BLOCKS = ["x", "s", "y", "v", "tau", "h", "z", "r", "w", "kappa"]


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    from paper_1611_01828_amd import cdcs
    cdcs.load()
    return cdcs


def _blocks(flat, prob):
    nE, ns, m = prob.nE, prob.ns, prob.m
    lens = [nE, ns, m, ns, 1] * 2
    return np.split(flat, np.cumsum(lens)[:-1])


def _cancellation_scales(cache, u, vt):
    """S_b of the step from (u, v~): the Sherman-Morrison term gamma zt_b."""
    omega = [a + b for a, b in zip(u, vt)]
    w3 = omega[4]
    t = [a - w3 * z for a, z in zip(omega[:4], cache.zeta)]
    p = cache.inner_solve(t)
    gamma = abs(cache.dot(cache.zeta, p) / cache.den)
    nz = [float(np.linalg.norm(z)) for z in cache.zt]
    st = w3 + gamma * abs(cache.den - 1.0)
    return {"x": gamma * nz[0], "s": gamma * nz[1], "y": gamma * nz[2], "v": gamma * nz[3], "tau": st,
            "h": 0.0, "z": gamma * nz[1], "r": 0.0, "w": 0.0, "kappa": st}


def lockstep(lib, inst, iters, alpha=1.0, tol=1e-10, eps_c=1e-12, **settings):
    whole_tol = tol if alpha == 1.0 else 3 * tol
    prob = hsde.build_problem(inst)
    cache = hsde.AffineCache(prob)
    sizes = hsde.clique_sizes(prob)
    u, vt = hsde.initial_point(prob)
    s = lib.Solver(inst, alpha=alpha, **settings)
    worst_whole, worst_blk = 0.0, {b: 0.0 for b in BLOCKS}
    try:
        for k in range(1, iters + 1):
            S = {b: max(1.0, alpha) * v for b, v in _cancellation_scales(cache, u, vt).items()}
            u, vt = hsde.iterate(prob, cache, u, vt, sizes, alpha)
            s.iterate(1)
            gu, gv = s.get_state()
            got = np.concatenate([gu, gv])
            want = hsde.state_vector(u, vt)
            nw = np.linalg.norm(want)
            s_norm = float(np.linalg.norm([S[b] for b in BLOCKS]))
            whole = np.linalg.norm(got - want) / nw
            worst_whole = max(worst_whole, whole)
            assert whole * nw <= whole_tol * nw + eps_c * s_norm, (k, whole, s_norm / nw)
            for name, g, w in zip(BLOCKS, _blocks(got, prob), _blocks(want, prob)):
                err = np.linalg.norm(g - w)
                nb = np.linalg.norm(w)
                bar = tol * nb + eps_c * S[name]
                worst_blk[name] = max(worst_blk[name], err / nb if nb > 0 else err)
                assert err <= bar, (k, name, err, nb, S[name])
    finally:
        s.close()
    _log(f"  worst whole-state rel {worst_whole:.2e}; per block " +
         ", ".join(f"{b} {worst_blk[b]:.1e}" for b in BLOCKS))
    return worst_whole, worst_blk


@pytest.mark.timeout(900)
@pytest.mark.parametrize("alpha", [1.0, 1.8])
def test_maxcut_random_2000_50_iterations(lib, alpha):
    _log(f"max-cut G(2000, 6000), cliques up to 673: 50 iterations, alpha={alpha}")
    lockstep(lib, configs.maxcut_random_2000(), 50, alpha)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("alpha,jmax", [(1.0, 0), (1.8, 0), (1.0, 64)])
def test_uneven_cliques_5000_50_iterations(lib, alpha, jmax):
    _log(f"uneven cliques n=5000, m=2000: 50 iterations, alpha={alpha}, jacobi_max={jmax}")
    lockstep(lib, configs.uneven_cliques_5000(), 50, alpha, jacobi_max=jmax)


@pytest.mark.timeout(600)
def test_uneven_twin_50_iterations(lib):
    _log("uneven-clique infeasible twin (m=2002): 50 iterations")
    lockstep(lib, configs.uneven_cliques_5000(twin=True), 50)
