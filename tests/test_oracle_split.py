"""Pins of the primal-only and dual-only ADMM oracle (oracle/split.py).

Against what the mathematics fixes, not against the oracle itself:
  * step 1 of each method against a dense solve of its KKT system (the plain
    definition of the equality-constrained least-squares step);
  * Moreau's decomposition after steps 2-3: the multiplier is in the cone
    (primal method) or its negative is (dual method) and complementary to
    the projected block;
  * closed-form optima: the trace-constrained minimum is lambda_min(C), the
    max-cut SDP of an odd cycle is -2n(1 + cos(pi/n)) and of the complete
    graph -n^2;
  * the solution of the self-dual oracle (a different algorithm) on the
    theta1-sized block-arrow problem;
  * a planted sign error in step 1 fails the first pin.
"""
import math

import numpy as np
import pytest

from oracle import hsde, split
from sdpgen import configs


def _rand_state(prob, rng):
    return rng.standard_normal(prob.ns), rng.standard_normal(prob.ns)


def _dense_kkt_primal(prob, rho, s, lam):
    """[[rho D, -A^T], [A, 0]] (x, y) = (H^T(rho s + lam) - c, b)."""
    nE, m = prob.nE, prob.m
    A = prob.A.toarray()
    M = np.zeros((nE + m, nE + m))
    M[:nE, :nE] = rho * np.diag(prob.D)
    M[:nE, nE:] = -A.T
    M[nE:, :nE] = A
    rhs = np.concatenate([prob.H.T @ (rho * s + lam) - prob.c, prob.b])
    sol = np.linalg.solve(M, rhs)
    return sol[:nE], sol[nE:]


def _dense_kkt_dual(prob, rho, z, lam):
    """Stationarity of -b^T y + rho/2 ||v - z + lam/rho||^2 + x^T(A^T y + H^T v - c)
    in (y, v, x), assembled densely: unknowns (y, v, x)."""
    nE, m, ns = prob.nE, prob.m, prob.ns
    A = prob.A.toarray()
    H = prob.H.toarray()
    N = m + ns + nE
    M = np.zeros((N, N))
    rhs = np.zeros(N)
    # d/dy: -b + A x = 0
    M[:m, m + ns:] = A
    rhs[:m] = prob.b
    # d/dv: rho (v - z + lam/rho) + H x = 0
    M[m:m + ns, m:m + ns] = rho * np.eye(ns)
    M[m:m + ns, m + ns:] = H
    rhs[m:m + ns] = rho * z - lam
    # equality: A^T y + H^T v = c
    M[m + ns:, :m] = A.T
    M[m + ns:, m:m + ns] = H.T
    rhs[m + ns:] = prob.c
    sol = np.linalg.solve(M, rhs)
    return sol[m + ns:], sol[:m], sol[m:m + ns]


@pytest.mark.parametrize("rho", [1.0, 0.3])
def test_step1_matches_dense_kkt(rho):
    inst = configs.small_block_arrow(3, n=14, block=4, arrow=2, m=5)
    prob = hsde.build_problem(inst)
    cache = split.SplitCache(prob, rho)
    rng = np.random.default_rng(1)
    s, lam = _rand_state(prob, rng)
    x, y = split.primal_step1(prob, cache, s, lam)
    xw, yw = _dense_kkt_primal(prob, rho, s, lam)
    assert np.linalg.norm(x - xw) <= 1e-12 * np.linalg.norm(xw)
    assert np.linalg.norm(y - yw) <= 1e-12 * np.linalg.norm(yw)
    assert np.linalg.norm(prob.A @ x - prob.b) <= 1e-12 * np.linalg.norm(prob.b)
    x, y, v = split.dual_step1(prob, cache, s, lam)
    xw, yw, vw = _dense_kkt_dual(prob, rho, s, lam)
    assert np.linalg.norm(x - xw) <= 1e-11 * np.linalg.norm(xw)
    assert np.linalg.norm(y - yw) <= 1e-11 * np.linalg.norm(yw)
    assert np.linalg.norm(v - vw) <= 1e-11 * np.linalg.norm(vw)
    assert np.linalg.norm(prob.A.T @ y + prob.H.T @ v - prob.c) <= 1e-11 * np.linalg.norm(prob.c)


@pytest.mark.parametrize("method", [split.PRIMAL, split.DUAL])
def test_iterate_invariants(method):
    inst = configs.block_arrow_n50()
    prob = hsde.build_problem(inst)
    cache = split.SplitCache(prob)
    sizes = hsde.clique_sizes(prob)
    st = split.initial_state(prob)
    sign = 1.0 if method == split.PRIMAL else -1.0
    for _ in range(15):
        st, _ = split.iterate(prob, cache, st, method, sizes)
        for k, K in enumerate(sizes):
            sl = slice(prob.slot_off[k], prob.slot_off[k + 1])
            L = hsde.smat_blocks(sign * st.lam[sl], int(K))
            S = hsde.smat_blocks(st.s[sl], int(K))
            scale = max(1.0, np.linalg.norm(L), np.linalg.norm(S))
            assert np.linalg.eigvalsh(L).min() >= -1e-12 * scale
            assert np.linalg.eigvalsh(S).min() >= -1e-12 * scale
            assert abs(float(st.lam[sl] @ st.s[sl])) <= 1e-11 * scale * scale
        if method == split.PRIMAL:
            assert np.linalg.norm(prob.A @ st.x - prob.b) <= 1e-11 * np.linalg.norm(prob.b)
        else:
            assert np.linalg.norm(prob.A @ st.x - prob.b) <= 1e-10 * np.linalg.norm(prob.b)


def _trace_problem(seed, n=12, block=3, arrow=2):
    rng = np.random.default_rng(seed)
    cliques, parent = configs.block_arrow_cliques(n, block, arrow)
    er, ec = configs.pattern_entries(cliques)
    vals = rng.standard_normal(len(er))
    C = (er.astype(np.int32), ec.astype(np.int32), vals)
    A = (np.zeros(n, np.int32), np.arange(n, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    inst = configs.SDPInstance(n, 1, C, A, np.array([1.0]), [np.asarray(c) for c in cliques], np.asarray(parent))
    Cd = np.zeros((n, n))
    Cd[er, ec] = vals
    Cd[ec, er] = vals
    return inst, Cd


@pytest.mark.parametrize("method", [split.PRIMAL, split.DUAL])
def test_trace_constrained_min_is_lambda_min(method):
    inst, Cd = _trace_problem(0)
    res = split.solve(inst, method, eps_tol=1e-10, max_iter=100000)
    assert res.status == hsde.SOLVED
    rec = split.recover(res, method)
    lam = np.linalg.eigvalsh(Cd).min()
    assert abs(rec["obj_p"] - lam) <= 1e-6 * max(1, abs(lam))
    assert abs(rec["obj_d"] - lam) <= 1e-6 * max(1, abs(lam))


@pytest.mark.parametrize("method", [split.PRIMAL, split.DUAL])
def test_maxcut_closed_forms(method):
    n = 7
    inst = configs.maxcut_from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    res = split.solve(inst, method, eps_tol=1e-10, max_iter=100000)
    assert res.status == hsde.SOLVED
    want = -2 * n * (1 + math.cos(math.pi / n))
    obj = split.recover(res, method)
    assert abs(obj["obj_p"] - want) <= 1e-6 * abs(want)
    assert abs(obj["obj_d"] - want) <= 1e-6 * abs(want)
    n = 5
    inst = configs.maxcut_from_edges(n, [(i, j) for i in range(n) for j in range(i)])
    res = split.solve(inst, method, eps_tol=1e-10, max_iter=100000)
    assert res.status == hsde.SOLVED
    assert abs(split.recover(res, method)["obj_p"] + n * n) <= 1e-6 * n * n


@pytest.mark.parametrize("method", [split.PRIMAL, split.DUAL])
def test_same_solution_as_the_self_dual_method(method):
    inst = configs.block_arrow_n50()
    ref = hsde.recover(hsde.solve(inst, eps_tol=1e-10, max_iter=100000))
    res = split.solve(inst, method, eps_tol=1e-10, max_iter=100000)
    assert res.status == hsde.SOLVED
    rec = split.recover(res, method)
    assert abs(rec["obj_p"] - ref["obj_p"]) <= 1e-6 * abs(ref["obj_p"])
    assert abs(rec["obj_d"] - ref["obj_d"]) <= 1e-6 * abs(ref["obj_d"])
    # y and Z = sum_k E_k^T Z_k E_k are unique here (strictly feasible data)
    assert np.linalg.norm(rec["y"] - ref["y"]) <= 1e-5 * np.linalg.norm(ref["y"])
    assert np.linalg.norm(rec["Zvec"] - ref["Zvec"]) <= 1e-5 * np.linalg.norm(ref["Zvec"])


def test_planted_sign_error_in_step1_is_caught(monkeypatch):
    inst = configs.small_block_arrow(3, n=14, block=4, arrow=2, m=5)
    prob = hsde.build_problem(inst)
    cache = split.SplitCache(prob)
    rng = np.random.default_rng(1)
    s, lam = _rand_state(prob, rng)
    real = split.primal_step1

    def planted(prob, cache, s, lam):
        return real(prob, cache, s, -lam)
    x, _ = planted(prob, cache, s, lam)
    xw, _ = _dense_kkt_primal(prob, 1.0, s, lam)
    assert np.linalg.norm(x - xw) > 1e-3 * np.linalg.norm(xw)
