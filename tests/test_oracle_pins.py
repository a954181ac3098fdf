"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, the plain definition of step 1 (dense LU of the assembled I + Q of
eq. (HomogeneousEmbedding)), the paper's literal n^2 coordinates, Moreau's
decomposition for the projection, Grone/Agler (Theorems 1-2) at solutions,
and validity of infeasibility certificates.
"""
import math

import numpy as np
import pytest

from oracle import hsde, literal
from sdpgen import chordal, configs


def _inst(n, m, C, A, b, cliques, parent=None):
    if parent is None:
        parent = np.full(len(cliques), -1)
    return configs.SDPInstance(n, m, C, A, np.asarray(b, float),
                               [np.asarray(c) for c in cliques], np.asarray(parent))


# ----------------------------------------------------------------------------
# projection onto the PSD cone (Step2)
# ----------------------------------------------------------------------------

def test_projection_2x2_closed_form():
    rng = np.random.default_rng(7)
    for _ in range(200):
        a, b, c = rng.standard_normal(3) * rng.choice([1e-3, 1.0, 1e3])
        disc = math.sqrt(((a - c) / 2) ** 2 + b * b)
        lp, lm = (a + c) / 2 + disc, (a + c) / 2 - disc
        if lm >= 0:
            want = np.array([[a, b], [b, c]])
        elif lp <= 0:
            want = np.zeros((2, 2))
        else:
            q = np.array([b, lp - a]) if abs(lp - a) > abs(lp - c) else np.array([lp - c, b])
            q = q / np.linalg.norm(q)
            want = lp * np.outer(q, q)
        got = hsde.proj_psd(np.array([[a, b], [b, c]]))
        scale = max(1.0, abs(a) + abs(b) + abs(c))
        assert np.allclose(got, want, atol=1e-12 * scale, rtol=0)
        # the packed path: svec with sqrt2 off-diagonal, projected, unpacked
        vec = np.array([a, math.sqrt(2) * b, c])
        out = hsde.proj_psd_packed(vec, [2], np.array([0]))
        assert np.allclose(hsde.smat_blocks(out, 2), want, atol=1e-12 * scale, rtol=0)


@pytest.mark.parametrize("K", [1, 2, 3, 7, 14, 40])
def test_projection_moreau(K):
    rng = np.random.default_rng(K)
    for _ in range(5):
        G = rng.standard_normal((K, K))
        Y = (G + G.T) / 2
        P = hsde.proj_psd(Y)
        N = P - Y                                  # = Pi_+(-Y)
        tol = 1e-12 * np.linalg.norm(Y)
        assert np.linalg.eigvalsh(P).min() >= -tol
        assert np.linalg.eigvalsh(N).min() >= -tol
        assert abs(np.sum(P * N)) <= tol * np.linalg.norm(Y)
        assert np.allclose(hsde.proj_psd(P), P, atol=tol)
        # nearest-point property against random PSD candidates
        d0 = np.linalg.norm(Y - P)
        for _ in range(10):
            B = rng.standard_normal((K, K))
            cand = B @ B.T
            assert np.linalg.norm(Y - cand) >= d0 - tol


# ----------------------------------------------------------------------------
# step 1 against its plain definition; cached quantities
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["tiny", "block_arrow_n50"])
def test_step1_matches_dense_lu(which):
    inst = configs.small_block_arrow(1) if which == "tiny" else configs.block_arrow_n50()
    prob = hsde.build_problem(inst)
    cache = hsde.AffineCache(prob)
    IQ, off = literal.dense_affine_matrix_svec(prob)
    rng = np.random.default_rng(3)
    for _ in range(3):
        w = rng.standard_normal(off[-1])
        want = np.linalg.solve(IQ, w)
        parts = [w[off[i]:off[i + 1]] for i in range(4)] + [float(w[-1])]
        got = cache.solve(parts)
        got = np.concatenate([np.atleast_1d(g) for g in got])
        assert np.linalg.norm(got - want) <= 1e-11 * np.linalg.norm(want)
    # matrix-free check of (I + Q) u_hat = omega along iterates
    u, vt = hsde.initial_point(prob)
    sizes = hsde.clique_sizes(prob)
    for _ in range(5):
        u, vt = hsde.iterate(prob, cache, u, vt, sizes)
    om = [a + b for a, b in zip(u, vt)]
    uh = cache.solve(om)
    Qu = hsde.apply_Q(prob, uh)
    lhs = np.concatenate([np.atleast_1d(a + b) for a, b in zip(uh, Qu)])
    rhs = np.concatenate([np.atleast_1d(a) for a in om])
    # Backward error.  The Sherman-Morrison route forms t = omega_12 -
    # omega_3 zeta and then cancels p against gamma M^{-1} zeta, so rounding
    # scales with ||I+Q|| (||omega|| + omega_3 ||zeta||), not with ||omega||.
    nrm_iq = np.linalg.norm(IQ, 2)
    nz = np.sqrt(sum(float(z @ z) for z in cache.zeta))
    scale = nrm_iq * (np.linalg.norm(rhs) + abs(om[4]) * nz)
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * scale


def test_Q_is_skew_and_cache_invariants():
    prob = hsde.build_problem(configs.block_arrow_n50())
    IQ, off = literal.dense_affine_matrix_svec(prob)
    Q = IQ - np.eye(off[-1])
    assert np.abs(Q + Q.T).max() == 0.0
    rng = np.random.default_rng(0)
    u = [rng.standard_normal(off[i + 1] - off[i]) for i in range(4)] + [0.7]
    Qu = hsde.apply_Q(prob, u)
    uQu = sum(float(np.dot(np.atleast_1d(a), np.atleast_1d(b))) for a, b in zip(u, Qu))
    assert abs(uQu) < 1e-10
    cache = hsde.AffineCache(prob)
    # zeta^T M^{-1} zeta = ||M^{-1} zeta||^2 because M - I is skew
    nz = sum(float(a @ a) for a in cache.zt)
    assert abs(cache.den - (1.0 + nz)) <= 1e-12 * cache.den
    assert np.linalg.eigvalsh(cache.K).min() >= 1.0 - 1e-12


# ----------------------------------------------------------------------------
# svec coordinates against the paper's literal vec coordinates
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_literal_vec_vs_svec_iterates(seed):
    inst = configs.small_block_arrow(seed, n=6, block=2, arrow=1, m=3)
    prob = hsde.build_problem(inst)
    res = hsde.solve(prob, max_iter=40, record=40, stop=False)
    L = literal.Literal(inst)
    u, vt = L.initial()
    for k in range(40):
        u, vt = L.iterate(u, vt)
        a = hsde.state_vector(L.to_svec(u, prob.erow, prob.ecol), L.to_svec(vt, prob.erow, prob.ecol))
        b = hsde.state_vector(*res.history[k])
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


def test_residuals_against_literal_formulas():
    inst = configs.small_block_arrow(2, n=6, block=2, arrow=1, m=3)
    prob = hsde.build_problem(inst)
    res = hsde.solve(prob, max_iter=25, record=25, stop=False)
    L = literal.Literal(inst)
    u, vt = L.initial()
    for _ in range(25):
        u, vt = L.iterate(u, vt)
    x, s, y, v, tau = L.split(u)
    z, kap = L.split(vt)[1], L.split(vt)[4]
    tau = float(tau[0])
    pri = np.concatenate([L.A @ x - tau * L.b, L.H @ x - s])
    dua = np.concatenate([L.A.T @ y + L.H.T @ v - tau * L.c, v - z])
    r = hsde.residuals(prob, res.u, res.vt)
    assert math.isclose(r["eps_p"], np.linalg.norm(pri) / (tau * (1 + np.linalg.norm(L.b))), rel_tol=1e-9)
    assert math.isclose(r["eps_d"], np.linalg.norm(dua) / (tau * (1 + np.linalg.norm(L.c))), rel_tol=1e-9)
    cx, by = float(L.c @ x), float(L.b @ y)
    assert math.isclose(r["eps_g"], abs(cx - by) / (tau + abs(cx) + abs(by)), rel_tol=1e-9)


# ----------------------------------------------------------------------------
# step 3 and Moreau invariants along iterates
# ----------------------------------------------------------------------------

def test_iterate_invariants():
    prob = hsde.build_problem(configs.block_arrow_n50())
    res = hsde.solve(prob, max_iter=60, record=60, stop=False)
    sizes = hsde.clique_sizes(prob)
    for u, vt in res.history:
        h, z, r, w, kap = vt
        assert not np.any(h) and not np.any(r) and not np.any(w)
        assert u[4] * kap == 0.0 and u[4] >= 0 and kap >= 0
        for k, K in enumerate(sizes):
            sl = slice(prob.slot_off[k], prob.slot_off[k + 1])
            S = hsde.smat_blocks(u[1][sl], K)
            Z = hsde.smat_blocks(z[sl], K)
            sc = 1e-12 * (1 + np.linalg.norm(S) + np.linalg.norm(Z))
            assert np.linalg.eigvalsh(S).min() >= -sc
            assert np.linalg.eigvalsh(Z).min() >= -sc
            assert abs(np.sum(S * Z)) <= sc * (1 + np.linalg.norm(S) + np.linalg.norm(Z))


# ----------------------------------------------------------------------------
# whole solves with closed-form optima
# ----------------------------------------------------------------------------

def _trace_problem(seed, n=12, block=3, arrow=2):
    rng = np.random.default_rng(seed)
    cliques, parent = configs.block_arrow_cliques(n, block, arrow)
    er, ec = configs.pattern_entries(cliques)
    vals = rng.standard_normal(len(er))
    C = (er.astype(np.int32), ec.astype(np.int32), vals)
    A = (np.zeros(n, np.int32), np.arange(n, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    inst = _inst(n, 1, C, A, [1.0], cliques, parent)
    Cd = np.zeros((n, n))
    Cd[er, ec] = vals
    Cd[ec, er] = vals
    return inst, Cd


@pytest.mark.parametrize("seed", [0, 1])
def test_trace_constrained_min_is_lambda_min(seed):
    inst, Cd = _trace_problem(seed)
    res = hsde.solve(inst, eps_tol=1e-9, max_iter=40000)
    assert res.status == hsde.SOLVED
    rec = hsde.recover(res)
    lam = np.linalg.eigvalsh(Cd).min()
    assert abs(rec["obj_p"] - lam) <= 1e-6 * max(1, abs(lam))
    assert abs(rec["obj_d"] - lam) <= 1e-6 * max(1, abs(lam))


def _maxcut_value(n, edges):
    inst = configs.maxcut_from_edges(n, edges)
    res = hsde.solve(inst, eps_tol=1e-9, max_iter=40000)
    assert res.status == hsde.SOLVED
    return hsde.recover(res)["obj_p"], res


@pytest.mark.parametrize("n", [5, 7])
def test_maxcut_odd_cycle(n):
    val, _ = _maxcut_value(n, [(i, (i + 1) % n) for i in range(n)])
    want = -2 * n * (1 + math.cos(math.pi / n))
    assert abs(val - want) <= 1e-6 * abs(want)


def test_maxcut_even_cycle_and_complete_graph():
    val, _ = _maxcut_value(8, [(i, (i + 1) % 8) for i in range(8)])
    assert abs(val + 32) <= 1e-6 * 32
    n = 5
    val, _ = _maxcut_value(n, [(i, j) for i in range(n) for j in range(i)])
    assert abs(val + n * n) <= 1e-6 * n * n


@pytest.mark.parametrize("rows,cols", [(4, 6), (3, 4), (3, 5)])
def test_maxcut_periodic_grid(rows, cols):
    """The periodic grid (torus C_rows x C_cols, the generator of the random
    max-cut's grid companion at a small size) is vertex-transitive, so its max-cut SDP value
    is the eigenvalue bound n lambda_max(L) / 4 (Delorme & Poljak 1993), with
    lambda_max(L) = lambda_max(L(C_rows)) + lambda_max(L(C_cols)) for the
    Cartesian product and lambda_max(L(C_k)) = 2 - 2 cos(2 pi floor(k/2) / k).
    min <-L, X> is -4 times that value: -n lambda_max(L).  With both sides
    even the graph is bipartite and the value is -4 |E|."""
    inst = configs.grid_maxcut(0, rows=rows, cols=cols)
    res = hsde.solve(inst, eps_tol=1e-9, max_iter=40000)
    assert res.status == hsde.SOLVED
    val = hsde.recover(res)["obj_p"]
    lam = sum(2 - 2 * math.cos(2 * math.pi * (k // 2) / k) for k in (rows, cols))
    want = -rows * cols * lam
    if rows % 2 == 0 and cols % 2 == 0:
        assert abs(want + 4 * len(inst.meta["edges"])) <= 1e-12
    assert abs(val - want) <= 1e-6 * abs(want)


def test_decomposed_equals_undecomposed():
    inst = configs.small_block_arrow(3, n=12, block=3, arrow=2, m=4)
    whole = configs.SDPInstance(inst.n, inst.m, inst.C, inst.A, inst.b,
                                [np.arange(inst.n)], np.array([-1]))
    r1 = hsde.solve(inst, eps_tol=1e-9, max_iter=40000)
    r2 = hsde.solve(whole, eps_tol=1e-9, max_iter=40000)
    assert r1.status == r2.status == hsde.SOLVED
    o1, o2 = hsde.recover(r1)["obj_p"], hsde.recover(r2)["obj_p"]
    assert abs(o1 - o2) <= 1e-6 * max(1, abs(o2))


def test_grone_and_agler_at_solution():
    inst = configs.block_arrow_n50()
    res = hsde.solve(inst, eps_tol=1e-8, max_iter=40000)
    assert res.status == hsde.SOLVED
    prob = res.prob
    rec = hsde.recover(res)
    X = hsde.svec_to_dense(prob, rec["x"])
    sizes = hsde.clique_sizes(prob)
    nX = np.linalg.norm(X)
    # Grone (Theorem 1): every clique block of the partial X is PSD
    for c in prob.cliques:
        assert np.linalg.eigvalsh(X[np.ix_(c, c)]).min() >= -1e-6 * nX
    # Agler (Theorem 2): Z = sum_k E_k^T Z_k E_k with Z_k PSD, and
    # C - sum_i y_i A_i - Z = 0 up to the tolerance
    z = res.vt[1] / res.u[4]
    for k, K in enumerate(sizes):
        Zk = hsde.smat_blocks(z[prob.slot_off[k]:prob.slot_off[k + 1]], K)
        assert np.linalg.eigvalsh(Zk).min() >= -1e-12 * (1 + np.linalg.norm(Zk))
    Z = hsde.svec_to_dense(prob, rec["Zvec"])
    Cd = literal.dense_sym(inst.n, inst.C)
    con, r, c, v = inst.A
    S = np.zeros_like(Cd)
    for i, j, val, q in zip(r, c, v, con):
        S[i, j] += rec["y"][q] * val
        if i != j:
            S[j, i] += rec["y"][q] * val
    assert np.linalg.norm(Cd - S - Z) <= 1e-5 * (1 + np.linalg.norm(Cd))
    # the returned X is Grone-completable: a PSD matrix agrees with it on E'
    Xc = _psd_completion(X, prob)
    assert np.linalg.eigvalsh(Xc).min() >= -1e-6 * nX


def _psd_completion(X, prob):
    """Fill the off-pattern entries by the clique-tree (max-determinant)
    rule X_{ab} = X_{aS} X_{SS}^{-1} X_{Sb} for block-arrow cliques: blocks
    are conditionally independent given the arrow separator."""
    Xc = X.copy()
    cl = prob.cliques
    sep = np.array(sorted(set(cl[0].tolist()).intersection(*[set(c.tolist()) for c in cl[1:]])))
    Sinv = np.linalg.pinv(X[np.ix_(sep, sep)])
    for i in range(len(cl)):
        for j in range(len(cl)):
            if i == j:
                continue
            a = np.setdiff1d(cl[i], sep)
            bb = np.setdiff1d(cl[j], sep)
            Xc[np.ix_(a, bb)] = X[np.ix_(a, sep)] @ Sinv @ X[np.ix_(sep, bb)]
    return Xc


# ----------------------------------------------------------------------------
# infeasibility certificates (Table 4's role)
# ----------------------------------------------------------------------------

def test_primal_infeasible_certificate():
    # X_00 = -1 with X PSD is impossible
    inst = _inst(2, 1, (np.array([0, 1], np.int32), np.array([0, 1], np.int32), np.array([1.0, 1.0])),
                 (np.array([0], np.int32), np.array([0], np.int32), np.array([0], np.int32), np.array([1.0])),
                 [-1.0], [[0, 1]])
    res = hsde.solve(inst, max_iter=5000)
    assert res.status == hsde.PRIMAL_INFEASIBLE
    prob = res.prob
    rec = hsde.recover(res)
    y, v = rec["y_cert"], rec["v_cert"]
    assert math.isclose(float(prob.b @ y), 1.0, rel_tol=1e-12)
    assert np.linalg.norm(prob.A.T @ y + prob.H.T @ v) <= 1e-3
    # -sum_i y_i A_i is PSD: the Farkas certificate of the primal
    M = -y[0] * np.array([[1.0, 0.0], [0.0, 0.0]])
    assert np.linalg.eigvalsh(M).min() >= -1e-3


def test_dual_infeasible_certificate():
    # min <-I, X> with X_10 = 0 is unbounded below
    inst = _inst(2, 1, (np.array([0, 1], np.int32), np.array([0, 1], np.int32), np.array([-1.0, -1.0])),
                 (np.array([0], np.int32), np.array([1], np.int32), np.array([0], np.int32), np.array([1.0])),
                 [0.0], [[0, 1]])
    res = hsde.solve(inst, max_iter=5000)
    assert res.status == hsde.DUAL_INFEASIBLE
    prob = res.prob
    rec = hsde.recover(res)
    x = rec["x_cert"]
    assert math.isclose(float(prob.c @ x), -1.0, rel_tol=1e-12)
    assert np.linalg.norm(prob.A @ x) <= 1e-3
    X = hsde.svec_to_dense(prob, x)
    assert np.linalg.eigvalsh(X).min() >= -1e-3


# ----------------------------------------------------------------------------
# planted mistakes: each must break at least one pin above
# ----------------------------------------------------------------------------

def test_planted_sign_error_in_step1_is_caught(monkeypatch):
    prob = hsde.build_problem(configs.small_block_arrow(1))
    cache = hsde.AffineCache(prob)
    IQ, off = literal.dense_affine_matrix_svec(prob)
    w = np.random.default_rng(0).standard_normal(off[-1])
    want = np.linalg.solve(IQ, w)
    orig = cache.inner_solve

    def wrong(t):
        p = orig(t)
        p[3] = -p[3]          # flip the v-block sign
        return p

    monkeypatch.setattr(cache, "inner_solve", wrong)
    parts = [w[off[i]:off[i + 1]] for i in range(4)] + [float(w[-1])]
    got = np.concatenate([np.atleast_1d(g) for g in cache.solve(parts)])
    assert np.linalg.norm(got - want) > 1e-3 * np.linalg.norm(want)


def test_planted_projection_error_is_caught():
    Y = np.diag([2.0, -1.0])
    bad = np.maximum(Y, 0) - 0.0 * Y
    good = hsde.proj_psd(Y)
    assert np.allclose(good, bad)
    # a projection that keeps |lambda| instead of max(lambda, 0) fails Moreau
    lam, V = np.linalg.eigh(Y)
    wrong = (V * np.abs(lam)) @ V.T
    N = wrong - Y
    assert abs(np.sum(wrong * N)) > 1e-3
