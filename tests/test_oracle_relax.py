"""Pins of the oracle's over-relaxed iteration (alpha != 1).

The paper applies the ADMM of O'Donoghue et al. 2016 (Section 4.1), whose
relaxed form replaces u_hat by alpha u_hat + (1 - alpha) u in steps 2 and 3.
Writing t = u - v~ (so that u = Pi_K(t) and v~ = u - t after every step),
the unrelaxed steps are t+ = T(t) for the Douglas-Rachford map
T(t) = t + (I + Q)^{-1}(2 Pi_K(t) - t) - Pi_K(t), and the relaxed steps are
its Krasnosel'skii-Mann average t+ = (1 - alpha) t + alpha T(t).  The tests
check the relaxed oracle against that identity (evaluated with the alpha = 1
oracle, itself pinned in test_oracle_pins.py), against u+ = Pi_K(t+), and
against closed-form optima and certificates, which a relaxed iteration must
reach unchanged (relaxation moves no fixed point).
"""
import math

import numpy as np
import pytest

from oracle import hsde
from sdpgen import configs

from test_oracle_pins import _inst, _trace_problem


def _state(prob, iters=7):
    res = hsde.solve(prob, max_iter=iters, stop=False)
    return res.u, res.vt


def _t_of(u, vt):
    return [a - b for a, b in zip(u, vt)]


def _flat(parts):
    return np.concatenate([np.atleast_1d(np.asarray(p, dtype=float)) for p in parts])


def _averaged_map_error(prob, iterate, alpha):
    """max relative deviation of one relaxed step from (1 - alpha) t + alpha T(t)."""
    cache = hsde.AffineCache(prob)
    sizes = hsde.clique_sizes(prob)
    u, vt = _state(prob)
    t0 = _flat(_t_of(u, vt))
    u1, v1 = hsde.iterate(prob, cache, u, vt, sizes, 1.0)
    Tt = _flat(_t_of(u1, v1))
    ua, va = iterate(prob, cache, u, vt, sizes, alpha)
    ta = _flat(_t_of(ua, va))
    want = (1.0 - alpha) * t0 + alpha * Tt
    err_t = np.linalg.norm(ta - want) / np.linalg.norm(want)
    # u+ = Pi_K(t+): free parts equal, PSD blocks projected, tau = max(0, .)
    tl = _t_of(ua, va)
    proj = [tl[0], hsde.proj_psd_packed(tl[1], sizes, prob.slot_off[:-1]), tl[2], tl[3], max(0.0, tl[4])]
    err_u = np.linalg.norm(_flat(ua) - _flat(proj)) / np.linalg.norm(_flat(ua))
    zero_parts = max(np.abs(va[0]).max(), np.abs(va[2]).max(), np.abs(va[3]).max())
    return err_t, err_u, zero_parts


@pytest.mark.parametrize("alpha", [0.5, 1.5, 1.8])
@pytest.mark.parametrize("which", ["block_arrow_n50", "odd"])
def test_relaxed_step_is_averaged_dr_map(alpha, which):
    inst = configs.block_arrow_n50() if which == "block_arrow_n50" else configs.small_block_arrow(5, n=23, block=4, arrow=3, m=6)
    prob = hsde.build_problem(inst)
    err_t, err_u, zero_parts = _averaged_map_error(prob, hsde.iterate, alpha)
    assert err_t <= 1e-12
    assert err_u <= 1e-12
    assert zero_parts == 0.0


@pytest.mark.parametrize("seed", [0])
def test_relaxed_trace_constrained_min_is_lambda_min(seed):
    inst, Cd = _trace_problem(seed)
    lam = np.linalg.eigvalsh(Cd).min()
    res = hsde.solve(inst, eps_tol=1e-9, max_iter=40000, alpha=1.7)
    assert res.status == hsde.SOLVED
    rec = hsde.recover(res)
    assert abs(rec["obj_p"] - lam) <= 1e-6 * max(1, abs(lam))
    assert abs(rec["obj_d"] - lam) <= 1e-6 * max(1, abs(lam))


def test_relaxed_maxcut_odd_cycle():
    n = 5
    inst = configs.maxcut_from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    res = hsde.solve(inst, eps_tol=1e-9, max_iter=40000, alpha=1.7)
    assert res.status == hsde.SOLVED
    want = -2 * n * (1 + math.cos(math.pi / n))
    assert abs(hsde.recover(res)["obj_p"] - want) <= 1e-6 * abs(want)


def test_relaxed_certificates():
    # X_00 = -1 with X PSD is impossible; min <-I, X> with X_10 = 0 is unbounded
    pinf = _inst(2, 1, (np.array([0, 1], np.int32), np.array([0, 1], np.int32), np.array([1.0, 1.0])),
                 (np.array([0], np.int32), np.array([0], np.int32), np.array([0], np.int32), np.array([1.0])),
                 [-1.0], [[0, 1]])
    res = hsde.solve(pinf, max_iter=5000, alpha=1.7)
    assert res.status == hsde.PRIMAL_INFEASIBLE
    rec = hsde.recover(res)
    prob = res.prob
    assert math.isclose(float(prob.b @ rec["y_cert"]), 1.0, rel_tol=1e-12)
    assert np.linalg.norm(prob.A.T @ rec["y_cert"] + prob.H.T @ rec["v_cert"]) <= 1e-3
    dinf = _inst(2, 1, (np.array([0, 1], np.int32), np.array([0, 1], np.int32), np.array([-1.0, -1.0])),
                 (np.array([0], np.int32), np.array([1], np.int32), np.array([0], np.int32), np.array([1.0])),
                 [0.0], [[0, 1]])
    res = hsde.solve(dinf, max_iter=5000, alpha=1.7)
    assert res.status == hsde.DUAL_INFEASIBLE
    rec = hsde.recover(res)
    prob = res.prob
    assert math.isclose(float(prob.c @ rec["x_cert"]), -1.0, rel_tol=1e-12)
    assert np.linalg.norm(prob.A @ rec["x_cert"]) <= 1e-3
    assert np.linalg.eigvalsh(hsde.svec_to_dense(prob, rec["x_cert"])).min() >= -1e-3


def test_relaxation_keeps_the_solution_of_block_arrow_n50():
    """Same fixed point: the relaxed and unrelaxed solves agree to the tolerance."""
    inst = configs.block_arrow_n50()
    r1 = hsde.solve(inst, eps_tol=1e-8, max_iter=20000)
    r2 = hsde.solve(inst, eps_tol=1e-8, max_iter=20000, alpha=1.6)
    assert r1.status == r2.status == hsde.SOLVED
    o1, o2 = hsde.recover(r1)["obj_p"], hsde.recover(r2)["obj_p"]
    assert abs(o1 - o2) <= 1e-6 * max(1.0, abs(o1))


# ----------------------------------------------------------------------------
# planted mistakes in the relaxed step: each must break the identity above
# ----------------------------------------------------------------------------

def _planted(kind):
    def iterate(prob, cache, u, vt, sizes, alpha):
        omega = [a + b for a, b in zip(u, vt)]
        uh = cache.solve(omega)
        base = vt if kind == "average_with_v" else u
        ub = [alpha * a + (1.0 - alpha) * b for a, b in zip(uh, base)]
        d = [a - b for a, b in zip(ub, vt)]
        un = [d[0].copy(), hsde.proj_psd_packed(d[1], sizes, prob.slot_off[:-1]), d[2].copy(), d[3].copy(),
              max(0.0, d[4])]
        step3 = uh if kind == "unrelaxed_step3" else ub
        vn = [a - b + c for a, b, c in zip(vt, step3, un)]
        return un, vn
    return iterate


@pytest.mark.parametrize("kind", ["average_with_v", "unrelaxed_step3"])
def test_planted_relaxation_errors_are_caught(kind):
    prob = hsde.build_problem(configs.block_arrow_n50())
    err_t, err_u, zero_parts = _averaged_map_error(prob, _planted(kind), 1.6)
    assert err_t > 1e-6 or err_u > 1e-6 or zero_parts > 1e-6
