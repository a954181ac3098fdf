"""Primal-only and dual-only ADMM on the GPU (settings.method = 1, 2 through
the C ABI) against oracle/split.py on the same seeded inputs.

Bars (FP64 on both sides):
  * iterates k = 1..K in lock step from the zero start: whole state
    (x, s or z, y, lam[, v]) within 1e-10 relative, and every block within
    1e-10 of its own norm plus 1e-14 of the whole state's;
  * whole solves: the oracle's status and stop iteration (status checked
    after every iteration), objectives within 1e-6, X, y, Z within 1e-8;
  * batch instance i == plain instance i to 1e-12.
The large-clique instance sends its 130- and 250-vertex cliques through the
tridiagonal path of the projection, the others through the Jacobi buckets.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import hsde, split  # noqa: E402
from sdpgen import configs  # noqa: E402

METHOD = {split.PRIMAL: 1, split.DUAL: 2}


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


def _blocks(vec, prob, method):
    lens = [prob.nE, prob.ns, prob.m, prob.ns] + ([prob.ns] if method == split.DUAL else [])
    return np.split(vec, np.cumsum(lens)[:-1])


def lockstep(lib, inst, iters, method, rho=1.0, tol=1e-10, floor=1e-14):
    prob = hsde.build_problem(inst)
    cache = split.SplitCache(prob, rho)
    sizes = hsde.clique_sizes(prob)
    st = split.initial_state(prob)
    s = lib.Solver(inst, method=METHOD[method], rho=rho)
    names = ["x", "s", "y", "lam", "v"]
    worst = 0.0
    try:
        for k in range(1, iters + 1):
            st, _ = split.iterate(prob, cache, st, method, sizes)
            s.iterate(1)
            u, vt = s.get_state()
            got = np.concatenate([u, vt])
            want = split.state_vector(prob, st, method)
            nw = np.linalg.norm(want)
            whole = np.linalg.norm(got - want) / nw
            worst = max(worst, whole)
            assert whole <= tol, (k, whole)
            for name, g, w in zip(names, _blocks(got, prob, method), _blocks(want, prob, method)):
                err = np.linalg.norm(g - w)
                assert err <= tol * np.linalg.norm(w) + floor * nw, (k, name, err, np.linalg.norm(w))
    finally:
        s.close()
    _log(f"  worst whole-state rel {worst:.2e}")
    return worst


@pytest.mark.parametrize("method", [split.PRIMAL, split.DUAL])
def test_iterates_block_arrow_n50(lib, method):
    _log(f"{method}: block_arrow_n50, 50 iterations")
    lockstep(lib, configs.block_arrow_n50(), 50, method)


@pytest.mark.parametrize("method", [split.PRIMAL, split.DUAL])
def test_iterates_penalty_and_odd_sizes(lib, method):
    _log(f"{method}: small odd sizes, rho = 0.4, 50 iterations")
    lockstep(lib, configs.small_block_arrow(1, n=23, block=5, arrow=3, m=7), 50, method, rho=0.4)


@pytest.mark.parametrize("method", [split.PRIMAL, split.DUAL])
def test_iterates_large_cliques(lib, method):
    _log(f"{method}: cliques of 130 and 250 vertices, 30 iterations")
    lockstep(lib, configs.small_block_arrow(7, n=500, block=120, arrow=10, m=30, per_row=8), 30, method)
    lockstep(lib, configs.small_block_arrow(8, n=510, block=240, arrow=10, m=12, per_row=8), 15, method)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("method", [split.PRIMAL, split.DUAL])
def test_iterates_uneven_cliques_5000(lib, method):
    _log(f"{method}: uneven cliques n=5000, m=2000, 50 iterations")
    lockstep(lib, configs.uneven_cliques_5000(), 50, method)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("method", [split.PRIMAL, split.DUAL])
def test_iterates_maxcut_random_2000(lib, method):
    _log(f"{method}: max-cut G(2000, 6000), cliques up to 673, 20 iterations")
    lockstep(lib, configs.maxcut_random_2000(), 20, method)


@pytest.mark.parametrize("method", [split.PRIMAL, split.DUAL])
def test_solve_matches_oracle(lib, method):
    inst = configs.block_arrow_n50()
    ref = split.solve(inst, method)
    s = lib.Solver(inst, method=METHOD[method], check_every=1)
    info = s.solve()[0]
    _log(f"{method}: GPU {lib.STATUS_NAMES[info['status']]} at {info['iter']}, "
         f"oracle {hsde.STATUS_NAMES[ref.status]} at {ref.iters}")
    assert info["status"] == ref.status == hsde.SOLVED
    assert info["iter"] == ref.iters
    rec = split.recover(ref, method)
    assert abs(info["obj_p"] - rec["obj_p"]) <= 1e-6 * max(1.0, abs(rec["obj_p"]))
    assert abs(info["obj_d"] - rec["obj_d"]) <= 1e-6 * max(1.0, abs(rec["obj_d"]))
    X, y, Z = s.solution()
    s.close()
    for got, want in ((X, rec["x"]), (y, rec["y"]), (Z, rec["Zvec"])):
        assert np.linalg.norm(got - want) <= 1e-8 * np.linalg.norm(want)


@pytest.mark.parametrize("method", [split.PRIMAL, split.DUAL])
def test_batch_equals_single(lib, method):
    insts = [configs.small_block_arrow(i, n=15 + 3 * i, block=3 + i, arrow=2, m=5 + i) for i in range(4)]
    b = lib.Solver(insts, method=METHOD[method])
    b.iterate(30)
    for i, inst in enumerate(insts):
        s = lib.Solver(inst, method=METHOD[method])
        s.iterate(30)
        u1, v1 = s.get_state()
        u2, v2 = b.get_state(i)
        s.close()
        ref = np.concatenate([u1, v1])
        assert np.linalg.norm(np.concatenate([u2, v2]) - ref) <= 1e-12 * np.linalg.norm(ref)
    b.close()


@pytest.mark.parametrize("method", [split.PRIMAL, split.DUAL])
def test_graph_replay_and_resume(lib, method):
    inst = configs.block_arrow_n50()
    a = lib.Solver(inst, method=METHOD[method])
    a.iterate(30)
    ua, va = a.get_state()
    g = lib.Solver(inst, method=METHOD[method], use_graph=1)
    g.iterate(30)
    ug, vg = g.get_state()
    assert np.array_equal(ua, ug) and np.array_equal(va, vg)
    r = lib.Solver(inst, method=METHOD[method])
    r.iterate(12)
    u, v = r.get_state()
    c = lib.Solver(inst, method=METHOD[method])
    c.set_state(u, v)
    c.iterate(18)
    uc, vc = c.get_state()
    assert np.array_equal(ua, uc) and np.array_equal(va, vc)
    for x in (a, g, r, c):
        x.close()


def test_settings_checks(lib):
    inst = configs.small_block_arrow(0, n=12, block=3, arrow=2, m=4)
    for kw in (dict(method=3), dict(method=1, rho=0.0), dict(method=2, alpha=1.5), dict(method=1, eig_warm=1)):
        with pytest.raises(lib.CDCSError) as e:
            lib.Solver(inst, **kw)
        assert e.value.code == -1
    s = lib.Solver(inst, method=1)
    s.iterate(3)
    with pytest.raises(lib.CDCSError) as e:
        s.certificate()
    assert e.value.code == -8
    s.close()
