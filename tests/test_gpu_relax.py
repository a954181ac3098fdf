"""Relaxed steps 2-3 (settings alpha != 1) on the GPU against the oracle.

The same bars as the unrelaxed path, against the oracle run with the same
alpha on the same seeded inputs:
  * iterates k = 1..K: ||(u,v)_gpu - (u,v)_oracle|| <= 1e-10 ||(u,v)_oracle||
    (Jacobi cliques, tridiagonal-path cliques, mixed, graph replay);
  * whole solves: same status and stop iteration, objectives within 1e-6;
  * batch instance i == plain instance i to 1e-12; a resumed run (set_state)
    is bitwise equal to an uninterrupted one (nothing is carried between
    iterations beyond (u, v~));
  * alpha outside (0, 2) is rejected at setup.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import hsde  # noqa: E402
from sdpgen import configs  # noqa: E402


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


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _iterate_parity(lib, inst, iters, alpha, tol=1e-10, graph=False):
    res = hsde.solve(inst, max_iter=iters, record=iters, stop=False, alpha=alpha)
    s = lib.Solver(inst, use_graph=int(graph), alpha=alpha)
    worst = 0.0
    for k in range(iters):
        s.iterate(1)
        u, vt = s.get_state()
        r = _rel(np.concatenate([u, vt]), hsde.state_vector(*res.history[k]))
        worst = max(worst, r)
        assert r <= tol, (k + 1, r)
    s.close()
    return worst


@pytest.mark.parametrize("alpha", [0.7, 1.6])
def test_relaxed_iterates_block_arrow_n50(lib, alpha):
    _log(f"relaxed iterates block_arrow_n50 alpha={alpha}")
    w = _iterate_parity(lib, configs.block_arrow_n50(), 50, alpha)
    _log(f"  worst rel {w:.2e}")


def test_relaxed_iterates_graph_replay(lib):
    _log("relaxed iterates block_arrow_n50 (graph replay)")
    _iterate_parity(lib, configs.block_arrow_n50(), 20, 1.6, graph=True)


def test_relaxed_iterates_small_odd_sizes(lib):
    _log("relaxed iterates small")
    inst = configs.small_block_arrow(1, n=23, block=5, arrow=3, m=7)
    w = _iterate_parity(lib, inst, 50, 1.8)
    _log(f"  worst rel {w:.2e}")


def test_relaxed_iterates_large_cliques(lib):
    """Cliques of 130 and 250 vertices: the tridiagonal path's gather and recon."""
    _log("relaxed iterates large cliques")
    inst = configs.small_block_arrow(7, n=500, block=120, arrow=10, m=30, per_row=8)
    w = _iterate_parity(lib, inst, 20, 1.6)
    _log(f"  worst rel {w:.2e}")
    inst = configs.small_block_arrow(8, n=510, block=240, arrow=10, m=12, per_row=8)
    w = _iterate_parity(lib, inst, 10, 1.8)
    _log(f"  worst rel {w:.2e}")


def test_relaxed_iterates_uneven_cliques_5000(lib):
    _log("relaxed iterates uneven_cliques_5000")
    w = _iterate_parity(lib, configs.uneven_cliques_5000(), 15, 1.6)
    _log(f"  worst rel {w:.2e}")


def test_relaxed_iterates_maxcut_random_2000(lib):
    _log("relaxed iterates maxcut_random_2000 (max-cut n=2000, cliques up to 673)")
    w = _iterate_parity(lib, configs.maxcut_random_2000(), 3, 1.8)
    _log(f"  worst rel {w:.2e}")


@pytest.mark.parametrize("alpha", [1.5, 1.8])
def test_relaxed_solve_block_arrow_n50(lib, alpha):
    _log(f"relaxed solve block_arrow_n50 alpha={alpha}")
    inst = configs.block_arrow_n50()
    ref = hsde.solve(inst, alpha=alpha)
    s = lib.Solver(inst, alpha=alpha)
    info = s.solve()[0]
    s.close()
    obj = hsde.recover(ref)["obj_p"]
    _log(f"  status {info['status']} iters {info['iter']} (oracle {ref.iters}), obj {info['obj_p']:.10g}")
    assert info["status"] == ref.status == hsde.SOLVED
    assert info["iter"] == ref.iters
    assert abs(info["obj_p"] - obj) <= 1e-6 * max(1.0, abs(obj))


def test_relaxed_infeasible_tiny(lib):
    _log("relaxed infeasible tiny")
    P = configs.SDPInstance(2, 1, (np.array([0, 1], np.int32), np.array([0, 1], np.int32), np.array([1.0, 1.0])),
                            (np.array([0], np.int32), np.array([0], np.int32), np.array([0], np.int32), np.array([1.0])),
                            np.array([-1.0]), [np.array([0, 1])], np.array([-1]))
    D = configs.SDPInstance(2, 1, (np.array([0, 1], np.int32), np.array([0, 1], np.int32), np.array([-1.0, -1.0])),
                            (np.array([0], np.int32), np.array([1], np.int32), np.array([0], np.int32), np.array([1.0])),
                            np.array([0.0]), [np.array([0, 1])], np.array([-1]))
    for inst, want in ((P, hsde.PRIMAL_INFEASIBLE), (D, hsde.DUAL_INFEASIBLE)):
        ref = hsde.solve(inst, max_iter=5000, alpha=1.7)
        s = lib.Solver(inst, max_iter=5000, alpha=1.7)
        info = s.solve()[0]
        s.close()
        assert info["status"] == ref.status == want
        assert info["iter"] == ref.iters


def test_relaxed_batch_equals_single(lib):
    _log("relaxed batch == single")
    insts = [configs.small_block_arrow(i, n=15 + 3 * i, block=3 + i, arrow=2, m=5 + i) for i in range(4)]
    b = lib.Solver(insts, alpha=1.6)
    b.iterate(30)
    for i, inst in enumerate(insts):
        s = lib.Solver(inst, alpha=1.6)
        s.iterate(30)
        u1, v1 = s.get_state()
        u2, v2 = b.get_state(i)
        s.close()
        assert _rel(np.concatenate([u2, v2]), np.concatenate([u1, v1])) <= 1e-12
    b.close()


def test_relaxed_resume_is_bitwise(lib):
    _log("relaxed state roundtrip")
    inst = configs.block_arrow_n50()
    a = lib.Solver(inst, alpha=1.6)
    a.iterate(40)
    ua, va = a.get_state()
    b = lib.Solver(inst, alpha=1.6)
    b.iterate(20)
    c = lib.Solver(inst, alpha=1.6)
    c.set_state(*b.get_state())
    c.iterate(20)
    uc, vc = c.get_state()
    assert np.array_equal(ua, uc) and np.array_equal(va, vc)
    for s in (a, b, c):
        s.close()


def test_alpha_one_is_the_unrelaxed_path(lib):
    """alpha = 1 takes the paper's form bit for bit."""
    inst = configs.block_arrow_n50()
    a = lib.Solver(inst)
    a.iterate(25)
    b = lib.Solver(inst, alpha=1.0)
    b.iterate(25)
    ua, va = a.get_state()
    ub, vb = b.get_state()
    assert np.array_equal(ua, ub) and np.array_equal(va, vb)
    a.close()
    b.close()


def test_alpha_out_of_range_is_rejected(lib):
    for bad in (0.0, 2.0, -1.0, float("nan")):
        with pytest.raises(lib.CDCSError):
            lib.Solver(configs.block_arrow_n50(), alpha=bad)
