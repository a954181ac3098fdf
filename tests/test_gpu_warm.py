"""Warm-started Jacobi (settings eig_warm = 1) on the GPU against the oracle.

The warm start changes how each clique's eigen-decomposition is reached, not
what it is (the projection onto the PSD cone is unique), so the bars are the
unrelaxed path's: iterates within 1e-10 of the oracle (over 70 iterations, so
that the cold restart at iteration 65 is crossed), the same stop iteration
and objective in a whole solve, batch == single.  That the warm path ran is
checked by its iterates differing from the cold path's in the last bits
while agreeing with them to 1e-11.
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


def _iterate_parity(lib, inst, iters, tol=1e-10, alpha=1.0, **settings):
    res = hsde.solve(inst, max_iter=iters, record=iters, stop=False, alpha=alpha)
    s = lib.Solver(inst, eig_warm=1, alpha=alpha, **settings)
    worst = 0.0
    for k in range(iters):
        s.iterate(1)
        u, vt = s.get_state()
        r = _rel(np.concatenate([u, vt]), hsde.state_vector(*res.history[k]))
        worst = max(worst, r)
        assert r <= tol, (k + 1, r)
    s.close()
    return worst


def test_warm_iterates_block_arrow_n50(lib):
    _log("warm iterates block_arrow_n50 (70, across the cold restart)")
    w = _iterate_parity(lib, configs.block_arrow_n50(), 70)
    _log(f"  worst rel {w:.2e}")


def test_warm_iterates_graph_replay(lib):
    _log("warm iterates block_arrow_n50 (graph replay)")
    _iterate_parity(lib, configs.block_arrow_n50(), 20, use_graph=1)


def test_warm_iterates_small_odd_sizes(lib):
    _log("warm iterates small odd sizes")
    w = _iterate_parity(lib, configs.small_block_arrow(2, n=23, block=5, arrow=3, m=7), 50)
    _log(f"  worst rel {w:.2e}")


def test_warm_iterates_uneven_cliques_5000(lib):
    """Cliques of every Jacobi bucket (4..64 vertices) beside tridiagonal-path ones (65..96)."""
    _log("warm iterates uneven_cliques_5000")
    w = _iterate_parity(lib, configs.uneven_cliques_5000(), 20)
    _log(f"  worst rel {w:.2e}")


def test_warm_iterates_relaxed(lib):
    _log("warm + relaxed iterates block_arrow_n50")
    w = _iterate_parity(lib, configs.block_arrow_n50(), 40, alpha=1.6)
    _log(f"  worst rel {w:.2e}")


def test_warm_fp32_iterates(lib):
    _log("warm FP32 iterates block_arrow_n50")
    w = _iterate_parity(lib, configs.block_arrow_n50(), 50, tol=1e-4, eig_fp32=1)
    _log(f"  worst rel {w:.2e}")
    assert w > 1e-12


def test_warm_differs_from_cold_only_in_rounding(lib):
    inst = configs.uneven_cliques_5000()
    a = lib.Solver(inst)
    a.iterate(10)
    b = lib.Solver(inst, eig_warm=1)
    b.iterate(10)
    ua, va = a.get_state()
    ub, vb = b.get_state()
    r = _rel(np.concatenate([ub, vb]), np.concatenate([ua, va]))
    _log(f"warm vs cold after 10 iterations: {r:.2e}")
    assert not (np.array_equal(ua, ub) and np.array_equal(va, vb))
    assert r <= 1e-11
    a.close()
    b.close()


def test_warm_solve_block_arrow_n50(lib):
    _log("warm solve block_arrow_n50")
    inst = configs.block_arrow_n50()
    ref = hsde.solve(inst)
    s = lib.Solver(inst, eig_warm=1)
    info = s.solve()[0]
    s.close()
    obj = hsde.recover(ref)["obj_p"]
    _log(f"  status {info['status']} iters {info['iter']} (oracle {ref.iters})")
    assert info["status"] == ref.status == hsde.SOLVED
    assert info["iter"] == ref.iters
    assert abs(info["obj_p"] - obj) <= 1e-6 * max(1.0, abs(obj))


def test_warm_batch_equals_single(lib):
    insts = [configs.small_block_arrow(i, n=15 + 3 * i, block=3 + i, arrow=2, m=5 + i) for i in range(4)]
    b = lib.Solver(insts, eig_warm=1)
    b.iterate(30)
    for i, inst in enumerate(insts):
        s = lib.Solver(inst, eig_warm=1)
        s.iterate(30)
        u1, v1 = s.get_state()
        u2, v2 = b.get_state(i)
        s.close()
        assert _rel(np.concatenate([u2, v2]), np.concatenate([u1, v1])) <= 1e-12
    b.close()


def test_warm_resume_matches_to_rounding(lib):
    """set_state forces a cold start: the resumed run matches to rounding."""
    inst = configs.block_arrow_n50()
    a = lib.Solver(inst, eig_warm=1)
    a.iterate(40)
    ua, va = a.get_state()
    b = lib.Solver(inst, eig_warm=1)
    b.iterate(20)
    c = lib.Solver(inst, eig_warm=1)
    c.set_state(*b.get_state())
    c.iterate(20)
    uc, vc = c.get_state()
    assert _rel(np.concatenate([uc, vc]), np.concatenate([ua, va])) <= 1e-11
    for s in (a, b, c):
        s.close()


def test_eig_warm_flag_validated(lib):
    with pytest.raises(lib.CDCSError):
        lib.Solver(configs.block_arrow_n50(), eig_warm=2)
