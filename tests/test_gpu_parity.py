"""GPU path (through the C-ABI) against the CPU oracle on the same seeded inputs.

Bars (floating point, FP64 on both sides):
  * PSD projection of a packed block: ||gpu - oracle||_F <= 1e-13 ||Y||_F
  * iterates k = 1..50: ||(u,v)_gpu - (u,v)_oracle|| <= 1e-10 ||(u,v)_oracle||
  * whole solve: same status and stop iteration with check_every = 1, and
    objectives within 1e-6 relative
  * batch instance i == plain instance i to 1e-12; reruns bitwise equal.
"""
import math
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
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch


@pytest.fixture(scope="module")
def lib():
    from paper_1611_01828_amd import cdcs
    cdcs.load()
    return cdcs


def _state(res_entry):
    u, vt = res_entry
    return hsde.state_vector(u, vt)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ----------------------------------------------------------------------------
# the conic step on its own
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("sizes", [
    [1, 2, 3, 4, 5, 7, 8, 9, 15, 16],
    [17, 20, 31, 32],
    [33, 40, 63, 64],
    [65, 77, 95, 96],
    [97, 128, 129, 200],
    [136, 137, 168, 169],        # tail only, one panel + tail, two panels + tail
    [333, 512, 673],
    [1024],
])
def test_psd_project_matches_oracle(lib, torch_cuda, sizes):
    torch = torch_cuda
    _log(f"psd_project sizes={sizes}")
    rng = np.random.default_rng(sum(sizes))
    blocks, offs, pos = [], [], 0
    for K in sizes:
        G = rng.standard_normal((K, K))
        Y = (G + G.T) / 2
        Y[0, 0] += 0.0
        blocks.append(hsde.svec_blocks(Y, K))
        offs.append(pos)
        pos += K * (K + 1) // 2
    vec = np.concatenate(blocks)
    want = hsde.proj_psd_packed(vec, sizes, np.asarray(offs))
    dev_in = torch.tensor(vec, dtype=torch.float64, device="cuda")
    dev_out = torch.empty_like(dev_in)
    lib.psd_project(sizes, offs, dev_in, dev_out)
    got = dev_out.cpu().numpy()
    for K, o in zip(sizes, offs):
        sl = slice(o, o + K * (K + 1) // 2)
        err = np.linalg.norm(got[sl] - want[sl]) / np.linalg.norm(vec[sl])
        _log(f"  K={K} rel err {err:.2e}")
        assert err <= (1e-13 if K <= 96 else 1e-12), K


@pytest.mark.parametrize("K", [12, 150, 300])
def test_psd_project_special_blocks(lib, torch_cuda, K):
    """Zero, PSD, NSD, rank-one and repeated-eigenvalue blocks."""
    torch = torch_cuda
    _log(f"special blocks K={K}")
    rng = np.random.default_rng(5)
    mats = []
    mats.append(np.zeros((K, K)))
    G = rng.standard_normal((K, K))
    mats.append(G @ G.T)
    mats.append(-G @ G.T)
    q = rng.standard_normal(K)
    mats.append(np.outer(q, q))
    Qm, _ = np.linalg.qr(rng.standard_normal((K, K)))
    mats.append(Qm @ np.diag([1.0] * (K // 2) + [-1.0] * (K - K // 2)) @ Qm.T)
    mats.append(Qm @ np.diag([2.0] * 3 + [0.0] * (K - 5) + [-1.0] * 2) @ Qm.T)
    mats.append(np.eye(K) * 3.0)
    vec = np.concatenate([hsde.svec_blocks(M, K) for M in mats])
    sizes = [K] * len(mats)
    offs = [i * K * (K + 1) // 2 for i in range(len(mats))]
    want = hsde.proj_psd_packed(vec, sizes, np.asarray(offs))
    dev_in = torch.tensor(vec, dtype=torch.float64, device="cuda")
    lib.psd_project(sizes, offs, dev_in, dev_in)        # in place
    got = dev_in.cpu().numpy()
    nb = K * (K + 1) // 2
    for i in range(len(mats)):
        sl = slice(i * nb, (i + 1) * nb)
        err = np.linalg.norm(got[sl] - want[sl]) / max(1.0, np.linalg.norm(vec[sl]))
        assert err <= (1e-13 if K <= 96 else 1e-12), (i, err)


# ----------------------------------------------------------------------------
# iterates and whole solves
# ----------------------------------------------------------------------------

def _iterate_parity(lib, inst, iters, tol=1e-10, graph=False):
    res = hsde.solve(inst, max_iter=iters, record=iters, stop=False)
    s = lib.Solver(inst, use_graph=int(graph))
    worst = 0.0
    for k in range(iters):
        s.iterate(1)
        u, vt = s.get_state()
        got = np.concatenate([u, vt])
        want = _state(res.history[k])
        r = _rel(got, want)
        worst = max(worst, r)
        assert r <= tol, (k + 1, r)
    s.close()
    return worst


def test_iterates_block_arrow_n50(lib, torch_cuda):
    _log("iterates block_arrow_n50")
    w = _iterate_parity(lib, configs.block_arrow_n50(), 50)
    _log(f"  worst rel {w:.2e}")


def test_iterates_block_arrow_n50_graph_replay(lib, torch_cuda):
    _log("iterates block_arrow_n50 (graph replay)")
    _iterate_parity(lib, configs.block_arrow_n50(), 20, graph=True)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_iterates_small_odd_sizes(lib, torch_cuda, seed):
    _log(f"iterates small seed={seed}")
    inst = configs.small_block_arrow(seed, n=23, block=5, arrow=3, m=7)
    _iterate_parity(lib, inst, 50)


def test_iterates_large_cliques(lib, torch_cuda):
    """Cliques of 130 and 250 vertices go through the tridiagonal path.

    Sparse constraints (8 entries each) keep the data well scaled: with
    dense constraints the step-1 Sherman-Morrison update cancels
    O(||zeta||) intermediates down to an O(1e-2) iterate and FP64 itself
    (either algebra route) carries ~1e-7 error there.
    """
    _log("iterates large cliques")
    inst = configs.small_block_arrow(7, n=500, block=120, arrow=10, m=30, per_row=8)
    w = _iterate_parity(lib, inst, 30)
    _log(f"  worst rel {w:.2e}")
    inst = configs.small_block_arrow(8, n=510, block=240, arrow=10, m=12, per_row=8)
    w = _iterate_parity(lib, inst, 15)
    _log(f"  worst rel {w:.2e}")


@pytest.mark.parametrize("m", [300, 600, 1100])
def test_iterates_dense_factor_orders(lib, torch_cuda, m):
    """Dense m x m factors of 300, 600 and 1100 rows: the dense triangular
    sweeps with 2, 4 and 8 rows per thread (constraints of 25 entries each
    make I + A P^-1 A^T about half full)."""
    _log(f"iterates dense factor m={m}")
    inst = configs.small_block_arrow(3, n=100, block=10, arrow=5, m=m, per_row=25)
    w = _iterate_parity(lib, inst, 20)
    _log(f"  worst rel {w:.2e}")


def test_batch_mixed_dense_orders(lib, torch_cuda):
    """A 20-row and a 600-row dense factor in one batch (the small one then
    runs with the sweep shape of the large one)."""
    _log("batch of dense factors m=20 and m=600")
    insts = [configs.block_arrow_n50(), configs.small_block_arrow(3, n=100, block=10, arrow=5, m=600, per_row=25)]
    b = lib.Solver(insts)
    b.iterate(15)
    for i, inst in enumerate(insts):
        s = lib.Solver(inst)
        s.iterate(15)
        u1, v1 = s.get_state()
        u2, v2 = b.get_state(i)
        assert _rel(np.concatenate([u2, v2]), np.concatenate([u1, v1])) <= 1e-12


def test_iterates_uneven_cliques_5000(lib, torch_cuda):
    _log("iterates uneven_cliques_5000")
    w = _iterate_parity(lib, configs.uneven_cliques_5000(), 20)
    _log(f"  worst rel {w:.2e}")


def test_iterates_maxcut_random_2000(lib, torch_cuda):
    _log("iterates maxcut_random_2000 (max-cut n=2000, cliques up to 673)")
    w = _iterate_parity(lib, configs.maxcut_random_2000(), 4)
    _log(f"  worst rel {w:.2e}")


def test_iterates_grid_companion(lib, torch_cuda):
    """Max-cut on the periodic 40 x 50 grid: 1487 Jacobi cliques, 11 in the LDS
    tail, one of 147 vertices through the per-column chain."""
    _log("iterates grid companion (max-cut 40x50 periodic grid, 1499 cliques)")
    w = _iterate_parity(lib, configs.grid_maxcut(1), 20)
    _log(f"  worst rel {w:.2e}")


def test_solve_block_arrow_n50_matches_oracle(lib, torch_cuda):
    _log("solve block_arrow_n50")
    inst = configs.block_arrow_n50()
    ref = hsde.solve(inst)
    s = lib.Solver(inst)
    info = s.solve()[0]
    assert info["status"] == ref.status == hsde.SOLVED
    assert info["iter"] == ref.iters
    obj = hsde.recover(ref)["obj_p"]
    assert abs(info["obj_p"] - obj) <= 1e-6 * max(1.0, abs(obj))
    X, y, Z = s.solution()
    rec = hsde.recover(ref)
    assert _rel(X, rec["x"]) <= 1e-8
    assert _rel(y, rec["y"]) <= 1e-8
    assert _rel(Z, rec["Zvec"]) <= 1e-8


def test_primal_and_dual_infeasible_tiny(lib, torch_cuda):
    _log("infeasible tiny")
    P = configs.SDPInstance(2, 1, (np.array([0, 1], np.int32), np.array([0, 1], np.int32), np.array([1.0, 1.0])),
                            (np.array([0], np.int32), np.array([0], np.int32), np.array([0], np.int32), np.array([1.0])),
                            np.array([-1.0]), [np.array([0, 1])], np.array([-1]))
    ref = hsde.solve(P, max_iter=5000)
    s = lib.Solver(P, max_iter=5000)
    info = s.solve()[0]
    assert info["status"] == ref.status == hsde.PRIMAL_INFEASIBLE
    assert info["iter"] == ref.iters
    y, _ = s.certificate()
    assert abs(float(P.b @ y) - 1.0) <= 1e-12
    D = configs.SDPInstance(2, 1, (np.array([0, 1], np.int32), np.array([0, 1], np.int32), np.array([-1.0, -1.0])),
                            (np.array([0], np.int32), np.array([1], np.int32), np.array([0], np.int32), np.array([1.0])),
                            np.array([0.0]), [np.array([0, 1])], np.array([-1]))
    ref = hsde.solve(D, max_iter=5000)
    s = lib.Solver(D, max_iter=5000)
    info = s.solve()[0]
    assert info["status"] == ref.status == hsde.DUAL_INFEASIBLE
    assert info["iter"] == ref.iters
    _, X = s.certificate()
    prob = hsde.build_problem(D)
    assert abs(float(prob.c @ X) + 1.0) <= 1e-12


def test_batch_equals_single(lib, torch_cuda):
    _log("batch == single")
    insts = [configs.small_block_arrow(i, n=15 + 3 * i, block=3 + i, arrow=2, m=5 + i) for i in range(4)]
    b = lib.Solver(insts)
    b.iterate(30)
    for i, inst in enumerate(insts):
        s = lib.Solver(inst)
        s.iterate(30)
        u1, v1 = s.get_state()
        u2, v2 = b.get_state(i)
        assert _rel(np.concatenate([u2, v2]), np.concatenate([u1, v1])) <= 1e-12


def test_state_roundtrip_and_determinism(lib, torch_cuda):
    _log("state roundtrip")
    inst = configs.block_arrow_n50()
    a = lib.Solver(inst)
    a.iterate(40)
    ua, va = a.get_state()
    b = lib.Solver(inst)
    b.iterate(20)
    u, v = b.get_state()
    c = lib.Solver(inst)
    c.set_state(u, v)
    c.iterate(20)
    uc, vc = c.get_state()
    assert np.array_equal(ua, uc) and np.array_equal(va, vc)
    d = lib.Solver(inst)
    d.iterate(40)
    ud, vd = d.get_state()
    assert np.array_equal(ua, ud) and np.array_equal(va, vd)


def test_setup_rejects_bad_inputs(lib, torch_cuda):
    inst = configs.small_block_arrow(0, n=12, block=3, arrow=2, m=4)
    bad = configs.SDPInstance(inst.n, inst.m, inst.C, inst.A, inst.b, inst.cliques[:-1], inst.parent[:-1])
    with pytest.raises(lib.CDCSError) as e:
        lib.Solver(bad)
    assert e.value.code in (-2, -3)
    bad = configs.SDPInstance(inst.n, inst.m, inst.C, inst.A, inst.b * np.nan, inst.cliques, inst.parent)
    with pytest.raises(lib.CDCSError) as e:
        lib.Solver(bad)
    assert e.value.code == -4


@pytest.mark.timeout(600)
def test_iterates_sparse_factor_beyond_lds(lib, torch_cuda):
    """Max-cut on the periodic 100 x 100 grid: m = 10000 constraints, above the
    8192 rows the sparse triangular solve keeps in LDS (its vector then lives
    in global memory) and above the order up to which K is summed densely on
    the host (K is assembled from its nonzero terms)."""
    _log("iterates: max-cut on the 100 x 100 periodic grid (m = 10000)")
    inst = configs.grid_maxcut(2, rows=100, cols=100)
    w = _iterate_parity(lib, inst, 5)
    _log(f"  worst rel {w:.2e}")
