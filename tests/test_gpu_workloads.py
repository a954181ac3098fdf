"""The configurations' own instances on the GPU, against the oracle or, where
the oracle cannot finish, against what makes the result checkable by itself.

* Batched block-arrow instances (256-instance workload): each GPU step
  against the oracle's step from the same state (the GPU's previous iterate),
  30 steps.  The first step, from (0, 0, 0, 0, 1), within 1e-11 (measured
  ~2e-12).  From the second step on tau is 0 on these instances (constraints
  on 30 % of the pattern) and step 1 cancels O(||zeta||) intermediates down
  to the iterate, so any two FP64 evaluations of it differ by ~1e-9 (measured
  1e-9..7e-9 per step, the same with the cached K^-1 or the triangular
  solves; against 80-bit arithmetic such a state carries ~1e-7): bar 2e-8.
  Whole trajectories are not compared: the iteration then amplifies those
  differences (in the oracle alone a 1e-15 perturbation of iterate 1 grows
  to ~1.5e-8 by iteration 30).  The two smallest instances, solved to the
  end: the oracle's status, stop iteration and objective (1e-6).
  The same instances inside the 256-instance batched handle (one launch per
  phase for all of them): the same per-step bars, and for eight instances
  spread over n = 50..400 the oracle's status, stop iteration and objective.
* The uneven-clique workload (n = 5000, m = 2000) and its twin (m = 2002,
  <A_1,X> = 1 and -1 appended), solved with the status checked every
  iteration: the oracle's status and stop iteration (stored by
  tests/golden/make_uneven_solves.py, which runs only the oracle), the
  objective within 1e-6 at that iteration; the twin's certificate is also
  checked directly: b^T y = 1, ||A^T y + H^T v|| within the tolerance, and
  every clique block of z PSD.
* Differentiated batch, one instance of its shape (n = 200, m = 100): the
  implicit gradient against the oracle's dense reference gradient (stored by
  tests/golden/make_grad_block_arrow_n200.py) within 1e-6 relative.
"""
import json
import os
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


@pytest.fixture(scope="module")
def batch_insts():
    return configs.block_arrow_batch256()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _split(prob, u, vt):
    """The solver's flat (u, v~) as the oracle's block lists."""
    nE, ns, m = prob.nE, prob.ns, prob.m
    cut = np.cumsum([nE, ns, m, ns])
    return ([*np.split(u[:-1], cut[:-1]), float(u[-1])], [*np.split(vt[:-1], cut[:-1]), float(vt[-1])])


@pytest.mark.parametrize("i", [0, 1, 2])
def test_batch_instance_steps(lib, batch_insts, i):
    inst = batch_insts[i]
    _log(f"batch instance {i} (n={inst.n}, m={inst.m}): 30 steps, each against the oracle's step")
    prob = hsde.build_problem(inst)
    cache = hsde.AffineCache(prob)
    sizes = hsde.clique_sizes(prob)
    s = lib.Solver(inst)
    prev = hsde.initial_point(prob)
    worst = 0.0
    for k in range(30):
        s.iterate(1)
        u, vt = s.get_state()
        want = hsde.state_vector(*hsde.iterate(prob, cache, prev[0], prev[1], sizes))
        r = _rel(np.concatenate([u, vt]), want)
        worst = max(worst, r)
        assert r <= (1e-11 if k == 0 else 2e-8), (k + 1, r)
        prev = _split(prob, u, vt)
    s.close()
    _log(f"  worst step error {worst:.2e}")


def test_batch_smallest_instances_solve_like_the_oracle(lib, batch_insts):
    small = sorted(range(len(batch_insts)), key=lambda i: batch_insts[i].n)[:2]
    for i in small:
        inst = batch_insts[i]
        ref = hsde.solve(inst)
        s = lib.Solver(inst)
        info = s.solve()[0]
        s.close()
        obj = hsde.recover(ref)["obj_p"]
        _log(f"instance {i} n={inst.n}: status {info['status']} iter {info['iter']} (oracle {ref.iters})")
        assert info["status"] == ref.status == hsde.SOLVED
        assert info["iter"] == ref.iters
        assert abs(info["obj_p"] - obj) <= 1e-6 * max(1.0, abs(obj))


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _spread(insts, count):
    """Indices of `count` instances spread evenly over the range of n."""
    order = sorted(range(len(insts)), key=lambda i: insts[i].n)
    return [order[round(j * (len(order) - 1) / (count - 1))] for j in range(count)]


def test_batch256_instance_steps_in_the_batched_handle(lib, batch_insts):
    picks = _spread(batch_insts, 4)
    _log(f"256-instance batched handle: 30 steps of instances {picks} "
         f"(n={[batch_insts[i].n for i in picks]}) against the oracle's steps")
    s = lib.Solver(batch_insts)
    probs = {i: hsde.build_problem(batch_insts[i]) for i in picks}
    caches = {i: hsde.AffineCache(probs[i]) for i in picks}
    sizes = {i: hsde.clique_sizes(probs[i]) for i in picks}
    prev = {i: hsde.initial_point(probs[i]) for i in picks}
    worst = 0.0
    for k in range(30):
        s.iterate(1)
        for i in picks:
            u, vt = s.get_state(i)
            want = hsde.state_vector(*hsde.iterate(probs[i], caches[i], prev[i][0], prev[i][1], sizes[i]))
            r = _rel(np.concatenate([u, vt]), want)
            worst = max(worst, r)
            assert r <= (1e-11 if k == 0 else 2e-8), (i, k + 1, r)
            prev[i] = _split(probs[i], u, vt)
    s.close()
    _log(f"  worst step error {worst:.2e}")


def test_batch256_solves_like_the_oracle(lib, batch_insts):
    picks = _spread(batch_insts, 8)
    _log(f"256-instance batched solve (status every iteration); oracle on instances {picks}")
    s = lib.Solver(batch_insts, check_every=1)
    infos = s.solve()
    s.close()
    for i in picks:
        ref = hsde.solve(batch_insts[i])
        info = infos[i]
        _log(f"  instance {i} n={batch_insts[i].n}: {lib.STATUS_NAMES[info['status']]} at {info['iter']} "
             f"(oracle {hsde.STATUS_NAMES[ref.status]} at {ref.iters})")
        assert info["status"] == ref.status
        assert info["iter"] == ref.iters
        if ref.status == hsde.SOLVED:
            obj = hsde.recover(ref)["obj_p"]
            assert abs(info["obj_p"] - obj) <= 1e-6 * max(1.0, abs(obj))


def _golden_uneven():
    with open(os.path.join(GOLDEN, "uneven_cliques_5000_oracle.json")) as f:
        return json.load(f)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("form", ["plain", "relaxed"])
def test_uneven_solve_matches_the_oracle(lib, form):
    ref = _golden_uneven()["feasible"][form]
    _log(f"uneven cliques n=5000 solve ({form}, alpha={ref['alpha']}); oracle: {ref['status']} at {ref['iterations']}")
    s = lib.Solver(configs.uneven_cliques_5000(), check_every=1, alpha=ref["alpha"])
    info = s.solve()[0]
    s.close()
    _log(f"  GPU: {lib.STATUS_NAMES[info['status']]} at {info['iter']}, obj_p {info['obj_p']:.12g} "
         f"(oracle {ref.get('obj_p')})")
    assert lib.STATUS_NAMES[info["status"]] == ref["status"]
    assert info["iter"] == ref["iterations"]
    assert abs(info["obj_p"] - ref["obj_p"]) <= 1e-6 * max(1.0, abs(ref["obj_p"]))
    assert abs(info["obj_d"] - ref["obj_d"]) <= 1e-6 * max(1.0, abs(ref["obj_d"]))


def test_uneven_twin_matches_the_oracle(lib):
    ref = _golden_uneven()["twin"]["plain"]
    s = lib.Solver(configs.uneven_cliques_5000(twin=True), check_every=1)
    info = s.solve()[0]
    s.close()
    _log(f"twin: GPU {lib.STATUS_NAMES[info['status']]} at {info['iter']}; oracle {ref['status']} at {ref['iterations']}")
    assert lib.STATUS_NAMES[info["status"]] == ref["status"] == "primal_infeasible"
    assert info["iter"] == ref["iterations"]


def test_grad_shape_instance_matches_the_dense_oracle_gradient(lib):
    """Instance 0 of the differentiated batch (n = 200, block 16, arrow 4,
    m = 100), loss <W, X*>: the GPU forward solve to eps_tol = 5e-11 and its
    implicit gradient against the oracle's dense reference (solved to 5e-11,
    just above the FP64 floor of this instance's residuals)."""
    path = os.path.join(GOLDEN, "grad_block_arrow_n200.txt")
    ref = np.loadtxt(path, comments="#")
    inst = configs.block_arrow_grad64(count=1)[0]
    prob = hsde.build_problem(inst)
    assert len(ref) == prob.nE + prob.m
    gc, gb = ref[:prob.nE], ref[prob.nE:]
    wr, wc, wv = inst.meta["W"]
    key = {(int(r), int(c)): e for e, (r, c) in enumerate(zip(prob.erow, prob.ecol))}
    w = np.zeros(prob.nE)
    for r, c, x in zip(wr, wc, wv):
        w[key[(int(r), int(c))]] = x * (1.0 if r == c else np.sqrt(2.0))
    s = lib.Solver(inst, eps_tol=5e-11, max_iter=100000, check_every=50)
    info = s.solve()[0]
    assert info["status"] == lib.SOLVED, info
    dc, db, it = s.adjoint(w, max_iter=200000, tol=1e-11)
    s.close()
    rc = np.linalg.norm(dc - gc) / np.linalg.norm(gc)
    rb = np.linalg.norm(db - gb) / np.linalg.norm(gb)
    _log(f"grad-shape instance: forward {info['iter']} iterations, adjoint {it} applications, "
         f"rel err dL/dc {rc:.2e}, dL/db {rb:.2e}")
    assert rc <= 1e-6 and rb <= 1e-6


def test_uneven_twin_is_primal_infeasible(lib):
    inst = configs.uneven_cliques_5000(twin=True)
    s = lib.Solver(inst, max_iter=20000, check_every=10)
    info = s.solve()[0]
    _log(f"twin: status {info['status']} after {info['iter']} iterations")
    assert info["status"] == hsde.PRIMAL_INFEASIBLE
    y_cert, _ = s.certificate()
    u, vt = s.get_state()
    s.close()
    prob = hsde.build_problem(inst)
    nE, ns, m = prob.nE, prob.ns, prob.m
    y = u[nE + ns: nE + ns + m]
    v = u[nE + ns + m: nE + 2 * ns + m]
    z = vt[nE: nE + ns]
    by = float(prob.b @ y)
    assert by > 0
    assert np.allclose(y_cert, y / by, rtol=1e-12, atol=0)
    assert abs(float(prob.b @ y_cert) - 1.0) <= 1e-12
    res = prob.A.T @ y_cert + prob.H.T @ (v / by)
    _log(f"  ||A^T y + H^T v|| = {np.linalg.norm(res):.2e}")
    assert np.linalg.norm(res) <= 1e-4
    sizes = hsde.clique_sizes(prob)
    for k, K in enumerate(sizes):
        Zk = hsde.smat_blocks(z[prob.slot_off[k]:prob.slot_off[k + 1]], K)
        assert np.linalg.eigvalsh(Zk).min() >= -1e-10 * max(1.0, np.linalg.norm(Zk))
