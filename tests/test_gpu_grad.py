"""GPU implicit gradient (cdcs_adjoint through the C-ABI) against the oracle's
dense adjoint on tightly solved instances; batched == single."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import grad, hsde  # noqa: E402
from sdpgen import configs  # noqa: E402


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_1611_01828_amd import cdcs
    cdcs.load()
    return cdcs


def _gpu_grad(lib, insts, ws, eps=1e-11):
    s = lib.Solver(insts, eps_tol=eps, max_iter=400000, check_every=50)
    infos = s.solve()
    assert all(i["status"] == 1 for i in infos), infos
    dc, db, it = s.adjoint(np.concatenate(ws), max_iter=200000, tol=1e-11)
    return s, dc, db, it


@pytest.mark.parametrize("shape", [dict(n=10, block=3, arrow=2, m=4), dict(n=30, block=6, arrow=3, m=10)])
def test_adjoint_matches_dense_oracle(lib, shape):
    _log(f"adjoint vs dense oracle {shape}")
    inst = configs.small_block_arrow(21, **shape)
    prob = hsde.build_problem(inst)
    w = np.random.default_rng(4).standard_normal(prob.nE)
    _, res = grad.objective_weight_loss(inst, w, eps_tol=1e-11)
    gc, gb = grad.adjoint_gradient_dense(res, w)
    s, dc, db, it = _gpu_grad(lib, [inst], [w])
    rc = np.linalg.norm(dc - gc) / np.linalg.norm(gc)
    rb = np.linalg.norm(db - gb) / max(np.linalg.norm(gb), 1e-12)
    _log(f"  adjoint iterations {it}, rel err dc {rc:.2e} db {rb:.2e}")
    assert rc <= 1e-6 and rb <= 1e-6


def test_adjoint_batch_equals_single(lib):
    _log("adjoint batch == single")
    insts = [configs.small_block_arrow(30 + i, n=12 + 2 * i, block=3, arrow=2, m=4 + i) for i in range(3)]
    ws = [np.random.default_rng(i).standard_normal(hsde.build_problem(x).nE) for i, x in enumerate(insts)]
    _, dcb, dbb, _ = _gpu_grad(lib, insts, ws)
    oe = or_ = 0
    for i, x in enumerate(insts):
        _, dc, db, _ = _gpu_grad(lib, [x], [ws[i]])
        assert np.linalg.norm(dcb[oe:oe + len(dc)] - dc) <= 1e-9 * np.linalg.norm(dc)
        assert np.linalg.norm(dbb[or_:or_ + len(db)] - db) <= 1e-9 * max(np.linalg.norm(db), 1e-12)
        oe += len(dc)
        or_ += len(db)


def test_torch_layer_gradient_matches_finite_differences(lib):
    """autograd through SDPLayer vs central differences of the GPU solve."""
    import torch
    from paper_1611_01828_amd.layer import SDPLayer
    _log("torch layer vs FD")
    insts = [configs.small_block_arrow(40 + i, n=14, block=4, arrow=2, m=5) for i in range(2)]
    layer = SDPLayer(insts, eps_tol=1e-11, adjoint_tol=1e-11)
    c0 = np.concatenate([layer.svec_of(i, x.C) for i, x in enumerate(insts)])
    b0 = np.concatenate([x.b for x in insts])
    rng = np.random.default_rng(9)
    W = torch.tensor(rng.standard_normal(sum(layer.nE)), dtype=torch.float64, device="cuda")
    c = torch.tensor(c0, dtype=torch.float64, device="cuda", requires_grad=True)
    b = torch.tensor(b0, dtype=torch.float64, device="cuda", requires_grad=True)
    L = (W * layer(c, b)).sum()
    L.backward()
    gc = c.grad.cpu().numpy()
    gb = b.grad.cpu().numpy()
    h = 1e-5
    for _ in range(3):
        dc = rng.standard_normal(len(c0))
        db = rng.standard_normal(len(b0))
        with torch.no_grad():
            Lp = float((W * layer(torch.tensor(c0 + h * dc, device="cuda"), torch.tensor(b0 + h * db, device="cuda"))).sum())
            Lm = float((W * layer(torch.tensor(c0 - h * dc, device="cuda"), torch.tensor(b0 - h * db, device="cuda"))).sum())
        fd = (Lp - Lm) / (2 * h)
        an = float(gc @ dc + gb @ db)
        _log(f"  fd {fd:.10f} autograd {an:.10f}")
        assert abs(fd - an) <= 1e-4 * (abs(an) + np.linalg.norm(gc) + np.linalg.norm(gb))


def test_adjoint_reports_its_outcome(lib):
    """cdcs_get_adjoint_info: the final relative residual of every instance and
    why GMRES stopped; a tiny iteration limit is reported as such, and
    SDPLayer turns it into a warning."""
    import warnings

    import torch
    from paper_1611_01828_amd.layer import SDPLayer
    _log("adjoint outcome reporting")
    insts = [configs.small_block_arrow(50 + i, n=14, block=4, arrow=2, m=5) for i in range(2)]
    ws = [np.random.default_rng(i).standard_normal(hsde.build_problem(x).nE) for i, x in enumerate(insts)]
    s, _, _, _ = _gpu_grad(lib, insts, ws)
    r, why = s.adjoint_info()
    assert np.all(np.isfinite(r)) and set(why.tolist()) <= {0, 1}
    assert all((why[i] == 0) == (r[i] <= 1e-11) for i in range(2))
    s.adjoint(np.concatenate(ws), max_iter=3, tol=1e-14)
    r3, why3 = s.adjoint_info()
    assert list(why3) == [2, 2] and np.all(r3 > 1e-14)
    s.close()
    layer = SDPLayer(insts, eps_tol=1e-9, adjoint_tol=1e-14, adjoint_max_iter=3)
    c0 = np.concatenate([layer.svec_of(i, x.C) for i, x in enumerate(insts)])
    b0 = np.concatenate([x.b for x in insts])
    c = torch.tensor(c0, dtype=torch.float64, device="cuda", requires_grad=True)
    b = torch.tensor(b0, dtype=torch.float64, device="cuda", requires_grad=True)
    L = layer(c, b).sum()
    with warnings.catch_warnings(record=True) as rec:
        warnings.simplefilter("always")
        L.backward()
    assert any("iteration limit" in str(x.message) for x in rec)


def _golden(name):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    with open(path) as f:
        head = json.loads(f.readline()[1:])
        vals = np.array([float(v) for v in f])
    return head, vals


def test_adjoint_clique_above_64_matches_stored_oracle_gradient(lib):
    """Cliques of 70 and 24 vertices: the 70-vertex one takes the adjoint's
    96-vertex eigen-cache.  Reference: the oracle's dense gradient stored by
    tests/golden/make_grad_block_arrow_k70.py (forward solve to 1e-11)."""
    import importlib.util
    import os
    _log("adjoint with a 70-vertex clique vs the stored dense oracle gradient")
    spec = importlib.util.spec_from_file_location(
        "make_k70", os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "make_grad_block_arrow_k70.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    inst = mk.instance()
    prob = hsde.build_problem(inst)
    head, ref = _golden("grad_block_arrow_k70.txt")
    assert sorted(head["cliques"]) == sorted(len(c) for c in inst.cliques) and max(head["cliques"]) > 64
    gc, gb = ref[:prob.nE], ref[prob.nE:]
    s, dc, db, it = _gpu_grad(lib, [inst], [mk.weights(prob)])
    r, why = s.adjoint_info()
    s.close()
    rc = np.linalg.norm(dc - gc) / np.linalg.norm(gc)
    rb = np.linalg.norm(db - gb) / max(np.linalg.norm(gb), 1e-12)
    _log(f"  adjoint iterations {it}, residual {r[0]:.1e} (reason {why[0]}), rel err dc {rc:.2e} db {rb:.2e}")
    assert rc <= 1e-6 and rb <= 1e-6


def test_adjoint_rejects_cliques_above_96(lib):
    _log("adjoint refuses a 98-vertex clique")
    inst = configs.small_block_arrow(62, n=98, block=96, arrow=2, m=6)
    assert max(len(c) for c in inst.cliques) == 98
    s = lib.Solver([inst], max_iter=5)
    s.solve()
    with pytest.raises(lib.CDCSError, match="96 vertices"):
        s.adjoint(np.ones(hsde.build_problem(inst).nE), max_iter=10, tol=1e-8)
    s.close()
