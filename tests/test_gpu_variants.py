"""The FP32-eigensolve variant and the Jacobi tile autotuner (through the C-ABI).

FP32 variant (settings eig_fp32 = 1): the Jacobi eigen-decompositions of
cliques up to 64 vertices run in FP32, everything else in FP64.  Bars, against
the FP64 oracle on the same seeded inputs:
  * iterates k = 1..50 within 1e-4 relative (FP32 rounding, ~1e-7 per conic
    step, accumulates at most linearly in a nonexpansive iteration), and not
    within 1e-12 (the FP32 kernels did run);
  * a whole solve reaches the same status, objective within 1e-4 relative,
    iteration count reported.
Autotuner (settings autotune = 1): the tile shape changes only the order of
the sweep sums, so iterates match the FP64 oracle to the usual 1e-10.
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


def _worst_iterate_error(lib, inst, iters, **settings):
    res = hsde.solve(inst, max_iter=iters, record=iters, stop=False)
    s = lib.Solver(inst, **settings)
    worst = 0.0
    for k in range(iters):
        s.iterate(1)
        u, vt = s.get_state()
        worst = max(worst, _rel(np.concatenate([u, vt]), hsde.state_vector(*res.history[k])))
    tuning = s.tuning()
    s.close()
    return worst, tuning


def test_fp32_eig_iterates_block_arrow_n50(lib):
    _log("FP32 eig: iterates block_arrow_n50")
    w, _ = _worst_iterate_error(lib, configs.block_arrow_n50(), 50, eig_fp32=1)
    _log(f"  worst rel {w:.2e}")
    assert 1e-12 < w <= 1e-4


def test_fp32_eig_iterates_uneven_cliques(lib):
    """Cliques of every Jacobi bucket (4..64 vertices) beside tridiagonal-path ones (65..96)."""
    _log("FP32 eig: iterates uneven_cliques_5000 (cliques 4..96)")
    w, _ = _worst_iterate_error(lib, configs.uneven_cliques_5000(), 20, eig_fp32=1)
    _log(f"  worst rel {w:.2e}")
    assert 1e-12 < w <= 1e-4


def test_fp32_eig_solve_block_arrow_n50(lib):
    _log("FP32 eig: solve block_arrow_n50")
    inst = configs.block_arrow_n50()
    ref = hsde.solve(inst)
    obj = hsde.recover(ref)["obj_p"]
    s = lib.Solver(inst, eig_fp32=1)
    info = s.solve()[0]
    s.close()
    _log(f"  status {info['status']} iters {info['iter']} (FP64 oracle {ref.iters}), "
         f"obj {info['obj_p']:.10g} vs {obj:.10g}")
    assert info["status"] == ref.status == hsde.SOLVED
    assert abs(info["obj_p"] - obj) <= 1e-4 * max(1.0, abs(obj))


def test_autotuned_iterates_match_oracle(lib):
    _log("autotune: iterates uneven_cliques_5000")
    w, tuning = _worst_iterate_error(lib, configs.uneven_cliques_5000(), 20, autotune=1)
    _log(f"  worst rel {w:.2e}; tuning {tuning}")
    assert w <= 1e-10
    allowed = {16: (64, 128), 32: (64, 128), 64: (128, 256), 96: (256, 512)}
    for b in tuning:
        assert b["threads"] in allowed[b["kmax"]]
        assert b["tuned"] == (b["cliques"] > 0)


def test_alternative_tile_shapes_match_oracle(lib):
    """autotune = 2 runs the other candidate shape of every bucket."""
    _log("alternative tile shapes: iterates uneven_cliques_5000")
    w, tuning = _worst_iterate_error(lib, configs.uneven_cliques_5000(), 20, autotune=2)
    _log(f"  worst rel {w:.2e}; tuning {tuning}")
    assert w <= 1e-10
    assert [b["threads"] for b in tuning] == [128, 64, 128, 256]
    w, _ = _worst_iterate_error(lib, configs.uneven_cliques_5000(), 20, autotune=2, eig_fp32=1)
    _log(f"  FP32, alternative shapes: worst rel {w:.2e}")
    assert 1e-12 < w <= 1e-4


def test_autotune_off_reports_defaults(lib):
    s = lib.Solver(configs.block_arrow_n50())
    t = s.tuning()
    s.close()
    assert [b["threads"] for b in t] == [64, 128, 256, 512]
    assert not any(b["tuned"] for b in t)
    assert sum(b["cliques"] for b in t) == len(configs.block_arrow_n50().cliques)


def test_settings_reject_bad_variant_flags(lib):
    with pytest.raises(lib.CDCSError):
        lib.Solver(configs.block_arrow_n50(), eig_fp32=2)
    with pytest.raises(lib.CDCSError):
        lib.Solver(configs.block_arrow_n50(), autotune=3)
