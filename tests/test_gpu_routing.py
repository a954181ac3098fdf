"""Routing of the clique projections (settings.jacobi_max): cliques above the
threshold take the tridiagonal path (reduction in LDS, bisection, inverse
iteration, back-transformation) instead of the Jacobi kernels.  The
projection is unique, so the iteration is the same up to rounding: against
the FP64 oracle on the same seeded inputs the bars are those of the default
routing (iterates within 1e-10 relative, solves at the oracle's status and
stop iteration with objectives within 1e-6).  The adjoint keeps its own
Jacobi lists, so gradients do not depend on the routing (to the forward
solve's accuracy)."""
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


def _iterate_parity(lib, inst, iters, **settings):
    res = hsde.solve(inst, max_iter=iters, record=iters, stop=False)
    s = lib.Solver(inst, **settings)
    worst = 0.0
    for k in range(iters):
        s.iterate(1)
        u, vt = s.get_state()
        r = _rel(np.concatenate([u, vt]), hsde.state_vector(*res.history[k]))
        worst = max(worst, r)
        assert r <= 1e-10, (k + 1, r)
    tuning = s.tuning()
    s.close()
    return worst, tuning


@pytest.mark.parametrize("jmax", [16, 32])
def test_small_cliques_through_the_tridiagonal_path(lib, jmax):
    """Cliques of 3..40 vertices (block-arrow, blocks of 3..33 + arrow 7)."""
    for seed, (n, block, arrow) in enumerate([(60, 33, 7), (45, 9, 6), (30, 3, 2)]):
        inst = configs.small_block_arrow(60 + seed, n=n, block=block, arrow=arrow, m=9, per_row=8)
        w, tun = _iterate_parity(lib, inst, 30, jacobi_max=jmax)
        _log(f"jacobi_max={jmax}, n={n} block={block} arrow={arrow}: worst rel {w:.2e}, "
             f"Jacobi buckets {[(t['kmax'], t['cliques']) for t in tun]}")


@pytest.mark.parametrize("jmax", [16, 32])
def test_uneven_cliques_routed(lib, jmax):
    _log(f"uneven cliques n=5000 (4..96 vertices), jacobi_max={jmax}: 20 iterations")
    w, tun = _iterate_parity(lib, configs.uneven_cliques_5000(), 20, jacobi_max=jmax)
    _log(f"  worst rel {w:.2e}, Jacobi buckets {[(t['kmax'], t['cliques']) for t in tun]}")


def test_solve_routed_matches_oracle(lib):
    inst = configs.small_block_arrow(70, n=48, block=20, arrow=5, m=10)
    ref = hsde.solve(inst)
    s = lib.Solver(inst, jacobi_max=16)
    info = s.solve()[0]
    s.close()
    _log(f"routed solve: GPU {info['iter']} iterations, oracle {ref.iters}")
    assert info["status"] == ref.status == hsde.SOLVED
    assert info["iter"] == ref.iters
    obj = hsde.recover(ref)["obj_p"]
    assert abs(info["obj_p"] - obj) <= 1e-6 * max(1.0, abs(obj))


def test_adjoint_independent_of_routing(lib):
    insts = [configs.small_block_arrow(80 + i, n=30, block=20, arrow=4, m=6) for i in range(2)]
    w = np.concatenate([np.random.default_rng(i).standard_normal(hsde.build_problem(x).nE)
                        for i, x in enumerate(insts)])
    out = []
    for jmax in (0, 16):
        s = lib.Solver(insts, eps_tol=1e-10, max_iter=200000, check_every=50, jacobi_max=jmax)
        infos = s.solve()
        assert all(i["status"] == 1 for i in infos)
        dc, db, _ = s.adjoint(w, max_iter=100000, tol=1e-11)
        s.close()
        out.append((dc, db))
    rc = _rel(out[1][0], out[0][0])
    rb = _rel(out[1][1], out[0][1])
    _log(f"adjoint with the 24-vertex cliques routed to the tridiagonal path: rel diff dc {rc:.1e}, db {rb:.1e}")
    assert rc <= 1e-6 and rb <= 1e-6


def test_bad_jacobi_max_rejected(lib):
    inst = configs.small_block_arrow(0, n=12, block=3, arrow=2, m=4)
    with pytest.raises(lib.CDCSError) as e:
        lib.Solver(inst, jacobi_max=48)
    assert e.value.code == -1


# ----------------------------------------------------------------------------
# the reduction to tridiagonal form (settings.band_min): two-stage (dense to
# band, band to tridiagonal) for cliques of band_min vertices or more, the
# one-stage blocked reduction below; the same eigenpairs up to rounding
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("band_min", [137, 200, 2000])
def test_reductions_against_oracle(lib, band_min):
    """Cliques of 130 and 250 vertices (the 250-vertex one through the
    two-stage reduction unless band_min = 2000)."""
    inst = configs.small_block_arrow(8, n=510, block=240, arrow=10, m=12, per_row=8)
    w, _ = _iterate_parity(lib, inst, 15, band_min=band_min)
    _log(f"band_min={band_min}, cliques of 250: worst rel {w:.2e}")


@pytest.mark.parametrize("band_min", [300, 2000])
def test_maxcut_mixed_reductions(lib, band_min):
    """Max-cut G(2000, 6000): with band_min = 300 the 29 cliques above 300
    vertices take the two-stage reduction and the 18 of 137..300 the
    one-stage one in the same step; 2000 keeps the one-stage reduction for
    all."""
    w, _ = _iterate_parity(lib, configs.maxcut_random_2000(), 4, band_min=band_min)
    _log(f"max-cut, band_min={band_min}: worst rel {w:.2e}")


def test_bad_band_min_rejected(lib):
    inst = configs.small_block_arrow(0, n=12, block=3, arrow=2, m=4)
    with pytest.raises(lib.CDCSError) as e:
        lib.Solver(inst, band_min=100)
    assert e.value.code == -1
