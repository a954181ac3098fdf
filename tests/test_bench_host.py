"""Host logic of bench.py: the algorithmic work models and the traffic records.

No GPU: these check the arithmetic that turns kernel durations into roofline
fractions against hand counts, and that a counter record is used only while
the kernel source it was taken from is unchanged.
"""
import importlib.util
import json
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_tail_start(bench):
    # the last <= 136 columns go to the LDS tail; global steps in whole panels of 32
    assert bench.trd_tail_start(96) == 0
    assert bench.trd_tail_start(136) == 0
    assert bench.trd_tail_start(137) == 32
    assert bench.trd_tail_start(168) == 32
    assert bench.trd_tail_start(169) == 64
    assert bench.trd_tail_start(673) == 544


def test_symv_work_hand_count(bench):
    # one clique of 200 through the one-stage reduction: panels 0..1 (tail
    # start 64), 32 columns each
    w = bench.phase_work([200], (0, 0, 0, 1), band_min=2000)
    tot = 0.0
    for j in range(64):
        i = j % 32
        n1 = 200 - j - 1
        tot += 8.0 * (n1 * n1 + 2 * i * n1)
    assert w["trd_symv"][1] == pytest.approx(tot / 64)
    assert w["trd_symv"][0] == "hbm"
    assert w["trd_tail"][1] == pytest.approx(4.0 / 3.0 * (200 - 64) ** 3)


def test_band_work_hand_count(bench):
    # one clique of 150 through the two-stage reduction: panels 0..17
    # (band_panels = ceil(141 / 8) = 18) and the closing launch 18
    w = bench.phase_work([150], (0, 0, 0, 1), rcounts=[40])
    assert bench.band_panels(150) == 18
    pan = trail = 0.0
    for p in range(19):
        n = 150 - 8 * p
        pan += 64.0 * n * (6 + (n + 127) // 128)
        n2 = n - 8
        if n2 > 0:
            trail += 8.0 * n2 * n2 * (2 if p else 1) + 8.0 * n2 * 24
    assert w["band_panel"] == ("hbm", pytest.approx(pan / 19), "GB/s")
    assert w["band_trail"] == ("hbm", pytest.approx(trail / 18), "GB/s")   # no trail launch at p = 18
    # sweep s has ceil((149 - s) / 8) steps
    steps = sum(-(-(149 - s) // 8) for s in range(148))
    assert bench.chase_steps(150) == steps
    assert w["band_chase"][1] == pytest.approx(950.0 * steps)
    assert w["band_q2"][1] == pytest.approx(32.0 * 40 * steps)
    assert w["bt_apply"][1] == pytest.approx(4.0 * 150 * 150 * 40)
    assert "trd_symv" not in w


def test_smaller_side_counts_from_the_state(bench):
    # a fake solver whose state holds Y = s - z for one clique of 70 with
    # 20 negative eigenvalues, beside a Jacobi clique of 3
    from oracle import hsde

    class Inst:
        cliques = [list(range(3)), list(range(70))]

    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((70, 70)))
    Y = Q @ np.diag(np.r_[-np.arange(1, 21), np.arange(1, 51)].astype(float)) @ Q.T
    small = hsde.svec_blocks(np.eye(3), 3)
    yv = np.r_[small, hsde.svec_blocks(Y, 70)]
    ns = yv.size

    class Solver:
        def dims(self):
            return (2, ns, 1, 2)

        def get_state(self):
            u = np.r_[np.zeros(2), yv, np.zeros(1 + ns + 1)]
            return u, np.zeros_like(u)

    assert bench.smaller_side_counts(Solver(), Inst()) == [None, 20]


def test_affine_work_hand_count(bench):
    class Inst:
        def __init__(self, nnz):
            self.A = (None, None, None, np.zeros(nnz))
    dims = [(10, 30, 4, 2), (6, 12, 3, 1)]
    w = bench.affine_work([Inst(20), Inst(9)], dims)
    nE, ns, M, nnz = 16, 42, 7, 29
    assert w["spmv_A"] == 12 * nnz + 8 * nE + 24 * M
    assert w["spmv_At"] == 12 * nnz + 8 * M + 40 * nE
    assert w["r0_scatter"] == 28 * ns + 4 * nE + 40 * nE
    assert w["trsv"] == 8 * 4 * 5 + 8 * 3 * 4 + 16 * M
    assert w["update_x"] == 64 * nE and w["update_y"] == 40 * M


def test_traffic_record_follows_the_source_hash(bench, tmp_path, monkeypatch):
    import hashlib
    prof = tmp_path / "profiles"
    src = tmp_path / "paper_1611_01828_amd" / "csrc"
    prof.mkdir()
    src.mkdir(parents=True)
    (src / "k.hip").write_text("kernel v1")
    digest = hashlib.sha256(b"kernel v1").hexdigest()
    rec = {"kernel": "spmv_At", "bytes_per_launch": 123, "source_sha256": digest}
    (prof / "t.md").write_text("x\n<!-- traffic: " + json.dumps(rec) + " -->\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("spmv_At", "t.md", "k.hip") == 123
    assert bench.measured_traffic("spmv_A", "t.md", "k.hip") is None
    (src / "k.hip").write_text("kernel v2")
    assert bench.measured_traffic("spmv_At", "t.md", "k.hip") is None


def test_gpus_above_one_exit_with_a_message():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_auto_band_min(bench):
    """settings.band_min = 0 as the library reads it: the two-stage reduction
    only when the largest clique has at least 320 vertices."""
    assert bench.auto_band_min([673, 600, 140, 40]) == 137
    assert bench.auto_band_min([320, 5]) == 137
    assert bench.auto_band_min([319, 200]) == 1025
    assert bench.auto_band_min([147, 64, 5]) == 1025


def test_traffic_summaries_named_in_bench_exist():
    """Every counter summary bench.py reads is a committed file with a record."""
    import re
    src = open(os.path.join(ROOT, "bench.py")).read()
    names = set(re.findall(r'"(\w+_traffic\.md)"', src))
    assert names, "bench.py names no traffic summary"
    for name in names:
        path = os.path.join(ROOT, "profiles", name)
        assert os.path.exists(path), name
        assert "<!-- traffic: " in open(path).read(), name
