"""The library's host factorisation of the m x m matrix of step 1 (K = shift I +
A P^{-1} A^T, eqs. ThirdBlkElm / FactorizationMatrix after the matrix
inversion lemma; shift 0 for the primal-only / dual-only methods), compiled
with g++ from its source together with a small driver (tests/host/), against
the definition of K on random sparse data: dense form for a small dense K,
sparse form for a sparse K summed densely (m <= 8192) and for one assembled
from its nonzero terms (m > 8192).  No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ is not available")
    out = str(tmp_path_factory.mktemp("factor") / "factor_check")
    src = [os.path.join(ROOT, "tests", "host", "factor_check.cpp"),
           os.path.join(ROOT, "paper_1611_01828_amd", "csrc", "setup.cpp")]
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), *src, "-o", out], check=True)
    return out


@pytest.mark.parametrize("m,nE,per_row,shift,form", [
    (60, 200, 40, 1.0, "dense"),
    (3000, 60000, 4, 1.0, "sparse"),
    (12000, 60000, 3, 1.0, "sparse"),
    (12000, 60000, 3, 0.0, "sparse"),
])
def test_factor_solves_the_defined_matrix(driver, m, nE, per_row, shift, form):
    r = subprocess.run([driver, str(m), str(nE), str(per_row), str(shift), "7"], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    kind, err = r.stdout.split()
    assert kind == form
    assert float(err) <= 1e-10, r.stdout
