"""cdcs_psd_project_noalloc (device scratch in a fixed library array, no
hipMalloc) against cdcs_psd_project through the C ABI, and both against the
oracle's projection.

Two calls in a row on the same GPU, the second with a smaller input, so the
second runs on scratch the first left behind.  Bar: the conic-step bar of the
parity tests (1e-13 relative per block up to order 96, 1e-12 above) against
the oracle; the two entry points run the same kernels, so they must agree
bit for bit.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import hsde  # noqa: E402


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


def _blocks(sizes, seed):
    rng = np.random.default_rng(seed)
    parts, offs, pos = [], [], 0
    for K in sizes:
        G = rng.standard_normal((K, K))
        parts.append(hsde.svec_blocks((G + G.T) / 2, K))
        offs.append(pos)
        pos += K * (K + 1) // 2
    return np.concatenate(parts), np.asarray(offs, dtype=np.int64)


def _check(lib, torch, sizes, seed):
    vec, offs = _blocks(sizes, seed)
    want = hsde.proj_psd_packed(vec, np.asarray(sizes), offs)
    dev_in = torch.tensor(vec, dtype=torch.float64, device="cuda")
    out_plain = torch.full_like(dev_in, float("nan"))
    out_noalloc = torch.full_like(dev_in, float("nan"))
    lib.psd_project(sizes, offs, dev_in, out_plain)
    lib.psd_project_noalloc(sizes, offs, dev_in, out_noalloc)
    plain = out_plain.cpu().numpy()
    got = out_noalloc.cpu().numpy()
    assert np.array_equal(got, plain), "no-allocation entry point differs from cdcs_psd_project"
    for K, o in zip(sizes, offs):
        sl = slice(o, o + K * (K + 1) // 2)
        err = np.linalg.norm(got[sl] - want[sl]) / np.linalg.norm(vec[sl])
        assert err <= (1e-13 if K <= 96 else 1e-12), (K, err)


def test_noalloc_projection_two_calls(lib, torch_cuda):
    first = [1, 5, 16, 20, 33, 64, 97, 150, 300, 673]
    second = [3, 17, 40, 130]             # smaller, on the scratch the first call left
    _log(f"noalloc call 1 sizes={first}")
    _check(lib, torch_cuda, first, 11)
    _log(f"noalloc call 2 sizes={second}")
    _check(lib, torch_cuda, second, 12)


def test_noalloc_projection_in_place_and_jacobi_only(lib, torch_cuda):
    torch = torch_cuda
    sizes = [8, 24, 48, 64, 2]
    vec, offs = _blocks(sizes, 13)
    want = hsde.proj_psd_packed(vec, np.asarray(sizes), offs)
    dev = torch.tensor(vec, dtype=torch.float64, device="cuda")
    _log("noalloc in place, Jacobi buckets only")
    lib.psd_project_noalloc(sizes, offs, dev, dev)
    got = dev.cpu().numpy()
    for K, o in zip(sizes, offs):
        sl = slice(o, o + K * (K + 1) // 2)
        assert np.linalg.norm(got[sl] - want[sl]) <= 1e-13 * np.linalg.norm(vec[sl]), K


def test_noalloc_projection_rejects_oversize(lib, torch_cuda):
    """Two blocks of order 1024 need about 84 MB of workspace, above the 64 MiB
    scratch: refused on the host before anything is launched."""
    torch = torch_cuda
    nb = 1024 * 1025 // 2
    sizes = [1024, 1024]
    offs = [0, nb]
    dev = torch.zeros(2 * nb, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.CDCSError) as ei:
        lib.psd_project_noalloc(sizes, offs, dev, dev)
    assert ei.value.code == -1 and "scratch" in str(ei.value)
    # the entry point still works afterwards
    _check(lib, torch, [1024], 14)
