"""Fixed workloads for counter and trace runs under rocprofv3.

Runs, on cuda:0: a 64 MiB FP64 copy three times (the runtime's copy kernel,
a kernel of known traffic that calibrates FETCH_SIZE / WRITE_SIZE), then K
ADMM iterations of one workload launched kernel by kernel (no graph replay,
so that every dispatch is seen by the counters) through the C ABI.

    python -u -m paper_1611_01828_amd.profile_run --workload maxcut --iters 4

Workloads: maxcut (G(2000, 6000) max-cut relaxation, cliques up to 673),
batch (256 block-arrow SDPs in one handle), uneven (uneven cliques 4..96,
n = 5000, m = 2000); --method 1 / 2 runs the primal-only / dual-only ADMM.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["maxcut", "batch", "uneven"], default="maxcut")
    ap.add_argument("--iters", type=int, default=4)
    ap.add_argument("--no-copy", action="store_true", help="skip the 64 MiB copy calibration")
    ap.add_argument("--method", type=int, default=0, choices=[0, 1, 2],
                    help="settings.method: 0 self-dual, 1 primal-only, 2 dual-only ADMM")
    args = ap.parse_args()

    import torch
    from paper_1611_01828_amd import cdcs
    from sdpgen import configs

    if not args.no_copy:
        n = (64 << 20) // 8
        a = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        print("[profile_run] 3 copies of 64 MiB done", flush=True)
    inst = {"maxcut": configs.maxcut_random_2000, "batch": configs.block_arrow_batch256, "uneven": configs.uneven_cliques_5000}[args.workload]()
    s = cdcs.Solver(inst, method=args.method)
    s.iterate(args.iters)
    torch.cuda.synchronize()
    s.close()
    print(f"[profile_run] {args.iters} iterations of {args.workload} done", flush=True)


if __name__ == "__main__":
    main()
