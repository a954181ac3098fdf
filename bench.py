"""Throughput of the HSDE-ADMM hot path on one MI355X.

A step is one ADMM iteration (steps 1-3 of the method: affine projection,
conic projection of every clique block, dual update, residual reductions)
over the max-cut relaxation on a random graph G(2000, 6000) (C = -L,
A_i = e_i e_i^T, b = 1, minimum-degree chordal extension; cliques up to 673
vertices), with all data resident on the GPU.  The JSON line reports
ADMM iterations/s, the roofline position of the dominant kernel (timed live
with HIP events on the solver's stream), time to the 1e-4 residual (the
paper's steps, and the over-relaxed form of the same ADMM with --alpha), and
the CPU oracle timed on a bounded sample of the same workload.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-solve] [--alpha A]

By default the timed region is the paper's whole iteration budget (2000 ADMM
iterations after one warm-up), since the cost of an iteration varies along
the solve (more eigenpairs per large clique later, clustered eigenvalues).

Secondary measurements (their own JSON line, not the headline):
  --workload batch   256 block-arrow SDPs in one batched solve vs the plain
                     path run instance by instance
  --workload grad    64 block-arrow SDPs: forward solve + implicit gradient
                     vs forward only
  --workload grid    the max-cut relaxation on a periodic 40 x 50 grid
                     (n = 2000, 1499 cliques of 5..147 vertices), measured
                     like the headline
  --workload uneven  the uneven-clique SDP (n = 5000, cliques of 4..96
                     vertices, m = 2000), measured like the headline
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ADMM iters/s + time-to-1e-4 residual; batched & grad vs plain; % HBM/FP64 roofline"
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector (and matrix) peak
PEAK_HBM_GBS = 8000.0
JACOBI_MAX = 64              # cliques up to this order: Jacobi in LDS; larger: the tridiagonal path


# settings every solver of the run gets (command-line options)
SOLVER_DEFAULTS = {}


def make_solver(cdcs, instances, **settings):
    return cdcs.Solver(instances, **{**SOLVER_DEFAULTS, **settings})


def trd_tail_start(K, tail=136, nb=32):
    """First column of a clique's tridiagonalisation done in LDS by the tail kernel."""
    return ((K - tail + nb - 1) // nb) * nb if K > tail else 0


BAND = 8                     # bandwidth of the two-stage reduction's first stage
BAND_MIN = 137               # smallest clique order of the two-stage reduction when it is on
BAND_AUTO = 320              # automatic setting: on when the largest clique has at least this order


def auto_band_min(sizes):
    """settings.band_min = 0 as the library reads it: 137 when the largest
    clique has at least BAND_AUTO vertices, otherwise no clique (1025)."""
    return BAND_MIN if max(sizes) >= BAND_AUTO else 1025


def band_panels(K):
    """Panels of the dense-to-band stage of a clique of order K."""
    return (K - 9 + BAND - 1) // BAND


def chase_steps(K):
    """Bulge-chasing steps of a clique of order K (sweeps 0..K-3)."""
    return sum((K - 1 - s + BAND - 1) // BAND for s in range(K - 2))


def smaller_side_counts(solver, inst):
    """Eigenvectors each large clique's projection computed at the last
    iteration: min(#negative, #nonnegative) eigenvalues of Y = s - z (the
    argument of the last conic step: s = Pi(Y), z = s - Y), from the
    solver's state; None for the Jacobi cliques."""
    import numpy as np
    nE, ns, m, _ = solver.dims()
    u, vt = solver.get_state()
    y = u[nE:nE + ns] - vt[nE:nE + ns]
    out, off = [], 0
    for c in inst.cliques:
        K = len(c)
        blk = y[off:off + K * (K + 1) // 2]
        off += K * (K + 1) // 2
        if K <= JACOBI_MAX:
            out.append(None)
            continue
        # svec over the lower triangle, column by column, off-diagonals x sqrt(2)
        Y = np.zeros((K, K))
        rows, cols = np.tril_indices(K)
        order = np.lexsort((rows, cols))
        Y[rows[order], cols[order]] = blk
        Y = np.tril(Y, -1) / np.sqrt(2.0) + np.diag(np.diag(Y))
        Y = Y + np.tril(Y, -1).T
        nneg = int(np.sum(np.linalg.eigvalsh(Y) < 0.0))
        out.append(min(nneg, K - nneg))
    return out


def phase_work(inst_sizes, prob_dims, band_min=BAND_MIN, rcounts=None):
    """Algorithmic work of one average launch of each kernel phase.

    Returns {phase: (bound, amount, unit)}; amount is bytes for memory-bound
    phases and flops for arithmetic ones.  Cliques of band_min vertices or
    more take the two-stage reduction: per panel of 8 columns one panel
    launch (the panel's columns, V, Y, U and the column-tile partials of
    A22 U once each) and one trailing-update launch (A22 read, and written
    after the first panel), then one bulge-chasing launch (~950 flops per
    8 x 8 step) and the back-transformation of its reflectors (32 flops per
    reflector and eigenvector; rcounts: eigenvectors per clique, in clique
    order, None where unknown).  The others: one symv and one update launch
    per column step of the panels (all such cliques in lockstep, each until
    its last <= 136 columns), one trailing update per panel of 32 and one
    LDS tail launch."""
    large = sorted((k for k in inst_sizes if k > JACOBI_MAX), reverse=True)
    small = [k for k in inst_sizes if k <= JACOBI_MAX]
    band = [k for k in large if k >= band_min]
    one = [k for k in large if k < band_min]
    nE, ns, m, p = prob_dims
    out = {}
    if band:
        npm = band_panels(band[0])
        pan_b = trail_b = 0.0
        for pp in range(npm + 1):
            for K in band:
                if band_panels(K) < pp:
                    break
                n = K - BAND * pp
                nct = (n + 127) // 128
                pan_b += 8.0 * BAND * n * (6 + nct)
                n2 = n - BAND
                if n2 > 0:
                    trail_b += 8.0 * n2 * n2 * (2 if pp > 0 else 1) + 8.0 * n2 * 3 * BAND
        ntrail = sum(1 for pp in range(npm + 1) if band[0] - BAND * pp - BAND > 0)
        out["band_panel"] = ("hbm", pan_b / (npm + 1), "GB/s")
        out["band_trail"] = ("hbm", trail_b / ntrail, "GB/s")
        out["band_chase"] = ("alu", sum(950.0 * chase_steps(K) for K in band), "TFLOP/s")
        if rcounts is not None:
            rk = [r for k, r in zip(inst_sizes, rcounts) if r is not None and k >= band_min]
            kb = [k for k, r in zip(inst_sizes, rcounts) if r is not None and k >= band_min]
            out["band_q2"] = ("alu", sum(32.0 * r * chase_steps(K) for K, r in zip(kb, rk)), "TFLOP/s")
    if rcounts is not None:
        # compact-WY back-transformation: 4 K^2 r flops per clique
        out["bt_apply"] = ("alu", sum(4.0 * k * k * r for k, r in zip(inst_sizes, rcounts) if r is not None),
                           "TFLOP/s")
    if one:
        nbp = 32
        npan = trd_tail_start(one[0]) // nbp
        symv_b = upd_b = trail_f = 0.0
        for pp in range(npan):
            for K in one:
                if trd_tail_start(K) <= pp * nbp:
                    break
                n2 = K - pp * nbp - nbp
                # trailing update A22 -= V Wp^T + Wp V^T, both triangles: 4 nb flops per entry
                trail_f += 4.0 * nbp * n2 * n2
                for i in range(nbp):
                    n1 = K - (pp * nbp + i) - 1
                    # y = A22 v plus the 2i panel dots: each operand read once
                    symv_b += 8.0 * (n1 * n1 + 2 * i * n1)
                    # w and the column update: y, 2i panel entries, v, column j+1 per row; Wp, W writes
                    upd_b += 8.0 * n1 * (2 * i + 6)
        if npan:
            out["trd_symv"] = ("hbm", symv_b / (npan * nbp), "GB/s")
            out["trd_update"] = ("hbm", upd_b / (npan * nbp), "GB/s")
            out["trd_trail"] = ("alu", trail_f / npan, "TFLOP/s")
        # the last n <= 136 columns of every clique, (4/3) n^3 flops each
        out["trd_tail"] = ("alu", sum(4.0 / 3.0 * (K - trd_tail_start(K)) ** 3 for K in one), "TFLOP/s")
    # Jacobi blocks: counted with the 10 K^3 eigen-decomposition convention
    for kmax, name in ((16, "cone_jacobi16"), (32, "cone_jacobi32"), (64, "cone_jacobi64"), (96, "cone_jacobi96")):
        lo = {16: 0, 32: 16, 64: 32, 96: 64}[kmax]
        out[name] = ("alu", sum(10.0 * k ** 3 for k in small if lo < k <= kmax), "TFLOP/s")
    # scatter H^T(s+z+v): read s,z,v (3 ns doubles) + slot ids + x, c, pinv; write hsum, q
    out["r0_scatter"] = ("hbm", 8.0 * 3 * ns + 4.0 * ns + 4.0 * (nE + 1) + 8.0 * 3 * nE + 8.0 * 2 * nE, "GB/s")
    return out


def measured_traffic(kernel, summary="trd_symv_maxcut_random_2000_traffic.md", source="kernels_large.hip"):
    """HBM bytes per launch of `kernel` from a committed counter summary
    (profiles/<summary>, one `<!-- traffic: {...} -->` record per kernel), or
    None when it is missing or the kernel's source file changed since."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", summary)
    src = os.path.join(ROOT, "paper_1611_01828_amd", "csrc", source)
    try:
        text = open(path).read()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    for m in re.finditer(r"<!-- traffic: (\{.*\}) -->", text):
        rec = json.loads(m.group(1))
        if rec.get("kernel") == kernel and rec.get("source_sha256") == digest:
            return rec.get("bytes_per_launch")
    return None


def affine_work(insts, dims):
    """Algorithmic HBM bytes of one launch of each streaming phase of the
    affine step over a batch (every operand read or written once; gathers of
    vectors that stay in cache counted once).  dims: per instance (nE, ns, m, p)."""
    nE = sum(d[0] for d in dims)
    ns = sum(d[1] for d in dims)
    M = sum(d[2] for d in dims)
    nnz = sum(len(inst.A[3]) for inst in insts)
    tri = sum(8.0 * d[2] * (d[2] + 1) for d in dims)       # L for the forward sweep, L^T for the backward
    return {
        # s, z, v and the slot lists; x, c, P^-1 in; H^T(s+z+v)/2 and P^-1 r0 out
        "r0_scatter": 8.0 * 3 * ns + 4.0 * ns + 4.0 * nE + 8.0 * 3 * nE + 8.0 * 2 * nE,
        # A (value + column index), P^-1 r0 once, y and b in, g' out
        "spmv_A": 12.0 * nnz + 8.0 * nE + 8.0 * 3 * M,
        # the dense factor twice, g' in, w' out
        "trsv": tri + 8.0 * 2 * M,
        # A^T (value + row index), w' once, q, P^-1, c in; A^T w' and p_x out
        "spmv_At": 12.0 * nnz + 8.0 * M + 8.0 * 3 * nE + 8.0 * 2 * nE,
        # p_x, zt_x, A^T w', A^T zt_y, H^T(s+z+v)/2, D/2, c in; x out
        "update_x": 8.0 * 7 * nE + 8.0 * nE,
        # b, zt_y, w', y in; y out
        "update_y": 8.0 * 4 * M + 8.0 * M,
    }


def measure_peaks(torch):
    """Measured ceilings on this GPU: device-to-device copy bandwidth of a
    1 GiB tensor (HBM-resident) and of a 32 MiB tensor copied repeatedly
    (resident in the 256 MB last-level cache), read + write bytes over the
    HIP-event time; and the FP64 rate of an 8192^3 matrix product (the
    vendor BLAS), the practical FP64 ceiling."""
    def ev_time(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) * 1e-3 / reps
    out = {}
    for label, nbytes, reps in (("copy_hbm_GBs", 1 << 30, 10), ("copy_cache_GBs", 32 << 20, 200)):
        x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        out[label] = round(2 * nbytes / ev_time(lambda: y.copy_(x), reps) / 1e9, 1)
        del x, y
    n = 8192
    g = torch.Generator(device="cuda").manual_seed(0)
    a = torch.rand(n, n, dtype=torch.float64, device="cuda", generator=g)
    b = torch.rand(n, n, dtype=torch.float64, device="cuda", generator=g)
    c = torch.empty_like(a)
    out["dgemm_TFLOPs"] = round(2 * n ** 3 / ev_time(lambda: torch.matmul(a, b, out=c), 3) / 1e12, 2)
    del a, b, c
    torch.cuda.empty_cache()
    print(f"[bench] measured peaks: {out}", file=sys.stderr, flush=True)
    return out


def timed_solve(cdcs, torch, inst, label, **settings):
    """Wall time of a fresh cdcs_solve (graph replay, status read every 10 iterations)."""
    import threading
    fresh = make_solver(cdcs, inst, check_every=10, use_graph=1, **settings)
    torch.cuda.synchronize()
    box = {}
    t0 = time.perf_counter()
    th = threading.Thread(target=lambda: box.setdefault("info", fresh.solve()[0]))
    th.start()
    while th.is_alive():          # the library call releases the GIL; report progress
        th.join(timeout=15.0)
        if th.is_alive():
            print(f"[bench] {label}... {time.perf_counter() - t0:.0f}s", file=sys.stderr, flush=True)
    tsolve = time.perf_counter() - t0
    info = box["info"]
    fresh.close()
    out = {"seconds": round(tsolve, 3), "iterations": info["iter"],
           "status": cdcs.STATUS_NAMES[info["status"]], "obj_p": info["obj_p"], "obj_d": info["obj_d"],
           "eps_p": info["eps_p"], "eps_d": info["eps_d"], "eps_g": info["eps_g"]}
    print(f"[bench] {label}: {out}", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed iterations (default: 2000 for maxcut, the paper's iteration limit, "
                         "whose cost per iteration varies along the solve; 20 otherwise)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed iterations first (default 1; 3 otherwise)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-1e-4 solve")
    ap.add_argument("--cpu-iters", type=int, default=None, help="oracle iterations timed (default 10; 30 for grid)")
    ap.add_argument("--eig-warm", type=int, default=0, choices=[0, 1],
                    help="warm-start the Jacobi eigen-decompositions (settings.eig_warm)")
    ap.add_argument("--alpha", type=float, default=1.8,
                    help="relaxation of the second solve (1 = skip it; the value is always alpha = 1)")
    ap.add_argument("--workload", choices=["maxcut", "batch", "grad", "grid", "uneven"], default="maxcut")
    ap.add_argument("--method", choices=["self_dual", "primal", "dual"], default="self_dual",
                    help="secondary lines only: the primal-only or dual-only ADMM (settings.method) in place of "
                         "the self-dual method (the headline line always measures the self-dual method)")
    ap.add_argument("--jacobi-max", type=int, default=0, choices=[0, 16, 32, 64],
                    help="largest clique order the Jacobi kernels take (settings.jacobi_max; 0 = automatic: "
                         "32, or 64 with the FP32 or warm-started Jacobi variants)")
    ap.add_argument("--band-min", type=int, default=0,
                    help="smallest clique order of the two-stage tridiagonalisation (settings.band_min; 0 = automatic: "
                         "137 when the largest clique has at least 320 vertices, otherwise none; above 1024 = the "
                         "one-stage reduction for every clique)")
    ap.add_argument("--no-extra", action="store_true",
                    help="leave out the compact batched and differentiated figures of the default line")
    args = ap.parse_args()
    if args.jacobi_max:
        SOLVER_DEFAULTS["jacobi_max"] = args.jacobi_max
    if args.band_min:
        SOLVER_DEFAULTS["band_min"] = args.band_min
    split = args.method != "self_dual"
    if split:
        if args.workload not in ("grid", "uneven") and not (args.workload == "maxcut" and args.no_extra):
            print("--method primal|dual measures a secondary line: use --workload grid|uneven, or maxcut with "
                  "--no-extra", file=sys.stderr)
            sys.exit(2)
        SOLVER_DEFAULTS["method"] = {"primal": 1, "dual": 2}[args.method]
        args.alpha = 1.0        # the relaxed form belongs to the self-dual method
    whole = args.workload in ("maxcut", "grid", "uneven")
    if args.steps is None:
        args.steps = 2000 if whole else 20
    if args.warmup is None:
        args.warmup = 1 if whole else 3
    if args.cpu_iters is None:
        args.cpu_iters = 30 if args.workload == "grid" else 10
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              f"(independent instances shard across GPUs without exchange)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    from paper_1611_01828_amd import cdcs
    from sdpgen import configs

    if args.workload == "batch":
        return bench_batch(args, cdcs, configs)
    if args.workload == "grad":
        return bench_grad(args, cdcs, configs)

    grid = args.workload in ("grid", "uneven")   # secondary single-SDP workloads (no extra objects)
    t0 = time.perf_counter()
    if args.workload == "grid":
        inst = configs.grid_maxcut(1)
    elif args.workload == "uneven":
        inst = configs.uneven_cliques_5000()
    else:
        inst = configs.maxcut_random_2000()
    gen_s = time.perf_counter() - t0
    sizes = [len(c) for c in inst.cliques]
    print(f"[bench] workload: {inst.name}, p={len(sizes)}, max clique {max(sizes)}, "
          f"generation {gen_s:.1f}s", file=sys.stderr, flush=True)

    # timed region: the iteration replayed from a captured HIP graph
    t0 = time.perf_counter()
    ew = args.eig_warm
    solver = make_solver(cdcs, inst, use_graph=1, eig_warm=ew)
    setup_s = time.perf_counter() - t0
    dims = solver.dims()
    print(f"[bench] setup {setup_s:.2f}s dims(nE, ns, m, p)={dims}", file=sys.stderr, flush=True)
    solver.iterate(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    left = args.steps
    while left > 0:                   # chunks of 500, with a progress line between them
        n = min(500, left)
        solver.iterate(n)
        left -= n
        if left:
            print(f"[bench] timed: {args.steps - left} iterations, {time.perf_counter() - t0:.1f}s",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    its = args.steps / dt
    print(f"[bench] {args.steps} iterations in {dt:.3f}s -> {its:.1f} it/s (graph replay)", file=sys.stderr, flush=True)
    solver.close()

    # per-kernel times: the first min(K, 200) of the same iterations launched
    # one by one with a HIP event pair around every launch on its stream
    ev_steps = min(args.steps, 200)
    timed = make_solver(cdcs, inst, timing=1, eig_warm=ew)
    timed.iterate(args.warmup)
    timed.reset_phase_times()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    timed.iterate(ev_steps)
    torch.cuda.synchronize()
    dt_ev = time.perf_counter() - t0
    phases = timed.phase_times()
    # eigenvectors each large clique's projection computed in the last timed
    # iteration (the back-transformations' work scales with them)
    rcounts = smaller_side_counts(timed, inst) if args.method == "self_dual" else None
    print(f"[bench] eigenvectors of the large cliques at the last event-timed iteration: "
          f"{sum(r for r in (rcounts or []) if r is not None)}", file=sys.stderr, flush=True)
    timed.close()
    print(f"[bench] event-timed pass ({ev_steps} iterations): {1e3 * dt_ev / ev_steps:.2f} ms/iteration",
          file=sys.stderr, flush=True)

    # dominant kernel and its roofline position (per-launch averages from HIP events)
    per_launch = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in phases.items()}
    dom = max(phases, key=lambda k: phases[k][0])
    work = phase_work(sizes, dims, band_min=args.band_min or auto_band_min(sizes), rcounts=rcounts)
    roof = None
    if dom in work:
        bound, amount, unit = work[dom]
        sec = per_launch[dom] * 1e-3
        if unit == "TFLOP/s":
            ach = amount / sec / 1e12
            peak = PEAK_FP64_TFLOPS
        else:
            ach = amount / sec / 1e9
            peak = PEAK_HBM_GBS
        roof = {"kernel": dom, "bound": bound, "achieved": round(ach, 4), "peak": peak, "unit": unit,
                # counter traffic is recorded for the random-graph workload only
                "frac": round(ach / peak, 6),
                "traffic": None if grid else measured_traffic(
                    dom, summary=("band_panel_maxcut_random_2000_traffic.md" if dom.startswith("band_")
                                  else "trd_symv_maxcut_random_2000_traffic.md")),
                "work_per_launch": amount, "avg_launch_ms": round(per_launch[dom], 5),
                "launches_per_step": phases[dom][1] / ev_steps,
                "ms_per_step_in_kernel": round(phases[dom][0] / ev_steps, 4)}

    peaks = measure_peaks(torch)
    if roof is not None:
        ref = peaks["copy_hbm_GBs"] if roof["unit"] == "GB/s" else peaks["dgemm_TFLOPs"]
        roof["frac_vs_measured"] = round(roof["achieved"] / ref, 6)

    tol = tol_relaxed = None
    if not args.no_solve:
        tol = timed_solve(cdcs, torch, inst, "solve", eig_warm=ew)
        tol["setup_s"] = round(setup_s, 3)
        if args.alpha != 1.0:
            # the over-relaxed form of the same ADMM: its cost per iteration
            # (graph replay, as the value) and its time to the tolerance
            rs = make_solver(cdcs, inst, use_graph=1, alpha=args.alpha, eig_warm=ew)
            rs.iterate(args.warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rs.iterate(args.steps)
            torch.cuda.synchronize()
            rit = args.steps / (time.perf_counter() - t0)
            rs.close()
            tol_relaxed = timed_solve(cdcs, torch, inst, f"relaxed solve (alpha {args.alpha})", alpha=args.alpha,
                                      eig_warm=ew)
            tol_relaxed = {"alpha": args.alpha, "iter_per_s": round(rit, 3), **tol_relaxed}

    cpu = None
    if not args.no_cpu:
        from oracle import hsde, split as osplit
        prob = hsde.build_problem(inst)
        csz = hsde.clique_sizes(prob)
        if split:
            scache = osplit.SplitCache(prob)

            def sample():
                st = osplit.initial_state(prob)
                for _ in range(args.cpu_iters):
                    st, _ = osplit.iterate(prob, scache, st, args.method, csz)
        else:
            cache = hsde.AffineCache(prob)

            def sample():
                u, vt = hsde.initial_point(prob)
                for _ in range(args.cpu_iters):
                    u, vt = hsde.iterate(prob, cache, u, vt, csz)
        t0 = time.perf_counter()
        sample()
        cdt = time.perf_counter() - t0
        cores = len(os.sched_getaffinity(0))
        # the same sample with the BLAS/LAPACK pools limited to one thread
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            sample()
            cdt1 = time.perf_counter() - t0
        cpu = {"value": round(args.cpu_iters / cdt, 5), "unit": "iter/s", "cores": cores, "kind": "oracle",
               "sample": f"{args.cpu_iters} ADMM iterations of the same workload from the initial point "
                         f"(FP64 NumPy/SciPy, LAPACK eigh per clique batched by size, setup excluded)",
               "seconds": round(cdt, 2),
               "one_thread": {"value": round(args.cpu_iters / cdt1, 5), "cores": 1, "seconds": round(cdt1, 2)}}
        print(f"[bench] cpu oracle: {cpu}", file=sys.stderr, flush=True)

    extra = {}
    if not grid and not args.no_extra:
        extra["batch"] = batch_summary(cdcs, configs, torch)
        extra["grad"] = grad_summary(cdcs, configs, torch)

    out = {
        "metric": METRIC if not (grid or split) else
                  f"ADMM iters/s + time-to-1e-4 residual ({args.workload} workload, {args.method} method)",
        "value": round(its, 3),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ("max-cut relaxation, periodic 40x50 grid (n=2000), C=-L, A_i=e_i e_i^T, b=1, "
                                "min-degree chordal extension") if args.workload == "grid" else
                               ("uneven-clique SDP: clique-tree growth, n=5000, cliques of 4-96 vertices, m=2000 "
                                "constraints of 8 entries, strictly feasible") if args.workload == "uneven" else
                               ("max-cut relaxation, G(n=2000, M=6000) random graph, C=-L, A_i=e_i e_i^T, b=1, "
                                "min-degree chordal extension"),
                   "n": inst.n, "m": inst.m, "cliques": len(sizes), "max_clique": max(sizes),
                   "nE": dims[0], "ns": dims[1], "eps_tol": 1e-4, "eig_warm": ew,
                   "jacobi_max": args.jacobi_max or ("64" if ew else "32 (automatic)"), "band_min": args.band_min or ("137 (automatic)" if auto_band_min(sizes) == BAND_MIN else "off (automatic)"),
                   "method": args.method},
        "roofline": roof,
        "measured_peaks": peaks,
        "cpu_baseline": cpu,
        "time_to_1e-4": tol,
        "time_to_1e-4_relaxed": tol_relaxed,
        "phases_ms_per_step": {k: round(v[0] / ev_steps, 4) for k, v in phases.items() if v[1]},
        "event_timed_ms_per_step": round(1e3 * dt_ev / ev_steps, 4),
        "event_timed_steps": ev_steps,
        **extra,
    }
    print(json.dumps(out))


def _status_counts(cdcs, infos):
    st = {}
    for x in infos:
        k = cdcs.STATUS_NAMES[x["status"]]
        st[k] = st.get(k, 0) + 1
    return st


def batch_summary(cdcs, configs, torch, steps=200, warmup=3):
    """Compact figures of the 256-SDP batched workload for the default line:
    instance-iterations/s of one batched handle (graph replay) against the
    plain path (one handle per instance, a sample of 16), and the time until
    every instance has stopped at eps_tol = 1e-4, in FP64 and with FP32
    Jacobi eigensolves."""
    insts = configs.block_arrow_batch256()

    def rate(solver, count):
        solver.iterate(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.iterate(steps)
        torch.cuda.synchronize()
        return count * steps / (time.perf_counter() - t0)

    out = {"workload": "256 block-arrow SDPs, n ~ U{50..400}, block ~ U{4..32}, arrow ~ U{2..8}, m = n/2",
           "unit": "instance-iter/s", "steps": steps}
    for label, settings in (("fp64", {}), ("fp32_eig", {"eig_fp32": 1})):
        s = make_solver(cdcs, insts, use_graph=1, **settings)
        r = rate(s, len(insts))
        s.close()
        f = make_solver(cdcs, insts, check_every=10, use_graph=1, **settings)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = f.solve()
        tsolve = time.perf_counter() - t0
        f.close()
        out[label] = {"value": round(r, 1), "ms_per_batch_iteration": round(1e3 * len(insts) / r, 4),
                      "time_to_1e-4": {"seconds": round(tsolve, 3), "max_iterations": max(x["iter"] for x in infos),
                                       "status_counts": _status_counts(cdcs, infos)}}
        print(f"[bench] batch {label}: {r:.0f} instance-iterations/s, all stopped in {tsolve:.2f}s", file=sys.stderr,
              flush=True)
    plain_t, sample = 0.0, insts[::16]
    for inst in sample:
        p = make_solver(cdcs, inst, use_graph=1)
        plain_t += steps / rate(p, 1)           # seconds for this instance's steps
        p.close()
    plain = len(sample) * steps / plain_t
    out["plain_value"] = round(plain, 1)
    out["speedup_vs_plain"] = round(out["fp64"]["value"] / plain, 2)
    print(f"[bench] batch plain per instance: {plain:.0f} instance-iterations/s", file=sys.stderr, flush=True)
    # the gather/scatter/solve phases of the affine step against the HBM
    # roofline: algorithmic bytes (affine_work) over the average launch
    # duration from HIP events on the launch stream, 20 iterations
    tm = make_solver(cdcs, insts, timing=1)
    tm.iterate(warmup)
    tm.reset_phase_times()
    tm.iterate(20)
    torch.cuda.synchronize()
    phases = tm.phase_times()
    dims = [tm.dims(i) for i in range(len(insts))]
    tm.close()
    aff = {}
    for name, nbytes in affine_work(insts, dims).items():
        ms, n = phases.get(name, (0.0, 0))
        if n:
            gbs = nbytes / (ms / n * 1e-3) / 1e9
            aff[name] = {"achieved": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4), "bytes_per_launch": nbytes,
                         "avg_launch_ms": round(ms / n, 5)}
    out["roofline_affine"] = {"bound": "hbm", "peak": PEAK_HBM_GBS, "unit": "GB/s", "kernels": aff}
    print(f"[bench] batch affine phases: {aff}", file=sys.stderr, flush=True)
    return out


def grad_loss_weights(cdcs, insts):
    """svec(W) over each instance's E' (W is drawn on the lower pattern entries)."""
    import numpy as np
    s = make_solver(cdcs, insts[:1])
    rows, cols = s.entries(0)
    s.close()
    out = []
    for inst in insts:
        wr, wc, wv = inst.meta["W"]
        key = {(int(r), int(c)): e for e, (r, c) in enumerate(zip(rows, cols))}
        v = np.zeros(len(rows))
        for r, c, x in zip(wr, wc, wv):
            v[key[(int(r), int(c))]] = x * (1.0 if r == c else np.sqrt(2.0))
        out.append(v)
    return np.concatenate(out)


def grad_summary(cdcs, configs, torch):
    """Compact figures of the differentiated 64-SDP batch for the default line:
    forward solve (eps_tol = 1e-4) + implicit gradient per second against the
    forward solve alone, and the adjoint's operator applications."""
    insts = configs.block_arrow_grad64()
    dX = grad_loss_weights(cdcs, insts)      # every instance has the same pattern
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f = make_solver(cdcs, insts, check_every=10, use_graph=1)
    infos = f.solve()
    tf = time.perf_counter() - t0
    t0 = time.perf_counter()
    dc, db, it = f.adjoint(dX, max_iter=20000, tol=1e-10)
    tb = time.perf_counter() - t0
    f.close()
    out = {"workload": "64 block-arrow SDPs, n=200, block 16, arrow 4, m=100; loss <W, X*>",
           "unit": "batches/s", "value": round(1.0 / (tf + tb), 4), "forward_only": round(1.0 / tf, 4),
           "forward_s": round(tf, 3), "backward_s": round(tb, 3), "adjoint_applications": it,
           "forward_iterations_max": max(x["iter"] for x in infos), "status_counts": _status_counts(cdcs, infos)}
    print(f"[bench] grad: forward {tf:.3f}s backward {tb:.3f}s ({it} applications)", file=sys.stderr, flush=True)
    return out


def bench_batch(args, cdcs, configs):
    """256 block-arrow SDPs: one batched handle for all instances vs one handle per instance;
    FP64 with the default and the autotuned Jacobi tiles, the FP32-eigensolve
    variant with its errors against FP64, and the warm-started Jacobi (FP64 and
    FP32)."""
    import numpy as np
    import torch
    t0 = time.perf_counter()
    insts = configs.block_arrow_batch256()
    print(f"[bench] 256 block-arrow instances generated in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)

    def run(label, **settings):
        t0 = time.perf_counter()
        s = make_solver(cdcs, insts, use_graph=1, **settings)
        setup = time.perf_counter() - t0
        s.iterate(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.iterate(args.steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tuning = s.tuning()
        s.close()
        f = make_solver(cdcs, insts, check_every=10, use_graph=1, **settings)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = f.solve()
        tsolve = time.perf_counter() - t0
        f.close()
        st = {}
        for x in infos:
            st[cdcs.STATUS_NAMES[x["status"]]] = st.get(cdcs.STATUS_NAMES[x["status"]], 0) + 1
        rate = len(insts) * args.steps / dt
        print(f"[bench] {label}: {rate:.0f} instance-iterations/s, solve {tsolve:.2f}s {st}", file=sys.stderr,
              flush=True)
        return {"value": round(rate, 1), "ms_per_step": round(1e3 * dt / args.steps, 4), "setup_s": round(setup, 2),
                "time_to_1e-4": {"seconds": round(tsolve, 3), "max_iterations": max(x["iter"] for x in infos),
                                 "status_counts": st},
                "tuning": [{"kmax": b["kmax"], "threads": b["threads"], "cliques": b["cliques"]} for b in tuning]}, infos

    fp64, inf64 = run("FP64, default tiles")
    tuned, _ = run("FP64, autotuned tiles", autotune=1)
    fp32, inf32 = run("FP32 eigensolves, autotuned tiles", eig_fp32=1, autotune=1)
    # warm-started Jacobi: the same projections (to rounding), fewer sweeps
    warm, infw = run("FP64, warm-started Jacobi", eig_warm=1)
    warm["iterations_vs_fp64"] = {"max_abs_delta": int(max(abs(infw[i]["iter"] - inf64[i]["iter"]) for i in range(len(insts)))),
                                  "obj_rel_max": float(max(abs(infw[i]["obj_p"] - inf64[i]["obj_p"]) /
                                                           max(1.0, abs(inf64[i]["obj_p"])) for i in range(len(insts))))}
    warm32, _ = run("FP32 eigensolves, warm-started Jacobi", eig_fp32=1, eig_warm=1)
    # FP32 against FP64 on every instance that both solved
    both = [i for i in range(len(insts)) if inf64[i]["status"] == cdcs.SOLVED and inf32[i]["status"] == cdcs.SOLVED]
    rel = [abs(inf32[i]["obj_p"] - inf64[i]["obj_p"]) / max(1.0, abs(inf64[i]["obj_p"])) for i in both]
    dit = [inf32[i]["iter"] - inf64[i]["iter"] for i in both]
    fp32["vs_fp64"] = {"instances": len(both), "obj_rel_max": float(max(rel)), "obj_rel_median": float(np.median(rel)),
                       "iter_delta_mean": float(np.mean(dit)), "iter_delta_max_abs": int(max(abs(d) for d in dit)),
                       "eps_p_max": float(max(inf32[i]["eps_p"] for i in both)),
                       "eps_d_max": float(max(inf32[i]["eps_d"] for i in both))}
    # and against the FP64 oracle on the two smallest instances
    from oracle import hsde
    small = sorted(range(len(insts)), key=lambda i: insts[i].n)[:2]
    orc = []
    for i in small:
        ref = hsde.solve(insts[i])
        o = hsde.recover(ref)["obj_p"] if ref.status == hsde.SOLVED else float("nan")
        orc.append({"instance": i, "n": insts[i].n, "oracle_iters": ref.iters, "fp32_iters": inf32[i]["iter"],
                    "fp64_iters": inf64[i]["iter"], "obj_rel_fp32_vs_oracle": abs(inf32[i]["obj_p"] - o) / max(1.0, abs(o)),
                    "obj_rel_fp64_vs_oracle": abs(inf64[i]["obj_p"] - o) / max(1.0, abs(o))})
    fp32["vs_oracle"] = orc
    print(f"[bench] FP32 vs FP64: {fp32['vs_fp64']}; vs oracle: {orc}", file=sys.stderr, flush=True)
    # plain path: a sample of instances, one handle each, same number of steps
    sample = insts[::16]
    plain_t = 0.0
    for inst in sample:
        p = make_solver(cdcs, inst, use_graph=1)
        p.iterate(args.warmup)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        p.iterate(args.steps)
        torch.cuda.synchronize()
        plain_t += time.perf_counter() - t1
        p.close()
    plain = len(sample) * args.steps / plain_t
    print(f"[bench] plain per instance: {plain:.0f} instance-iterations/s", file=sys.stderr, flush=True)
    # the streaming phases of the affine step against the HBM roofline
    # (per-launch durations from HIP events on the launch stream)
    tm = make_solver(cdcs, insts, timing=1)
    tm.iterate(args.warmup)
    tm.reset_phase_times()
    tm.iterate(args.steps)
    torch.cuda.synchronize()
    phases = tm.phase_times()
    dims = [tm.dims(i) for i in range(len(insts))]
    tm.close()
    work = affine_work(insts, dims)
    affine = []
    for name, nbytes in work.items():
        ms, n = phases.get(name, (0.0, 0))
        if not n:
            continue
        gbs = nbytes / (ms / n * 1e-3) / 1e9
        affine.append({"kernel": name, "bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                       "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4), "bytes_per_launch": nbytes,
                       "avg_launch_ms": round(ms / n, 5),
                       "traffic": measured_traffic(name, "affine_block_arrow_batch256_traffic.md", "kernels_iter.hip")})
    peaks = measure_peaks(torch)
    for e in affine:
        e["frac_vs_measured"] = round(e["achieved"] / peaks["copy_hbm_GBs"], 4)
    print(f"[bench] affine-step phases: {affine}", file=sys.stderr, flush=True)
    out = {"metric": "batched instance-iterations/s (256 block-arrow SDPs)", "value": fp64["value"],
           "unit": "instance-iter/s", "plain_value": round(plain, 1),
           "speedup_vs_plain": round(fp64["value"] / plain, 2), "steps": args.steps, "dtype": "f64",
           "fp64": fp64, "fp64_autotuned": tuned, "fp32_eig_autotuned": fp32,
           "fp64_warm_jacobi": warm, "fp32_eig_warm_jacobi": warm32,
           "roofline_affine": affine, "measured_peaks": peaks,
           "phases_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in phases.items() if v[1]}}
    print(json.dumps(out))


def bench_grad(args, cdcs, configs):
    """64 block-arrow SDPs: forward (solve) + backward (implicit adjoint) vs forward only."""
    import numpy as np
    import torch
    insts = configs.block_arrow_grad64()
    W = np.concatenate([i.meta["W"][2] for i in insts])
    # W is drawn on the lower pattern entries; map to svec over each instance's E'
    s = make_solver(cdcs, insts, check_every=10)
    dX = []
    for i, inst in enumerate(insts):
        rows, cols = s.entries(i)
        wr, wc, wv = inst.meta["W"]
        key = {(int(r), int(c)): e for e, (r, c) in enumerate(zip(rows, cols))}
        v = np.zeros(len(rows))
        for r, c, x in zip(wr, wc, wv):
            v[key[(int(r), int(c))]] = x * (1.0 if r == c else np.sqrt(2.0))
        dX.append(v)
    dX = np.concatenate(dX)
    s.close()

    def run(**settings):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = make_solver(cdcs, insts, check_every=10, use_graph=1, **settings)
        infos = f.solve()
        tf = time.perf_counter() - t0
        t0 = time.perf_counter()
        dc, db, it = f.adjoint(dX, max_iter=20000, tol=1e-10)
        tb = time.perf_counter() - t0
        f.close()
        return infos, tf, tb, dc, db, it

    infos, tf, tb, dc, db, it = run()
    nsolved = sum(1 for x in infos if x["status"] == cdcs.SOLVED)
    print(f"[bench] FP64: forward {tf:.3f}s backward {tb:.3f}s ({it} GMRES applications)", file=sys.stderr,
          flush=True)
    # FP32-eigensolve forward (the adjoint's eigen-cache stays FP64)
    inf32, tf32, tb32, dc32, db32, it32 = run(eig_fp32=1)
    fp32 = {"forward_s": round(tf32, 3), "backward_s": round(tb32, 3), "adjoint_iterations": it32,
            "solved": sum(1 for x in inf32 if x["status"] == cdcs.SOLVED),
            "grad_c_rel_vs_fp64": float(np.linalg.norm(dc32 - dc) / np.linalg.norm(dc)),
            "grad_b_rel_vs_fp64": float(np.linalg.norm(db32 - db) / np.linalg.norm(db)),
            "value": round(1.0 / (tf32 + tb32), 4)}
    print(f"[bench] FP32 eig forward: {fp32}", file=sys.stderr, flush=True)
    out = {"metric": "differentiated batch (64 SDPs): forward+backward per second vs forward only",
           "value": round(1.0 / (tf + tb), 4), "unit": "batches/s", "forward_only": round(1.0 / tf, 4),
           "forward_s": round(tf, 3), "backward_s": round(tb, 3), "adjoint_iterations": it,
           "forward_iterations_max": max(x["iter"] for x in infos), "solved": nsolved, "dtype": "f64",
           "grad_norm_c": float(np.linalg.norm(dc)), "grad_norm_b": float(np.linalg.norm(db)),
           "fp32_eig_forward": fp32}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
