"""Seeded synthetic SDP instances shaped like the paper's workloads.

The paper measures on SDPLIB (Section 5, Table 1), which is not available
here; these generators stand in for it with the shapes its tables describe
(a theta1-sized block-arrow problem, a maxG32-shaped max-cut relaxation, an
infeasible problem like infp1) plus the batched and differentiated sets.

Every instance is a plain data record:
    n, m            order of X and number of equality constraints
    C               (rows, cols, vals) lower-triangular COO (row >= col)
    A               (con, rows, cols, vals) lower-triangular COO per constraint
    b               float64[m]
    cliques         list of sorted int arrays (natural vertex order)
    parent          int array, clique-tree parent (-1 = root)

Entries are matrix values, not scaled; off-diagonal (i, j) stands for both
X_ij and X_ji.  This module draws random numbers and builds patterns; it
holds none of the solver's arithmetic.

Seeds: numpy default_rng(SeedSequence([161101828, stream, instance])), one
stream number per workload generator.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import chordal

SEED_ROOT = 161101828


@dataclass
class SDPInstance:
    n: int
    m: int
    C: tuple
    A: tuple
    b: np.ndarray
    cliques: List[np.ndarray]
    parent: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)


def rng_for(stream: int, instance: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, stream, instance]))


# ----------------------------------------------------------------------------
# pattern helpers
# ----------------------------------------------------------------------------

def pattern_entries(cliques):
    """Sorted lower-triangular entries (row >= col) of the union of C_k x C_k.

    Sorted by column, then row (column-major order of the lower triangle).
    """
    keys = set()
    for c in cliques:
        c = np.asarray(c, dtype=np.int64)
        a, bb = np.tril_indices(len(c))
        r = c[a]
        q = c[bb]
        lo = np.minimum(r, q)
        hi = np.maximum(r, q)
        keys.update(zip(lo.tolist(), hi.tolist()))
    arr = np.array(sorted(keys), dtype=np.int64).reshape(-1, 2)
    # arr[:,0] = col, arr[:,1] = row
    return arr[:, 1].copy(), arr[:, 0].copy()


def _clique_psd_sum(rng, n, cliques, keys):
    """Sum_k E_k^T W_k E_k with W_k = G G^T / |C_k| (Wishart), on the sorted
    lower-triangular entry keys (row * n + col) of the pattern."""
    out = np.zeros(len(keys))
    for c in cliques:
        c = np.asarray(c, dtype=np.int64)
        k = len(c)
        G = rng.standard_normal((k, k))
        W = G @ G.T / k
        a, bb = np.tril_indices(k)
        r = np.maximum(c[a], c[bb])
        q = np.minimum(c[a], c[bb])
        pos = np.searchsorted(keys, r * n + q)
        np.add.at(out, pos, W[a, bb])
    return out


def _random_constraints(rng, m, er, ec, per_row):
    """m constraints, each N(0,1) on `per_row` distinct pattern entries."""
    nE = len(er)
    con, rr, cc, vv = [], [], [], []
    for i in range(m):
        pick = np.sort(rng.choice(nE, size=per_row, replace=False))
        con.append(np.full(per_row, i, dtype=np.int32))
        rr.append(er[pick])
        cc.append(ec[pick])
        vv.append(rng.standard_normal(per_row))
    return (np.concatenate(con).astype(np.int32), np.concatenate(rr).astype(np.int32),
            np.concatenate(cc).astype(np.int32), np.concatenate(vv).astype(np.float64))


def _apply_constraints(n, A, keys, xval):
    """<A_i, X> for symmetric X given on the lower pattern entries
    (off-diagonals count twice)."""
    con, r, c, v = A
    w = np.where(r == c, 1.0, 2.0)
    m = int(con.max()) + 1 if len(con) else 0
    pos = np.searchsorted(keys, r.astype(np.int64) * n + c)
    out = np.zeros(m)
    np.add.at(out, con, w * v * xval[pos])
    return out


def _feasible_data(rng, n, m, cliques, A):
    """b = A(X0), C = Z0 + sum_i y0_i A_i with X0, Z0 clique-PSD sums (strictly feasible)."""
    er, ec = pattern_entries(cliques)
    keys = er.astype(np.int64) * n + ec
    order = np.argsort(keys)
    keys_s = keys[order]
    X0 = _clique_psd_sum(rng, n, cliques, keys_s)
    b = _apply_constraints(n, A, keys_s, X0)
    y0 = rng.standard_normal(m)
    Z0 = _clique_psd_sum(rng, n, cliques, keys_s)
    con, r, c, v = A
    Cv = Z0.copy()
    pos = np.searchsorted(keys_s, r.astype(np.int64) * n + c)
    np.add.at(Cv, pos, y0[con] * v)
    rows = (keys_s // n).astype(np.int32)
    cols = (keys_s % n).astype(np.int32)
    keep = Cv != 0.0
    C = (rows[keep], cols[keep], Cv[keep])
    return b, C, dict(X0=(rows, cols, X0), Z0=(rows, cols, Z0), y0=y0)


def block_arrow_cliques(n, block, arrow):
    """Diagonal blocks of size `block` over vertices 0..n-arrow-1 (the last
    block takes the remainder) plus an arrow of the last `arrow` vertices
    adjacent to everything.  Natural order is a perfect elimination order."""
    body = n - arrow
    arrow_v = np.arange(body, n)
    cl = []
    start = 0
    while start < body:
        end = min(start + block, body)
        cl.append(np.concatenate([np.arange(start, end), arrow_v]).astype(np.int64))
        start = end
    p = len(cl)
    parent = np.array([k + 1 if k + 1 < p else -1 for k in range(p)], dtype=np.int64)
    return cl, parent


def block_arrow_instance(stream, instance, n, block, arrow, m, density=0.3, per_row=None):
    """Block-arrow SDP; each A_i has `per_row` N(0,1) entries (default: a
    fraction `density` of the pattern), made strictly feasible."""
    rng = rng_for(stream, instance)
    cliques, parent = block_arrow_cliques(n, block, arrow)
    er, ec = pattern_entries(cliques)
    if per_row is None:
        per_row = int(np.floor(density * len(er) + 0.5))
    A = _random_constraints(rng, m, er, ec, per_row)
    b, C, meta = _feasible_data(rng, n, m, cliques, A)
    meta.update(block=block, arrow=arrow)
    return SDPInstance(n, m, C, A, b, cliques, parent,
                       name=f"block-arrow n={n} b={block} a={arrow} m={m}", meta=meta)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def block_arrow_n50():
    """Plain block-arrow SDP: n=50, 5 blocks of 9 + arrow 5, cliques of 14, m=20."""
    return block_arrow_instance(0, 0, n=50, block=9, arrow=5, m=20)


def maxcut_instance(stream, instance, n, n_edges):
    """min <-L, X> s.t. X_ii = 1 on a uniform random graph G(n, M)."""
    rng = rng_for(stream, instance)
    edges = set()
    while len(edges) < n_edges:
        need = n_edges - len(edges)
        i = rng.integers(0, n, size=2 * need)
        j = rng.integers(0, n, size=2 * need)
        for a, bb in zip(i.tolist(), j.tolist()):
            if a == bb:
                continue
            e = (max(a, bb), min(a, bb))
            if e not in edges:
                edges.add(e)
                if len(edges) == n_edges:
                    break
    return maxcut_from_edges(n, sorted(edges), name=f"max-cut G(n={n}, M={n_edges})")


def maxcut_from_edges(n, edges, name="max-cut"):
    edges = [(max(int(a), int(b)), min(int(a), int(b))) for a, b in edges]
    deg = np.zeros(n)
    for i, j in edges:
        deg[i] += 1
        deg[j] += 1
    # C = -L = A_graph - Deg  (unit weights)
    rows = list(range(n)) + [i for i, j in edges]
    cols = list(range(n)) + [j for i, j in edges]
    vals = list(-deg) + [1.0] * len(edges)
    C = (np.asarray(rows, np.int32), np.asarray(cols, np.int32), np.asarray(vals, np.float64))
    cliques, parent, order = chordal.chordal_extension(n, edges)
    A = (np.arange(n, dtype=np.int32), np.arange(n, dtype=np.int32),
         np.arange(n, dtype=np.int32), np.ones(n))
    b = np.ones(n)
    return SDPInstance(n, n, C, A, b, cliques, parent, name=name,
                       meta=dict(edges=edges, order=order))


def maxcut_random_2000():
    """Max-cut relaxation on G(2000, 6000) (average degree 6), min-degree extension."""
    return maxcut_instance(1, 0, n=2000, n_edges=6000)


def grid_maxcut(stream, rows=40, cols=50):
    """Companion of the random max-cut: max-cut relaxation on the 2-D periodic
    rows x cols grid (torus)."""
    n = rows * cols
    edges = []
    for r in range(rows):
        for c in range(cols):
            v = r * cols + c
            edges.append((v, r * cols + (c + 1) % cols))
            edges.append((v, ((r + 1) % rows) * cols + c))
    return maxcut_from_edges(n, edges, name=f"max-cut periodic grid {rows}x{cols}")


def clique_tree_growth(rng, n, smin=4, smax=96):
    """Random chordal graph grown clique by clique (a perfect elimination
    construction): each new clique keeps a random proper subset of a random
    existing clique as separator and adds fresh vertices."""
    cliques = []
    parent = []
    s = int(rng.integers(smin, smax + 1))
    s = min(s, n)
    cliques.append(np.arange(s, dtype=np.int64))
    parent.append(-1)
    nv = s
    while nv < n:
        s = int(rng.integers(smin, smax + 1))
        par = int(rng.integers(0, len(cliques)))
        pc = cliques[par]
        smax_sep = min(s - 1, len(pc) - 1)
        sig = int(rng.integers(1, smax_sep + 1))
        sep = np.sort(rng.choice(pc, size=sig, replace=False))
        new = min(s - sig, n - nv)
        fresh = np.arange(nv, nv + new, dtype=np.int64)
        nv += new
        cliques.append(np.sort(np.concatenate([sep, fresh])))
        parent.append(par)
    return cliques, np.asarray(parent, dtype=np.int64)


def uneven_cliques_5000(twin=False):
    """Uneven cliques (4..96) on n=5000, m=2000 sparse constraints (8 entries
    each); the infeasible twin appends <A_1,X> = 1 and <A_1,X> = -1."""
    rng = rng_for(2, 0)
    n, m = 5000, 2000
    cliques, parent = clique_tree_growth(rng, n)
    er, ec = pattern_entries(cliques)
    A = _random_constraints(rng, m, er, ec, 8)
    b, C, meta = _feasible_data(rng, n, m, cliques, A)
    name = "uneven cliques n=5000 m=2000"
    if twin:
        con, r, c, v = A
        first = con == 0
        A = (np.concatenate([con, np.full(first.sum(), m, np.int32), np.full(first.sum(), m + 1, np.int32)]),
             np.concatenate([r, r[first], r[first]]), np.concatenate([c, c[first], c[first]]),
             np.concatenate([v, v[first], v[first]]))
        b = np.concatenate([b, [1.0, -1.0]])
        m += 2
        name += " (infeasible twin, m=2002)"
    return SDPInstance(n, m, C, A, b, cliques, parent, name=name, meta=meta)


def block_arrow_batch256(count=256):
    """256 block-arrow SDPs: n~U{50..400}, block~U{4..32}, arrow~U{2..8}, m=n//2."""
    out = []
    for i in range(count):
        rng = rng_for(3, 10_000 + i)
        n = int(rng.integers(50, 401))
        blk = int(rng.integers(4, 33))
        arw = int(rng.integers(2, 9))
        out.append(block_arrow_instance(3, i, n=n, block=blk, arrow=arw, m=n // 2))
    return out


def block_arrow_grad64(count=64):
    """64 block-arrow SDPs with n=200, block 16, arrow 4, m=100 (+ loss weights W)."""
    out = []
    for i in range(count):
        inst = block_arrow_instance(4, i, n=200, block=16, arrow=4, m=100)
        rng = rng_for(4, 10_000 + i)
        er, ec = pattern_entries(inst.cliques)
        inst.meta["W"] = (er.astype(np.int32), ec.astype(np.int32), rng.standard_normal(len(er)))
        out.append(inst)
    return out


def small_block_arrow(instance, n=12, block=3, arrow=2, m=4, per_row=None):
    """Tiny instances for the oracle's pins and quick parity checks."""
    return block_arrow_instance(90, instance, n=n, block=block, arrow=arrow, m=m, per_row=per_row)
