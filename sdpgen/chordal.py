"""Host-side chordal tools: chordal extension, maximal cliques, clique tree.

These build the *input* of the solver (the cliques C_1..C_p of a chordal
extension of the aggregate sparsity pattern, Section 2.1 and the assumption
stated after the primal/dual pair in Section 3).  They are preprocessing done
once per problem, not part of the ADMM iteration, and hold none of its
arithmetic.

Methods (standard, written from their published descriptions):
  * minimum-degree elimination (Tinney-Walker; the AMD family of
    Amestoy-Davis-Duff 1996 approximates it) to obtain a fill-reducing
    perfect elimination ordering of the filled graph;
  * fundamental supernodes of the elimination tree give the maximal cliques
    and a clique tree (Vandenberghe & Andersen 2014, Sections 4.4-4.8);
  * maximum-cardinality search (Tarjan-Yannakakis 1984) to test chordality.
"""
from __future__ import annotations

import heapq
from typing import List, Sequence, Tuple

import numpy as np


def adjacency_from_edges(n: int, edges) -> List[set]:
    """Undirected simple adjacency sets (no self loops)."""
    adj = [set() for _ in range(n)]
    for i, j in edges:
        i = int(i)
        j = int(j)
        if i == j:
            continue
        adj[i].add(j)
        adj[j].add(i)
    return adj


def min_degree_elimination(adj: Sequence[set]) -> Tuple[np.ndarray, List[set]]:
    """Eliminate vertices by minimum current degree (ties: lowest index).

    Returns (order, higher) where order[t] is the t-th eliminated vertex and
    higher[v] is the set of neighbours of v in the filled graph that are
    eliminated after v.  {v} U higher[v] is a clique of the filled graph.
    """
    n = len(adj)
    work = [set(a) for a in adj]
    done = np.zeros(n, dtype=bool)
    heap = [(len(work[v]), v) for v in range(n)]
    heapq.heapify(heap)
    order = []
    higher: List[set] = [set() for _ in range(n)]
    while heap:
        d, v = heapq.heappop(heap)
        if done[v] or d != len(work[v]):
            continue
        done[v] = True
        order.append(v)
        nb = work[v]
        higher[v] = set(nb)
        for u in nb:
            wu = work[u]
            wu.discard(v)
            wu |= nb
            wu.discard(u)
            heapq.heappush(heap, (len(wu), u))
        work[v] = set()
    return np.asarray(order, dtype=np.int64), higher


def cliques_from_elimination(order: np.ndarray, higher: Sequence[set]):
    """Maximal cliques and clique-tree parents from a perfect elimination order.

    Returns (cliques, parent): cliques[k] is a sorted int array (natural
    vertex order, as the clique convention of Section 2.1 requires) and
    parent[k] is the index of the parent clique (-1 for a root).  Cliques are
    listed in elimination order of their representative vertex, so every
    parent comes after its children.
    """
    n = len(order)
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    # elimination-tree parent: earliest-eliminated higher neighbour
    etp = np.full(n, -1, dtype=np.int64)
    for v in range(n):
        if higher[v]:
            etp[v] = min(higher[v], key=lambda u: pos[u])
    # v is absorbed into the supernode of a child u when col(v) = col(u) minus u
    absorbed_into = np.full(n, -1, dtype=np.int64)
    for t in range(n):
        u = int(order[t])
        p = etp[u]
        if p >= 0 and absorbed_into[p] < 0 and len(higher[u]) == len(higher[p]) + 1:
            absorbed_into[p] = u
    # supernode id: follow the absorption chain downward to its representative
    snode = np.full(n, -1, dtype=np.int64)
    reps = []
    for t in range(n):
        v = int(order[t])
        if absorbed_into[v] < 0:
            snode[v] = len(reps)
            reps.append(v)
        else:
            snode[v] = snode[absorbed_into[v]]
    # last vertex of each supernode and its separator
    last = [None] * len(reps)
    for t in range(n):
        v = int(order[t])
        last[snode[v]] = v
    cliques = []
    parent = np.full(len(reps), -1, dtype=np.int64)
    for k, r in enumerate(reps):
        cl = np.array(sorted(higher[r] | {r}), dtype=np.int64)
        cliques.append(cl)
        sep = higher[last[k]]
        if sep:
            f = min(sep, key=lambda u: pos[u])
            parent[k] = snode[f]
    return cliques, parent


def chordal_extension(n: int, edges):
    """Minimum-degree chordal extension; returns (cliques, parent, order)."""
    adj = adjacency_from_edges(n, edges)
    order, higher = min_degree_elimination(adj)
    cliques, parent = cliques_from_elimination(order, higher)
    return cliques, parent, order


def is_chordal(n: int, edges) -> bool:
    """Maximum-cardinality search + zero-fill test of the reversed visit order."""
    adj = adjacency_from_edges(n, edges)
    weight = np.zeros(n, dtype=np.int64)
    visited = np.zeros(n, dtype=bool)
    visit = []
    for _ in range(n):
        cand = np.where(~visited)[0]
        v = int(cand[np.argmax(weight[cand])])
        visited[v] = True
        visit.append(v)
        for u in adj[v]:
            if not visited[u]:
                weight[u] += 1
    # reverse of the MCS visit order is a perfect elimination order iff chordal
    peo = visit[::-1]
    pos = {v: i for i, v in enumerate(peo)}
    for v in peo:
        later = [u for u in adj[v] if pos[u] > pos[v]]
        if not later:
            continue
        w = min(later, key=lambda u: pos[u])
        rest = set(later) - {w}
        if not rest <= (adj[w] | {w}):
            return False
    return True


def clique_tree_ok(n: int, cliques, parent) -> bool:
    """Induced-subtree (running intersection) property of a clique tree.

    For every vertex the cliques containing it must form a connected subtree:
    with c_v cliques containing v and e_v tree edges whose both ends contain
    v, connectivity holds iff e_v = c_v - 1.
    """
    cnt = np.zeros(n, dtype=np.int64)
    edge = np.zeros(n, dtype=np.int64)
    sets = [set(int(x) for x in c) for c in cliques]
    for k, c in enumerate(sets):
        for v in c:
            cnt[v] += 1
        p = int(parent[k])
        if p >= 0:
            for v in c & sets[p]:
                edge[v] += 1
    covered = cnt > 0
    return bool(np.all(covered) and np.all(edge[covered] == cnt[covered] - 1))


def clique_edges(cliques):
    """All undirected edges (i > j) of the union of the cliques."""
    out = set()
    for c in cliques:
        c = [int(x) for x in c]
        for a in range(len(c)):
            for b in range(a):
                i, j = c[a], c[b]
                out.add((max(i, j), min(i, j)))
    return out
