"""Host chordal tools (input preparation) against brute force on small graphs."""
import itertools

import numpy as np
import pytest

from sdpgen import chordal, configs


def _brute_maximal_cliques(n, edge_set):
    adj = [[False] * n for _ in range(n)]
    for i, j in edge_set:
        adj[i][j] = adj[j][i] = True
    cl = []
    for r in range(1, n + 1):
        for sub in itertools.combinations(range(n), r):
            if all(adj[a][b] for a, b in itertools.combinations(sub, 2)):
                cl.append(frozenset(sub))
    return {c for c in cl if not any(c < d for d in cl)}


@pytest.mark.parametrize("seed", range(12))
def test_min_degree_extension_gives_maximal_cliques_and_tree(seed):
    rng = np.random.default_rng(seed)
    n = 9
    edges = [(i, j) for i in range(n) for j in range(i) if rng.random() < 0.35]
    cliques, parent, order = chordal.chordal_extension(n, edges)
    filled = chordal.clique_edges(cliques)
    assert {(max(a, b), min(a, b)) for a, b in edges} <= filled
    assert chordal.is_chordal(n, list(filled))
    assert {frozenset(int(x) for x in c) for c in cliques} == _brute_maximal_cliques(n, filled)
    assert len(cliques) == len({frozenset(c.tolist()) for c in cliques})
    for c in cliques:
        assert np.all(np.diff(c) > 0)
    assert chordal.clique_tree_ok(n, cliques, parent)


def test_is_chordal():
    assert not chordal.is_chordal(4, [(0, 1), (1, 2), (2, 3), (3, 0)])
    assert chordal.is_chordal(4, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)])


def test_block_arrow_and_growth_patterns():
    cl, par = configs.block_arrow_cliques(200, 16, 4)
    assert [len(c) for c in cl] == [20] * 12 + [8]
    assert chordal.clique_tree_ok(200, cl, par)
    rng = configs.rng_for(99, 0)
    cl, par = configs.clique_tree_growth(rng, 400, 4, 30)
    assert chordal.clique_tree_ok(400, cl, par)
    assert chordal.is_chordal(400, list(chordal.clique_edges(cl)))
    sets = [frozenset(c.tolist()) for c in cl]
    assert not any(a < b for a in sets for b in sets)
