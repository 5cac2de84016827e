"""Host logic of the exploratory driver: the variants of each level against
an independent enumeration (networkx isomorphism classes of the connected
spanning edge subsets), on small labelled templates."""
import itertools

import networkx as nx
import pytest

from paper_1912_08453_amd import explore


def _classes_nx(labels, edges, k):
    n0 = len(labels)
    reps = []
    for removed in itertools.combinations(range(len(edges)), k):
        es = [e for i, e in enumerate(edges) if i not in removed]
        g = nx.Graph()
        g.add_nodes_from((q, {"l": labels[q]}) for q in range(n0))
        g.add_edges_from(es)
        if not nx.is_connected(g):
            continue
        if not any(nx.is_isomorphic(g, h, node_match=lambda a, b: a["l"] == b["l"])
                   for h in reps):
            reps.append(g)
    return len(reps)


CASES = [
    ([0, 1, 2, 3], [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2), (1, 3)]),          # K4, distinct
    ([0, 0, 0, 0], [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2), (1, 3)]),          # K4, one label
    ([1, 2, 1, 2, 3], [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4), (2, 4)]),
    ([5, 5, 6, 7, 6, 5], [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 0), (1, 4)]),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_variant_classes_match_networkx(case):
    labels, edges = CASES[case]
    for k in range(len(edges) + 1):
        vs = explore.variants(labels, edges, k)
        assert len(vs) == _classes_nx(labels, edges, k), f"level {k}"
        for es in vs:
            assert len(es) == len(edges) - k
            assert set(map(tuple, map(sorted, es))) <= set(map(tuple, map(sorted, edges)))


def test_level_zero_is_the_template_and_disconnecting_levels_are_empty():
    labels, edges = CASES[0]
    assert explore.variants(labels, edges, 0) == [[tuple(sorted(e)) for e in edges]]
    # a spanning tree of 4 vertices has 3 edges: removing 4 of 6 disconnects
    assert explore.variants(labels, edges, 4) == []
