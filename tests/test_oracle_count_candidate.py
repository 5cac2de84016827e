"""Pins of the oracle's match enumeration (counting on the reduced graph,
termination and output section) and of its candidate set (interactive
incremental search), against networkx, closed forms from the adjacency
matrix, and brute force over every template variant."""
import itertools

import networkx as nx
import numpy as np
import pytest
from networkx.algorithms import isomorphism as iso

import oracle
from paper_1912_08453_amd import inputs as I


def _nx_maps(g, t):
    G = nx.Graph()
    for v in range(g.n):
        G.add_node(v, label=int(g.labels[v]))
    for u in range(g.n):
        for e in range(g.row_ptr[u], g.row_ptr[u + 1]):
            G.add_edge(u, int(g.col[e]))
    H = nx.Graph()
    for q, lab in enumerate(t.labels):
        H.add_node(q, label=lab)
    H.add_edges_from(t.edges)
    gm = iso.GraphMatcher(G, H, node_match=lambda a, b: a["label"] == b["label"])
    out = set()
    for mapping in gm.subgraph_monomorphisms_iter():
        phi = {q: v for v, q in mapping.items()}
        out.add(tuple(phi[q] for q in range(len(t.labels))))
    return out


def _random(seed):
    rng = np.random.Generator(np.random.Philox(9100 + seed))
    g = I.random_graph(int(rng.integers(6, 16)), float(rng.uniform(0.15, 0.5)),
                       int(rng.integers(1, 3)), 9100 + seed)
    kind = seed % 4
    n0 = int(rng.integers(2, 6))
    if kind == 0:
        edges = I.shape_tree(rng, n0)
    elif kind == 1:
        edges = I.shape_one_cycle(rng, max(n0, 3))
    elif kind == 2:
        edges = I.shape_two_cycles(rng, 5)
    else:
        edges = I.shape_k4(rng, 4)
    n0 = max(max(e) for e in edges) + 1
    labels = [int(x) for x in rng.integers(0, int(g.labels.max()) + 1, size=n0)]
    return g, I.Template(labels, edges)


@pytest.mark.parametrize("seed", range(40))
def test_enumeration_equals_networkx_monomorphisms(seed):
    g, t = _random(seed)
    cnt, maps = oracle.enumerate_maps(g.row_ptr, g.col, g.labels, t.labels, t.edges)
    want = _nx_maps(g, t)
    assert cnt == len(want)
    assert {tuple(int(x) for x in r) for r in maps} == want
    # the brute-force union counts the same maps
    assert oracle.bruteforce(g.row_ptr, g.col, g.labels, t.labels, t.edges)[2] == cnt


def _adjacency(g):
    A = np.zeros((g.n, g.n), dtype=np.int64)
    for u in range(g.n):
        for e in range(g.row_ptr[u], g.row_ptr[u + 1]):
            A[u, int(g.col[e])] = 1
    return A


@pytest.mark.parametrize("seed", range(8))
def test_counts_closed_forms_unlabeled(seed):
    """Unlabeled templates: an edge has 2|E| maps; a triangle trace(A^3);
    a two-edge path sum d(d-1); a three-leaf star sum d(d-1)(d-2)."""
    g = I.random_graph(14, 0.35, 1, 9300 + seed)
    A = _adjacency(g)
    d = A.sum(1)
    lab = np.zeros(g.n, dtype=np.uint8)

    def cnt(edges):
        n0 = max(max(e) for e in edges) + 1
        return oracle.enumerate_maps(g.row_ptr, g.col, lab, [0] * n0, edges, cap=1)[0]
    assert cnt([(0, 1)]) == int(A.sum())
    assert cnt([(0, 1), (1, 2), (0, 2)]) == int(np.trace(A @ A @ A))
    assert cnt([(0, 1), (1, 2)]) == int((d * (d - 1)).sum())
    assert cnt([(0, 1), (0, 2), (0, 3)]) == int((d * (d - 1) * (d - 2)).sum())


def _variants(t):
    """Every connected spanning edge subset of the template (deleting edges,
    keeping all vertices)."""
    n0 = len(t.labels)
    out = []
    for k in range(len(t.edges) + 1):
        for keep in itertools.combinations(t.edges, len(t.edges) - k):
            G = nx.Graph()
            G.add_nodes_from(range(n0))
            G.add_edges_from(keep)
            if nx.is_connected(G):
                out.append(list(keep))
    return out


@pytest.mark.parametrize("seed", range(40))
def test_candidate_set_holds_every_edge_deleted_variant(seed):
    g, t = _random(seed)
    cand, cedge = oracle.candidate_set(g.row_ptr, g.col, g.labels, t.labels, t.edges)
    for keep in _variants(t):
        role, edge, _ = oracle.bruteforce(g.row_ptr, g.col, g.labels, t.labels, keep)
        assert not np.any(role & ~cand), keep
        assert not np.any(edge & ~cedge), keep
    # the relaxed rule keeps at least what the full local rule keeps
    gg, tt = oracle._G(g.row_ptr, g.col, g.labels), oracle._T(t.labels, t.edges)
    om = oracle.init_roles(gg, tt)
    oracle.lcc(gg, tt, om)
    assert not np.any(om & ~cand)


def test_candidate_set_by_hand():
    """Template path q0(A) - q1(B) - q2(C) (so its only connected variant is
    itself; q1 needs an A or a C neighbour in the candidate rule).
    Background: v0(A) - v1(B), v2(B) isolated from A and C but adjacent to
    v3(B), v4(C) - v5(B).  Candidate set: v0 {q0}, v1 {q1}, v4 {q2},
    v5 {q1}; v2 and v3 lose q1 (no A or C neighbour)."""
    labels = np.array([0, 1, 1, 1, 2, 1], dtype=np.uint8)
    rp, col = I.csr_from_edges(6, np.array([(0, 1), (2, 3), (4, 5)]))
    cand, _ = oracle.candidate_set(rp, col, labels, [0, 1, 2], [(0, 1), (1, 2)])
    assert cand.tolist() == [1, 2, 0, 0, 4, 2]


@pytest.mark.parametrize("seed", range(10))
def test_sampled_sweep_equals_one_jacobi_sweep(seed):
    """The timing sampler applies the same local rule: on every vertex it
    gives exactly one synchronous sweep of the oracle's LCC."""
    g, t = _random(seed)
    gg, tt = oracle._G(g.row_ptr, g.col, g.labels), oracle._T(t.labels, t.edges)
    om = oracle.init_roles(gg, tt)
    one = om.copy()
    oracle.lcc(gg, tt, one, max_sweeps=1)
    got, entries = oracle.lcc_sample(gg, tt, om, np.arange(g.n))
    assert np.array_equal(got, one)
    assert entries == g.m
