"""Direct pins of the oracle's non-local constraint check (NLCC algorithm and
its token-generation paragraph) for ONE constraint at a time.

The other oracle pins reach the NLCC only through the final output, which
the exact final step fixes regardless of what the constraint loop did; a
sound but wrong head rule (say, checking only one terminal of a path
constraint) would pass them.  These tests state the surviving head roles of
single constraints by hand on small drawn graphs, and compare the oracle's
per-(vertex, head) decisions with a plain Python enumeration of rooted
injective embeddings over the snapshot state.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import constraints as C
from paper_1912_08453_amd import inputs as I


def _graph(n, edges):
    rp, col = I.csr_from_edges(n, np.asarray(edges, dtype=np.int64))
    return rp, col


def _roles(labels, tlabels):
    """Initial role sets (vertex state and initialisation): role q on v iff
    the labels agree."""
    om = np.zeros(len(labels), dtype=np.uint64)
    for v, lv in enumerate(labels):
        for q, lq in enumerate(tlabels):
            if lv == lq:
                om[v] |= np.uint64(1 << q)
    return om


def _bits(*qs):
    return sum(1 << q for q in qs)


def test_path_constraint_both_terminals_by_hand():
    """Template path q0(A) - q1(B) - q2(C) - q3(A): the repeated label A sits
    at both ends, three hops apart, so the constraint is a path constraint
    whose token sources are both terminals.

    Background (labels A=0, B=1, C=2):
      v0(A) - v1(B) - v2(C) - v3(A)          a straight path
      v4(A) - v5(B) - v6(C) - v4             a triangle: the only A at
                                             distance 3 would be v4 itself
    Hand-derived survivors of the head roles (non-head roles untouched):
      v0: q0 yes (v0 v1 v2 v3), q3 no (v0 has no C neighbour)
      v3: q3 yes (v3 v2 v1 v0), q0 no (v3 has no B neighbour)
      v4: q0 no (v4 v5 v6 would have to end at an A other than v4),
          q3 no (v4 v6 v5 likewise) -- injectivity of the repeated label
    """
    tl = [0, 1, 2, 0]
    te = [(0, 1), (1, 2), (2, 3)]
    labels = [0, 1, 2, 0, 0, 1, 2]
    rp, col = _graph(7, [(0, 1), (1, 2), (2, 3), (4, 5), (5, 6), (6, 4)])
    g = oracle._G(rp, col, labels)
    om = _roles(labels, tl)
    K0 = C.non_local_constraints(tl, te)
    pcs = [c for c in K0 if c.kind == C.PC]
    assert len(pcs) == 1
    pc = pcs[0]
    assert pc.edges == ((0, 1), (1, 2), (2, 3)) and pc.heads == _bits(0, 3)
    changed = oracle.nlcc(g, om, pc)
    want = np.array([_bits(0), _bits(1), _bits(2), _bits(3), 0, _bits(1), _bits(2)],
                    dtype=np.uint64)
    assert np.array_equal(om, want), om
    assert changed == 3          # v0, v3 and v4 lost head roles


def test_cycle_constraint_every_vertex_is_a_head_by_hand():
    """Template 4-cycle q0(A) q1(B) q2(C) q3(D): a cycle constraint whose
    token sources are all four vertices.

    Background: a closed 4-cycle v0 v1 v2 v3 (labels A B C D) and an open
    copy v4 v5 v6 v7 (the same labels, no edge v7 - v4), plus v8(A) adjacent
    to v1 only.  Every role on the closed cycle survives; every role of the
    open copy and of v8 goes."""
    tl = [0, 1, 2, 3]
    te = [(0, 1), (1, 2), (2, 3), (3, 0)]
    labels = [0, 1, 2, 3, 0, 1, 2, 3, 0]
    rp, col = _graph(9, [(0, 1), (1, 2), (2, 3), (3, 0), (4, 5), (5, 6), (6, 7), (8, 1)])
    g = oracle._G(rp, col, labels)
    om = _roles(labels, tl)
    ccs = [c for c in C.non_local_constraints(tl, te) if c.kind == C.CC]
    assert len(ccs) == 1 and ccs[0].heads == _bits(0, 1, 2, 3)
    changed = oracle.nlcc(g, om, ccs[0])
    want = np.array([_bits(0), _bits(1), _bits(2), _bits(3), 0, 0, 0, 0, 0], dtype=np.uint64)
    assert np.array_equal(om, want), om
    assert changed == 5


def test_constraint_reads_the_snapshot_not_its_own_removals():
    """Path q0(A)-q1(B)-q2(A), heads q0 and q2 (the repeated-label ends), on
    the background path v0(A) - v1(B) - v2(A) - v3(B) where v3 holds no
    role.  v0 and v2 support each other's paths (v0 v1 v2 and v2 v1 v0): no
    role goes and no vertex counts as changed.  With v1's role cleared
    beforehand, neither end has a path any more and both lose both head
    roles in one pass."""
    tl = [0, 1, 0]
    te = [(0, 1), (1, 2)]
    labels = [0, 1, 0, 1]
    rp, col = _graph(4, [(0, 1), (1, 2), (2, 3)])
    g = oracle._G(rp, col, labels)
    pc = C.Constraint(C.PC, ((0, 1), (1, 2)), _bits(0, 2), 0)
    om = _roles(labels, tl)
    om[3] = 0
    before = om.copy()
    assert oracle.nlcc(g, om, pc) == 0
    assert np.array_equal(om, before)
    om[1] = 0
    assert oracle.nlcc(g, om, pc) == 2
    assert om[0] == 0 and om[2] == 0


# ----------------------------------------------- brute-force enumeration
def _python_nlcc(n, adj, om, edges, heads):
    """Plain enumeration: (v, h) survives iff some injective map of the
    substructure's vertices into V, with h at v, gives every vertex a role
    it holds in the snapshot and maps every substructure edge onto an edge."""
    verts = sorted({a for e in edges for a in e})
    sat = np.zeros(n, dtype=np.uint64)
    for h in verts:
        if not (heads >> h) & 1:
            continue
        rest = [q for q in verts if q != h]
        for v in range(n):
            if not (int(om[v]) >> h) & 1:
                continue
            for imgs in itertools.permutations([x for x in range(n) if x != v], len(rest)):
                phi = dict(zip(rest, imgs))
                phi[h] = v
                if all((int(om[phi[q]]) >> q) & 1 for q in rest) and \
                        all(phi[b] in adj[phi[a]] for a, b in edges):
                    sat[v] |= np.uint64(1 << h)
                    break
    out = om.copy()
    for v in range(n):
        out[v] = np.uint64(int(om[v]) & (~heads | int(sat[v])) & 0xFFFFFFFFFFFFFFFF)
    return out


@pytest.mark.parametrize("seed", range(60))
def test_nlcc_equals_enumeration_of_rooted_embeddings(seed):
    """Random small graphs, random substructures (paths, cycles, small
    trees with a cycle), random head sets and random snapshot states that
    are subsets of the label roles: the oracle's per-head decisions equal
    the enumeration above."""
    rng = np.random.Generator(np.random.Philox(7000 + seed))
    n = int(rng.integers(5, 9))
    nl = int(rng.integers(1, 3))
    g = I.random_graph(n, float(rng.uniform(0.25, 0.6)), nl, 7000 + seed)
    kind = seed % 3
    if kind == 0:
        k = int(rng.integers(2, 5))
        edges = [(i, i + 1) for i in range(k - 1)]
    elif kind == 1:
        k = int(rng.integers(3, 5))
        edges = [(i, (i + 1) % k) for i in range(k)]
    else:
        edges = I.shape_one_cycle(rng, 4)
        k = 4
    edges = [tuple(sorted(e)) for e in edges]
    tl = [int(x) for x in rng.integers(0, nl, size=k)]
    heads = 0
    while heads == 0:
        heads = int(rng.integers(0, 1 << k))
    om = _roles([int(x) for x in g.labels], tl)
    drop = rng.integers(0, 1 << 62, size=n, dtype=np.int64).astype(np.uint64)
    om &= drop | np.uint64(rng.integers(0, 1 << 62))
    adj = [set() for _ in range(n)]
    for u in range(n):
        for e in range(g.row_ptr[u], g.row_ptr[u + 1]):
            adj[u].add(int(g.col[e]))
    want = _python_nlcc(n, adj, om, edges, heads)
    got = om.copy()
    ch = oracle.nlcc(oracle._G(g.row_ptr, g.col, g.labels), got,
                     C.Constraint(C.CC, tuple(edges), heads, 0))
    assert np.array_equal(got, want), (edges, heads, om, got, want)
    assert ch == int((got != om).sum())


def test_cycle_cap_keeps_the_shortest_cycles_and_the_output():
    """The reading of the cycle generator keeps at most MAX_CYCLES simple
    cycles, the shortest first in canonical order.  K5 has 10 triangles, 15
    four-cycles and 12 five-cycles (37 in all, enumerated in full because
    the first two lengths give only 25); the constraint list keeps the 10 +
    15 shorter ones and the first 7 five-cycles as cycle constraints (32),
    plus the TDS union.  The final output does not depend on the cap: it
    equals the brute-force union on a small graph."""
    n0 = 5
    te = [(a, b) for a in range(n0) for b in range(a + 1, n0)]
    cyc = C.simple_cycles(n0, te, (1 << n0) - 1)
    assert len(cyc) == 37
    lens = [len(c) for c in cyc]
    assert lens[:10] == [3] * 10 and lens[10:25] == [4] * 15 and lens[25:] == [5] * 12
    assert cyc == sorted(cyc, key=lambda c: (len(c), c))
    K0 = C.non_local_constraints([0] * n0, te)
    ccs = [k for k in K0 if k.kind == C.CC]
    assert len(ccs) == C.MAX_CYCLES == 32
    assert [len(k.edges) for k in ccs] == [3] * 10 + [4] * 15 + [5] * 7
    g = I.random_graph(12, 0.7, 1, 4242)
    t = I.Template([0] * n0, te)
    ref = oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges)
    role, edge, _ = oracle.bruteforce(g.row_ptr, g.col, g.labels, t.labels, t.edges)
    assert np.array_equal(ref.role_mask, role) and np.array_equal(ref.edge_bits, edge)
