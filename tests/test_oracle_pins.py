"""Pins for the CPU oracle against facts fixed outside the oracle itself:
an independent library (networkx monomorphism search), closed forms,
the paper's counterexample constructions (the three-template figure in the
solution overview), complexity claims, and invariants of monotone pruning.
"""
import itertools

import networkx as nx
import numpy as np
import pytest
from networkx.algorithms import isomorphism as iso

import oracle
from oracle import constraints as C
from paper_1912_08453_amd import inputs as I


# ---------------------------------------------------------------- helpers
def edge_set_from_bits(row_ptr, col, bits):
    """Set of directed CSR pairs (u, w) whose bit is set."""
    out = set()
    n = len(row_ptr) - 1
    for u in range(n):
        for e in range(row_ptr[u], row_ptr[u + 1]):
            if (int(bits[e >> 6]) >> (e & 63)) & 1:
                out.add((u, int(col[e])))
    return out


def nx_graph(g):
    G = nx.Graph()
    for v in range(g.n):
        G.add_node(v, label=int(g.labels[v]))
    for u in range(g.n):
        for e in range(g.row_ptr[u], g.row_ptr[u + 1]):
            G.add_edge(u, int(g.col[e]))
    return G


def nx_union(g, t):
    """Union of all monomorphisms (non-induced matches) via networkx."""
    G = nx_graph(g)
    H = nx.Graph()
    for q, lab in enumerate(t.labels):
        H.add_node(q, label=lab)
    H.add_edges_from(t.edges)
    gm = iso.GraphMatcher(G, H, node_match=lambda a, b: a["label"] == b["label"])
    roles = np.zeros(g.n, dtype=np.uint64)
    edges = set()
    for mapping in gm.subgraph_monomorphisms_iter():
        phi = {q: v for v, q in mapping.items()}
        for q, v in phi.items():
            roles[v] |= np.uint64(1 << q)
        for a, b in t.edges:
            edges.add((phi[a], phi[b]))
            edges.add((phi[b], phi[a]))
    return roles, edges


def random_case(seed, n_lo=8, n_hi=28):
    rng = np.random.Generator(np.random.Philox(seed))
    n = int(rng.integers(n_lo, n_hi))
    p = float(rng.uniform(0.08, 0.45))
    nl = int(rng.integers(1, 4))
    g = I.random_graph(n, p, nl, seed)
    kind = seed % 4
    n0 = int(rng.integers(2, 6))
    if kind == 0:
        edges = I.shape_tree(rng, n0)
    elif kind == 1:
        edges = I.shape_one_cycle(rng, max(n0, 3))
    elif kind == 2:
        edges = I.shape_two_cycles(rng, max(n0, 5))
    else:
        edges = I.shape_k4(rng, max(n0, 4))
    n0 = max(max(a, b) for a, b in edges) + 1
    labels = [int(x) for x in rng.integers(0, nl, size=n0)]
    return g, I.Template(labels, edges)


def run_prune(g, t, **kw):
    return oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges, **kw)


def run_brute(g, t):
    return oracle.bruteforce(g.row_ptr, g.col, g.labels, t.labels, t.edges)


def graph_from_edges(n, edges, labels):
    rp, col = I.csr_from_edges(n, np.asarray(edges))
    return I.Graph(rp, col, np.asarray(labels, dtype=np.uint8))


# ------------------------------------------------ brute force vs networkx
@pytest.mark.parametrize("seed", range(40))
def test_bruteforce_equals_networkx(seed):
    g, t = random_case(seed, 6, 18)
    role, ebits, _ = run_brute(g, t)
    nroles, nedges = nx_union(g, t)
    assert np.array_equal(role, nroles)
    assert edge_set_from_bits(g.row_ptr, g.col, ebits) == nedges


# ------------------------------------------ method steps vs the definition
@pytest.mark.parametrize("seed", range(150))
def test_prune_equals_bruteforce(seed):
    g, t = random_case(seed)
    r = run_prune(g, t)
    role, ebits, _ = run_brute(g, t)
    assert np.array_equal(r.role_mask, role)
    assert np.array_equal(r.edge_bits, ebits)


def test_prune_equals_bruteforce_square_pendant():
    """Square plus pendant on a scale-10 R-MAT graph with 8 uniform labels."""
    rp, col = I.rmat_csr(10, seed=7)
    g = I.Graph(rp, col, I.labels_uniform(rp.shape[0] - 1, 8, 99))
    t = I.template_square_pendant()
    r = run_prune(g, t)
    role, ebits, cnt = run_brute(g, t)
    assert np.array_equal(r.role_mask, role)
    assert np.array_equal(r.edge_bits, ebits)


# ------------------------------------------------------------ closed forms
def test_single_edge_template_closed_form():
    g = I.random_graph(60, 0.1, 3, 5)
    t = I.Template([0, 1], [(0, 1)])
    r = run_prune(g, t)
    exp_edges = set()
    exp_roles = np.zeros(g.n, dtype=np.uint64)
    for u in range(g.n):
        for e in range(g.row_ptr[u], g.row_ptr[u + 1]):
            w = int(g.col[e])
            if g.labels[u] == 0 and g.labels[w] == 1:
                exp_edges |= {(u, w), (w, u)}
                exp_roles[u] |= np.uint64(1)
                exp_roles[w] |= np.uint64(2)
    assert edge_set_from_bits(g.row_ptr, g.col, r.edge_bits) == exp_edges
    assert np.array_equal(r.role_mask, exp_roles)


def test_unlabeled_triangle_edge_support():
    """Edge in E* iff its endpoints have a common neighbour (edge support)."""
    g = I.random_graph(50, 0.12, 1, 11)
    t = I.Template([0, 0, 0], [(0, 1), (1, 2), (0, 2)])
    r = run_prune(g, t)
    nb = [set(g.col[g.row_ptr[v]:g.row_ptr[v + 1]].tolist()) for v in range(g.n)]
    exp = {(u, w) for u in range(g.n) for w in nb[u] if nb[u] & nb[w]}
    assert edge_set_from_bits(g.row_ptr, g.col, r.edge_bits) == exp
    for v in range(g.n):
        in_tri = any(nb[v] & nb[w] for w in nb[v])
        assert (int(r.role_mask[v]) == 0b111) == in_tri
        assert int(r.role_mask[v]) in (0, 0b111)


def test_unlabeled_k4_clique_edges():
    g = I.random_graph(40, 0.3, 1, 3)
    t = I.Template([0] * 4, [(a, b) for a in range(4) for b in range(a + 1, 4)])
    r = run_prune(g, t)
    G = nx_graph(g)
    exp = set()
    for cl in nx.enumerate_all_cliques(G):
        if len(cl) == 4:
            for a, b in itertools.permutations(cl, 2):
                exp.add((a, b))
        if len(cl) > 4:
            break
    assert edge_set_from_bits(g.row_ptr, g.col, r.edge_bits) == exp


def test_star_distinct_leaf_labels_closed_form():
    """K_{1,3} with centre label 0 and leaves 1, 2, 3: a centre needs one
    neighbour of each leaf label; a leaf needs a valid centre."""
    g = I.random_graph(80, 0.06, 4, 21)
    t = I.Template([0, 1, 2, 3], [(0, 1), (0, 2), (0, 3)])
    r = run_prune(g, t)
    nb = [g.col[g.row_ptr[v]:g.row_ptr[v + 1]].tolist() for v in range(g.n)]
    centre = [g.labels[v] == 0 and {1, 2, 3} <= {int(g.labels[u]) for u in nb[v]}
              for v in range(g.n)]
    for v in range(g.n):
        exp = 0
        if centre[v]:
            exp |= 1
        lab = int(g.labels[v])
        if lab in (1, 2, 3) and any(centre[u] for u in nb[v]):
            exp |= 1 << lab
        assert int(r.role_mask[v]) == exp


@pytest.mark.parametrize("seed", range(30))
def test_lcc_alone_exact_for_acyclic_unique_labels(seed):
    """Acyclic templates with unique labels need LCC only (solution overview);
    the LCC fixpoint and its edge state already equal the complete set."""
    rng = np.random.Generator(np.random.Philox(1000 + seed))
    n0 = int(rng.integers(2, 7))
    edges = I.shape_tree(rng, n0)
    labels = [int(x) for x in rng.permutation(6)[:n0]]
    g = I.random_graph(int(rng.integers(20, 60)), float(rng.uniform(0.05, 0.2)), 6, 2000 + seed)
    t = I.Template(labels, edges)
    assert C.non_local_constraints(labels, edges) == []
    lcc_state = run_prune(g, t, stop_after=0)
    role, ebits, _ = run_brute(g, t)
    assert np.array_equal(lcc_state.role_mask, role)
    assert np.array_equal(lcc_state.edge_bits, ebits)


def _template_diameter(n0, edges):
    G = nx.Graph()
    G.add_nodes_from(range(n0))
    G.add_edges_from(edges)
    return nx.diameter(G)


@pytest.mark.parametrize("seed", range(30))
def test_lcc_sweeps_bounded_by_diameter_plus_one(seed):
    """Complexity section: for acyclic unique-label templates LCC stops
    eliminating after at most diam(G0) + 1 iterations."""
    rng = np.random.Generator(np.random.Philox(3000 + seed))
    n0 = int(rng.integers(2, 8))
    edges = I.shape_tree(rng, n0)
    labels = [int(x) for x in rng.permutation(8)[:n0]]
    rp, col = I.rmat_csr(9, seed=4000 + seed)
    g = I.Graph(rp, col, I.labels_uniform(rp.shape[0] - 1, 8, seed))
    r = run_prune(g, I.Template(labels, edges), stop_after=0)
    assert r.lcc_sweeps[0] <= _template_diameter(n0, edges) + 1


# --------------------------------------- the paper's counterexample figure
def test_cycle_counterexample_lcc_keeps_cc_prunes():
    """3-cycle template; a 3k-cycle whose labels repeat survives LCC and the
    cycle constraint removes it."""
    k = 5
    n = 3 * k
    g = graph_from_edges(n, [(i, (i + 1) % n) for i in range(n)], [i % 3 for i in range(n)])
    t = I.Template([0, 1, 2], [(0, 1), (1, 2), (2, 0)])
    after_lcc = run_prune(g, t, stop_after=0)
    assert all(int(x) != 0 for x in after_lcc.role_mask)
    K0 = C.non_local_constraints(t.labels, t.edges)
    assert [c.kind for c in K0] == [C.CC]
    after_cc = run_prune(g, t, stop_after=1)
    assert not after_cc.role_mask.any() and not after_cc.edge_bits.any()
    assert not run_prune(g, t).role_mask.any()


def test_torus_counterexample_survives_cycles_needs_tds():
    """Two 4-cliques sharing a triangle against a doubly periodic 4x3 torus:
    local and cycle constraints all pass, only the full-template search
    removes every vertex."""
    R, S = 4, 3
    vid = lambda i, j: (i % R) * S + (j % S)
    edges = []
    for i in range(R):
        for j in range(S):
            edges.append((vid(i, j), vid(i + 1, j)))
            edges.append((vid(i, j), vid(i, j + 1)))
    g = graph_from_edges(R * S, edges, [0] * (R * S))
    t_edges = [(a, b) for a in range(5) for b in range(a + 1, 5) if (a, b) != (3, 4)]
    t = I.Template([0] * 5, t_edges)
    lcc_state = run_prune(g, t, stop_after=0)
    assert all(int(x) == 0b11111 for x in lcc_state.role_mask)
    K0 = C.non_local_constraints(t.labels, t.edges)
    all_cc = [i for i, c in enumerate(K0) if c.kind == C.CC]
    # the triangle constraints alone leave every vertex (the torus has triangles)
    tri = [i for i in all_cc if len(K0[i].edges) == 3]
    r = run_prune(g, t, order=tri + [i for i in range(len(K0)) if i not in tri],
                  stop_after=len(tri))
    assert all(int(x) != 0 for x in r.role_mask)
    final = run_prune(g, t)
    assert not final.role_mask.any() and not final.edge_bits.any()
    role, _, cnt = run_brute(g, t)
    assert cnt == 0 and not role.any()


def test_path_counterexample_needs_path_constraint():
    """Same-label template vertices three hops apart: a triangle with a
    single vertex of the repeated label passes LCC but has no match."""
    g = graph_from_edges(3, [(0, 1), (1, 2), (2, 0)], [0, 1, 2])
    t = I.Template([0, 1, 2, 0], [(0, 1), (1, 2), (2, 3)])
    lcc_state = run_prune(g, t, stop_after=0)
    assert all(int(x) != 0 for x in lcc_state.role_mask)
    K0 = C.non_local_constraints(t.labels, t.edges)
    assert [c.kind for c in K0] == [C.PC]
    assert not run_prune(g, t, stop_after=1).role_mask.any()


# -------------------------------------------------------------- invariants
@pytest.mark.parametrize("seed", range(20))
def test_monotone_and_recall_along_the_pipeline(seed):
    g, t = random_case(500 + seed)
    truth, _, _ = run_brute(g, t)
    K0 = C.non_local_constraints(t.labels, t.edges)
    prev = None
    for k in range(len(K0) + 1):
        st = run_prune(g, t, stop_after=k).role_mask
        assert np.all((truth & ~st) == 0)              # 100% recall
        if prev is not None:
            assert np.all((st & ~prev) == 0)           # monotone
        prev = st
    final = run_prune(g, t).role_mask
    assert np.all((final & ~prev) == 0)


@pytest.mark.parametrize("seed", range(15))
def test_order_independence(seed):
    g, t = random_case(700 + seed)
    K0 = C.non_local_constraints(t.labels, t.edges)
    base = run_prune(g, t)
    rng = np.random.Generator(np.random.Philox(seed))
    for _ in range(3):
        r = run_prune(g, t, order=list(rng.permutation(len(K0))))
        assert np.array_equal(r.role_mask, base.role_mask)
        assert np.array_equal(r.edge_bits, base.edge_bits)


@pytest.mark.parametrize("seed", range(10))
def test_permutation_equivariance(seed):
    g, t = random_case(800 + seed)
    r = run_prune(g, t)
    perm = np.random.Generator(np.random.Philox(seed)).permutation(g.n)
    inv = np.argsort(perm)
    edges = [(perm[u], perm[int(g.col[e])]) for u in range(g.n)
             for e in range(g.row_ptr[u], g.row_ptr[u + 1])]
    labels = np.zeros(g.n, dtype=np.uint8)
    labels[perm] = g.labels
    h = graph_from_edges(g.n, edges if edges else np.zeros((0, 2)), labels)
    rh = run_prune(h, t)
    assert np.array_equal(rh.role_mask[perm], r.role_mask)
    assert edge_set_from_bits(h.row_ptr, h.col, rh.edge_bits) == {
        (perm[u], perm[w]) for u, w in edge_set_from_bits(g.row_ptr, g.col, r.edge_bits)}


@pytest.mark.parametrize("seed", range(10))
def test_idempotence_on_the_solution_subgraph(seed):
    g, t = random_case(900 + seed)
    r = run_prune(g, t)
    keep = edge_set_from_bits(g.row_ptr, g.col, r.edge_bits)
    h = graph_from_edges(g.n, list(keep) if keep else np.zeros((0, 2)), g.labels)
    rh = run_prune(h, t)
    assert np.array_equal(rh.role_mask, r.role_mask)
    assert edge_set_from_bits(h.row_ptr, h.col, rh.edge_bits) == keep


@pytest.mark.parametrize("seed", range(20))
def test_structural_invariants_of_the_output(seed):
    g, t = random_case(1100 + seed)
    r = run_prune(g, t)
    es = edge_set_from_bits(g.row_ptr, g.col, r.edge_bits)
    adj = t.adjacency()
    for u, w in es:
        assert (w, u) in es                                   # symmetric
        ru, rw = int(r.role_mask[u]), int(r.role_mask[w])
        assert any((ru >> q) & 1 and (rw >> q2) & 1 for q in range(t.n0) for q2 in adj[q])
    if t.n0 >= 2:
        touched = {u for u, _ in es}
        for v in range(g.n):
            assert (int(r.role_mask[v]) != 0) == (v in touched)
    # closure under label-preserving template automorphisms
    H = nx.Graph()
    for q, lab in enumerate(t.labels):
        H.add_node(q, label=lab)
    H.add_edges_from(t.edges)
    for auto in iso.GraphMatcher(H, H, node_match=lambda a, b: a["label"] == b["label"]).isomorphisms_iter():
        for v in range(g.n):
            rv = int(r.role_mask[v])
            img = 0
            for q in range(t.n0):
                if (rv >> q) & 1:
                    img |= 1 << auto[q]
            assert img == rv


def test_single_vertex_template_is_label_match():
    g = I.random_graph(30, 0.2, 3, 8)
    t = I.Template([2], [])
    r = run_prune(g, t)
    assert np.array_equal(r.role_mask, (g.labels == 2).astype(np.uint64))
    assert not r.edge_bits.any()


def test_empty_and_edgeless_background():
    g = graph_from_edges(5, np.zeros((0, 2)), [0, 1, 0, 1, 0])
    t = I.Template([0, 1], [(0, 1)])
    r = run_prune(g, t)
    assert not r.role_mask.any() and r.edge_bits.shape[0] == 0


# ------------------------------------------------ constraint generation
def test_constraints_square_with_unique_pendant():
    """Step 1 drops the unique-label leaf; the square is the only cycle."""
    K0 = C.non_local_constraints([0, 1, 2, 3, 4], [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4)])
    assert len(K0) == 1 and K0[0].kind == C.CC
    assert K0[0].edges == ((0, 1), (0, 3), (1, 2), (2, 3)) and K0[0].heads == 0b1111


def test_constraints_triangle_square_pendant_by_hand():
    """Worked by hand from Steps 1-5: three simple cycles (triangle, square,
    outer 5-cycle), one path constraint q2-q1-q3-q5 between the repeated
    labels (3 hops, not inside one cycle), and one TDS union of the cycles."""
    labels = [10, 11, 12, 13, 14, 12]
    K0 = C.non_local_constraints(labels, I.TRI_SQUARE_EDGES)
    kinds = [(c.kind, len(c.edges)) for c in K0]
    assert kinds == [(C.CC, 3), (C.PC, 3), (C.CC, 4), (C.CC, 5), (C.TDS_CC, 6)]
    assert K0[1].edges == ((1, 2), (1, 3), (3, 5)) and K0[1].heads == (1 << 2) | (1 << 5)
    assert K0[4].heads == 0b11111


def test_constraints_path_inside_cycle_is_dropped():
    """Step 4(ii): same-label pairs whose shortest path lies in a cycle."""
    labels = [0, 1, 2, 0, 1, 2]
    K0 = C.non_local_constraints(labels, [(i, (i + 1) % 6) for i in range(6)])
    assert [c.kind for c in K0] == [C.CC]


def test_constraints_k4():
    K0 = C.non_local_constraints([0] * 4, [(a, b) for a in range(4) for b in range(a + 1, 4)])
    assert [(c.kind, len(c.edges)) for c in K0] == [(C.CC, 3)] * 4 + [(C.CC, 4)] * 3 + [(C.TDS_CC, 6)]


def test_constraints_tds_path_union():
    """Two repeated-label pairs whose paths share a vertex merge into a TDS
    path constraint reduced to a spanning tree."""
    # path 0-1-2-3-4-5-6 with labels A B C A B C D: pairs (0,3), (1,4), (2,5)
    labels = [0, 1, 2, 0, 1, 2, 3]
    edges = [(i, i + 1) for i in range(6)]
    K0 = C.non_local_constraints(labels, edges)
    kinds = [c.kind for c in K0]
    assert kinds == [C.PC, C.PC, C.PC, C.TDS_PC]
    assert K0[3].edges == ((0, 1), (1, 2), (2, 3), (3, 4), (4, 5))
    assert K0[3].heads == 0b111111


# ---------------------------------------------------------------- inputs
def test_philox_known_answers():
    """Published known-answer vectors of Philox4x32-10 (Random123)."""
    assert I.philox4x32_10([0] * 4, [0] * 2) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    assert I.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == (
        0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)
    assert I.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344],
                           [0xA4093822, 0x299F31D0]) == (0xD16CFE09, 0x94FDCCEB, 0x5001E420,
                                                          0x24126EA1)


def test_rmat_csr_is_simple_symmetric_sorted():
    rp, col = I.rmat_csr(11, seed=3)
    n = rp.shape[0] - 1
    src = np.repeat(np.arange(n), np.diff(rp))
    assert np.all(src != col)
    for v in range(0, n, 37):
        row = col[rp[v]:rp[v + 1]]
        assert np.all(np.diff(row) > 0)
    fwd = set(zip(src.tolist(), col.tolist()))
    assert all((w, u) in fwd for u, w in list(fwd)[:20000])
    assert I.labels_log2deg(rp).tolist() == [int(d).bit_length() for d in np.diff(rp)]


@pytest.mark.parametrize("k", [2, 3])
def test_distinct_count_rule_star_with_repeated_leaf_labels(k):
    """K_{1,k} whose leaves share one label: the LCC rule's distinct-neighbour
    count makes the LCC fixpoint exact -- a centre needs k distinct
    neighbours of the leaf label, a leaf needs a valid centre."""
    g = I.random_graph(90, 0.04, 2, 40 + k)
    t = I.Template([0] + [1] * k, [(0, i) for i in range(1, k + 1)])
    st = run_prune(g, t, stop_after=0)
    nb = [g.col[g.row_ptr[v]:g.row_ptr[v + 1]].tolist() for v in range(g.n)]
    centre = [g.labels[v] == 0 and sum(int(g.labels[u]) == 1 for u in nb[v]) >= k
              for v in range(g.n)]
    leaves = ((1 << (k + 1)) - 1) & ~1
    for v in range(g.n):
        exp = 1 if centre[v] else 0
        if g.labels[v] == 1 and any(centre[u] for u in nb[v]):
            exp |= leaves
        assert int(st.role_mask[v]) == exp
    role, _, _ = run_brute(g, t)
    assert np.array_equal(st.role_mask, role)


@pytest.mark.parametrize("seed", range(40))
def test_exact_sample_equals_bruteforce_on_sampled_vertices(seed):
    """The sampled exact step (used for parity at sizes where the whole
    exact step is too slow on the CPU) gives, for every sampled vertex, the
    brute-force role mask and membership of each of its entries -- from the
    label-only state and from the state after the constraint loop."""
    g, t = random_case(seed)
    role, ebits, _ = oracle.bruteforce(g.row_ptr, g.col, g.labels, t.labels, t.edges)
    gg = oracle._G(g.row_ptr, g.col, g.labels)
    tt = oracle._T(t.labels, t.edges)
    rng = np.random.Generator(np.random.Philox(seed))
    verts = np.sort(rng.choice(g.n, size=min(g.n, 12), replace=False))
    for om in (oracle.init_roles(gg, tt),
               oracle.state(g.row_ptr, g.col, g.labels, t.labels, t.edges)):
        r, inc, off = oracle.exact_sample(gg, tt, om, verts)
        assert np.array_equal(r, role[verts])
        for i, v in enumerate(verts):
            for j, e in enumerate(range(g.row_ptr[v], g.row_ptr[v + 1])):
                want = (int(ebits[e >> 6]) >> (e & 63)) & 1
                assert inc[off[i] + j] == want, (seed, v, e)


def test_relaxations_are_the_connected_deletion_variants_up_to_isomorphism():
    def nxt(t):
        H = nx.Graph()
        for q, lab in enumerate(t.labels):
            H.add_node(q, label=lab)
        H.add_edges_from(t.edges)
        return H
    nm = iso.categorical_node_match("label", None)
    for labels in ([1, 2, 3, 4, 5, 6, 7, 4], [1, 1, 1, 1, 1, 1, 1, 1], [1, 2, 1, 2, 1, 2, 1, 2]):
        base = I.Template(labels, I.THETA8_EDGES, "b")
        rel = I.relaxations(base)
        assert rel[0] is base
        Hs = [nxt(t) for t in rel]
        for i in range(len(Hs)):
            assert nx.is_connected(Hs[i]) and Hs[i].number_of_nodes() == 8
            assert 7 <= Hs[i].number_of_edges() <= 9
            for j in range(i):
                assert not nx.is_isomorphic(Hs[i], Hs[j], node_match=nm)
        # every connected variant with one or two deletions is one of them
        for d in (1, 2):
            for dels in itertools.combinations(range(9), d):
                es = [e for k, e in enumerate(I.THETA8_EDGES) if k not in dels]
                H = nxt(I.Template(labels, es))
                if not nx.is_connected(H):
                    continue
                assert any(nx.is_isomorphic(H, K, node_match=nm) for K in Hs)
    # distinct labels but the repeated pair: 1 + 8 + 19 variants
    assert len(I.relaxations(I.Template([1, 2, 3, 4, 5, 6, 7, 4], I.THETA8_EDGES))) == 28
