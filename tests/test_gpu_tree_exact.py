"""GPU parity of the search-free final step for acyclic templates whose
labels are unique except for one pair of vertices (setting "tree_exact"):
the complete sets equal the oracle's on hand-built graphs where the path
between the pair can only close on one vertex (LCC keeps those roles, no
match uses them), on tiny random graphs over few labels with random trees
of 2-8 vertices, on trees extracted from R-MAT graphs, and on the theta8
relaxations (19 of 28 are trees), with the setting on and off; with it on
no search runs for such templates, neither a non-local check nor a final
search.  A prune that stops after some constraints still checks them."""
import sys

import numpy as np
import pytest

import oracle
from paper_1912_08453_amd import inputs as I

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda", 0)


@pytest.fixture(scope="module")
def pmmod():
    from paper_1912_08453_amd import pm
    pm.load_library()
    return pm


def csr(n, edges):
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    rp = np.zeros(n + 1, dtype=np.int64)
    col = []
    for v in range(n):
        col += sorted(adj[v])
        rp[v + 1] = len(col)
    return rp, np.array(col, dtype=np.int32)


def one_pair_tree(t):
    """Acyclic, connected, one label on exactly two vertices, the rest unique."""
    n0 = len(t.labels)
    if len(t.edges) != n0 - 1 or n0 < 2:
        return False
    _, counts = np.unique(np.asarray(t.labels), return_counts=True)
    return sorted(counts.tolist()) == [1] * (n0 - 2) + [2]


def check(pmmod, torch_dev, g, ts, what, tree_exact_values=(1, 0)):
    torch, dev = torch_dev
    refs = [oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges) for t in ts]
    ctx = pmmod.PM(0)
    ctx.load_graph(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                   torch.from_numpy(np.ascontiguousarray(g.labels)).to(dev))
    first = ctx.load_templates(ts)
    for te in tree_exact_values:
        ctx.set_param("tree_exact", te)
        for i, (t, ref) in enumerate(zip(ts, refs)):
            role, edge, st = ctx.prune(first + i)
            r, e = pmmod.to_u64(role[0]), pmmod.to_u64(edge[0])
            tag = f"{what} tree_exact={te} template {i} {t.labels}/{t.edges}"
            bad_v = np.nonzero(r != ref.role_mask)[0]
            assert bad_v.size == 0, f"{tag}: {bad_v.size} role masks differ, e.g. vertex {bad_v[:5]}"
            bad_e = np.nonzero(e != ref.edge_bits)[0]
            assert bad_e.size == 0, f"{tag}: {bad_e.size} edge words differ"
            if te and one_pair_tree(t):
                assert st["vertex_queries"] == 0 and st["edge_queries"] == 0, \
                    f"{tag}: a search ran"
                # the path sweeps decide the path constraint: no search-based
                # non-local check runs either
                assert st["constraints"] == 0, f"{tag}: a non-local check ran"
    ctx.close()
    return refs


def test_path_that_closes_on_one_vertex(pmmod, torch_dev):
    # template a-x-y-b, labels A X Y A (path of 3 edges between the pair).
    # Vertex 0 (A), 1 (X), 2 (Y) form a triangle: every homomorphism through
    # 1 or 2 puts a and b both on 0.  Vertices 3 (A) - 4 (X) - 5 (Y) - 6 (A)
    # form a real match.  Vertex 7 (Y) hangs on 4 and reaches only A-vertex 3
    # through 4, so it is not in a match either.
    E = [(0, 1), (1, 2), (2, 0), (3, 4), (4, 5), (5, 6), (4, 7)]
    rp, col = csr(8, E)
    g = I.Graph(rp, col, np.array([0, 1, 2, 0, 1, 2, 0, 2], dtype=np.uint8))
    t = I.Template([0, 1, 2, 0], [(0, 1), (1, 2), (2, 3)])
    ref = check(pmmod, torch_dev, g, [t], "closing path")[0]
    assert ref.role_mask[0] == 0 and ref.role_mask[1] == 0 and ref.role_mask[7] == 0
    assert ref.role_mask[3] != 0


def test_pair_with_branches_and_adjacent_pair(pmmod, torch_dev):
    # template: a(A)-x(X)-b(A) with a pendant p(P) on a and q(Q) on x; and the
    # single edge A-A.  Graph: a star centred on X-vertex 0 with A-leaves 1
    # and 2 (only 1 has a P neighbour), Q-vertex 3 on 0; A-vertices 4-5
    # adjacent; X-vertex 6 with a single A neighbour 7 (closes on one vertex).
    E = [(0, 1), (0, 2), (1, 8), (0, 3), (4, 5), (6, 7), (7, 9), (6, 10)]
    lab = [1, 0, 0, 3, 0, 0, 1, 0, 2, 2, 3]
    rp, col = csr(len(lab), E)
    g = I.Graph(rp, col, np.array(lab, dtype=np.uint8))
    t1 = I.Template([0, 1, 0, 2, 3], [(0, 1), (1, 2), (0, 3), (1, 4)])
    t2 = I.Template([0, 0], [(0, 1)])
    refs = check(pmmod, torch_dev, g, [t1, t2], "branches")
    assert refs[0].role_mask[6] == 0 and refs[0].role_mask[0] != 0


def random_case(seed):
    rng = np.random.Generator(np.random.Philox(seed + 7000))
    n0 = int(rng.integers(2, 9))
    edges = I.shape_tree(rng, n0)
    nl = n0 - 1 + int(rng.integers(0, 2))
    labs = [int(x) for x in rng.permutation(nl)[:n0 - 1]]
    a, b = (int(x) for x in rng.choice(n0, size=2, replace=False))
    order = [q for q in range(n0) if q != b]
    labels = [0] * n0
    for q, L in zip(order, labs):
        labels[q] = L
    labels[b] = labels[a]
    n = int(rng.integers(12, 60))
    p = float(rng.uniform(0.06, 0.3))
    g = I.random_graph(n, p, nl, seed + 7000)
    return g, I.Template(labels, edges)


@pytest.mark.parametrize("chunk", range(6))
def test_random_one_pair_trees(pmmod, torch_dev, chunk):
    for seed in range(chunk * 25, chunk * 25 + 25):
        g, t = random_case(seed)
        assert one_pair_tree(t)
        check(pmmod, torch_dev, g, [t], f"seed {seed}")


@pytest.mark.parametrize("scale", [12, 14])
def test_extracted_trees_on_rmat(pmmod, torch_dev, scale):
    rp, col = I.rmat_csr(scale, seed=scale + 300)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    rng = np.random.Generator(np.random.Philox(scale + 300))
    ts = []
    while len(ts) < 10:
        n0 = int(rng.integers(3, 9))
        edges = I.shape_tree(rng, n0)
        a, b = (int(x) for x in rng.choice(n0, size=2, replace=False))
        try:
            t = I.extract_template(g, n0, edges, int(rng.integers(1 << 30)), repeat_pairs=[(a, b)])
        except RuntimeError:
            continue
        if one_pair_tree(t):
            ts.append(t)
    check(pmmod, torch_dev, g, ts, f"rmat scale {scale}")


@pytest.mark.parametrize("scale", [14, 16])
def test_theta8_relaxations(pmmod, torch_dev, scale):
    rp, col = I.rmat_csr(scale, seed=scale + 100)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    ts = I.relaxations(I.template_theta8(g, 0))
    assert sum(one_pair_tree(t) for t in ts) == 19
    check(pmmod, torch_dev, g, ts, f"theta8 scale {scale}", tree_exact_values=(1,))
