"""GPU parity of the witness joins of the exact step: a candidate edge is
certified without a search when the recorded matches of its two ends,
joined across a bridge of the template, form a match.  The complete sets
must equal the oracle's with the joins on, on a hand-built graph where the
only join on offer puts two vertices of one label on the same image (it
must be refused), on a cycle whose two recorded matches share a vertex but
cannot be spliced, on tiny random graphs over few labels with cyclic
templates, on trees and one-cycle templates with repeated labels, and on
the theta8 relaxations (mostly trees) at two scales."""
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


def ctx_on(pmmod, torch_dev, g, settings):
    torch, dev = torch_dev
    ctx = pmmod.PM(0)
    ctx.load_graph(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                   torch.from_numpy(np.ascontiguousarray(g.labels)).to(dev))
    for k, v in settings.items():
        ctx.set_param(k, v)
    return ctx


def check_all(pmmod, ctx, g, ts, refs, what):
    first = ctx.load_templates(ts)
    joins = 0
    for i, (t, ref) in enumerate(zip(ts, refs)):
        role, edge, st = ctx.prune(first + i)
        r, e = pmmod.to_u64(role[0]), pmmod.to_u64(edge[0])
        bad_v = np.nonzero(r != ref.role_mask)[0]
        assert bad_v.size == 0, f"{what} template {i}: {bad_v.size} role masks differ"
        bad_e = np.nonzero(e != ref.edge_bits)[0]
        assert bad_e.size == 0, f"{what} template {i}: {bad_e.size} edge words differ"
        joins += st["join_edges"]
    return joins


JOIN_ON = [{"witness": 1}, {"witness": 1, "expand_edges": 0},
           {"witness": 1, "expand": 0, "search_grid": 3},
           {"witness": 1, "relist": 0, "expand_max": -1}]


@pytest.mark.parametrize("settings", JOIN_ON)
def test_join_refuses_two_images_of_one_label(pmmod, torch_dev, settings):
    # path template X-Y-Z-X (a, b, c, d).  u=0 X, w=1 Y, z=2 Z form a
    # triangle; u'=3 X hangs on w; u-w2-z2-x2 (4, 5, 6) is a second path.
    # The only match through b=w is (3, 1, 2, 0); the only one through a=u
    # is (0, 4, 5, 6).  Joining them across the bridge (a, b) for the edge
    # {0, 1} would put a and d both on vertex 0, and no match uses {0, 1}.
    rp, col = csr(7, [(0, 1), (1, 2), (2, 0), (3, 1), (0, 4), (4, 5), (5, 6)])
    g = I.Graph(rp, col, np.array([0, 1, 2, 0, 1, 2, 0], dtype=np.uint8))
    t = I.Template([0, 1, 2, 0], [(0, 1), (1, 2), (2, 3)])
    ref = oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges)
    k01 = int(np.nonzero(g.col[g.row_ptr[0]:g.row_ptr[1]] == 1)[0][0])
    assert not (int(ref.edge_bits[0]) >> k01) & 1, "the oracle keeps edge {0, 1}"
    ctx = ctx_on(pmmod, torch_dev, g, settings)
    check_all(pmmod, ctx, g, [t], [ref], f"hand case {settings}")
    ctx.close()


@pytest.mark.parametrize("settings", JOIN_ON)
def test_cycle_edge_between_two_recorded_matches(pmmod, torch_dev, settings):
    # 6-cycle template a-b-c-d-e-f labelled A B Z D Z F.  The only match
    # through a=u (vertex 0) is (0, 2, 4, 7, 5, 8), the only one through b=w
    # (vertex 1) is (3, 1, 5, 7, 6, 9).  Both put d on vertex 7, so the
    # edge {0, 1} would close a cycle from halves of the two -- but e (from
    # the first) and c (from the second) are both vertex 5, and no match
    # uses the edge: neither a swap nor a join may certify it.
    E = [(0, 2), (2, 4), (4, 7), (7, 5), (5, 8), (8, 0), (3, 1), (1, 5), (7, 6), (6, 9),
         (9, 3), (0, 1)]
    rp, col = csr(10, E)
    g = I.Graph(rp, col, np.array([0, 1, 1, 0, 2, 2, 2, 3, 4, 4], dtype=np.uint8))
    t = I.Template([0, 1, 2, 3, 2, 4], [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 0)])
    ref = oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges)
    k01 = int(np.nonzero(g.col[g.row_ptr[0]:g.row_ptr[1]] == 1)[0][0])
    assert not (int(ref.edge_bits[0]) >> k01) & 1, "the oracle keeps edge {0, 1}"
    ctx = ctx_on(pmmod, torch_dev, g, settings)
    check_all(pmmod, ctx, g, [t], [ref], f"cycle case {settings}")
    ctx.close()


def random_cyclic_case(seed):
    # tiny random graphs over 1-3 labels (many same-label pairs, so joins
    # that would reuse an image are frequent) and cyclic templates
    rng = np.random.Generator(np.random.Philox(seed + 5000))
    n = int(rng.integers(10, 48))
    p = float(rng.uniform(0.08, 0.35))
    nl = int(rng.integers(1, 4))
    g = I.random_graph(n, p, nl, seed + 5000)
    n0 = int(rng.integers(3, 8))
    kind = seed % 3
    if kind == 0:
        edges = I.shape_one_cycle(rng, n0)
    elif kind == 1:
        edges = I.shape_two_cycles(rng, max(n0, 5))
    else:
        edges = I.shape_tree(rng, n0)
    n0 = max(max(a, b) for a, b in edges) + 1
    labels = [int(x) for x in rng.integers(0, nl, size=n0)]
    return g, I.Template(labels, edges)


@pytest.mark.parametrize("seed", range(90))
def test_random_tiny_cases_with_joins(pmmod, torch_dev, seed):
    g, t = random_cyclic_case(seed)
    ref = oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges)
    for settings in JOIN_ON[:2]:
        ctx = ctx_on(pmmod, torch_dev, g, settings)
        check_all(pmmod, ctx, g, [t], [ref], f"seed {seed} {t.labels}/{t.edges} {settings}")
        ctx.close()


@pytest.fixture(scope="module")
def mixed_case():
    rp, col = I.rmat_csr(14, seed=414)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    rng = np.random.Generator(np.random.Philox(414))
    ts = []
    while len(ts) < 12:
        n0 = int(rng.integers(4, 9))
        edges = I.shape_tree(rng, n0) if len(ts) % 2 == 0 else I.shape_one_cycle(rng, n0)
        n0 = max(max(a, b) for a, b in edges) + 1
        # labels of a seeded occurrence in which vertices 0 and n0 - 1 share one
        try:
            t = I.extract_template(g, n0, edges, int(rng.integers(1 << 30)),
                                   repeat_pairs=[(0, n0 - 1)])
        except RuntimeError:
            continue
        ts.append(t)
    refs = [oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges) for t in ts]
    return g, ts, refs


@pytest.mark.parametrize("settings", JOIN_ON)
def test_trees_and_cycles_with_repeated_labels(pmmod, torch_dev, mixed_case, settings):
    g, ts, refs = mixed_case
    ctx = ctx_on(pmmod, torch_dev, g, settings)
    joins = check_all(pmmod, ctx, g, ts, refs, f"mixed {settings}")
    log(f"mixed {settings}: {joins} joined edges")
    ctx.close()


@pytest.mark.parametrize("scale", [14, 16])
def test_theta8_relaxations_with_joins(pmmod, torch_dev, scale):
    rp, col = I.rmat_csr(scale, seed=scale + 100)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    ts = I.relaxations(I.template_theta8(g, 0))
    refs = [oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges) for t in ts]
    for settings in JOIN_ON[:2]:
        ctx = ctx_on(pmmod, torch_dev, g, settings)
        joins = check_all(pmmod, ctx, g, ts, refs, f"theta8 s{scale} {settings}")
        log(f"theta8 scale {scale} {settings}: {joins} joined edges")
        assert joins > 0, "no candidate edge was certified by a join"
        ctx.close()
