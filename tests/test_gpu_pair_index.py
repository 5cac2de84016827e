"""GPU checks of the label-pair subgraph (pm_build_pair_index): its size is
the number of entries whose label pair is that of a template edge (counted
here with numpy), prunes that start their first compaction from it give the
oracle's complete sets (batched and one call per template, with the
witness joins on), a template whose label pairs it does not hold and the
edge-elimination ablation fall back to the whole graph, match counts are
unchanged, and count 0 frees it.  The first LCC sweep of a covered template
reads the subgraph's own count index (also past 16-bit row counts)."""
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


def load(pmmod, torch_dev, g):
    torch, dev = torch_dev
    ctx = pmmod.PM(0)
    ctx.load_graph(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                   torch.from_numpy(np.ascontiguousarray(g.labels)).to(dev))
    return ctx


def pair_entries(g, ts):
    nl = int(max(max(t.labels) for t in ts)) + 1
    adj = np.zeros((max(nl, int(g.labels.max()) + 1),) * 2, dtype=bool)
    for t in ts:
        for a, b in t.edges:
            adj[t.labels[a], t.labels[b]] = adj[t.labels[b], t.labels[a]] = True
    src = np.repeat(g.labels.astype(np.int64), np.diff(g.row_ptr))
    return int(adj[src, g.labels[g.col].astype(np.int64)].sum())


def same_as(pmmod, role, edge, ref, what):
    r, e = pmmod.to_u64(role), pmmod.to_u64(edge)
    assert np.array_equal(r, ref.role_mask), f"{what}: roles differ"
    assert np.array_equal(e, ref.edge_bits), f"{what}: edges differ"


@pytest.fixture(scope="module", params=[14, 16])
def relax_case(request):
    scale = request.param
    rp, col = I.rmat_csr(scale, seed=scale + 200)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    ts = I.relaxations(I.template_theta8(g, 1))
    refs = [oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges) for t in ts]
    return scale, g, ts, refs


def test_size_and_parity_of_relaxation_batches(pmmod, torch_dev, relax_case):
    torch, dev = torch_dev
    scale, g, ts, refs = relax_case
    ctx = load(pmmod, torch_dev, g)
    first = ctx.load_templates(ts)
    assert ctx.graph_info()["pair_entries"] == -1
    ms = ctx.build_pair_index(first, len(ts))
    info = ctx.graph_info()
    want = pair_entries(g, ts)
    log(f"scale {scale}: pair subgraph {info['pair_entries']} of {g.m} entries, {ms:.2f} ms")
    assert info["pair_entries"] == want and info["ms_pair_index"] > 0
    for settings in ({}, {"witness": 1, "expand_edges": 0, "relist": 0},
                     {"search_grid": 64, "search_grid_solo": 2048}):
        for k, v in settings.items():
            ctx.set_param(k, v)
        T = len(ts)
        rb = torch.empty((T, g.n), dtype=torch.int64, device=dev)
        eb = torch.empty((T, (g.m + 63) // 64), dtype=torch.int64, device=dev)
        ctx.prune(first, count=T, role_mask=rb, edge_bits=eb, batch_streams=4)
        for i, ref in enumerate(refs):
            same_as(pmmod, rb[i], eb[i], ref, f"scale {scale} {settings} batched template {i}")
        for i in (0, 1, T - 1):
            role, edge, _ = ctx.prune(first + i)
            same_as(pmmod, role[0], edge[0], refs[i], f"scale {scale} {settings} template {i}")
    ctx.close()


def test_uncovered_template_and_ablation_fall_back(pmmod, torch_dev):
    rp, col = I.rmat_csr(14, seed=321)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    a = I.template_tri_square(g, 3)
    b = I.templates_batch(g, 5, count=6)
    ts = [a] + b
    refs = [oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges) for t in ts]
    pairs_a = {(a.labels[x], a.labels[y]) for x, y in a.edges}
    pairs_a |= {(q, p) for p, q in pairs_a}
    uncovered = [i for i, t in enumerate(b, 1)
                 if any((t.labels[x], t.labels[y]) not in pairs_a for x, y in t.edges)]
    assert uncovered, "every batch template is covered by the first one's pairs"
    ctx = load(pmmod, torch_dev, g)
    first = ctx.load_templates(ts)
    ctx.build_pair_index(first, 1)
    assert ctx.graph_info()["pair_entries"] == pair_entries(g, [a])
    for i, ref in enumerate(refs):
        role, edge, _ = ctx.prune(first + i)
        same_as(pmmod, role[0], edge[0], ref, f"template {i} (covered: {i not in uncovered})")
    role, edge, _ = ctx.prune(first, ablate=pmmod.PM_ABLATE_EDGE_ELIMINATION)
    same_as(pmmod, role[0], edge[0], refs[0], "edge elimination ablated")
    ctx.close()


def test_counts_unchanged_and_count_zero_frees(pmmod, torch_dev):
    rp, col = I.rmat_csr(13, seed=77)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    t = I.template_tri_square(g, 2)
    ctx = load(pmmod, torch_dev, g)
    tid = ctx.load_templates([t])
    before = ctx.count_matches(tid)
    ctx.build_pair_index(tid, 1)
    after = ctx.count_matches(tid)
    n_maps, _ = oracle.enumerate_maps(g.row_ptr, g.col, g.labels, t.labels, t.edges, cap=1)
    assert before["maps"] == after["maps"] == n_maps and after["complete"] == 1
    ctx.build_pair_index(tid, 0)
    assert ctx.graph_info()["pair_entries"] == -1
    with pytest.raises(pmmod.PMError):
        ctx.build_pair_index(tid + 5, 1)
    ctx.close()


def test_first_sweep_from_pair_counts(pmmod, torch_dev, relax_case):
    """With the label-pair subgraph built, the first LCC sweep of a covered
    template reads the subgraph's own count index: the LCC fixpoint (no
    non-local check) still equals the oracle's, and so does the state after
    the first constraints."""
    scale, g, ts, _ = relax_case
    ctx = load(pmmod, torch_dev, g)
    first = ctx.load_templates(ts)
    ctx.build_pair_index(first, len(ts))
    for i in (0, 1, 5, len(ts) - 1):
        t = ts[i]
        for k in (0, 1):
            ref = oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges, stop_after=k)
            role, edge, st = ctx.prune(first + i, stop_after=k)
            same_as(pmmod, role[0], edge[0], ref, f"scale {scale} template {i} after {k}")
    ctx.close()


def test_pair_counts_saturate_on_rows_past_16_bits(pmmod, torch_dev):
    """A row of the label-pair subgraph with more than 65,535 entries of one
    label: the 16-bit tile counters must saturate instead of wrapping.  A
    star whose centre (label 0) has 65,546 leaves (label 2); the template is
    a star with 20 leaves of label 2, so the centre keeps its role only if
    its count of label-2 neighbours reads at least 20 (a wrapped counter
    would read 10)."""
    leaves = 65546
    n = leaves + 1
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1] = leaves
    rp[2:] = leaves + np.arange(1, leaves + 1)
    col = np.concatenate([np.arange(1, n, dtype=np.int32), np.zeros(leaves, dtype=np.int32)])
    lab = np.full(n, 2, dtype=np.uint8)
    lab[0] = 0
    g = I.Graph(rp, col, lab)
    t = I.Template([0] + [2] * 20, [(0, j) for j in range(1, 21)])
    ref = oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges, stop_after=0)
    assert ref.role_mask[0] == 1
    ctx = load(pmmod, torch_dev, g)
    tid = ctx.load_templates([t])
    for built in (False, True):
        if built:
            ctx.build_pair_index(tid, 1)
            assert ctx.graph_info()["pair_entries"] == 2 * leaves
        role, edge, _ = ctx.prune(tid, stop_after=0)
        same_as(pmmod, role[0], edge[0], ref, f"star, pair subgraph built: {built}")
    ctx.close()
