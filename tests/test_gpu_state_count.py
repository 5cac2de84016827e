"""GPU parity of the state, reuse, counting and workspace entry points
against the oracle: export of the pruning state after k constraints and its
import into a fresh context (checkpoint and resume), the candidate set and
solution reuse of the interactive incremental search, match counting and
enumeration on the pruned graph, the design-decision ablations (same
output, other work), and a caller-owned workspace.  Everything is integer
and bit-exact."""
import itertools
import sys

import networkx as nx
import numpy as np
import pytest

import oracle
from oracle import constraints as C
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


def case(seed):
    rng = np.random.Generator(np.random.Philox(4400 + seed))
    n = int(rng.integers(10, 40))
    nl = int(rng.integers(1, 4))
    g = I.random_graph(n, float(rng.uniform(0.08, 0.4)), nl, 4400 + seed)
    kind = seed % 4
    n0 = int(rng.integers(3, 7))
    if kind == 0:
        edges = I.shape_tree(rng, n0)
    elif kind == 1:
        edges = I.shape_one_cycle(rng, n0)
    elif kind == 2:
        edges = I.shape_two_cycles(rng, max(n0, 5))
    else:
        edges = I.shape_k4(rng, max(n0, 4))
    n0 = max(max(a, b) for a, b in edges) + 1
    labels = [int(x) for x in rng.integers(0, nl, size=n0)]
    return g, I.Template(labels, edges)


def rmat_case(scale, seed, tseed=0):
    rp, col = I.rmat_csr(scale, seed=seed)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    return g, I.template_tri_square(g, tseed)


def load(pmmod, torch_dev, g):
    torch, dev = torch_dev
    ctx = pmmod.PM(0)
    ctx.load_graph(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                   torch.from_numpy(np.ascontiguousarray(g.labels)).to(dev))
    return ctx


def u64(pmmod, t):
    return pmmod.to_u64(t.reshape(-1))


CASES = [("random", s) for s in range(16)] + [("rmat12", 12), ("rmat14", 14)]


def get_case(kind, s):
    if kind == "random":
        return case(s)
    return rmat_case(s, 100 + s)


# ------------------------------------------------------- export / import
@pytest.mark.parametrize("kind,s", CASES)
def test_export_then_import_into_a_fresh_context(pmmod, torch_dev, kind, s):
    torch, dev = torch_dev
    g, t = get_case(kind, s)
    log(f"export/import {kind} {s} labels={t.labels} edges={t.edges}")
    K = len(C.non_local_constraints(t.labels, t.edges))
    ref = oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges)
    a = load(pmmod, torch_dev, g)
    b = load(pmmod, torch_dev, g)
    ta = a.load_templates([t])
    tb = b.load_templates([t])
    for k in sorted({0, K // 2, K}):
        state, done = a.export_state(ta, stop_after=k)
        want = oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges, stop_after=k)
        assert np.array_equal(u64(pmmod, state), want.role_mask), f"state after {k}"
        assert done & ~((1 << k) - 1) == 0
        # resume in the other context: the oracle's complete set
        r, e, st = b.import_state(tb, state.clone(), done)
        assert np.array_equal(u64(pmmod, r), ref.role_mask), f"resume from {k}: roles"
        assert np.array_equal(u64(pmmod, e), ref.edge_bits), f"resume from {k}: edges"
        assert st["done_mask"] & done == done
        # resume to the end of the constraint loop only: the oracle's state
        r2, e2, _ = b.import_state(tb, state.clone(), done, stop_after=K)
        want2 = oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges, stop_after=K)
        assert np.array_equal(u64(pmmod, r2), want2.role_mask), f"state {k} -> {K}"
        assert np.array_equal(u64(pmmod, e2), want2.edge_bits)
    a.close()
    b.close()


# ----------------------------------------------- incremental search reuse
def connected(n0, edges):
    G = nx.Graph()
    G.add_nodes_from(range(n0))
    G.add_edges_from(edges)
    return nx.is_connected(G)


@pytest.mark.parametrize("kind,s", CASES)
def test_candidate_set_equals_oracle(pmmod, torch_dev, kind, s):
    g, t = get_case(kind, s)
    ctx = load(pmmod, torch_dev, g)
    tid = ctx.load_templates([t])
    r, e, _ = ctx.prune(tid, mode=pmmod.PM_MODE_CANDIDATE)
    want_r, want_e = oracle.candidate_set(g.row_ptr, g.col, g.labels, t.labels, t.edges)
    assert np.array_equal(u64(pmmod, r), want_r)
    assert np.array_equal(u64(pmmod, e), want_e)
    ctx.close()


@pytest.mark.parametrize("kind,s", CASES)
def test_edge_edits_reuse_the_previous_solution(pmmod, torch_dev, kind, s):
    """Adding an edge: start from the previous complete set.  Deleting an
    edge: start from the candidate set with the previous complete set as
    known roles and edges.  Both equal the oracle's prune of the edited
    template."""
    torch, dev = torch_dev
    g, t = get_case(kind, s)
    n0 = len(t.labels)
    ctx = load(pmmod, torch_dev, g)
    tid = ctx.load_templates([t])
    r0, e0, _ = ctx.prune(tid)
    r0, e0 = r0.clone(), e0.clone()
    cand, _, _ = ctx.prune(tid, mode=pmmod.PM_MODE_CANDIDATE)
    cand = cand.clone()
    missing = [(a, b) for a in range(n0) for b in range(a + 1, n0) if (a, b) not in set(t.edges)]
    if missing:
        plus = I.Template(t.labels, sorted(t.edges + [missing[s % len(missing)]]))
        tp = ctx.load_templates([plus])
        r, e, _ = ctx.prune(tp, init_state=r0)
        ref = oracle.prune(g.row_ptr, g.col, g.labels, plus.labels, plus.edges)
        assert np.array_equal(u64(pmmod, r), ref.role_mask), f"add {plus.edges}"
        assert np.array_equal(u64(pmmod, e), ref.edge_bits)
    for drop in t.edges:
        keep = [x for x in t.edges if x != drop]
        if not connected(n0, keep):
            continue
        minus = I.Template(t.labels, keep)
        tm = ctx.load_templates([minus])
        r, e, st = ctx.prune(tm, init_state=cand, known_roles=r0, known_edges=e0)
        ref = oracle.prune(g.row_ptr, g.col, g.labels, minus.labels, minus.edges)
        assert np.array_equal(u64(pmmod, r), ref.role_mask), f"delete {drop}"
        assert np.array_equal(u64(pmmod, e), ref.edge_bits), f"delete {drop}"
        break
    ctx.close()


# ------------------------------------------------------ counting
def automorphisms(t):
    n0 = len(t.labels)
    E = {tuple(sorted(e)) for e in t.edges}
    c = 0
    for p in itertools.permutations(range(n0)):
        if all(t.labels[p[q]] == t.labels[q] for q in range(n0)) and \
                {tuple(sorted((p[a], p[b]))) for a, b in E} == E:
            c += 1
    return c


@pytest.mark.parametrize("kind,s", CASES)
def test_match_count_and_enumeration(pmmod, torch_dev, kind, s):
    torch, dev = torch_dev
    g, t = get_case(kind, s)
    cnt, _ = oracle.enumerate_maps(g.row_ptr, g.col, g.labels, t.labels, t.edges, cap=1)
    cnt, maps = oracle.enumerate_maps(g.row_ptr, g.col, g.labels, t.labels, t.edges,
                                      cap=max(cnt, 1))
    log(f"count {kind} {s}: {cnt} maps")
    ctx = load(pmmod, torch_dev, g)
    tid = ctx.load_templates([t])
    r, _, _ = ctx.prune(tid)
    aut = automorphisms(t) if len(t.labels) <= 8 else None
    for state in (r, None):
        res = ctx.count_matches(tid, state=state, cap=max(cnt, 1))
        assert res["maps"] == cnt, (res, cnt)
        assert res["written"] == cnt
        got = res["maps_out"].cpu().numpy()
        if cnt:
            got = got[np.lexsort(got.T[::-1])]
        assert np.array_equal(got, maps)
        if aut is not None:
            assert res["automorphisms"] == aut
            assert res["subgraphs"] * aut == cnt
    # a small cap writes that many valid maps and still counts them all
    if cnt > 3:
        res = ctx.count_matches(tid, state=r, cap=3)
        assert res["maps"] == cnt and res["written"] == 3
        allm = {tuple(x) for x in maps.tolist()}
        assert all(tuple(x) in allm for x in res["maps_out"].cpu().numpy().tolist())
    ctx.close()


def test_match_count_with_split_searches(pmmod, torch_dev):
    """A one-step split budget splits nearly every counting search; the
    count is the same."""
    g, t = rmat_case(14, 114)
    cnt, _ = oracle.enumerate_maps(g.row_ptr, g.col, g.labels, t.labels, t.edges, cap=1)
    ctx = load(pmmod, torch_dev, g)
    tid = ctx.load_templates([t])
    r, _, _ = ctx.prune(tid)
    for budget in (1, 5, 0):
        ctx.set_param("split_budget", budget)
        res = ctx.count_matches(tid, state=r)
        assert res["maps"] == cnt and res["complete"] == 1
    # a limit stops the searches early with a lower bound; far above the
    # count it changes nothing
    ctx.set_param("split_budget", 8192)
    assert cnt > 100000
    low = ctx.count_matches(tid, state=r, max_maps=1000)
    assert low["complete"] == 0 and 1000 <= low["maps"] <= cnt
    high = ctx.count_matches(tid, state=r, max_maps=10 * cnt + 1)
    assert high["complete"] == 1 and high["maps"] == cnt
    ctx.close()


# ------------------------------------------------------ ablations
@pytest.mark.parametrize("kind,s", CASES[:8] + CASES[-2:])
def test_ablations_leave_the_output_unchanged(pmmod, torch_dev, kind, s):
    g, t = get_case(kind, s)
    ref = oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges)
    ctx = load(pmmod, torch_dev, g)
    tid = ctx.load_templates([t])
    for ab in (1, 2, 3):
        r, e, _ = ctx.prune(tid, ablate=ab)
        assert np.array_equal(u64(pmmod, r), ref.role_mask), f"ablate {ab}"
        assert np.array_equal(u64(pmmod, e), ref.edge_bits), f"ablate {ab}"
    ctx.close()


# ------------------------------------------------------ workspace
def test_caller_workspace(pmmod, torch_dev):
    torch, dev = torch_dev
    g, t = rmat_case(14, 114)
    ts = [t] + I.templates_batch(g, 5, count=6)
    ctx = load(pmmod, torch_dev, g)
    first = ctx.load_templates(ts)
    n, words = g.n, (g.m + 63) // 64
    r0 = torch.empty((len(ts), n), dtype=torch.int64, device=dev)
    e0 = torch.empty((len(ts), words), dtype=torch.int64, device=dev)
    ctx.prune(first, count=len(ts), role_mask=r0, edge_bits=e0)
    bound = ctx.workspace_size(first, len(ts), batch_streams=2)
    ws = torch.empty(bound, dtype=torch.uint8, device=dev)
    ctx.set_workspace(ws)
    r1 = torch.empty_like(r0)
    e1 = torch.empty_like(e0)
    _, _, st = ctx.prune(first, count=len(ts), role_mask=r1, edge_bits=e1, batch_streams=2)
    assert torch.equal(r0, r1) and torch.equal(e0, e1)
    assert 0 < st["workspace_bytes"] <= bound // 2
    # too small: a clean error, and the context still works afterwards
    ctx.set_workspace(torch.empty(1 << 16, dtype=torch.uint8, device=dev))
    with pytest.raises(pmmod.PMError) as ei:
        ctx.prune(first)
    assert ei.value.code == -10
    ctx.set_workspace(None)
    r2, e2, _ = ctx.prune(first)
    assert torch.equal(r2[0], r0[0]) and torch.equal(e2[0], e0[0])
    ctx.close()
