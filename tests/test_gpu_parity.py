"""GPU parity: libpm's HIP path against the CPU oracle, element by element,
on the same seeded inputs -- final complete-set masks and the intermediate
state after the first LCC fixpoint and after every non-local constraint.
All arithmetic is integer/bitset, so the bar is bit-exact."""
import sys

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


def random_case(seed, n_lo=8, n_hi=40):
    rng = np.random.Generator(np.random.Philox(seed))
    n = int(rng.integers(n_lo, n_hi))
    p = float(rng.uniform(0.05, 0.4))
    nl = int(rng.integers(1, 4))
    g = I.random_graph(n, p, nl, seed)
    kind = seed % 4
    n0 = int(rng.integers(2, 7))
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


def load(pmmod, torch_dev, g, on_device=True):
    torch, dev = torch_dev
    ctx = pmmod.PM(0)
    if on_device:
        ctx.load_graph(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                       torch.from_numpy(np.ascontiguousarray(g.labels)).to(dev))
    else:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
    return ctx


def compare(pmmod, ctx, tid, g, t, stop_after=-1, order=None, what=""):
    role, edge, st = ctx.prune(tid, stop_after=stop_after, order=order)
    ref = oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges, order=order,
                       stop_after=None if stop_after < 0 else stop_after)
    r = pmmod.to_u64(role[0])
    e = pmmod.to_u64(edge[0])
    bad_v = np.nonzero(r != ref.role_mask)[0]
    assert bad_v.size == 0, f"{what}: {bad_v.size} role masks differ, first v={bad_v[:5]} " \
                            f"gpu={r[bad_v[:5]]} oracle={ref.role_mask[bad_v[:5]]}"
    bad_e = np.nonzero(e != ref.edge_bits)[0]
    assert bad_e.size == 0, f"{what}: {bad_e.size} edge words differ, first {bad_e[:5]}"
    return st, ref


@pytest.mark.parametrize("seed", range(120))
def test_random_small_full_and_every_intermediate_state(pmmod, torch_dev, seed):
    g, t = random_case(seed)
    log(f"case seed={seed} n={g.n} m={g.m} t={t.labels}/{t.edges}")
    ctx = load(pmmod, torch_dev, g, on_device=seed % 2 == 0)
    tid = ctx.load_templates([t])
    K0 = C.non_local_constraints(t.labels, t.edges)
    assert ctx.constraints(tid) == [(c.kind, c.edges, c.heads) for c in K0]
    for k in range(len(K0) + 1):
        compare(pmmod, ctx, tid, g, t, stop_after=k, what=f"seed {seed} after {k}")
    compare(pmmod, ctx, tid, g, t, what=f"seed {seed} full")
    ctx.close()


def test_square_pendant_scale12_uniform_labels(pmmod, torch_dev):
    """R-MAT scale 12, 8 uniform labels, square plus pendant: final masks
    against the oracle and against brute-force enumeration; every
    intermediate state against the oracle."""
    rp, col = I.rmat_csr(12, seed=1)
    g = I.Graph(rp, col, I.labels_uniform(rp.shape[0] - 1, 8, 12))
    t = I.template_square_pendant()
    log(f"square+pendant n={g.n} m={g.m}")
    ctx = load(pmmod, torch_dev, g)
    tid = ctx.load_templates([t])
    for k in range(len(C.non_local_constraints(t.labels, t.edges)) + 1):
        compare(pmmod, ctx, tid, g, t, stop_after=k, what=f"square+pendant after {k}")
    st, ref = compare(pmmod, ctx, tid, g, t, what="square+pendant full")
    role, ebits, cnt = oracle.bruteforce(g.row_ptr, g.col, g.labels, t.labels, t.edges)
    assert np.array_equal(role, ref.role_mask) and np.array_equal(ebits, ref.edge_bits)
    assert cnt > 0 and (role != 0).sum() > 0
    ctx.close()


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_rmat_scale16_degree_labels_tri_square(pmmod, torch_dev, seed):
    """Triangle + square + pendant with a repeated label on an R-MAT scale-16
    graph with log2-degree labels (several tiles, hubs split over
    wavefronts)."""
    rp, col = I.rmat_csr(16, seed=100 + seed)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    t = I.template_tri_square(g, seed)
    log(f"scale16 seed={seed} labels={t.labels} m={g.m}")
    ctx = load(pmmod, torch_dev, g)
    tid = ctx.load_templates([t])
    for k in range(len(C.non_local_constraints(t.labels, t.edges)) + 1):
        compare(pmmod, ctx, tid, g, t, stop_after=k, what=f"s16/{seed} after {k}")
    compare(pmmod, ctx, tid, g, t, what=f"s16/{seed} full")
    ctx.close()


def test_batch_of_templates_in_one_call(pmmod, torch_dev):
    torch, dev = torch_dev
    rp, col = I.rmat_csr(14, seed=5)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    ts = I.templates_batch(g, 3, count=16)
    ctx = load(pmmod, torch_dev, g)
    tid = ctx.load_templates(ts)
    role, edge, st = ctx.prune(tid, count=len(ts))
    for i, t in enumerate(ts):
        log(f"batch template {i} {t.name} {t.labels} {t.edges}")
        ref = oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges)
        assert np.array_equal(pmmod.to_u64(role[i]), ref.role_mask), t.name
        assert np.array_equal(pmmod.to_u64(edge[i]), ref.edge_bits), t.name
    ctx.close()


@pytest.mark.parametrize("seed", range(6))
def test_given_orders_same_final_output(pmmod, torch_dev, seed):
    g, t = random_case(3000 + seed, 20, 60)
    K0 = C.non_local_constraints(t.labels, t.edges)
    ctx = load(pmmod, torch_dev, g)
    tid = ctx.load_templates([t])
    base = pmmod.to_u64(ctx.prune(tid)[0][0])
    rng = np.random.Generator(np.random.Philox(seed))
    for _ in range(3):
        order = [int(x) for x in rng.permutation(len(K0))]
        compare(pmmod, ctx, tid, g, t, stop_after=len(K0), order=order, what="given order")
        r = pmmod.to_u64(ctx.prune(tid, order=order)[0][0])
        assert np.array_equal(r, base)
    ctx.close()


@pytest.mark.parametrize("split_budget", [8192, 1])
@pytest.mark.parametrize("n0", [10, 20, 40])
def test_wider_role_masks(pmmod, torch_dev, n0, split_budget):
    """Templates of 10/20/40 vertices exercise 16/32/64-bit role masks; with
    a one-step split budget the searches hand work on at every step, up to
    the prefix limit of a split task (deeper levels then stay unsplit)."""
    rng = np.random.Generator(np.random.Philox(n0))
    nl = n0 // 2 + 1
    g = I.random_graph(400, 0.05, nl, n0)
    edges = I.shape_one_cycle(rng, n0)
    labels = [q % nl for q in range(n0)]
    t = I.Template(labels, edges)
    ctx = load(pmmod, torch_dev, g)
    ctx.set_param("split_budget", split_budget)
    tid = ctx.load_templates([t])
    compare(pmmod, ctx, tid, g, t, stop_after=0, what=f"n0={n0} lcc")
    compare(pmmod, ctx, tid, g, t, what=f"n0={n0} full")
    ctx.close()


def test_uint16_labels(pmmod, torch_dev):
    rp, col = I.rmat_csr(11, seed=9)
    n = rp.shape[0] - 1
    lab = (I.labels_uniform(n, 6, 3).astype(np.uint16) * 211 + 300).astype(np.uint16)
    g = I.Graph(rp, col, lab)
    t = I.Template([300, 511, 722, 300], [(0, 1), (1, 2), (2, 3), (3, 0)])
    ctx = load(pmmod, torch_dev, g)
    tid = ctx.load_templates([t])
    compare(pmmod, ctx, tid, g, t, what="uint16 labels")
    ctx.close()


def test_edge_cases(pmmod, torch_dev):
    # no edges at all
    g = I.Graph(np.zeros(6, np.int64), np.zeros(0, np.int32), np.array([0, 1, 0, 1, 2], np.uint8))
    ctx = load(pmmod, torch_dev, g, on_device=False)
    ts = [I.Template([0, 1], [(0, 1)]), I.Template([1], []), I.Template([7, 8], [(0, 1)])]
    tid = ctx.load_templates(ts)
    for i, t in enumerate(ts):
        compare(pmmod, ctx, tid + i, g, t, what=f"edgeless {i}")
    ctx.close()
    # single-vertex template and absent labels on a real graph
    gg, _ = random_case(5)
    ctx = load(pmmod, torch_dev, gg)
    ts = [I.Template([1], []), I.Template([9, 9, 9], [(0, 1), (1, 2), (0, 2)])]
    tid = ctx.load_templates(ts)
    for i, t in enumerate(ts):
        compare(pmmod, ctx, tid + i, gg, t, what=f"special {i}")
    ctx.close()


def test_repeated_calls_are_identical(pmmod, torch_dev):
    rp, col = I.rmat_csr(14, seed=11)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    t = I.template_tri_square(g, 4)
    ctx = load(pmmod, torch_dev, g)
    tid = ctx.load_templates([t])
    outs = [tuple(pmmod.to_u64(x[0]).tobytes() for x in ctx.prune(tid)[:2]) for _ in range(3)]
    assert outs[0] == outs[1] == outs[2]
    ctx.close()


def test_error_codes(pmmod, torch_dev):
    ctx = pmmod.PM(0)
    with pytest.raises(pmmod.PMError) as ei:
        ctx.prune(0)
    assert ei.value.code in (-5, -8)
    bad_rp = np.array([0, 1, 1], np.int64)          # 0 -> 1 without 1 -> 0
    with pytest.raises(pmmod.PMError) as ei:
        ctx.load_graph(bad_rp, np.array([1], np.int32), np.zeros(2, np.uint8), validate=True)
    assert ei.value.code == -3
    g, t = random_case(7)
    ctx.load_graph(g.row_ptr, g.col, g.labels, validate=True)
    with pytest.raises(pmmod.PMError) as ei:
        ctx.prune(3)
    assert ei.value.code == -8
    with pytest.raises(pmmod.PMError) as ei:
        ctx.load_templates([I.Template([0, 1, 2], [(0, 1)])])
    assert ei.value.code == -4
    ctx.close()


def test_concurrent_batch_equals_one_at_a_time(pmmod, torch_dev):
    """Batched prune (templates on concurrent streams with separate scratch)
    gives the same masks as one template at a time, and as the oracle, also
    with the searches of concurrent templates sharing one grid."""
    rp, col = I.rmat_csr(14, seed=6)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    ts = I.templates_batch(g, 4, count=24)
    ctx = load(pmmod, torch_dev, g)
    tid = ctx.load_templates(ts)
    r1, e1, _ = ctx.prune(tid, count=len(ts))
    r1, e1 = pmmod.to_u64(r1), pmmod.to_u64(e1)
    r4, e4, _ = ctx.prune(tid, count=len(ts), batch_streams=4)
    assert np.array_equal(pmmod.to_u64(r4), r1) and np.array_equal(pmmod.to_u64(e4), e1)
    # searches sharing a grid that a lone one fills
    ctx.set_param("search_grid", 16)
    ctx.set_param("search_grid_solo", 4096)
    r5, e5, _ = ctx.prune(tid, count=len(ts), batch_streams=3)
    assert np.array_equal(pmmod.to_u64(r5), r1) and np.array_equal(pmmod.to_u64(e5), e1)
    for i in (0, 7, 13, 23):
        ref = oracle.prune(g.row_ptr, g.col, g.labels, ts[i].labels, ts[i].edges)
        assert np.array_equal(r1[i], ref.role_mask) and np.array_equal(e1[i], ref.edge_bits)
    ctx.close()


def test_count_index_unaligned_labels_and_gather_path_agree(pmmod, torch_dev, monkeypatch):
    """The first sweep from the neighbour-label count index, with a label
    array that starts at an odd address (scalar loads) and with the index
    switched off (gather sweep over the CSR), against the oracle at every
    intermediate state."""
    torch, dev = torch_dev
    rp, col = I.rmat_csr(13, seed=77)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    t = I.template_tri_square(g, 3)
    big = torch.zeros(g.n + 1, dtype=torch.uint8, device=dev)
    big[1:] = torch.from_numpy(g.labels).to(dev)
    for mode in ("unaligned", "no_index"):
        if mode == "no_index":
            monkeypatch.setenv("PM_NO_COUNT_INDEX", "1")
        ctx = pmmod.PM(0)
        lab = big[1:] if mode == "unaligned" else big[1:].clone()
        if mode == "unaligned":
            assert lab.data_ptr() % 4 != 0
        ctx.load_graph(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev), lab)
        tid = ctx.load_templates([t])
        for k in range(len(C.non_local_constraints(t.labels, t.edges)) + 1):
            compare(pmmod, ctx, tid, g, t, stop_after=k, what=f"{mode} after {k}")
        compare(pmmod, ctx, tid, g, t, what=f"{mode} full")
        ctx.close()


@pytest.mark.parametrize("env", [{"PM_RELIST": "0"}, {"PM_WITNESS": "1"}, {"PM_EXPAND": "0"},
                                 {"PM_EXPAND_MAX": "32"}, {"PM_EDGE_CHUNK": "1"},
                                 {"PM_EDGE_STRIPES": "1"}, {"PM_EDGE_STRIPES": "7"},
                                 {"PM_SPLIT_BUDGET": "0"}, {"PM_SPLIT_BUDGET": "1"},
                                 {"PM_SPLIT_BUDGET": "5", "PM_EDGE_CHUNK": "1"}])
def test_exact_step_switches_give_the_same_result(pmmod, torch_dev, monkeypatch, env):
    """The exact step's optional savings (role lists rebuilt from the exact
    roles, witness swaps, swap scans, their length cap, task chunking,
    splitting of long searches) only change how much work is done: the
    complete set equals the oracle's with each one switched off or changed
    (a split budget of one step splits nearly every search, down to the
    deepest level, and fills the split lists)."""
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    rp, col = I.rmat_csr(14, seed=91)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    ts = [I.template_tri_square(g, 5)] + I.templates_multicycle(g, 77, count=2)
    ctx = load(pmmod, torch_dev, g)
    for t in ts:
        tid = ctx.load_templates([t])
        compare(pmmod, ctx, tid, g, t, what=f"{env} {t.labels}")
    ctx.close()
