"""GPU checks of the tuning settings: they round-trip through the C ABI,
bad names and values are refused, extreme values (one search block, one
task per chunk, no swap scans) leave the complete set equal to the oracle's,
and an autotuned context gives the same masks as the default one."""
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


@pytest.fixture(scope="module")
def case():
    rp, col = I.rmat_csr(14, seed=91)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    ts = [I.template_tri_square(g, 5)] + I.templates_multicycle(g, 77, count=3)
    refs = [oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges) for t in ts]
    return g, ts, refs


def _ctx(pmmod, torch_dev, g, ts):
    torch, dev = torch_dev
    ctx = pmmod.PM(0)
    ctx.load_graph(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                   torch.from_numpy(np.ascontiguousarray(g.labels)).to(dev))
    return ctx, ctx.load_templates(ts)


def _check(pmmod, ctx, tid, refs, what):
    splits = 0
    for i, ref in enumerate(refs):
        role, edge, st = ctx.prune(tid + i)
        assert np.array_equal(pmmod.to_u64(role[0]), ref.role_mask), f"{what}: template {i} roles"
        assert np.array_equal(pmmod.to_u64(edge[0]), ref.edge_bits), f"{what}: template {i} edges"
        splits += st["split_tasks"]
    return splits


def test_params_round_trip_and_refusals(pmmod, torch_dev, case):
    g, ts, _ = case
    ctx, _ = _ctx(pmmod, torch_dev, g, ts)
    p = ctx.params()
    assert p["expand"] == 1 and p["witness"] == 0 and p["relist"] == 1
    assert p["edge_chunk"] == 16 and p["edge_stripes"] == 64 and p["expand_max"] == 4096
    assert p["search_grid"] >= 256 and p["split_budget"] == 8192
    assert p["search_grid_solo"] == 0
    for k, v in (("edge_chunk", 3), ("edge_stripes", 5), ("expand_max", -1), ("search_grid", 9),
                 ("witness", 1), ("relist", 0), ("expand", 0), ("search_grid_solo", 5000)):
        ctx.set_param(k, v)
        assert ctx.get_param(k) == v
    assert p["lcc_bin_small"] == 8 and p["lcc_bin_mid"] == 64
    for k, v in (("edge_chunk", 0), ("edge_stripes", 1 << 17), ("search_grid", 0),
                 ("search_grid_solo", -1), ("search_grid_solo", 1 << 17),
                 ("split_budget", -1), ("split_capacity", 0), ("expand_table_log2", 31),
                 ("lcc_bin_mid", 4097), ("lcc_bin_small", 65), ("lcc_bin_small", -1),
                 ("nope", 1)):
        with pytest.raises(pmmod.PMError):
            ctx.set_param(k, v)
    with pytest.raises(pmmod.PMError):
        ctx.get_param("nope")
    ctx.close()


@pytest.mark.parametrize("setting", [
    {"search_grid": 1}, {"search_grid": 7, "edge_chunk": 1, "edge_stripes": 3},
    {"expand": 0, "relist": 0, "search_grid": 4096},
    {"witness": 1, "expand_max": 8, "edge_chunk": 64, "edge_stripes": 1024},
    {"split_budget": 1}, {"split_budget": 2, "search_grid": 3}, {"split_budget": 0},
    {"split_budget": 1, "split_capacity": 20}, {"expand_table_log2": 10},
    {"read_first": 1, "witness": 1},
    {"lcc_bin_small": 0, "lcc_bin_mid": 0}, {"lcc_bin_mid": 4096, "lcc_bin_small": 4096},
    {"lcc_bin_small": 1, "lcc_bin_mid": 2},
    {"search_grid": 2, "search_grid_solo": 8192}, {"search_grid": 3, "search_grid_solo": 5}])
def test_extreme_settings_keep_the_complete_set(pmmod, torch_dev, case, setting):
    g, ts, refs = case
    ctx, tid = _ctx(pmmod, torch_dev, g, ts)
    for k, v in setting.items():
        ctx.set_param(k, v)
    log(f"settings {ctx.params()}")
    splits = _check(pmmod, ctx, tid, refs, str(setting))
    log(f"split tasks {splits}")
    if setting.get("split_budget") == 1:
        assert splits > 0, "a one-step budget must split searches"
    if setting.get("split_budget") == 0:
        assert splits == 0
    ctx.close()


def test_autotuned_context_gives_the_same_masks(pmmod, torch_dev, case):
    from paper_1912_08453_amd import autotune
    g, ts, refs = case
    ctx, tid = _ctx(pmmod, torch_dev, g, ts)
    space = autotune.default_space(ctx)
    start = ctx.params()
    best, table = autotune.autotune(ctx, list(range(tid, tid + len(ts))), reps=1, log=log)
    for k, v in best.items():
        assert v in space[k] and ctx.get_param(k) == v
    assert len(table) == 1 + sum(len([v for v in c if v != start[k]]) for k, c in space.items())
    _check(pmmod, ctx, tid, refs, f"autotuned {best}")
    ctx.close()
