"""GPU check of the exploratory driver against the oracle: levels before
the one it stops at have no match in any variant, and at that level the
union of the complete sets (vertices with a role, role bits, edges) equals
the union of the oracle's complete sets of the same level's variants (the
variants enumerated independently, with the input generator's relaxation
list).  With and without the candidate set of the base template as every
variant's starting state."""
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


K4 = [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2), (1, 3)]


@pytest.mark.parametrize("cand", [True, False])
@pytest.mark.parametrize("seed,labels,max_del", [
    (1, [0, 1, 2, 3], None),
    (2, [0, 1, 0, 1], None),
    (3, [0, 1, 2, 3], 0),
])
def test_explore_against_oracle(pmmod, torch_dev, seed, labels, max_del, cand):
    from paper_1912_08453_amd import explore
    torch, dev = torch_dev
    g = I.random_graph(300, 0.03, 4, seed)
    ctx = pmmod.PM(0)
    ctx.load_graph(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                   torch.from_numpy(np.ascontiguousarray(g.labels)).to(dev))
    res = explore.explore(ctx, labels, K4, max_deletions=max_del, use_candidate_set=cand,
                          log=log)
    base = I.Template(list(labels), list(K4))
    rel = I.relaxations(base, max_deletions=len(K4))
    by_level = {}
    for t in rel:
        by_level.setdefault(len(K4) - len(t.edges), []).append(t)
    stop = res.level if res.level >= 0 else (len(K4) if max_del is None else max_del)
    n, words = g.n, (g.m + 63) // 64
    for k in range(stop + 1):
        ts = by_level.get(k, [])
        r_un = np.zeros(n, np.uint64)
        e_un = np.zeros(words, np.uint64)
        any_match = False
        for t in ts:
            ref = oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges)
            any_match = any_match or bool(ref.role_mask.any())
            r_un |= ref.role_mask
            e_un |= ref.edge_bits
        log(f"level {k}: {len(ts)} variants, oracle match {any_match}")
        if k < res.level or res.level < 0:
            assert not any_match, f"oracle finds a match at level {k}"
        else:
            assert any_match
            assert len(res.variants) == len(ts)
            assert np.array_equal(pmmod.to_u64(res.role_union), r_un)
            assert np.array_equal(pmmod.to_u64(res.edge_union), e_un)
    ctx.close()
