"""GPU check of the interactive incremental search driver against the
oracle: a scripted sequence of edge additions and deletions, each revision
pruned with reuse (from the previous complete set, or from the candidate
set with the previous complete set pre-certified), equals the oracle's
prune of the revised template and the library's own prune from scratch."""
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


def script(edges_full):
    """Start from a spanning path-like tree of the full template, add the
    other edges one at a time, then delete edges while the template stays
    connected."""
    edges_full = sorted(tuple(sorted(e)) for e in edges_full)
    tree, rest, seen = [], [], {0}
    for a, b in edges_full:
        if (a in seen) != (b in seen):
            tree.append((a, b))
            seen |= {a, b}
        else:
            rest.append((a, b))
    # edges whose both ends were not yet seen when met: add them to the tree
    # pass until it spans
    while len(seen) < max(max(e) for e in edges_full) + 1:
        for e in list(rest):
            a, b = e
            if (a in seen) != (b in seen):
                tree.append(e)
                rest.remove(e)
                seen |= {a, b}
    ops = [("add", e) for e in rest] + [("delete", e) for e in rest[::-1]] + \
          [("delete", e) for e in tree[:1]]
    return tree, ops


@pytest.mark.parametrize("scale,seed", [(12, 212), (14, 214), (16, 216)])
def test_incremental_session_against_oracle(pmmod, torch_dev, scale, seed):
    from paper_1912_08453_amd import incremental
    torch, dev = torch_dev
    rp, col = I.rmat_csr(scale, seed=seed)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    t = I.template_tri_square(g, 0)
    tree, ops = script(sorted(t.edges))
    ctx = pmmod.PM(0)
    ctx.load_graph(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                   torch.from_numpy(g.labels).to(dev))
    s = incremental.Session(ctx, t.labels, tree, compare=True)
    cur = sorted(tree)
    for op, e in ops:
        if op == "add":
            rec = s.add_edge(*e)
            cur = sorted(cur + [e])
        else:
            if e not in cur:
                continue
            try:
                rec = s.delete_edge(*e)
            except ValueError:
                continue
            cur = [x for x in cur if x != e]
        ref = oracle.prune(g.row_ptr, g.col, g.labels, t.labels, cur)
        log(f"{op} {e}: {len(cur)} edges |V*|={int((ref.role_mask != 0).sum())} "
            f"{rec['ms']:.2f} ms (naive {rec['naive_ms']:.2f} ms)")
        assert rec["identical"], f"{op} {e}: differs from the library's own full prune"
        assert np.array_equal(pmmod.to_u64(s.role), ref.role_mask), f"{op} {e}: roles"
        assert np.array_equal(pmmod.to_u64(s.edge), ref.edge_bits), f"{op} {e}: edges"
    ctx.close()
