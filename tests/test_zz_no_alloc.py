"""The no-allocation prune (pm_prune_noalloc, scratch in the library's static
device array) against pm_prune through the C ABI: two calls in a row on
one device, the second on a smaller input, each equal to pm_prune's output
bit for bit (and to the oracle's), and a graph too large for the array
refused with PM_ERR_WORKSPACE.  Collected last so that a failure here does
not hide the other tests."""
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


def graph(scale, seed):
    rp, col = I.rmat_csr(scale, seed=seed)
    return I.Graph(rp, col, I.labels_log2deg(rp))


def run_both(pmmod, torch_dev, g, t):
    torch, dev = torch_dev
    ctx = pmmod.PM(0)
    ctx.load_graph(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                   torch.from_numpy(g.labels).to(dev))
    tid = ctx.load_templates([t])
    r0, e0, _ = ctx.prune(tid)
    words = (g.m + 63) // 64
    # outputs pre-filled with garbage: the call must overwrite every word
    r1 = torch.full((1, g.n), -1, dtype=torch.int64, device=dev)
    e1 = torch.full((1, words), -1, dtype=torch.int64, device=dev)
    st = ctx.prune_noalloc(tid, r1, e1)
    torch.cuda.synchronize()
    assert torch.equal(r0, r1), "role masks differ from pm_prune"
    assert torch.equal(e0, e1), "edge bits differ from pm_prune"
    ref = oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges)
    assert np.array_equal(pmmod.to_u64(r1[0]), ref.role_mask)
    assert np.array_equal(pmmod.to_u64(e1[0]), ref.edge_bits)
    assert 0 < st["workspace_bytes"] <= pmmod.NOALLOC_SCRATCH_BYTES
    ctx.close()
    return int((ref.role_mask != 0).sum())


def test_noalloc_two_calls_second_smaller(pmmod, torch_dev):
    g1 = graph(14, 114)
    t1 = I.template_tri_square(g1, 0)
    log(f"no-alloc call 1: scale 14 m={g1.m} t={t1.labels}")
    v1 = run_both(pmmod, torch_dev, g1, t1)
    g2 = graph(11, 111)
    t2 = I.template_tri_square(g2, 0)
    log(f"no-alloc call 2: scale 11 m={g2.m} t={t2.labels}")
    v2 = run_both(pmmod, torch_dev, g2, t2)
    log(f"  |V*| {v1} then {v2}")


def test_noalloc_refuses_inputs_beyond_the_array(pmmod, torch_dev):
    torch, dev = torch_dev
    g = graph(17, 117)
    t = I.template_tri_square(g, 0)
    ctx = pmmod.PM(0)
    ctx.load_graph(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                   torch.from_numpy(g.labels).to(dev))
    tid = ctx.load_templates([t])
    assert ctx.workspace_size(tid) > pmmod.NOALLOC_SCRATCH_BYTES
    words = (g.m + 63) // 64
    r = torch.empty((1, g.n), dtype=torch.int64, device=dev)
    e = torch.empty((1, words), dtype=torch.int64, device=dev)
    with pytest.raises(pmmod.PMError) as ei:
        ctx.prune_noalloc(tid, r, e)
    assert ei.value.code == -10
    # the context is still usable
    r0, e0, _ = ctx.prune(tid)
    assert int((r0 != 0).sum()) >= 0
    ctx.close()
