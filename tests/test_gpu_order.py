"""GPU checks of the learned constraint order: the perceptron's forward pass,
loss gradient and Adam training in libpm's kernels against the fp64 oracle
(fp32 tolerances derived in the design notes), the features the library
computes at every step against the oracle's replay of the same order, the
validity of every greedy choice, and -- the bar that matters -- the pruning
output, which must be bit-identical to the fixed order and to the oracle
whatever the model and the stopping threshold."""
import sys

import numpy as np
import pytest

import oracle
from oracle import constraints as C
from oracle import order_model as OM
from paper_1912_08453_amd import inputs as I

pytestmark = pytest.mark.gpu

# fp32 sums of at most 64 products of O(1) terms: relative error well under
# 1e-5; the bounds below leave a factor of ten.
FWD_RTOL, FWD_ATOL = 1e-4, 1e-4
FEAT_ATOL = 1e-5          # log2f within a few ulp on values below 32, /16
SCORE_TOL = 1e-3          # greedy choice: chosen score >= best - tol


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
def ctx0(pmmod, torch_dev):
    c = pmmod.PM(0)
    yield c
    c.close()


def _rng(seed):
    return np.random.Generator(np.random.Philox(seed))


def _data(seed, n):
    rng = _rng(seed)
    X = rng.uniform(0.0, 1.5, size=(n, 12)).astype(np.float32)
    T = rng.normal(2.0, 1.0, size=(n, 2)).astype(np.float32)
    return X, T


def _away_from_kinks(w, X, T, eps=1e-4):
    """Drop the samples with a pre-activation within eps of 0, where fp32
    and fp64 may take different ReLU branches (the gradient is not
    continuous there)."""
    W1, b1, W2, b2, W3, b3 = OM.unpack(np.asarray(w, np.float64))
    Z1 = X.astype(np.float64) @ W1.T + b1
    Z2 = np.maximum(Z1, 0) @ W2.T + b2
    keep = (np.abs(Z1).min(axis=1) > eps) & (np.abs(Z2).min(axis=1) > eps)
    return X[keep], T[keep]


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 70001])
def test_mlp_forward_matches_oracle(pmmod, ctx0, n):
    w = I.model_params(n)
    X, _ = _data(n + 1, n)
    log(f"forward n={n}")
    y = ctx0.mlp_forward(w, X).cpu().numpy()
    ref = OM.forward(w.astype(np.float64), X.astype(np.float64))
    assert np.allclose(y, ref, rtol=FWD_RTOL, atol=FWD_ATOL), np.abs(y - ref).max()


@pytest.mark.parametrize("n", [1, 5, 64, 777, 128 * 64 * 2 + 5])
def test_mlp_gradient_matches_oracle(pmmod, ctx0, n):
    w = I.model_params(100 + n)
    X, T = _away_from_kinks(w, *_data(200 + n, n))
    assert X.shape[0] >= 0.9 * n
    n = X.shape[0]
    log(f"grad n={n}")
    loss, g = ctx0.mlp_grad(w, X, T)
    g = g.cpu().numpy()
    ref_loss, ref_g = OM.loss_grad(w.astype(np.float64), X.astype(np.float64),
                                   T.astype(np.float64))
    assert loss == pytest.approx(ref_loss, rel=1e-4)
    scale = np.abs(ref_g).max()
    err = np.abs(g - ref_g).max()
    assert err <= 1e-4 * scale + 1e-7, (err, scale)


def test_mlp_gradient_is_deterministic(pmmod, ctx0):
    w = I.model_params(7)
    X, T = _data(8, 5000)
    _, g1 = ctx0.mlp_grad(w, X, T)
    _, g2 = ctx0.mlp_grad(w, X, T)
    assert np.array_equal(g1.cpu().numpy(), g2.cpu().numpy())


def test_mlp_train_follows_oracle_adam(pmmod, ctx0):
    w = I.model_params(9)
    X, T = _away_from_kinks(w, *_data(10, 300))
    w_gpu, hist = ctx0.mlp_train(w, X, T, steps=60, lr=1e-3)
    w_ref, ref_hist = OM.adam_train(w.astype(np.float64), X.astype(np.float64),
                                    T.astype(np.float64), steps=60, lr=1e-3)
    assert np.allclose(hist, ref_hist, rtol=2e-3, atol=1e-5)
    assert hist[-1] < 0.5 * hist[0]
    y = ctx0.mlp_forward(w_gpu, X).cpu().numpy()
    assert np.allclose(y, OM.forward(w_ref, X.astype(np.float64)), rtol=2e-2, atol=2e-2)


def test_model_argument_errors(pmmod, ctx0):
    with pytest.raises(pmmod.PMError) as e:
        ctx0.load_model(np.zeros(100, np.float32))
    assert e.value.code == -1
    bad = I.model_params(1)
    bad[17] = np.nan
    with pytest.raises(pmmod.PMError) as e:
        ctx0.load_model(bad)
    assert e.value.code == -9


def _graph14(seed):
    rp, col = I.rmat_csr(14, seed=300 + seed)
    return I.Graph(rp, col, I.labels_log2deg(rp))


def _load(pmmod, torch_dev, g):
    torch, dev = torch_dev
    ctx = pmmod.PM(0)
    ctx.load_graph(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                   torch.from_numpy(np.ascontiguousarray(g.labels)).to(dev))
    return ctx


def test_learned_order_needs_a_model(pmmod, torch_dev):
    g = _graph14(0)
    ctx = _load(pmmod, torch_dev, g)
    tid = ctx.load_templates([I.template_tri_square(g, 0)])
    with pytest.raises(pmmod.PMError) as e:
        ctx.prune(tid, order="learned")
    assert e.value.code == -9
    ctx.close()


def _templates(g, seed):
    ts = [I.template_tri_square(g, seed)]
    ts += I.templates_multicycle(g, 500 + seed, count=3)
    return ts


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_trace_features_and_role_totals_match_oracle_replay(pmmod, torch_dev, seed):
    """Fixed order with a trace: at every step the features the library
    computed and the role-bit totals before and after equal the oracle's
    replay of the same order."""
    g = _graph14(seed)
    ctx = _load(pmmod, torch_dev, g)
    for t in _templates(g, seed):
        tid = ctx.load_templates([t])
        _, _, st = ctx.prune(tid, trace=True, stop_after=len(C.non_local_constraints(
            t.labels, t.edges)))
        tr = st["trace"]
        order = [e["constraint"] for e in tr]
        log(f"seed {seed} t={t.labels}/{t.edges} steps={len(order)}")
        assert order == list(range(len(order)))
        rep = OM.replay(g.row_ptr, g.col, g.labels, t.labels, t.edges, order)
        for e, r in zip(tr, rep):
            k = e["constraint"]
            assert e["roles_before"] == r["roles_before"]
            assert e["roles_after"] == r["roles_after"]
            assert e["active_before"] == r["n_active"]
            assert e["changed"] == r["changed"]
            assert np.allclose(e["features"], r["features"][k], rtol=0, atol=FEAT_ATOL), \
                (k, e["features"], r["features"][k])
    ctx.close()


def _check_greedy(g, t, tr, w, min_score=None):
    order = [e["constraint"] for e in tr if e["constraint"] >= 0]
    rep = OM.replay(g.row_ptr, g.col, g.labels, t.labels, t.edges, order)
    K = len(C.non_local_constraints(t.labels, t.edges))
    remaining = [True] * K
    w64 = np.asarray(w, np.float64)
    for e, r in zip(tr, rep):
        k = e["constraint"]
        assert remaining[k]
        s = OM.scores(w64, r["features"])
        best = max(s[i] for i in range(K) if remaining[i])
        assert s[k] >= best - SCORE_TOL, (k, s[k], best)
        assert e["score"] == pytest.approx(s[k], abs=SCORE_TOL)
        if min_score is not None:
            assert s[k] >= min_score - SCORE_TOL
        remaining[k] = False
    if tr and tr[-1]["constraint"] == -1:
        f = OM.final_state_features(g.row_ptr, g.col, g.labels, t.labels, t.edges, order)
        s = OM.scores(w64, f)
        best = max(s[i] for i in range(K) if remaining[i])
        assert best < min_score + SCORE_TOL


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_learned_order_output_is_exact_and_choices_are_greedy(pmmod, torch_dev, seed):
    g = _graph14(seed)
    ctx = _load(pmmod, torch_dev, g)
    w = I.model_params(40 + seed)
    ctx.load_model(w)
    for t in _templates(g, seed):
        tid = ctx.load_templates([t])
        ref = oracle.prune(g.row_ptr, g.col, g.labels, t.labels, t.edges)
        role_f, edge_f, _ = ctx.prune(tid)
        role_f = role_f.clone()
        edge_f = edge_f.clone()
        for thr in (None, 0.0, 1e30):
            role, edge, st = ctx.prune(tid, order="learned", learned_min_score=thr, trace=True)
            tr = st["trace"]
            log(f"seed {seed} t={t.labels} thr={thr} order={[e['constraint'] for e in tr]}")
            r = pmmod.to_u64(role[0])
            e = pmmod.to_u64(edge[0])
            assert np.array_equal(r, ref.role_mask)
            assert np.array_equal(e, ref.edge_bits)
            assert np.array_equal(r, pmmod.to_u64(role_f[0]))
            assert np.array_equal(e, pmmod.to_u64(edge_f[0]))
            if thr == 1e30 and len(ref.order):
                assert tr[0]["constraint"] == -1 and st["constraints"] == 0
            _check_greedy(g, t, tr, w, thr)
    ctx.close()


def test_learned_order_tiny_random_cases_exact(pmmod, torch_dev):
    """Many small graphs and shapes: learned order (random models, several
    thresholds) gives exactly the brute-force complete set."""
    torch, dev = torch_dev
    for seed in range(40):
        rng = _rng(seed)
        n = int(rng.integers(10, 40))
        g = I.random_graph(n, float(rng.uniform(0.1, 0.4)), int(rng.integers(1, 3)), seed)
        edges = I.shape_two_cycles(rng, int(rng.integers(5, 8))) if seed % 2 else \
            I.shape_k4(rng, int(rng.integers(4, 7)))
        n0 = max(max(a, b) for a, b in edges) + 1
        t = I.Template([int(x) for x in rng.integers(0, 2, size=n0)], edges)
        ctx = pmmod.PM(0)
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        tid = ctx.load_templates([t])
        ctx.load_model(I.model_params(1000 + seed))
        brute_r, brute_e, _ = oracle.bruteforce(g.row_ptr, g.col, g.labels, t.labels, t.edges)
        for thr in (None, float(rng.normal(0, 2))):
            role, edge, _ = ctx.prune(tid, order="learned", learned_min_score=thr)
            assert np.array_equal(pmmod.to_u64(role[0]), brute_r), seed
            assert np.array_equal(pmmod.to_u64(edge[0]), brute_e), seed
        ctx.close()
