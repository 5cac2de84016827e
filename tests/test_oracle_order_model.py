"""Pins of the oracle's learned-ordering model (CPU only).

The perceptron, its gradient and the Adam update are pinned against facts
that do not come from the oracle's own formulas: central finite differences
of the loss, networks built by hand to compute known functions, the closed
form of the loss and its gradient for a constant network, Adam's first-step
property and its limit on a convex problem.  The features are pinned by
special cases whose values are exact and by invariances.
"""
import dataclasses

import numpy as np
import pytest

from oracle import order_model as OM


def _rng(seed):
    return np.random.Generator(np.random.Philox(seed))


def _random_params(seed, scale=0.3):
    return _rng(seed).normal(0.0, scale, OM.N_PARAMS)


def test_parameter_count_matches_layer_sizes():
    assert OM.N_PARAMS == 12 * 64 + 64 + 64 * 64 + 64 + 2 * 64 + 2 == 5122


def test_hand_built_network_computes_absolute_difference():
    # h1_0 = relu(x0 - x1), h1_1 = relu(x1 - x0), h2_0 = h1_0 + h1_1 = |x0 - x1|
    W1 = np.zeros((64, 12)); b1 = np.zeros(64)
    W2 = np.zeros((64, 64)); b2 = np.zeros(64)
    W3 = np.zeros((2, 64)); b3 = np.array([0.0, 7.0])
    W1[0, 0], W1[0, 1] = 1.0, -1.0
    W1[1, 0], W1[1, 1] = -1.0, 1.0
    W2[0, 0] = W2[0, 1] = 1.0
    W3[0, 0] = 1.0
    # second output: 3 * relu(x2 + 5) + 7 (pins b1, row 1 of W3 and b3[1])
    W1[2, 2] = 1.0; b1[2] = 5.0
    W2[5, 2] = 1.0
    W3[1, 5] = 3.0
    w = OM.pack(W1, b1, W2, b2, W3, b3)
    X = _rng(1).uniform(-10, 10, (200, 12))
    Y = OM.forward(w, X)
    assert np.allclose(Y[:, 0], np.abs(X[:, 0] - X[:, 1]), rtol=0, atol=1e-12)
    assert np.allclose(Y[:, 1], 3.0 * np.maximum(X[:, 2] + 5.0, 0.0) + 7.0, rtol=0, atol=1e-12)


def test_forward_is_piecewise_linear_and_positively_homogeneous_without_biases():
    # with zero biases a ReLU network satisfies f(a x) = a f(x) for a > 0
    W1, b1, W2, b2, W3, b3 = OM.unpack(_random_params(2).copy())
    w = OM.pack(W1, 0 * b1, W2, 0 * b2, W3, 0 * b3)
    X = _rng(3).normal(size=(50, 12))
    assert np.allclose(OM.forward(w, 2.5 * X), 2.5 * OM.forward(w, X), rtol=1e-12, atol=1e-12)
    assert np.allclose(OM.forward(w, 0 * X), 0.0)


def test_constant_network_loss_and_gradient_closed_form():
    W1, b1, W2, b2, W3, b3 = (np.zeros((64, 12)), np.zeros(64), np.zeros((64, 64)),
                              np.zeros(64), np.zeros((2, 64)), np.array([1.5, -2.0]))
    w = OM.pack(W1, b1, W2, b2, W3, b3)
    T = _rng(4).normal(size=(37, 2))
    X = _rng(5).normal(size=(37, 12))
    loss, g = OM.loss_grad(w, X, T)
    want = (((1.5 - T[:, 0]) ** 2).sum() + ((-2.0 - T[:, 1]) ** 2).sum()) / (2 * 37)
    assert loss == pytest.approx(want, rel=1e-12)
    gb3 = OM.unpack(g)[5]
    assert np.allclose(gb3, [np.mean(1.5 - T[:, 0]), np.mean(-2.0 - T[:, 1])], atol=1e-12)
    # every hidden unit is at z = 0, where ReLU' = 0: no other gradient
    assert np.count_nonzero(g[:-2]) == 0


def test_gradient_matches_central_finite_differences():
    w = _random_params(6)
    X = _rng(7).normal(size=(16, 12))
    T = _rng(8).normal(size=(16, 2))
    _, g = OM.loss_grad(w, X, T)
    h = 1e-6
    idx = _rng(9).choice(OM.N_PARAMS, 300, replace=False)
    for i in idx:
        wp = w.copy(); wp[i] += h
        wm = w.copy(); wm[i] -= h
        fd = (OM.loss_grad(wp, X, T)[0] - OM.loss_grad(wm, X, T)[0]) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-8), i


def test_gradient_layout_every_block_checked_by_finite_differences():
    # one parameter from each block of the packed layout
    w = _random_params(10)
    X = _rng(11).normal(size=(8, 12))
    T = _rng(12).normal(size=(8, 2))
    _, g = OM.loss_grad(w, X, T)
    starts = [0, 768, 832, 4928, 4992, 5120]
    h = 1e-6
    for s in starts:
        for i in (s, s + 1):
            wp = w.copy(); wp[i] += h
            wm = w.copy(); wm[i] -= h
            fd = (OM.loss_grad(wp, X, T)[0] - OM.loss_grad(wm, X, T)[0]) / (2 * h)
            assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-8)


def test_adam_first_step_moves_each_parameter_by_lr_times_sign():
    w = _random_params(13)
    X = _rng(14).normal(size=(20, 12))
    T = _rng(15).normal(size=(20, 2))
    _, g = OM.loss_grad(w, X, T)
    # bias-corrected moments of step 1 are g and g^2: the step is
    # lr * g / (|g| + eps)
    w1, losses = OM.adam_train(w, X, T, steps=1, lr=1e-3, eps=1e-30)
    d = w1 - w
    nz = np.abs(g) > 1e-20
    assert nz.sum() > 1000
    assert np.allclose(d[nz], -1e-3 * np.sign(g[nz]), rtol=1e-9, atol=0)
    assert np.all(d[g == 0] == 0)
    assert losses[0] == pytest.approx(OM.loss_grad(w, X, T)[0])


def test_adam_fits_the_mean_of_the_targets_for_a_constant_network():
    # only b3 receives a gradient; the loss is convex in it, minimum at mean(T)
    w = OM.pack(np.zeros((64, 12)), np.zeros(64), np.zeros((64, 64)), np.zeros(64),
                np.zeros((2, 64)), np.zeros(2))
    X = _rng(16).normal(size=(30, 12))
    T = _rng(17).normal(3.0, 1.0, size=(30, 2))
    w1, losses = OM.adam_train(w, X, T, steps=3000, lr=0.01)
    assert np.allclose(OM.unpack(w1)[5], T.mean(axis=0), atol=1e-3)
    assert losses[-1] < losses[0]


def test_training_reduces_loss_on_a_learnable_target():
    rng = _rng(18)
    X = rng.uniform(0, 1, size=(256, 12))
    T = np.stack([X[:, 0] + 2 * X[:, 5], np.abs(X[:, 1] - X[:, 2])], axis=1)
    w0 = _random_params(19, scale=0.2)
    _, losses = OM.adam_train(w0, X, T, steps=300, lr=3e-3)
    assert losses[-1] < 0.1 * losses[0]


@dataclasses.dataclass
class _K:
    kind: int
    edges: tuple
    heads: int


def test_features_exact_special_case():
    # lg(2^a - 1) = a exactly
    k = _K(kind=0, edges=((0, 1), (1, 2), (0, 2)), heads=0b111)
    counts = [3, 7, 15, 1000]
    counts0 = [15, 7, 15, 1000]
    F = [1, 3, 255, 9]
    f = OM.features([k], counts, counts0, n_active=65535, role_freq=F, done=2, total=8)[0]
    want = [3 / 8, 3 / 8, 1, 0, 1, 2 / 16, 3 / 16, 4 / 16, 16 / 16, (1 + 2 + 8) / 3 / 16,
            (4 - 2) / 3 / 16, 2 / 8]
    assert np.allclose(f, want, rtol=0, atol=1e-15)


def test_features_of_a_path_and_tds_kinds():
    p = _K(kind=1, edges=((0, 1), (1, 3)), heads=(1 << 0) | (1 << 3))
    f = OM.features([p], [1, 1, 1, 1], [1, 1, 1, 1], 1, [1, 1, 1, 1], 0, 1)[0]
    assert (f[2], f[3]) == (0.0, 0.0)
    assert f[4] == pytest.approx(2 / 3)
    assert f[10] == 0.0 and f[11] == 0.0
    for kind, flags in ((2, (1.0, 1.0)), (3, (0.0, 1.0)), (0, (1.0, 0.0))):
        f = OM.features([_K(kind, p.edges, p.heads)], [1] * 4, [1] * 4, 1, [1] * 4, 0, 1)[0]
        assert (f[2], f[3]) == flags


def test_features_invariant_under_renaming_template_vertices():
    rng = _rng(20)
    k = _K(kind=2, edges=((0, 1), (1, 2), (2, 3), (0, 3), (1, 4)), heads=0b11111)
    counts = rng.integers(0, 10**6, 6)
    counts0 = counts + rng.integers(0, 10**5, 6)
    F = rng.integers(1, 10**6, 6)
    base = OM.features([k], counts, counts0, 12345, F, 3, 9)
    perm = rng.permutation(6)
    inv = np.argsort(perm)
    k2 = _K(kind=2, edges=tuple(tuple(sorted((int(perm[a]), int(perm[b])))) for a, b in k.edges),
            heads=sum(1 << int(perm[q]) for q in range(5)))
    moved = OM.features([k2], counts[inv], counts0[inv], 12345, F[inv], 3, 9)
    assert np.allclose(base, moved, rtol=0, atol=1e-15)


def test_choose_takes_largest_score_ties_to_lowest_index_and_skips_done():
    # network whose score is x0 - x1 (y0 = relu(x0), y1 = relu(x1), inputs >= 0)
    W1 = np.zeros((64, 12)); W2 = np.zeros((64, 64)); W3 = np.zeros((2, 64))
    W1[0, 0] = W1[1, 1] = 1.0
    W2[0, 0] = W2[1, 1] = 1.0
    W3[0, 0] = W3[1, 1] = 1.0
    w = OM.pack(W1, np.zeros(64), W2, np.zeros(64), W3, np.zeros(2))
    F = np.zeros((4, 12))
    F[:, 0] = [1.0, 3.0, 3.0, 5.0]
    F[:, 1] = [0.0, 1.0, 1.0, 0.5]
    assert OM.choose(w, F, [True] * 4) == (3, 4.5)
    assert OM.choose(w, F, [True, True, True, False]) == (1, 2.0)
    assert OM.choose(w, F, [False] * 4)[0] == -1


def test_role_counts_and_frequencies():
    om = np.array([0b101, 0b001, 0, 0b110], dtype=np.uint64)
    assert list(OM.role_counts(om, 3)) == [2, 1, 2]
    assert list(OM.role_frequencies(np.array([1, 2, 1, 0]), [1, 0, 5])) == [2, 1, 0]
