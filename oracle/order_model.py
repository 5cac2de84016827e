"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Plain fp64 reference of the learned ordering of non-local constraints: the
per-constraint feature vector, the multilayer perceptron that predicts a
constraint's yield and cost, its loss gradient and the Adam update, and the
greedy choice.  Only tests, the smoke check and the benchmark's CPU-baseline
leg may use it; the library never does.

The paper names constraint selection and ordering by modelling as an open
question (conclusion) and ranks constraints by label frequency, edge count
and kind (ordering heuristics of the constraint generation section); the
model here is this build's extension, so its definitions are the ones below
(also listed in the design notes):

  features of constraint k with vertex set V_k, edges E_k, heads H_k, kind
  kappa, at a state with active role counts c[q], counts c0[q] at the first
  LCC fixpoint, n_A active vertices, background label frequency F[q] of
  role q's label, d constraints applied of K; lg(x) = log2(1 + x):
     f0  = |E_k| / 8                 f6  = mean lg(c[q]) / 16
     f1  = |V_k| / 8                 f7  = max  lg(c[q]) / 16
     f2  = kappa is a cycle kind     f8  = lg(n_A) / 16
     f3  = kappa is a TDS kind       f9  = mean lg(F[q]) / 16
     f4  = |H_k| / |V_k|             f10 = mean (lg(c0[q]) - lg(c[q])) / 16
     f5  = min lg(c[q]) / 16         f11 = d / K
  (min, mean and max over q in V_k).

  model: 12 -> 64 (ReLU) -> 64 (ReLU) -> 2, fp32 parameters packed as
     W1[64][12], b1[64], W2[64][64], b2[64], W3[2][64], b3[2]  (5122 floats)
  outputs: y0 = predicted lg(role bits removed by the constraint and the
  LCC fixpoint after it), y1 = predicted lg(microseconds spent on both).
  score = y0 - y1 (log2 of the yield/cost ratio); the greedy choice takes
  the remaining constraint of largest score, ties to the lowest index.
  loss = sum over samples and outputs of (y - t)^2 / (2 N); ReLU'(0) = 0.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

N_FEATURES = 12
HIDDEN = 64
N_OUT = 2
N_PARAMS = HIDDEN * N_FEATURES + HIDDEN + HIDDEN * HIDDEN + HIDDEN + N_OUT * HIDDEN + N_OUT

CYCLE_KINDS = (0, 2)   # cycle, TDS-cycle
TDS_KINDS = (2, 3)     # TDS-cycle, TDS-path


def unpack(w: np.ndarray):
    """Views of the packed parameter vector: W1, b1, W2, b2, W3, b3."""
    w = np.asarray(w)
    if w.shape != (N_PARAMS,):
        raise ValueError(f"expected {N_PARAMS} parameters")
    o = 0
    out = []
    for shape in ((HIDDEN, N_FEATURES), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (N_OUT, HIDDEN),
                  (N_OUT,)):
        size = int(np.prod(shape))
        out.append(w[o:o + size].reshape(shape))
        o += size
    return tuple(out)


def pack(W1, b1, W2, b2, W3, b3) -> np.ndarray:
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel()
                           for a in (W1, b1, W2, b2, W3, b3)])


def forward(w: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Outputs [N][2] of the perceptron for inputs X [N][12] (fp64)."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(w, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64).reshape(-1, N_FEATURES)
    H1 = np.maximum(X @ W1.T + b1, 0.0)
    H2 = np.maximum(H1 @ W2.T + b2, 0.0)
    return H2 @ W3.T + b3


def loss_grad(w: np.ndarray, X: np.ndarray, T: np.ndarray) -> Tuple[float, np.ndarray]:
    """Mean squared error (halved) and its gradient in the packed layout,
    by the chain rule through the three layers."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(w, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64).reshape(-1, N_FEATURES)
    T = np.asarray(T, dtype=np.float64).reshape(-1, N_OUT)
    n = X.shape[0]
    Z1 = X @ W1.T + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2.T + b2
    H2 = np.maximum(Z2, 0.0)
    Y = H2 @ W3.T + b3
    R = Y - T
    loss = float((R * R).sum() / (2.0 * n))
    dY = R / n                                  # dL/dY
    gW3 = dY.T @ H2
    gb3 = dY.sum(axis=0)
    dZ2 = (dY @ W3) * (Z2 > 0.0)                # ReLU'(z) = 1 for z > 0, else 0
    gW2 = dZ2.T @ H1
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * (Z1 > 0.0)
    gW1 = dZ1.T @ X
    gb1 = dZ1.sum(axis=0)
    return loss, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam_train(w: np.ndarray, X: np.ndarray, T: np.ndarray, steps: int, lr: float,
               beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """Full-batch Adam (Kingma and Ba, Algorithm 1) from zero moments.
    Returns the final parameters and the loss before each step."""
    w = np.array(w, dtype=np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    losses = []
    for t in range(1, steps + 1):
        loss, g = loss_grad(w, X, T)
        losses.append(loss)
        m = beta1 * m + (1.0 - beta1) * g
        v = beta2 * v + (1.0 - beta2) * g * g
        mhat = m / (1.0 - beta1 ** t)
        vhat = v / (1.0 - beta2 ** t)
        w = w - lr * mhat / (np.sqrt(vhat) + eps)
    return w, losses


def lg(x) -> np.ndarray:
    return np.log2(1.0 + np.asarray(x, dtype=np.float64))


def constraint_vertices(edges: Sequence[Tuple[int, int]]) -> List[int]:
    s = set()
    for a, b in edges:
        s.add(int(a))
        s.add(int(b))
    return sorted(s)


def features(cons, counts: Sequence[int], counts0: Sequence[int], n_active: int,
             role_freq: Sequence[int], done: int, total: int) -> np.ndarray:
    """Feature matrix [len(cons)][12] (definitions in the module docstring).
    cons: constraints with .kind, .edges, .heads; counts, counts0, role_freq
    indexed by template vertex."""
    c = np.asarray(counts, dtype=np.float64)
    c0 = np.asarray(counts0, dtype=np.float64)
    F = np.asarray(role_freq, dtype=np.float64)
    out = np.zeros((len(cons), N_FEATURES), dtype=np.float64)
    for i, k in enumerate(cons):
        vs = constraint_vertices(k.edges)
        nv = len(vs)
        heads = sum(1 for q in vs if (int(k.heads) >> q) & 1)
        lc = lg(c[vs])
        out[i, 0] = len(k.edges) / 8.0
        out[i, 1] = nv / 8.0
        out[i, 2] = 1.0 if k.kind in CYCLE_KINDS else 0.0
        out[i, 3] = 1.0 if k.kind in TDS_KINDS else 0.0
        out[i, 4] = heads / nv
        out[i, 5] = lc.min() / 16.0
        out[i, 6] = lc.mean() / 16.0
        out[i, 7] = lc.max() / 16.0
        out[i, 8] = float(lg(n_active)) / 16.0
        out[i, 9] = lg(F[vs]).mean() / 16.0
        out[i, 10] = (lg(c0[vs]) - lc).mean() / 16.0
        out[i, 11] = done / total if total else 0.0
    return out


def scores(w: np.ndarray, feats: np.ndarray) -> np.ndarray:
    y = forward(w, feats)
    return y[:, 0] - y[:, 1]


def choose(w: np.ndarray, feats: np.ndarray, remaining: Sequence[bool]) -> Tuple[int, float]:
    """Greedy choice: the remaining constraint of largest score, ties to the
    lowest index.  Returns (index, score), or (-1, -inf) if none remain."""
    s = scores(w, feats)
    best, best_s = -1, -np.inf
    for i, r in enumerate(remaining):
        if r and s[i] > best_s:
            best, best_s = i, float(s[i])
    return best, best_s


def role_counts(omega: np.ndarray, n0: int) -> np.ndarray:
    """c[q] = number of vertices whose role set holds q."""
    om = np.asarray(omega, dtype=np.uint64)
    return np.array([int(((om >> np.uint64(q)) & np.uint64(1)).sum()) for q in range(n0)],
                    dtype=np.int64)


def role_frequencies(labels: np.ndarray, t_labels: Sequence[int]) -> np.ndarray:
    """F[q] = number of background vertices carrying role q's label."""
    lab = np.asarray(labels)
    return np.array([int((lab == L).sum()) for L in t_labels], dtype=np.int64)


def replay(row_ptr, col, labels, t_labels, t_edges, order: Sequence[int]) -> List[Dict]:
    """Run the oracle's constraint loop in the given order and record, before
    each step, the features of every constraint and the role-bit total, and
    after it the role-bit total (after the NLCC step and its LCC fixpoint).
    `order` may be a prefix of a permutation."""
    import oracle
    from oracle import constraints as C
    g = oracle._G(row_ptr, col, labels)
    t = oracle._T(t_labels, t_edges)
    K0 = C.non_local_constraints(t.label_list, t.edge_list)
    om = oracle.init_roles(g, t)
    oracle.lcc(g, t, om)
    c0 = role_counts(om, t.n0)
    F = role_frequencies(g.labels, t.label_list)
    steps = []
    for d, k in enumerate(order):
        c = role_counts(om, t.n0)
        n_active = int((om != 0).sum())
        feats = features(K0, c, c0, n_active, F, d, len(K0))
        before = int(c.sum())
        ch = oracle.nlcc(g, om, K0[k])
        if ch:
            oracle.lcc(g, t, om)
        after = int(role_counts(om, t.n0).sum())
        steps.append({"constraint": int(k), "features": feats, "roles_before": before,
                      "roles_after": after, "changed": int(ch), "n_active": n_active})
    return steps


def final_state_features(row_ptr, col, labels, t_labels, t_edges, order: Sequence[int]):
    """Features of every constraint after the given order has been applied
    (the state a stopping decision is taken on)."""
    import oracle
    from oracle import constraints as C
    g = oracle._G(row_ptr, col, labels)
    t = oracle._T(t_labels, t_edges)
    K0 = C.non_local_constraints(t.label_list, t.edge_list)
    om = oracle.init_roles(g, t)
    oracle.lcc(g, t, om)
    c0 = role_counts(om, t.n0)
    F = role_frequencies(g.labels, t.label_list)
    for k in order:
        if oracle.nlcc(g, om, K0[k]):
            oracle.lcc(g, t, om)
    c = role_counts(om, t.n0)
    return features(K0, c, c0, int((om != 0).sum()), F, len(order), len(K0))
