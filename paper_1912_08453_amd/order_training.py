"""Training of the constraint-ordering model (runs on the GPU through libpm).

Logs come from pruning runs that check the non-local constraints in random
orders and record, for every step, the features the library computed and
what the step did: role bits removed by the NLCC step and the LCC fixpoint
after it, and the device time of both.  The model learns
    y0 = log2(1 + role bits removed),  y1 = log2(1 + microseconds)
by full-batch Adam in libpm's kernels.  A stopping threshold on the score
y0 - y1 is then chosen on the training templates by measuring the whole
prune (final search included) for each candidate threshold.

    python -m paper_1912_08453_amd.order_training [--scale 22] [--out DIR]

writes order_model.npy (float32[5122]) and order_model.json (training
description, loss, chosen threshold) next to this file.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import List, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(HERE, "order_model.npy")
META_PATH = os.path.join(HERE, "order_model.json")

# template seeds: training draws never overlap the evaluation workload
# (multi-cycle templates of seed 4)
TRAIN_TRI_SQUARE_SEEDS = tuple(range(1000, 1024))
TRAIN_MULTICYCLE_SEED = 9
TRAIN_MULTICYCLE_COUNT = 24
THRESHOLDS = (None, -6.0, -4.0, -2.0, 0.0)


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def load_model(path: str = MODEL_PATH) -> np.ndarray:
    w = np.load(path, allow_pickle=False)
    return np.ascontiguousarray(w, dtype=np.float32)


def load_threshold(path: str = META_PATH):
    with open(path) as f:
        return json.load(f).get("min_score")


def training_templates(graph, tri_square_seeds: Sequence[int] = TRAIN_TRI_SQUARE_SEEDS,
                       mc_seed: int = TRAIN_MULTICYCLE_SEED,
                       mc_count: int = TRAIN_MULTICYCLE_COUNT):
    from . import inputs as I
    ts = []
    for s in tri_square_seeds:
        try:
            ts.append(I.template_tri_square(graph, s))
        except RuntimeError:
            pass
    ts += I.templates_multicycle(graph, mc_seed, count=mc_count)
    return ts


def targets(entry) -> List[float]:
    removed = max(0, int(entry["roles_before"]) - int(entry["roles_after"]))
    return [float(np.log2(1.0 + removed)), float(np.log2(1.0 + 1000.0 * float(entry["ms"])))]


def collect(ctx, tids: Sequence[int], n_cons: Sequence[int], orders_per_template: int,
            seed: int):
    """Random-order runs (constraint loop only, no final search); returns
    features [N][12] and targets [N][2] as float32."""
    rng = np.random.Generator(np.random.Philox(seed))
    X, T = [], []
    for tid, K in zip(tids, n_cons):
        if K == 0:
            continue
        for r in range(orders_per_template):
            order = list(range(K)) if r == 0 else [int(x) for x in rng.permutation(K)]
            _, _, st = ctx.prune(tid, order=order, stop_after=K, trace=True)
            for e in st["trace"]:
                if e["constraint"] >= 0:
                    X.append(e["features"])
                    T.append(targets(e))
    return np.asarray(X, np.float32), np.asarray(T, np.float32)


def total_ms(ctx, tids, order=None, min_score=None, reps: int = 1) -> float:
    import torch
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for tid in tids:
            ctx.prune(tid, order=order, learned_min_score=min_score)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        best = ms if best is None else min(best, ms)
    return best


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--graph-seed", type=int, default=22)
    ap.add_argument("--orders", type=int, default=4, help="random orders per template")
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--init-seed", type=int, default=5)
    ap.add_argument("--out", default=HERE)
    args = ap.parse_args(argv)

    import torch
    from . import inputs as I
    from . import pm

    t0 = time.time()
    rp, col = I.rmat_csr(args.scale, seed=args.graph_seed)
    labels = I.labels_log2deg(rp)
    g = I.Graph(rp, col, labels)
    log(f"graph scale {args.scale}: n={g.n} m={g.m} ({time.time() - t0:.1f}s)")
    dev = torch.device("cuda", 0)
    ctx = pm.PM(0)
    ctx.load_graph(torch.from_numpy(rp).to(dev), torch.from_numpy(col).to(dev),
                   torch.from_numpy(labels).to(dev))
    ts = training_templates(g)
    first = ctx.load_templates(ts)
    tids = list(range(first, first + len(ts)))
    n_cons = [len(ctx.constraints(t)) for t in tids]
    log(f"{len(ts)} training templates, {sum(n_cons)} constraints")

    t1 = time.time()
    X, T = collect(ctx, tids, n_cons, args.orders, seed=args.init_seed)
    log(f"logs: {X.shape[0]} steps in {time.time() - t1:.1f}s")

    w0 = I.model_params(args.init_seed)
    w, hist = ctx.mlp_train(w0, X, T, steps=args.steps, lr=args.lr)
    w = w.cpu().numpy().astype(np.float32)
    log(f"loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    ctx.load_model(w)

    # stopping threshold: whole prune on the training templates
    total_ms(ctx, tids)                                   # warm-up
    fixed = total_ms(ctx, tids)
    timing = {"fixed": fixed}
    for thr in THRESHOLDS:
        timing[str(thr)] = total_ms(ctx, tids, order="learned", min_score=thr)
        log(f"threshold {thr}: {timing[str(thr)]:.1f} ms (fixed order {fixed:.1f} ms)")
    best = min(THRESHOLDS, key=lambda t: timing[str(t)])

    os.makedirs(args.out, exist_ok=True)
    np.save(os.path.join(args.out, "order_model.npy"), w, allow_pickle=False)
    meta = {
        "graph": f"R-MAT scale {args.scale} seed {args.graph_seed}, log2-degree labels",
        "templates": f"triangle+square+pendant seeds {TRAIN_TRI_SQUARE_SEEDS[0]}.."
                     f"{TRAIN_TRI_SQUARE_SEEDS[-1]} and "
                     f"{TRAIN_MULTICYCLE_COUNT} multi-cycle templates of seed "
                     f"{TRAIN_MULTICYCLE_SEED}",
        "orders_per_template": args.orders, "samples": int(X.shape[0]),
        "adam_steps": args.steps, "lr": args.lr, "init_seed": args.init_seed,
        "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
        "threshold_ms_on_training_templates": timing, "min_score": best,
    }
    with open(os.path.join(args.out, "order_model.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
