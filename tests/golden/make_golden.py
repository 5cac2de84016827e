#!/usr/bin/env python3
"""Writes prune_digests.json: SHA-256 digests of the oracle's complete sets
(role masks and edge words) for the full-size workloads, so that the GPU
tests compare every vertex and every edge of their output with the oracle
without running the oracle's exact step (minutes on the host) at test time.

Only the oracle and the seeded input generators are called here; nothing
comes from the library.  Run from the repository root:

    python tests/golden/make_golden.py [--budget-s SECONDS]

Workloads (R-MAT scale 22, graph seed 22, log2-degree labels):
  * tri-square seed 0: the triangle + 4-cycle + pendant template;
  * mixed batch seed 3: as many of the 64 templates as finish within the
    per-template time budget (the oracle's exact step grows steeply with
    the number of surviving matches);
  * multi-cycle seed 4: likewise.
Digest of an array: SHA-256 of its little-endian uint64 words.
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "prune_digests.json")


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


def record(workload, index, t, res, secs):
    bits = np.unpackbits(res.edge_bits.view(np.uint8))
    return {"workload": workload, "index": index, "labels": [int(x) for x in t.labels],
            "edges": [[int(a), int(b)] for a, b in t.edges],
            "role_sha256": digest(res.role_mask), "edge_sha256": digest(res.edge_bits),
            "result_vertices": int((res.role_mask != 0).sum()),
            "result_entries": int(bits.sum()), "oracle_s": round(secs, 1)}


_GRAPH = None   # (row_ptr, col, labels) in a worker process


def _init_worker(paths):
    global _GRAPH
    sys.path.insert(0, ROOT)
    _GRAPH = tuple(np.load(p, mmap_mode="r") for p in paths)


def _one(args):
    """Oracle prune of one template in a child process (so a template over
    budget can be abandoned)."""
    import oracle
    rp, col, labels = _GRAPH
    labels_t, edges_t = args
    t0 = time.time()
    res = oracle.prune(rp, col, labels, labels_t, edges_t)
    return res.role_mask, res.edge_bits, time.time() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--budget-s", type=float, default=240.0,
                    help="per-template time limit for the batch workloads")
    ap.add_argument("--only", default="tri-square,batch,multicycle")
    args = ap.parse_args()
    from paper_1912_08453_amd import inputs as I
    rp, col = I.rmat_csr(22, seed=22)
    labels = I.labels_log2deg(rp)
    g = I.Graph(rp, col, labels)
    # the workers are spawned (an OpenMP runtime does not survive fork) and
    # map the graph from files
    tmpdir = os.path.join(os.path.dirname(OUT), ".graph_tmp")
    os.makedirs(tmpdir, exist_ok=True)
    paths = []
    for name, arr in (("rp", rp), ("col", col), ("labels", labels)):
        paths.append(os.path.join(tmpdir, name + ".npy"))
        np.save(paths[-1], arr)
    out = {"graph": {"scale": 22, "graph_seed": 22, "labels": "log2-degree",
                     "n": int(g.n), "m": int(g.m)}, "records": []}
    if os.path.exists(OUT):
        old = json.load(open(OUT))
        if old.get("graph", {}).get("m") == g.m:
            out["records"] = old["records"]
    have = {(r["workload"], r["index"]) for r in out["records"]}
    work = []
    only = args.only.split(",")
    if "tri-square" in only:
        work.append(("tri-square-seed0", 0, I.template_tri_square(g, 0)))
    if "batch" in only:
        work += [("batch-seed3", i, t) for i, t in enumerate(I.templates_batch(g, 3, count=64))]
    if "multicycle" in only:
        work += [("multicycle-seed4", i, t)
                 for i, t in enumerate(I.templates_multicycle(g, 4, count=64))]
    ctx = mp.get_context("spawn")
    for wl, i, t in work:
        if (wl, i) in have:
            continue
        budget = 1e9 if wl.startswith("tri-square") else args.budget_s
        with ctx.Pool(1, initializer=_init_worker, initargs=(paths,)) as pool:
            job = pool.apply_async(_one, ((list(t.labels), list(t.edges)),))
            try:
                role, edge, secs = job.get(timeout=budget)
            except mp.TimeoutError:
                print(f"{wl} {i}: over {budget:.0f}s, skipped", flush=True)
                pool.terminate()
                continue

        class R:
            pass
        res = R()
        res.role_mask, res.edge_bits = role, edge
        rec = record(wl, i, t, res, secs)
        out["records"].append(rec)
        print(f"{wl} {i}: {secs:.1f}s |V*|={rec['result_vertices']}", flush=True)
        json.dump(out, open(OUT + ".tmp", "w"), indent=1)
        os.replace(OUT + ".tmp", OUT)
    json.dump(out, open(OUT + ".tmp", "w"), indent=1)
    os.replace(OUT + ".tmp", OUT)
    for p in paths:
        os.remove(p)
    os.rmdir(tmpdir)


if __name__ == "__main__":
    main()
