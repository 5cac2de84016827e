#!/usr/bin/env python3
"""Benchmark of the complete-set prune on one MI355X.

Workload (one step): prune an R-MAT scale-22 graph (Graph500 parameters,
edge factor 16, undirected, log2-degree labels) to the complete set of a
6-vertex template (triangle and 4-cycle sharing an edge, a pendant, one
repeated label), through the C ABI: first LCC sweep, candidate-subgraph
compaction, LCC fixpoint, every non-local constraint, and the exact
full-template step.  Inputs are resident in HBM before timing starts.

Prints one JSON line: metric GTEPS = directed CSR entries / time-to-fixpoint,
with time-to-fixpoint, per-phase device times, a roofline entry for the
first LCC sweep kernel and the CPU oracle's rate on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--graph-seed", type=int, default=22)
    ap.add_argument("--template-seed", type=int, default=0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (for HBM counter scaling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-s", type=float, default=20.0)
    ap.add_argument("--legs", default="batched,learned,autotune",
                    help="extra legs on the same resident graph: batched (64 mixed templates, "
                         "one call per template vs concurrent streams), learned (64 multi-cycle "
                         "templates, fixed vs learned constraint order), autotune (coordinate "
                         "search of the tuning settings on the timed template; the timed "
                         "steps above use the defaults), explore (opt-in: exploratory search "
                         "from the 6-clique on the timed template's labels, relaxed level "
                         "by level until a variant matches); '' for none")
    ap.add_argument("--batch-streams", type=int, default=4)
    ap.add_argument("--workload", default="tri-square-s22", choices=["tri-square-s22", "theta8-s26"],
                    help="tri-square-s22: one template at scale 22 (default); theta8-s26: scale-26 base template "
                         "and its 1-2 edge-deletion relaxations, one call per variant vs one "
                         "batched call with the learned order")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1912_08453_amd import inputs as I
    from paper_1912_08453_amd import pm

    if args.copy_calibration:
        # a plain copy of known size: 1 GiB read + 1 GiB written per launch
        x = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        x.fill_(1)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30,
                          "launches": 3}))
        return

    if args.workload == "theta8-s26":
        return exploratory(args)

    t0 = time.time()
    rp, col = I.rmat_csr(args.scale, seed=args.graph_seed)
    labels = I.labels_log2deg(rp)
    g = I.Graph(rp, col, labels)
    tmpl = I.template_tri_square(g, args.template_seed)
    n, m = g.n, g.m
    log(f"graph scale {args.scale}: n={n} m={m} (directed entries), built in "
        f"{time.time() - t0:.1f}s; template labels {tmpl.labels}")

    dev = torch.device("cuda", 0)
    d_rp = torch.from_numpy(rp).to(dev)
    d_col = torch.from_numpy(col).to(dev)
    d_lab = torch.from_numpy(labels).to(dev)
    ctx = pm.PM(0)
    torch.cuda.synchronize()
    t_load = time.perf_counter()
    ctx.load_graph(d_rp, d_col, d_lab)
    torch.cuda.synchronize()
    load_ms = 1e3 * (time.perf_counter() - t_load)
    tid = ctx.load_templates([tmpl])
    words = (m + 63) // 64
    role = torch.empty((1, n), dtype=torch.int64, device=dev)
    edge = torch.empty((1, words), dtype=torch.int64, device=dev)

    for i in range(args.warmup):
        _, _, st = ctx.prune(tid, role_mask=role, edge_bits=edge)
        log(f"warmup {i}: {st['ms_total']:.2f} ms")
    torch.cuda.synchronize()
    stats = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        _, _, st = ctx.prune(tid, role_mask=role, edge_bits=edge)
        stats.append(st)
    torch.cuda.synchronize()
    t_el = time.perf_counter() - t_start
    ms_per_step = 1e3 * t_el / args.steps
    gteps = m / (ms_per_step / 1e3) / 1e9
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {gteps:.3f} GTEPS")

    def avg(k):
        return sum(s[k] for s in stats) / len(stats)

    # roofline of the first LCC sweep kernel (HBM-bound).  From the
    # neighbour-label count index: compulsory bytes = labels (1 B per
    # vertex) + the count bytes each vertex's initial roles need + omega
    # written (s B per vertex), computed by the library.  Without the index
    # (gather sweep over the CSR): 4 B worklist id + 16 B row_ptr pair per
    # active vertex, 4 B col per entry, omega read once and written once per
    # active vertex.
    s_bytes = 1 if tmpl.n0 <= 8 else 2 if tmpl.n0 <= 16 else 4 if tmpl.n0 <= 32 else 8
    if stats[-1]["first_sweep_bytes"] > 0:
        alg_bytes = stats[-1]["first_sweep_bytes"]
        kname = "first_sweep_counts_kernel (first LCC sweep from the neighbour-label count index)"
    else:
        na = stats[-1]["first_sweep_vertices"]
        ma = stats[-1]["first_sweep_entries"]
        alg_bytes = 20 * na + 4 * ma + s_bytes * (n + na)
        kname = "lcc_sweep_kernel (first LCC sweep over the CSR)"
    k_ms = avg("ms_sweep_kernel")
    achieved = alg_bytes / (k_ms / 1e3) / 1e9 if k_ms > 0 else 0.0
    traffic = None
    if stats[-1]["first_sweep_bytes"] > 0:
        traffic = recorded_traffic("first_sweep_counts_kernel", args.scale, args.graph_seed,
                                   args.template_seed)
    roofline = {"bound": "hbm", "kernel": kname,
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_launch": int(alg_bytes), "ms_per_launch": round(k_ms, 5)}

    phases = {k: round(avg(k), 4) for k in stats[-1] if k.startswith("ms_")}
    search = {k: round(avg(k), 3) for k in stats[-1] if k.startswith("wave_ms_")}
    counts = {k: stats[-1][k] for k in stats[-1]
              if not k.startswith("ms_") and not k.startswith("wave_ms_")}
    r = pm.to_u64(role[0])
    counts["result_vertices"] = int((r != 0).sum())
    counts["result_entries"] = int(np.unpackbits(pm.to_u64(edge[0]).view(np.uint8)).sum())

    legs = [x for x in args.legs.split(",") if x]
    batched = learned = tuned = None
    if "autotune" in legs:
        tuned = autotune_leg(ctx, tid, role, edge)
        log(f"autotune: {json.dumps(tuned)}")
    explored = None
    if "explore" in legs:
        explored = explore_leg(ctx, tmpl)
        log(f"explore: {json.dumps(explored)}")
    if "batched" in legs:
        batched = batched_leg(ctx, g, args.batch_streams)
        log(f"batched: {json.dumps(batched)}")
    if "learned" in legs:
        learned = learned_leg(ctx, g)
        log(f"learned: {json.dumps(learned)}")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(g, tmpl, args.cpu_sample_s)

    out = {
        "metric": "GTEPS (directed CSR entries / time-to-fixpoint, bit-exact complete set)",
        "value": round(gteps, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"R-MAT scale {args.scale} (a,b,c)=(0.57,0.19,0.19) ef16, "
                               f"log2-degree uint8 labels; 6-vertex triangle+4-cycle+pendant "
                               f"template, repeated label (seed {args.template_seed})",
                   "n": n, "m_directed": m, "template_labels": tmpl.labels,
                   "parallelism": "single GPU"},
        "time_to_fixpoint_ms": round(ms_per_step, 4),
        "graph_load_ms": round(load_ms, 2),
        "phases_ms": phases,
        "counts": counts,
        "search_wave_ms": search,
        "roofline": roofline,
        "dominant_phase": {"phase": "exact step (edge_search_kernel, vertex_search_kernel)",
                           "share_of_step": round(avg("ms_exact") / max(avg("ms_total"), 1e-9), 4),
                           "bound": "search latency / random gathers (no roofline claim)"},
        "cpu_baseline": cpu,
        "batched": batched,
        "autotune": tuned,
        "explore": explored,
        "learned_order": learned,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def recorded_traffic(kernel, scale, graph_seed, template_seed):
    """HBM bytes per launch of `kernel` from the counter record under
    profiles/ (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration), or
    None when there is no record for this workload or the kernel's source has
    changed since the counters were taken."""
    import hashlib
    if graph_seed != 22:
        return None
    path = os.path.join(ROOT, "profiles",
                        f"first_sweep_counts_tri_square_scale{scale}_seed{template_seed}.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#") and "=" in line:
            k, v = line.split("=", 1)
            rec[k] = v
    if rec.get("kernel") != kernel:
        return None
    src = os.path.join(ROOT, rec.get("source", ""))
    if not os.path.exists(src) or hashlib.sha1(open(src, "rb").read()).hexdigest() != rec.get("source_sha1"):
        return None
    return int(float(rec["fetch_kib_per_dispatch"]) * 1024 * float(rec["fetch_scale"]) +
               float(rec["write_kib_per_dispatch"]) * 1024 * float(rec["write_scale"]))


def exploratory(args, scale=26, graph_seed=26, template_seed=0):
    """Scale-26 exploratory workload: the 8-vertex two-cycle base template
    (repeated-label pair 4 hops apart) and its connected 1- and 2-edge
    deletion relaxations, deduplicated up to labelled isomorphism.  Plain:
    one pm_prune call per variant, fixed order.  Batched: one call for all
    variants on concurrent streams with the learned order.  Value: directed
    entries x variants / batched wall time."""
    import numpy as np
    import torch
    from paper_1912_08453_amd import inputs as I
    from paper_1912_08453_amd import order_training as OT
    from paper_1912_08453_amd import pm
    t0 = time.time()
    rp, col = I.rmat_csr(scale, seed=graph_seed)
    labels = I.labels_log2deg(rp)
    g = I.Graph(rp, col, labels)
    base = I.template_theta8(g, template_seed)
    ts = I.relaxations(base)
    log(f"graph scale {scale}: n={g.n} m={g.m} built in {time.time() - t0:.1f}s; "
        f"{len(ts)} variants of {base.labels}")
    dev = torch.device("cuda", 0)
    ctx = pm.PM(0)
    ctx.load_graph(torch.from_numpy(rp).to(dev), torch.from_numpy(col).to(dev),
                   torch.from_numpy(labels).to(dev))
    first = ctx.load_templates(ts)
    ctx.load_model(OT.load_model())
    thr = OT.load_threshold()
    T = len(ts)
    n, words = g.n, (g.m + 63) // 64
    rb = torch.empty((T, n), dtype=torch.int64, device=dev)
    eb = torch.empty((T, words), dtype=torch.int64, device=dev)
    r1 = torch.empty((1, n), dtype=torch.int64, device=dev)
    e1 = torch.empty((1, words), dtype=torch.int64, device=dev)
    ctx.prune(first, role_mask=r1, edge_bits=e1)      # warm-up
    plain_ms, batched_ms = [], []
    per = []
    for step in range(args.steps):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for i in range(T):
            _, _, st = ctx.prune(first + i, role_mask=r1, edge_bits=e1)
            if step == 0:
                per.append({"edges": len(ts[i].edges), "ms": round(st["ms_total"], 2),
                            "ms_exact": round(st["ms_exact"], 2),
                            "result_vertices": st["result_vertices"]})
        torch.cuda.synchronize()
        plain_ms.append(1e3 * (time.perf_counter() - ta))
        ta = time.perf_counter()
        _, _, stb = ctx.prune(first, count=T, role_mask=rb, edge_bits=eb,
                              batch_streams=args.batch_streams, order="learned",
                              learned_min_score=thr)
        torch.cuda.synchronize()
        batched_ms.append(1e3 * (time.perf_counter() - ta))
        log(f"step {step}: one per call {plain_ms[-1]:.1f} ms, batched+learned {batched_ms[-1]:.1f} ms")
    # the last variant of the plain pass is still in r1/e1: same output
    same = bool(torch.equal(r1[0], rb[T - 1]) and torch.equal(e1[0], eb[T - 1]))
    bm = float(np.median(batched_ms))
    pmed = float(np.median(plain_ms))
    out = {
        "metric": "GTEPS (directed CSR entries x variants / time-to-fixpoint, bit-exact complete "
                  "sets)",
        "value": round(g.m * T / (bm / 1e3) / 1e9, 4), "unit": "GTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": round(bm, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"R-MAT scale {scale} ef16 log2-degree labels; 8-vertex two-cycle "
                               f"template with a repeated-label pair 4 hops apart and its "
                               f"{T - 1} connected 1-2 edge-deletion relaxations",
                   "n": n, "m_directed": g.m, "variants": T, "base_labels": base.labels,
                   "parallelism": "single GPU"},
        "one_variant_per_call_fixed_order_ms": round(pmed, 2),
        "batched_learned_ms": round(bm, 2), "batch_streams": args.batch_streams,
        "speedup": round(pmed / bm, 4), "last_variant_identical": same,
        "batched_stats": {k: round(v, 2) if isinstance(v, float) else v
                          for k, v in stb.items() if k.startswith("ms_") or k in
                          ("constraints", "result_vertices", "edge_queries")},
        "per_variant_plain": per,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def explore_leg(ctx, tmpl, max_deletions=4):
    """Exploratory search (the paper's 6-clique scenario): the complete
    graph on the timed template's vertex labels, relaxed level by level
    (connected variants, one per isomorphism class) until a variant has a
    match; per-level variant counts, matches and wall time."""
    from paper_1912_08453_amd import explore
    n0 = len(tmpl.labels)
    clique = [(a, b) for a in range(n0) for b in range(a + 1, n0)]
    t0 = time.perf_counter()
    res = explore.explore(ctx, tmpl.labels, clique, max_deletions=max_deletions, log=log)
    total = 1e3 * (time.perf_counter() - t0)
    out = {"workload": f"K{n0} on labels {list(tmpl.labels)}, up to {max_deletions} edges "
                       f"removed", "levels": res.levels, "stop_level": res.level,
           "total_ms": round(total, 1)}
    if res.level >= 0:
        out["union_vertices"] = int((res.role_union != 0).sum().item())
    return out


def autotune_leg(ctx, tid, role, edge):
    """Coordinate search of the tuning settings on the timed template (best
    of 3 prunes per candidate), the tuned time against the defaults' on the
    same timer, and the output with the tuned settings against the timed
    steps' output.  The defaults are restored afterwards."""
    import torch
    from paper_1912_08453_amd import autotune
    start = ctx.params()
    best, table = autotune.autotune(ctx, [tid], reps=3)
    timer = autotune.prune_timer(ctx, [tid], reps=5)
    tuned_ms = timer()
    r2, e2, _ = ctx.prune(tid)
    same = bool(torch.equal(r2, role) and torch.equal(e2, edge))
    for k, v in start.items():
        ctx.set_param(k, v)
    default_ms = timer()
    return {"defaults": start, "tuned": {k: v for k, v in best.items() if v != start[k]},
            "candidates_timed": len(table) - 1, "default_ms": round(default_ms, 2),
            "tuned_ms": round(tuned_ms, 2), "outputs_identical": same}


def batched_leg(ctx, g, streams, seed=3, count=64):
    """64 mixed templates (paths/trees, one- and two-cycle, K4; some with a
    repeated label) against the resident graph: one pm_prune call per
    template in the fixed order, then one call for all of them on `streams`
    concurrent streams.  Outputs must be identical."""
    import torch
    from paper_1912_08453_amd import inputs as I
    ts = I.templates_batch(g, seed, count=count)
    first = ctx.load_templates(ts)
    n, words = g.n, (g.m + 63) // 64
    dev = torch.device("cuda", 0)
    r1 = torch.empty((count, n), dtype=torch.int64, device=dev)
    e1 = torch.empty((count, words), dtype=torch.int64, device=dev)
    r2 = torch.empty_like(r1)
    e2 = torch.empty_like(e1)
    ctx.prune(first, count=count, role_mask=r2, edge_bits=e2, batch_streams=streams)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phase = {"ms_exact": 0.0, "ms_nlcc": 0.0, "ms_lcc": 0.0}
    for i in range(count):
        _, _, st = ctx.prune(first + i, role_mask=r1[i:i + 1], edge_bits=e1[i:i + 1])
        for k in phase:
            phase[k] += st[k]
    torch.cuda.synchronize()
    seq_ms = 1e3 * (time.perf_counter() - t0)
    t0 = time.perf_counter()
    ctx.prune(first, count=count, role_mask=r2, edge_bits=e2, batch_streams=streams)
    torch.cuda.synchronize()
    bat_ms = 1e3 * (time.perf_counter() - t0)
    same = bool(torch.equal(r1, r2) and torch.equal(e1, e2))
    del r1, e1, r2, e2
    return {"workload": f"{count} templates (3-8 vertices; trees, one/two cycles, K4; "
                        f"seed {seed}) on the same graph",
            "one_template_per_call_ms": round(seq_ms, 2),
            "batched_ms": round(bat_ms, 2), "batch_streams": streams,
            "speedup": round(seq_ms / bat_ms, 4), "outputs_identical": same,
            "one_per_call_phase_ms": {k: round(v, 2) for k, v in phase.items()}}


def learned_leg(ctx, g, seed=4, count=64):
    """64 seeded 7-8 vertex templates with cyclomatic number >= 2 (seeds
    disjoint from the model's training templates): whole prune with the
    fixed order and with the learned order (model and stopping threshold
    shipped with the package).  Outputs must be identical."""
    import torch
    from paper_1912_08453_amd import inputs as I
    from paper_1912_08453_amd import order_training as OT
    ts = I.templates_multicycle(g, seed, count=count)
    first = ctx.load_templates(ts)
    ctx.load_model(OT.load_model())
    thr = OT.load_threshold()
    n, words = g.n, (g.m + 63) // 64
    dev = torch.device("cuda", 0)
    ra = torch.empty((1, n), dtype=torch.int64, device=dev)
    ea = torch.empty((1, words), dtype=torch.int64, device=dev)
    rb = torch.empty_like(ra)
    eb = torch.empty_like(ea)
    keys = ("ms_total", "ms_nlcc", "ms_lcc", "ms_exact", "constraints")
    tot = {"fixed": dict.fromkeys(keys, 0.0), "learned": dict.fromkeys(keys, 0.0)}
    same = True
    ctx.prune(first, role_mask=ra, edge_bits=ea)   # warm-up
    for i in range(count):
        _, _, sf = ctx.prune(first + i, role_mask=ra, edge_bits=ea)
        _, _, sl = ctx.prune(first + i, order="learned", learned_min_score=thr,
                             role_mask=rb, edge_bits=eb)
        same = same and bool(torch.equal(ra, rb) and torch.equal(ea, eb))
        for k in keys:
            tot["fixed"][k] += sf[k]
            tot["learned"][k] += sl[k]
    out = {"workload": f"{count} multi-cycle templates (7-8 vertices, cyclomatic >= 2, "
                       f"seed {seed}) on the same graph",
           "min_score": thr, "outputs_identical": same}
    for mode in ("fixed", "learned"):
        out[mode] = {k: round(v, 2) for k, v in tot[mode].items()}
    out["speedup_total"] = round(tot["fixed"]["ms_total"] / tot["learned"]["ms_total"], 4)
    cl_f = tot["fixed"]["ms_nlcc"] + tot["fixed"]["ms_lcc"]
    cl_l = tot["learned"]["ms_nlcc"] + tot["learned"]["ms_lcc"]
    out["speedup_nlcc_plus_lcc"] = round(cl_f / cl_l, 4) if cl_l > 0 else None
    return out


def cpu_baseline(g, tmpl, budget_s):
    """The oracle, as it stands, on a bounded sample of the same workload:
    init, LCC fixpoint and every non-local constraint on the full graph,
    then the exact final step's searches for a uniform random sample of the
    surviving vertices, scaled to all of them.  Rate = directed entries per
    second of the estimated whole prune."""
    import numpy as np
    import oracle
    from oracle import constraints as C
    cores = oracle.num_threads()
    gg = oracle._G(g.row_ptr, g.col, g.labels)
    tt = oracle._T(tmpl.labels, tmpl.edges)
    t0 = time.perf_counter()
    om = oracle.init_roles(gg, tt)
    oracle.lcc(gg, tt, om)
    t_lcc = time.perf_counter() - t0
    K0 = C.non_local_constraints(tmpl.labels, tmpl.edges)
    done = 0
    for c in K0:
        if time.perf_counter() - t0 > budget_s:
            break
        if oracle.nlcc(gg, om, c):
            oracle.lcc(gg, tt, om)
        done += 1
    t_nlcc = time.perf_counter() - t0 - t_lcc
    active = np.nonzero(om)[0].astype(np.int32)
    rng = np.random.Generator(np.random.Philox(7))
    sample = np.sort(rng.permutation(active)[:min(2000, active.shape[0])]) if active.size else active
    t1 = time.perf_counter()
    oracle.exact_subset(gg, tt, om, sample)
    t_s = time.perf_counter() - t1
    t_exact = t_s * (active.shape[0] / max(sample.shape[0], 1))
    total = t_lcc + t_nlcc + t_exact
    complete = done == len(K0)
    return {"value": round(g.m / total / 1e9, 6), "unit": "GTEPS", "cores": cores,
            "kind": "oracle",
            "sample": f"oracle on the same graph and template: init + LCC fixpoint "
                      f"({t_lcc:.2f}s) + {done}/{len(K0)} non-local constraints ({t_nlcc:.2f}s) "
                      f"measured in full; exact step timed on {sample.shape[0]} of "
                      f"{active.shape[0]} surviving vertices ({t_s:.2f}s) and scaled to all "
                      f"(est. {t_exact:.1f}s)" + ("" if complete else "; constraint list cut "
                      "by the time budget")}


if __name__ == "__main__":
    main()
