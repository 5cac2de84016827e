#!/usr/bin/env python3
"""Benchmark of complete-set pruning (constraint checking) on one MI355X.

Default workload (one step): R-MAT scale 26 (Graph500 parameters, edge
factor 16, 67.1 M vertices, 2.1 G directed CSR entries, log2-degree uint8
labels), the 8-vertex two-cycle template with a repeated-label pair four
hops apart and all its connected 1- and 2-edge-deletion relaxations (28
templates in all), pruned to their complete sets through the C ABI:

  * the neighbour-label count index (one streaming pass over the CSR; the
    first LCC sweep of every template reads it),
  * the label-pair subgraph of the batch (the entries whose label pair is
    that of a template edge; every template's first compaction reads it
    instead of the whole CSR), then
  * one batched pm_prune call for all 28 templates on 4 concurrent streams
    with the learned constraint order: first LCC sweep, compaction, LCC
    fixpoint, every non-local constraint, the exact final search.

Inputs are resident in HBM before timing starts.  The plain path -- the
same two index passes, then one pm_prune call per template with the fixed order
-- is timed beside it, and every template's output must be identical.

Prints one JSON line: metric GTEPS = directed CSR entries x templates /
time-to-fixpoint of the step, the roofline of the CSR-streaming kernel (the
count-index pass), the CPU oracle's rate on a bounded sample, and legs on a
resident scale-22 graph (single template, 64-template batch, learned order
with ablations, incremental search, match counting, exploratory search,
topology sweep and design ablations).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
GRAPH500 = (0.57, 0.19, 0.19)
CHAKRABARTI = (0.45, 0.15, 0.15)
UNIFORM = (0.25, 0.25, 0.25)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="theta8-s26", choices=["theta8-s26", "tri-square-s22"],
                    help="theta8-s26 (default): the scale-26 batch of a base template and its "
                         "relaxations; tri-square-s22: one template at scale 22")
    ap.add_argument("--legs",
                    default="single,batched,learned,autotune,incremental,count,explore,topology",
                    help="comma-separated legs on a resident scale-22 graph; '' for none")
    ap.add_argument("--batch-streams", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (for HBM counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path, so --gpus must be 1 "
              "(templates would shard across GPUs with no communication; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
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

    legs = [x for x in args.legs.split(",") if x]
    if args.workload == "theta8-s26":
        out = theta8_s26(args)
    else:
        out = None
    ctx22 = g22 = None
    leg_out = {}
    if legs or out is None:
        g22 = build_graph(22, 22)
        ctx22 = load(g22)
    if out is None:
        out = single_leg(ctx22, g22, args, primary=True)
    else:
        if "single" in legs:
            leg_out["single_template_s22"] = single_leg(ctx22, g22, args, primary=False)
    for name, fn in (("batched", batched_leg), ("learned", learned_leg),
                     ("autotune", autotune_leg),
                     ("incremental", incremental_leg), ("count", count_leg),
                     ("explore", explore_leg), ("topology", topology_leg)):
        if name in legs:
            t0 = time.time()
            leg_out[name] = fn(ctx22, g22, args)
            log(f"leg {name} ({time.time() - t0:.0f}s): {json.dumps(leg_out[name])[:400]}")
    out["legs"] = leg_out
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ helpers
def build_graph(scale, seed, abc=GRAPH500):
    import numpy as np  # noqa: F401
    from paper_1912_08453_amd import inputs as I
    t0 = time.time()
    rp, col = I.rmat_csr(scale, seed=seed, abc=abc)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    log(f"graph scale {scale} abc={abc}: n={g.n} m={g.m} built in {time.time() - t0:.1f}s")
    return g


def load(g):
    import torch
    from paper_1912_08453_amd import pm
    dev = torch.device("cuda", 0)
    ctx = pm.PM(0)
    ctx.load_graph(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                   torch.from_numpy(g.labels).to(dev))
    torch.cuda.synchronize()
    return ctx


def wall(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0), r


def index_bytes(ctx):
    """Algorithmic bytes of one count-index pass (the first LCC sweep's
    input for every template): row_ptr (8(n+1)), col (4m), every vertex's
    label once (n, the compulsory part of the label gather) and the index
    written (labels x padded n)."""
    gi = ctx.graph_info()
    n, m = gi["n"], gi["m"]
    return 8 * (n + 1) + 4 * m + n + gi["index_bytes"]


def recorded_traffic(kernel_file):
    """HBM bytes per launch from a counter record under profiles/
    (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration), or None when
    there is none or the kernel's source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", kernel_file)
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#") and "=" in line:
            k, v = line.split("=", 1)
            rec[k.strip()] = v.strip()
    # every source the counted kernels come from, unchanged since
    srcs = [x.strip() for x in rec.get("source", "").split(",") if x.strip()]
    shas = [x.strip() for x in rec.get("source_sha1", "").split(",")]
    if not srcs or len(srcs) != len(shas):
        return None
    for name, sha in zip(srcs, shas):
        src = os.path.join(ROOT, name)
        if not os.path.exists(src) or hashlib.sha1(open(src, "rb").read()).hexdigest() != sha:
            return None
    try:
        return int(float(rec["fetch_kib_per_dispatch"]) * 1024 * float(rec["fetch_scale"]) +
                   float(rec["write_kib_per_dispatch"]) * 1024 * float(rec["write_scale"]))
    except (KeyError, ValueError):
        return None


def roofline_of_index(ctx, ms_list, workload_key):
    b = index_bytes(ctx)
    k_ms = sum(ms_list) / len(ms_list)
    achieved = b / (k_ms / 1e3) / 1e9
    return {"bound": "hbm",
            "kernel": "label_count_tiles_kernel + label_count_hub_kernel (neighbour-label count "
                      "index: one pass over row_ptr and col, labels gathered, index written)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": recorded_traffic(f"label_count_{workload_key}.txt"),
            "bytes_per_launch": int(b), "ms_per_launch": round(k_ms, 4),
            "launches_timed": len(ms_list)}


def pair_bytes(g, ts, ctx):
    """Algorithmic bytes of one label-pair subgraph build for templates ts,
    the batch's one pass over the CSR: every label once (n), the row bounds
    (8 n_a) and columns (4 m_a) of the n_a vertices whose label is on a
    template edge (every other row is skipped), the role byte of those
    vertices written (n_a), the subgraph written (row_ptr 8(n+1), column and
    original offset 8 m_p for its m_p entries) and its count index written
    (labels x padded n)."""
    import numpy as np
    labs = sorted({t.labels[q] for t in ts for e in t.edges for q in e})
    held = np.isin(g.labels, np.asarray(labs, dtype=g.labels.dtype))
    deg = np.diff(g.row_ptr)
    n_a, m_a = int(held.sum()), int(deg[held].sum())
    n, m_p = g.n, int(ctx.graph_info()["pair_entries"])
    nlab = int(g.labels.max()) + 1
    b = n + 8 * n_a + 4 * m_a + n_a + 8 * (n + 1) + 8 * m_p + nlab * ((n + 255) // 256 * 256)
    return b, {"n_a": n_a, "m_a": m_a, "m_p": m_p}


def roofline_of_pair(g, ts, ctx, ms_list, workload_key):
    b, sizes = pair_bytes(g, ts, ctx)
    k_ms = sum(ms_list) / len(ms_list)
    achieved = b / (k_ms / 1e3) / 1e9
    return {"bound": "hbm",
            "kernel": "label-pair subgraph build (role init, compaction count/scan/fill over the "
                      "rows of vertices with a template-edge label, labels gathered; then its "
                      "neighbour-label counts, label_count_tiles_kernel<true>): the batch's one "
                      "pass over the CSR, which every template's first LCC sweep and first "
                      "compaction read",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": recorded_traffic(f"pair_subgraph_{workload_key}.txt"),
            "bytes_per_launch": int(b), "sizes": sizes, "ms_per_launch": round(k_ms, 4),
            "launches_timed": len(ms_list)}


# ------------------------------------------------------ config 5 (default)
def theta8_s26(args, scale=26, seed=26, template_seed=0):
    import numpy as np
    import torch
    from paper_1912_08453_amd import inputs as I
    from paper_1912_08453_amd import order_training as OT
    g = build_graph(scale, seed)
    base = I.template_theta8(g, template_seed)
    ts = I.relaxations(base)
    T = len(ts)
    log(f"{T} templates: base labels {base.labels}")
    ms_load, ctx = wall(lambda: load(g))
    first = ctx.load_templates(ts)
    ctx.load_model(OT.load_model())
    # settings the project's autotuner chose for this workload (search
    # switches and grid, LCC bin bounds; results do not depend on them),
    # used by the batched and the plain path alike
    from paper_1912_08453_amd import autotune
    tuned = autotune.apply_tuned(ctx, "theta8-s26")
    thr = OT.load_threshold()
    dev = torch.device("cuda", 0)
    n, words = g.n, (g.m + 63) // 64
    rb = torch.empty((T, n), dtype=torch.int64, device=dev)
    eb = torch.empty((T, words), dtype=torch.int64, device=dev)

    # per step: the label-pair subgraph of the batch's template edges and
    # its neighbour-label counts (the batch's one pass over the CSR: every
    # template's first LCC sweep reads the counts, its first compaction the
    # subgraph), then the batch.  The graph's full count index, built at
    # load, is not read by these templates.
    pair_ms = []

    def step(order="learned", min_score=None):
        k_ms = ctx.build_pair_index(first, T)
        pair_ms.append(k_ms)
        _, _, st = ctx.prune(first, count=T, role_mask=rb, edge_bits=eb,
                             batch_streams=args.batch_streams, order=order,
                             learned_min_score=min_score)
        return k_ms, st

    for i in range(args.warmup):
        ms, _ = wall(step)
        log(f"warmup {i}: {ms:.1f} ms")
    times, k_ms_list, stats = [], [], []
    for i in range(args.steps):
        ms, (k_ms, st) = wall(step)
        times.append(ms)
        k_ms_list.append(k_ms)
        stats.append(st)
        log(f"step {i}: {ms:.1f} ms (label-pair subgraph and its counts {k_ms:.2f} ms)")
    ms_step = float(np.mean(times))
    value = g.m * T / (ms_step / 1e3) / 1e9

    # the plain path: the same pass over the CSR, one call per template,
    # fixed order
    r1 = torch.empty((T, n), dtype=torch.int64, device=dev)
    e1 = torch.empty((T, words), dtype=torch.int64, device=dev)

    def plain():
        ctx.build_pair_index(first, T)
        per = []
        for i in range(T):
            _, _, st = ctx.prune(first + i, role_mask=r1[i:i + 1], edge_bits=e1[i:i + 1])
            per.append(st)
        return per
    plain_ms = []
    per_plain = None
    for _ in range(min(args.steps, 3)):
        ms, per_plain = wall(plain)
        plain_ms.append(ms)
    identical = bool(torch.equal(r1, rb) and torch.equal(e1, eb))
    log(f"plain {np.mean(plain_ms):.1f} ms, batched+learned {ms_step:.1f} ms, identical {identical}")
    if not identical:
        raise SystemExit("batched output differs from the one-template-per-call output")
    # other batched modes (one timing each), same outputs
    alt = {}
    for name, order, ms_thr in (("batched_fixed", None, None),
                                ("batched_learned_stop", "learned", thr)):
        ms, _ = wall(lambda: step(order, ms_thr))
        same = bool(torch.equal(r1, rb) and torch.equal(e1, eb))
        alt[name] = {"ms": round(ms, 2), "identical": same}
        if not same:
            raise SystemExit(f"{name} output differs")
    del r1, e1
    roof = roofline_of_pair(g, ts, ctx, k_ms_list, "theta8_rmat26")
    phases = {k: round(float(np.mean([s[k] for s in stats])), 3) for k in stats[-1]
              if k.startswith("ms_")}
    per_variant = [{"edges": len(ts[i].edges), "ms": round(p["ms_total"], 2),
                    "ms_exact": round(p["ms_exact"], 2),
                    "result_vertices": p["result_vertices"]} for i, p in enumerate(per_plain)]
    out = {
        "metric": "GTEPS (directed CSR entries x templates / time-to-fixpoint, bit-exact "
                  "complete sets; batched + learned order vs one template per call, fixed "
                  "order)",
        "value": round(value, 4), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"R-MAT scale {scale} (a,b,c)=(0.57,0.19,0.19) ef16, "
                               f"log2-degree uint8 labels; 8-vertex two-cycle template with a "
                               f"repeated-label pair 4 hops apart and its {T - 1} connected "
                               f"1-2 edge-deletion relaxations ({T} templates), one batch",
                   "n": n, "m_directed": g.m, "templates": T, "base_labels": base.labels,
                   "batch_streams": args.batch_streams, "order": "learned (every non-local "
                   "constraint checked; the one-repeated-pair trees' path constraints decided "
                   "by path sweeps)", "settings": tuned, "parallelism": "single GPU"},
        "time_to_fixpoint_ms": round(ms_step, 3),
        "plain_one_template_per_call_ms": round(float(np.mean(plain_ms)), 2),
        "speedup_vs_plain": round(float(np.mean(plain_ms)) / ms_step, 4),
        "outputs_identical": identical,
        "other_batched_modes": alt,
        "pair_index_ms": round(float(np.mean(pair_ms)), 3),
        "count_index_at_load_ms": round(float(ctx.graph_info()["ms_count_index"]), 3),
        "pair_index_entries": ctx.graph_info()["pair_entries"],
        "graph_load_ms": round(ms_load, 1),
        "phases_ms_sum_over_templates": phases,
        "per_template_plain": per_variant,
        "roofline": roof,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle sweep on a vertex sample")
        out["cpu_baseline"] = cpu_sweep_baseline(g, ts, T)
        log(f"cpu baseline: {out['cpu_baseline']['value']} GTEPS")
    ctx.close()
    del rb, eb
    torch.cuda.empty_cache()
    return out


def cpu_sweep_baseline(g, ts, T, budget_s=20.0, target_1t_s=4.0):
    """The oracle's local rule (one LCC sweep from the label roles) timed for
    every template of the batch in turn, each sweep over all vertices that
    hold one of the template's roles (the only rows a sweep scans), until the
    templates are done or budget_s has passed; the mean sweep time stands for
    the templates not reached.  Every template's prune needs at least this
    first sweep and the oracle's later steps (LCC fixpoint, constraints,
    exact step) only add time, so m x T / (sum of first-sweep times) bounds
    its rate in entries x templates per second from above.  Also timed on one
    thread, on a uniform vertex sample of the base template."""
    import numpy as np
    import oracle
    gg = oracle._G(g.row_ptr, g.col, g.labels)
    cores = oracle.num_threads()
    sweeps, ents, t_start = [], 0, time.perf_counter()
    for t in ts:
        tt = oracle._T(t.labels, t.edges)
        om = oracle.init_roles(gg, tt)
        v = np.nonzero(om)[0].astype(np.int32)
        t0 = time.perf_counter()
        _, ent = oracle.lcc_sample(gg, tt, om, v)
        sweeps.append(time.perf_counter() - t0)
        ents += ent
        if time.perf_counter() - t_start > budget_s:
            break
    est_s = float(np.mean(sweeps)) * T
    # one thread: a vertex sample of the base template's sweep
    tt = oracle._T(ts[0].labels, ts[0].edges)
    om = oracle.init_roles(gg, tt)
    active = np.nonzero(om)[0].astype(np.int32)
    perm = np.random.Generator(np.random.Philox(7)).permutation(active)
    # a full sweep on one thread takes about cores x the threaded one
    k1 = int(min(active.size, max(1 << 10, active.size * target_1t_s /
                                  max(sweeps[0] * cores, 1e-6))))
    v1 = np.sort(perm[:k1])
    oracle.set_threads(1)
    t0 = time.perf_counter()
    _, ent1 = oracle.lcc_sample(gg, tt, om, v1)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(cores)
    sweep1_s = dt1 * active.size / max(v1.size, 1)
    return {"value": round(g.m * T / est_s / 1e9, 6), "unit": "GTEPS", "cores": cores,
            "kind": "oracle",
            "sample": f"oracle's LCC rule, the first sweep (from the label roles) of "
                      f"{len(sweeps)} of the {T} templates, each over every vertex holding one "
                      f"of its roles in the same scale-26 graph ({ents} entries scanned, "
                      f"{sum(sweeps):.2f}s; mean {np.mean(sweeps):.3f}s per sweep, est. "
                      f"{est_s:.1f}s for all {T}); every template needs at least this sweep, so "
                      f"m x {T} / that time bounds the oracle's rate from above",
            "one_thread": {"value": round(g.m / sweep1_s / 1e9, 6), "unit": "GTEPS", "cores": 1,
                           "sample": f"base template's sweep on {v1.size} of its {active.size} "
                                     f"role-holding vertices ({ent1} entries, {dt1:.1f}s), "
                                     f"est. {sweep1_s:.1f}s per sweep"}}


# ------------------------------------------------- config 2 (single template)
def single_leg(ctx, g, args, primary):
    """The triangle + 4-cycle + pendant template (repeated label) on the
    scale-22 graph: time-to-fixpoint of one prune, with the count-index pass
    in the step."""
    import numpy as np
    import torch
    from paper_1912_08453_amd import inputs as I
    t = I.template_tri_square(g, 0)
    tid = ctx.load_templates([t])
    dev = torch.device("cuda", 0)
    role = torch.empty((1, g.n), dtype=torch.int64, device=dev)
    edge = torch.empty((1, (g.m + 63) // 64), dtype=torch.int64, device=dev)

    def step():
        k_ms = ctx.build_count_index()
        _, _, st = ctx.prune(tid, role_mask=role, edge_bits=edge)
        return k_ms, st
    steps = args.steps if primary else max(args.steps, 5)
    for _ in range(args.warmup):
        wall(step)
    times, kms, stats = [], [], []
    for _ in range(steps):
        ms, (k, st) = wall(step)
        times.append(ms)
        kms.append(k)
        stats.append(st)
    ms_step = float(np.mean(times))
    prune_ms = float(np.mean([s["ms_total"] for s in stats]))
    phases = {k: round(float(np.mean([s[k] for s in stats])), 4) for k in stats[-1]
              if k.startswith("ms_")}
    search = {k: round(float(np.mean([s[k] for s in stats])), 3) for k in stats[-1]
              if k.startswith("wave_ms_")}
    r = role[0].cpu().numpy().view(np.uint64)
    res = {"workload": f"R-MAT scale 22 ef16 log2-degree labels; 6-vertex triangle+4-cycle+"
                       f"pendant template {t.labels} (repeated label)",
           "value": round(g.m / (ms_step / 1e3) / 1e9, 4), "unit": "GTEPS",
           "ms_per_step": round(ms_step, 3), "steps": steps,
           "prune_device_ms": round(prune_ms, 3),
           "value_prune_only": round(g.m / (prune_ms / 1e3) / 1e9, 4),
           "count_index_ms": round(float(np.mean(kms)), 4),
           "phases_ms": phases, "search_wave_ms": search,
           "result_vertices": int((r != 0).sum()),
           "roofline": roofline_of_index(ctx, kms, "rmat22_log2deg"),
           "dominant_phase": {"phase": "exact step (edge_search_kernel, vertex_search_kernel)",
                              "share_of_prune": round(phases["ms_exact"] /
                                                      max(phases["ms_total"], 1e-9), 4),
                              "bound": "search latency / random gathers (no byte roofline)"}}
    log(f"single template: {ms_step:.2f} ms/step")
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle prune of the single template (bounded sample)")
        res["cpu_baseline"] = cpu_oracle_prune_baseline(g, t)
    if primary:
        res.update({"metric": "GTEPS (directed CSR entries / time-to-fixpoint, bit-exact "
                              "complete set)", "n_gpus": 1, "warmup": args.warmup,
                    "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                    "dtype": "u8", "data": "synthetic",
                    "config": {"workload": res["workload"], "n": g.n, "m_directed": g.m,
                               "parallelism": "single GPU"},
                    "cpu_baseline": res.get("cpu_baseline")})
    return res


def cpu_oracle_prune_baseline(g, t, budget_s=20.0, sample=2000):
    """The oracle on the same graph and template: init, LCC fixpoint and
    every non-local constraint in full, then the exact step for a uniform
    sample of the surviving vertices, scaled to all of them."""
    import numpy as np
    import oracle
    from oracle import constraints as C
    cores = oracle.num_threads()
    gg = oracle._G(g.row_ptr, g.col, g.labels)
    tt = oracle._T(t.labels, t.edges)
    t0 = time.perf_counter()
    om = oracle.init_roles(gg, tt)
    oracle.lcc(gg, tt, om)
    t_lcc = time.perf_counter() - t0
    K0 = C.non_local_constraints(t.labels, t.edges)
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
    smp = np.sort(rng.permutation(active)[:min(sample, active.shape[0])]) if active.size else active
    t1 = time.perf_counter()
    oracle.exact_subset(gg, tt, om, smp)
    t_s = time.perf_counter() - t1
    t_exact = t_s * (active.shape[0] / max(smp.shape[0], 1))
    total = t_lcc + t_nlcc + t_exact
    return {"value": round(g.m / total / 1e9, 6), "unit": "GTEPS", "cores": cores,
            "kind": "oracle",
            "sample": f"init + LCC fixpoint ({t_lcc:.2f}s) + {done}/{len(K0)} non-local "
                      f"constraints ({t_nlcc:.2f}s) in full; exact step on {smp.shape[0]} of "
                      f"{active.shape[0]} surviving vertices ({t_s:.2f}s) scaled to all "
                      f"(est. {t_exact:.1f}s)"}


# ----------------------------------------------------------- config 3 batch
def batched_leg(ctx, g, args, seed=3, count=64):
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
    ctx.prune(first, count=count, role_mask=r2, edge_bits=e2, batch_streams=args.batch_streams)

    def one_by_one():
        for i in range(count):
            ctx.prune(first + i, role_mask=r1[i:i + 1], edge_bits=e1[i:i + 1])
    seq_ms, _ = wall(one_by_one)
    bat_ms, _ = wall(lambda: ctx.prune(first, count=count, role_mask=r2, edge_bits=e2,
                                       batch_streams=args.batch_streams))
    same = bool(torch.equal(r1, r2) and torch.equal(e1, e2))
    # the same batch drawing all scratch from one caller-owned workspace
    ws_bytes = ctx.workspace_size(first, count, batch_streams=args.batch_streams)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    ctx.set_workspace(ws)
    ws_ms, _ = wall(lambda: ctx.prune(first, count=count, role_mask=r2, edge_bits=e2,
                                      batch_streams=args.batch_streams))
    same_ws = bool(torch.equal(r1, r2) and torch.equal(e1, e2))
    ctx.set_workspace(None)
    del ws, r1, e1, r2, e2
    torch.cuda.empty_cache()
    return {"workload": f"{count} templates (3-8 vertices; trees, one/two cycles, K4; seed {seed})"
                        f" on the scale-22 graph",
            "one_template_per_call_ms": round(seq_ms, 2), "batched_ms": round(bat_ms, 2),
            "batch_streams": args.batch_streams, "speedup": round(seq_ms / bat_ms, 4),
            "outputs_identical": same,
            "caller_workspace": {"bytes": ws_bytes, "batched_ms": round(ws_ms, 2),
                                 "outputs_identical": same_ws}}


# ------------------------------------------------------ config 4 learned
def learned_leg(ctx, g, args, seed=4, count=64):
    """Multi-cycle templates: fixed order; learned order with every
    constraint checked; learned order with the stopping threshold; and, to
    separate ordering from skipping, the fixed order stopped after as many
    constraints as the learned run checked, and no non-local constraint at
    all (stop_after = 0, then the exact step).  All outputs identical."""
    import torch
    from paper_1912_08453_amd import inputs as I
    from paper_1912_08453_amd import order_training as OT
    ts = I.templates_multicycle(g, seed, count=count)
    first = ctx.load_templates(ts)
    ctx.load_model(OT.load_model())
    thr = OT.load_threshold()
    keys = ("ms_total", "ms_nlcc", "ms_lcc", "ms_exact", "constraints")
    modes = ("fixed", "learned_all", "learned_stop", "fixed_stop_same_count", "no_nonlocal")
    tot = {m: dict.fromkeys(keys, 0.0) for m in modes}
    same = True
    ra = None
    ctx.prune(first)   # warm-up
    for i in range(count):
        outs = {}
        _, _, s_l = ctx.prune(first + i, order="learned", learned_min_score=thr)
        k_stop = int(s_l["constraints"])
        for m, kw in (("fixed", {}), ("learned_all", {"order": "learned"}),
                      ("learned_stop", {"order": "learned", "learned_min_score": thr}),
                      ("fixed_stop_same_count", {}), ("no_nonlocal", {})):
            if m == "fixed_stop_same_count":
                r, e, st = ctx.prune(first + i, max_checks=k_stop)
            elif m == "no_nonlocal":
                r, e, st = ctx.prune(first + i, max_checks=0)
            else:
                r, e, st = ctx.prune(first + i, **kw)
            outs[m] = (r.clone(), e.clone())
            for k in keys:
                tot[m][k] += st[k]
        if i % 16 == 15:
            log(f"learned leg: {i + 1}/{count} templates")
        ra, ea = outs["fixed"]
        for m in modes:
            same = same and bool(torch.equal(ra, outs[m][0]) and torch.equal(ea, outs[m][1]))
    res = {"workload": f"{count} multi-cycle templates (7-8 vertices, cyclomatic >= 2, "
                       f"seed {seed}) on the scale-22 graph", "min_score": thr,
           "outputs_identical": same}
    for m in modes:
        res[m] = {k: round(v, 2) for k, v in tot[m].items()}
    f = tot["fixed"]["ms_total"]
    res["speedup_vs_fixed"] = {m: round(f / tot[m]["ms_total"], 4) for m in modes}
    return res


# ------------------------------------------------------------- autotuner
def autotune_leg(ctx, g, args):
    """Coordinate search of the settings (search switches and grid, LCC bin
    bounds) on the config-2 template, best of 3 prunes per candidate; the
    tuned time against the defaults' on the same timer, same output.  The
    defaults are restored afterwards."""
    import torch
    from paper_1912_08453_amd import autotune
    from paper_1912_08453_amd import inputs as I
    t = I.template_tri_square(g, 0)
    tid = ctx.load_templates([t])
    start = ctx.params()
    r0, e0, _ = ctx.prune(tid)
    r0, e0 = r0.clone(), e0.clone()
    best, table = autotune.autotune(ctx, [tid], reps=3)
    timer = autotune.prune_timer(ctx, [tid], reps=5)
    tuned_ms = timer()
    r1, e1, _ = ctx.prune(tid)
    same = bool(torch.equal(r0, r1) and torch.equal(e0, e1))
    for k, v in start.items():
        ctx.set_param(k, v)
    default_ms = timer()
    return {"defaults": start, "tuned": {k: v for k, v in best.items() if v != start[k]},
            "candidates_timed": len(table) - 1, "default_ms": round(default_ms, 2),
            "tuned_ms": round(tuned_ms, 2), "outputs_identical": same}


# ----------------------------------------------------- incremental (f2)
def incremental_leg(ctx, g, args):
    """Interactive incremental search: the triangle + 4-cycle + pendant
    template reached from a spanning tree by adding its two other edges,
    then relaxed again by deleting them; each revision reuses the previous
    complete set (additions) or the candidate set with the previous complete
    set pre-certified (deletions), timed against a full prune."""
    from paper_1912_08453_amd import incremental
    from paper_1912_08453_amd import inputs as I
    t = I.template_tri_square(g, 0)
    edges = sorted(tuple(sorted(e)) for e in t.edges)
    tree = [(0, 1), (0, 2), (0, 4), (1, 3), (3, 5)]
    extra = [e for e in edges if e not in tree]
    s = incremental.Session(ctx, t.labels, tree, compare=True)
    for e in extra:
        s.add_edge(*e)
    for e in extra[::-1]:
        s.delete_edge(*e)
    recs = s.history[1:]
    inc = sum(r["ms"] + r.get("candidate_ms", 0.0) for r in recs)
    naive = sum(r["naive_ms"] for r in recs)
    return {"workload": f"scale-22 graph, template labels {t.labels}: start from the tree "
                        f"{tree}, add {extra}, delete them again",
            "steps": [{k: (list(v) if isinstance(v, tuple) else v) for k, v in r.items()}
                      for r in recs],
            "incremental_ms": round(inc, 2), "naive_ms": round(naive, 2),
            "speedup": round(naive / inc, 4) if inc > 0 else None,
            "outputs_identical": all(r["identical"] for r in recs)}


# --------------------------------------------------------- counting (f3)
def count_leg(ctx, g, args, max_maps=1 << 34):
    """Match counting on the pruned graph: every match of the config-2
    template and of the scale-22 batch's first templates, counted within
    their complete sets (each count stops past 2^34 maps; "complete" says
    whether it did), with the pruning time beside the counting time."""
    from paper_1912_08453_amd import inputs as I
    t = I.template_tri_square(g, 0)
    ts = [t] + I.templates_batch(g, 3, count=64)[:3]
    first = ctx.load_templates(ts)
    out = []
    for i, tt in enumerate(ts):
        prune_ms, (r, _, _) = wall(lambda: ctx.prune(first + i))
        r = r.clone()
        cnt_ms, res = wall(lambda: ctx.count_matches(first + i, state=r, max_maps=max_maps))
        rec = {"labels": list(tt.labels), "edges": len(tt.edges), "maps": res["maps"],
               "complete": bool(res["complete"]), "automorphisms": res["automorphisms"],
               "matches": res["subgraphs"] if res["complete"] else None,
               "roots": res["roots"], "prune_ms": round(prune_ms, 2),
               "count_ms": round(cnt_ms, 2)}
        log(f"count: {rec}")
        out.append(rec)
    return {"workload": "scale-22 graph: triangle+4-cycle+pendant and three batch templates",
            "templates": out}


# ------------------------------------------------------- exploratory (f1)
def explore_leg(ctx, g, args, max_deletions=4):
    """The 6-clique on the config-2 template's labels, relaxed level by
    level until a variant matches, with and without the candidate set."""
    from paper_1912_08453_amd import explore
    from paper_1912_08453_amd import inputs as I
    t = I.template_tri_square(g, 0)
    n0 = len(t.labels)
    clique = [(a, b) for a in range(n0) for b in range(a + 1, n0)]
    res = {}
    # one untimed run of each mode first (scratch growth), then the timed ones
    for cand in (False, True, False, True):
        log(f"explore: candidate set {cand}")
        ms, r = wall(lambda: explore.explore(ctx, t.labels, clique, max_deletions=max_deletions,
                                             use_candidate_set=cand))
        res["with_candidate_set" if cand else "from_label_roles"] = {
            "levels": r.levels, "stop_level": r.level, "total_ms": round(ms, 1),
            "union_vertices": int((r.role_union != 0).sum().item()) if r.level >= 0 else 0}
    return {"workload": f"K{n0} on labels {list(t.labels)}, up to {max_deletions} edges removed",
            **res}


# ------------------------------------------------- topology + ablations (f4)
def topology_leg(ctx22, g22, args, scale=20, seed=20):
    """R-MAT graphs of one scale with the paper's three parameter sets
    (Graph500, Chakrabarti et al., uniform), log2-degree labels, the
    triangle + 4-cycle + pendant shape with labels from an occurrence in
    each graph: complete-set size, match count and time; then the design
    ablations (edge elimination off, work aggregation off) on the scale-22
    graph, same output."""
    import numpy as np
    import torch
    from paper_1912_08453_amd import inputs as I
    from paper_1912_08453_amd import pm
    rows = []
    shapes = (("tri+square+pendant", I.TRI_SQUARE_EDGES),
              ("square+pendant", [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4)]))
    for name, abc in (("graph500", GRAPH500), ("chakrabarti", CHAKRABARTI),
                      ("uniform", UNIFORM)):
        g = build_graph(scale, seed, abc)
        ctx = load(g)
        log(f"topology: {name}")
        for sname, edges in shapes:
            n0 = max(max(e) for e in edges) + 1
            try:
                # labels of an occurrence, repeats allowed: a log2-degree
                # labelling of the uniform graph has too few labels for
                # pairwise distinct ones
                t = I.extract_template(g, n0, edges, 11, distinct=False, name=sname)
            except RuntimeError:
                rows.append({"graph": name, "shape": sname, "template": "no occurrence found"})
                continue
            tid = ctx.load_templates([t])
            ctx.prune(tid)
            ms, (r, e, st) = wall(lambda: ctx.prune(tid))
            r = r.clone()
            bits = int(np.unpackbits(e[0].cpu().numpy().view(np.uint8)).sum())
            cms, cnt = wall(lambda: ctx.count_matches(tid, state=r, max_maps=1 << 34))
            rows.append({"graph": name, "abc": abc, "n": g.n, "m": g.m,
                         "d_max": int(np.diff(g.row_ptr).max()),
                         "labels": int(g.labels.max()) + 1, "shape": sname,
                         "template_labels": list(t.labels),
                         "result_vertices": int((r[0] != 0).sum().item()),
                         "result_entries": bits, "maps": cnt["maps"],
                         "count_complete": bool(cnt["complete"]),
                         "matches": cnt["subgraphs"] if cnt["complete"] else None,
                         "prune_ms": round(ms, 2), "count_ms": round(cms, 2),
                         "phases_ms": {k: round(v, 3) for k, v in st.items()
                                       if k.startswith("ms_")}})
        ctx.close()
        del g
    t = I.template_tri_square(g22, 0)
    tid = ctx22.load_templates([t])
    abl = {}
    ref = None
    for name, bits in (("default", 0), ("no_edge_elimination", pm.PM_ABLATE_EDGE_ELIMINATION),
                       ("no_work_aggregation", pm.PM_ABLATE_WORK_AGGREGATION)):
        ctx22.prune(tid, ablate=bits)
        ms, (r, e, st) = wall(lambda: ctx22.prune(tid, ablate=bits))
        if ref is None:
            ref = (r.clone(), e.clone())
        abl[name] = {"ms": round(ms, 2), "ms_lcc": round(st["ms_lcc"], 3),
                     "ms_compact": round(st["ms_compact"], 3), "ms_nlcc": round(st["ms_nlcc"], 3),
                     "ms_exact": round(st["ms_exact"], 3),
                     "candidate_entries": st["candidate_entries"],
                     "edge_queries": st["edge_queries"], "vertex_queries": st["vertex_queries"],
                     "identical": bool(torch.equal(ref[0], r) and torch.equal(ref[1], e))}
    return {"topology": {"workload": f"R-MAT scale {scale} ef16, log2-degree labels",
                         "graphs": rows},
            "ablations": {"workload": f"scale-22 graph, template {t.labels}", **abl}}


if __name__ == "__main__":
    main()
