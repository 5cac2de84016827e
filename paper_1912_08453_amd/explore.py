"""Exploratory search: progressive relaxation of an over-constrained template.

The paper's exploratory usage scenario starts from a template that may have
no match and relaxes it level by level: level k holds every variant with k
template edges removed, and the levels are searched in order until one of
them has a variant with a match; the answer is the union of all matches at
that level.  Here a variant keeps all template vertices and must stay
connected (as in the incremental scenario), variants that are the same up
to a label-preserving relabelling are searched once (they have the same
matches as vertex and edge sets), and each level is pruned by batched
pm_prune calls on the resident graph.

Candidate set (the key enabler the paper names for this scenario): before
level 0 the base template is pruned in PM_MODE_CANDIDATE -- local checks
only, with the rule relaxed so that the result holds the complete set of
every connected variant obtained by deleting edges -- and every variant of
every level then starts from that set (one shared init_state) instead of
from the label roles of the whole graph.  The library ORs the complete sets
of a level into its union buffers (a vertex is in the union iff it holds a
role in some variant's complete set; its bits are the roles it holds in the
class representatives searched, not in every isomorphic copy).

    from paper_1912_08453_amd import explore
    res = explore.explore(ctx, labels, edges, max_deletions=3)

Non-local constraint results are not carried from one variant to the next:
each variant's checks run against its own state, which is sound only for
that variant.
"""
from __future__ import annotations

import itertools
import time
from collections import namedtuple
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple


_Variant = namedtuple("_Variant", "labels edges")


def _spans_connected(n0: int, edges: Sequence[Tuple[int, int]]) -> bool:
    """Do the edges connect all n0 template vertices?"""
    parent = list(range(n0))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    parts = n0
    for a, b in edges:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
            parts -= 1
    return parts == 1


def _pair_index(n0: int):
    idx = {}
    for a in range(n0):
        for b in range(a + 1, n0):
            idx[(a, b)] = len(idx)
    return idx


def _class_key(labels: Sequence[int], edges: Sequence[Tuple[int, int]], perms, pidx) -> int:
    """Smallest edge bitmask (bit = unordered vertex pair) over the given
    label-preserving vertex permutations: equal keys <=> isomorphic."""
    best = None
    for p in perms:
        m = 0
        for a, b in edges:
            x, y = p[a], p[b]
            m |= 1 << pidx[(x, y) if x < y else (y, x)]
        if best is None or m < best:
            best = m
    return best


def _label_perms(labels: Sequence[int]):
    n0 = len(labels)
    classes = {}
    for q in range(n0):
        classes.setdefault(labels[q], []).append(q)
    groups = list(classes.values())
    perms = []
    for images in itertools.product(*[itertools.permutations(g) for g in groups]):
        p = [0] * n0
        for g, img in zip(groups, images):
            for q, r in zip(g, img):
                p[q] = r
        perms.append(p)
    return perms


def variants(labels: Sequence[int], edges: Sequence[Tuple[int, int]], k: int
             ) -> List[List[Tuple[int, int]]]:
    """Edge lists of the level-k variants: k edges removed, all template
    vertices still connected, one per label-preserving isomorphism class
    (the first in order of the removed edges' indices)."""
    n0 = len(labels)
    edges = [tuple(sorted(e)) for e in edges]
    perms = _label_perms(labels)
    pidx = _pair_index(n0)
    seen = set()
    out = []
    for removed in itertools.combinations(range(len(edges)), k):
        drop = set(removed)
        es = [e for i, e in enumerate(edges) if i not in drop]
        if not _spans_connected(n0, es):
            continue
        key = _class_key(labels, es, perms, pidx)
        if key in seen:
            continue
        seen.add(key)
        out.append(es)
    return out


@dataclass
class ExploreResult:
    level: int                       # first level with a match, -1 if none
    variants: List[List[Tuple[int, int]]] = field(default_factory=list)
    matched: List[bool] = field(default_factory=list)
    # int64 tensor [n]: OR of the role masks of the matched variants, one
    # representative per label-preserving isomorphism class; its bits are
    # that representative's template vertices, so read it as an indicator of
    # the vertices in some match (nonzero) rather than per role
    role_union: object = None
    edge_union: object = None        # int64 tensor [ceil(m/64)]: OR of the edge bits
    levels: List[dict] = field(default_factory=list)   # per level: variants, matched, ms


def explore(ctx, labels: Sequence[int], edges: Sequence[Tuple[int, int]],
            max_deletions: Optional[int] = None, batch: int = 32, batch_streams: int = 4,
            use_candidate_set: bool = True, log=None) -> ExploreResult:
    """Search levels 0, 1, ... (at most max_deletions, default: as long as
    variants remain) until a level has a variant with a match; see the
    module docstring."""
    import torch
    from . import pm as _pm
    labels = [int(x) for x in labels]
    edges = [tuple(int(v) for v in e) for e in edges]
    top = len(edges) if max_deletions is None else min(max_deletions, len(edges))
    dev = ctx.device
    n, words = ctx.n, (ctx.m + 63) // 64
    res = ExploreResult(level=-1)
    cand = None
    if use_candidate_set:
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        base = ctx.load_templates([_Variant(labels, edges)])
        role, _, _ = ctx.prune(base, mode=_pm.PM_MODE_CANDIDATE)
        cand = role[0].contiguous()
        torch.cuda.synchronize(dev)
        ms = 1e3 * (time.perf_counter() - t0)
        res.levels.append({"level": "candidate set", "ms": round(ms, 2)})
        if log:
            log(f"candidate set: {ms:.1f} ms")
    for k in range(top + 1):
        vs = variants(labels, edges, k)
        if not vs:
            break
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        matched: List[bool] = []
        r_un = torch.zeros(n, dtype=torch.int64, device=dev)
        e_un = torch.zeros(words, dtype=torch.int64, device=dev)
        for s in range(0, len(vs), batch):
            chunk = vs[s:s + batch]
            first = ctx.load_templates([_Variant(labels, es) for es in chunk])
            _, _, st = ctx.prune(first, count=len(chunk), batch_streams=batch_streams,
                                 init_state=cand, shared_inputs=True, union_roles=r_un,
                                 union_edges=e_un, per_template=True)
            matched += [p["result_vertices"] > 0 for p in st["per_template"]]
        torch.cuda.synchronize(dev)
        ms = 1e3 * (time.perf_counter() - t0)
        res.levels.append({"level": k, "variants": len(vs), "matched": int(sum(matched)),
                           "ms": round(ms, 2)})
        if log:
            log(f"level {k}: {len(vs)} variants, {sum(matched)} with matches, {ms:.1f} ms")
        if any(matched):
            res.level, res.variants, res.matched = k, vs, matched
            res.role_union, res.edge_union = r_un, e_un
            return res
    return res
