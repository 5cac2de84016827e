"""Interactive incremental search (the paper's usage scenario of that name).

The user starts from a template, looks at its complete set, and edits the
template by adding or deleting edges (vertices stay, the template stays
connected).  Two facts let each revision reuse earlier work, with the
result still exactly the revised template's complete set:

  * adding an edge only adds a constraint: the complete set of the revised
    template lies inside the current one, so the revision is pruned
    starting from the current complete set (init_state);
  * deleting an edge only drops a constraint: the current complete set lies
    inside the revised one (every match survives the deletion), so its
    roles and edges are certified in advance (known_roles, known_edges) and
    the final search runs only for the rest; the revision starts from the
    candidate set of the current template -- local checks with the rule
    that every connected edge-deleted variant satisfies -- which holds the
    revised complete set.

    s = Session(ctx, labels, edges)
    s.add_edge(a, b); s.delete_edge(c, d)      # each returns a record

Every step's naive counterpart (a full prune of the revised template from
the label roles) can be timed beside it with compare=True; the outputs must
be identical.
"""
from __future__ import annotations

import time
from collections import namedtuple
from typing import List, Sequence, Tuple

from . import pm as _pm

_T = namedtuple("_T", "labels edges")


def _connected(n0: int, edges) -> bool:
    adj = [[] for _ in range(n0)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    seen = {0}
    stack = [0]
    while stack:
        x = stack.pop()
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                stack.append(y)
    return len(seen) == n0


class Session:
    """Incremental search on one context's resident graph."""

    def __init__(self, ctx, labels: Sequence[int], edges: Sequence[Tuple[int, int]],
                 compare: bool = False):
        self.ctx = ctx
        self.labels = [int(x) for x in labels]
        self.edges = sorted(tuple(sorted((int(a), int(b)))) for a, b in edges)
        self.compare = compare
        self.history: List[dict] = []
        self.role = self.edge = self.cand = None
        t0 = self._now()
        tid = self._load(self.edges)
        role, edge, st = ctx.prune(tid)
        self.role, self.edge = role[0].clone(), edge[0].clone()
        ms = self._now() - t0
        self.history.append({"op": "start", "edges": len(self.edges), "ms": round(ms, 3),
                             "result_vertices": st["result_vertices"]})

    def _now(self):
        self.ctx.torch.cuda.synchronize(self.ctx.device)
        return 1e3 * time.perf_counter()

    def _load(self, edges):
        return self.ctx.load_templates([_T(self.labels, list(edges))])

    def _candidate(self):
        """Candidate set of the current template (computed when first needed
        after a change)."""
        if self.cand is None:
            tid = self._load(self.edges)
            r, _, _ = self.ctx.prune(tid, mode=_pm.PM_MODE_CANDIDATE)
            self.cand = r[0].clone()
        return self.cand

    def _naive(self, tid, rec, role, edge):
        t0 = self._now()
        r, e, _ = self.ctx.prune(tid)
        rec["naive_ms"] = round(self._now() - t0, 3)
        rec["identical"] = bool(self.ctx.torch.equal(r[0], role[0]) and
                                self.ctx.torch.equal(e[0], edge[0]))

    def add_edge(self, a: int, b: int) -> dict:
        e = tuple(sorted((int(a), int(b))))
        if e in self.edges or e[0] == e[1] or e[1] >= len(self.labels):
            raise ValueError(f"cannot add edge {e}")
        new = sorted(self.edges + [e])
        tid = self._load(new)
        t0 = self._now()
        role, edge, st = self.ctx.prune(tid, init_state=self.role)
        rec = {"op": "add", "edge": e, "edges": len(new), "ms": round(self._now() - t0, 3),
               "result_vertices": st["result_vertices"]}
        if self.compare:
            self._naive(tid, rec, role, edge)
        self.edges, self.role, self.edge, self.cand = new, role[0].clone(), edge[0].clone(), None
        self.history.append(rec)
        return rec

    def delete_edge(self, a: int, b: int) -> dict:
        e = tuple(sorted((int(a), int(b))))
        if e not in self.edges:
            raise ValueError(f"edge {e} not in the template")
        new = [x for x in self.edges if x != e]
        if not _connected(len(self.labels), new):
            raise ValueError(f"deleting {e} disconnects the template")
        t0 = self._now()
        cand = self._candidate()
        t_cand = self._now() - t0
        tid = self._load(new)
        t0 = self._now()
        role, edge, st = self.ctx.prune(tid, init_state=cand, known_roles=self.role,
                                        known_edges=self.edge)
        rec = {"op": "delete", "edge": e, "edges": len(new), "ms": round(self._now() - t0, 3),
               "candidate_ms": round(t_cand, 3), "result_vertices": st["result_vertices"]}
        if self.compare:
            self._naive(tid, rec, role, edge)
        # the candidate set of the current template also holds the complete
        # set of every later deletion from it: keep it
        self.edges, self.role, self.edge = new, role[0].clone(), edge[0].clone()
        self.history.append(rec)
        return rec
