"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Non-local constraint generation written out from the paper's constraint
generation table (Steps 1-5) and the TDS constraint generation algorithm,
independently of the library's template compiler.  Only tests, the smoke
check and the benchmark's CPU baseline may use it.

Readings of passages the paper leaves open (each is also listed in the design
notes):
  * FIND_CIRCLES: the simple cycles of G'0, canonicalised as the vertex
    sequence that starts at its smallest vertex and whose second vertex is
    smaller than its last; sorted by (length, sequence); at most 32 kept,
    enumerated length by length so only the lengths that contribute are
    explored (a template with more than 100000 cycles of one length is
    refused).
  * FIND_SHORTEST_PATH(G0, qi, qj, 3): breadth-first search over G0 from qi,
    neighbours in ascending index, first discoverer is the parent; the path
    is used only if it has at least 3 hops (Step 4).  Step 4(ii) drops a path
    whose edges all lie in one cycle constraint.
  * TDS_CONSTRAINTS: constraints are merged while some pair qualifies (cycle
    type: a common vertex and a common edge; path type: a common vertex); a
    merged group keeps the position of its first member.  Only groups with at
    least two members are new constraints (a single member repeats an
    existing one).  Path-type unions are replaced by the breadth-first
    spanning tree from their lowest vertex, neighbours in ascending index.
  * Step 5(3), the full-template search, is the exact final step that always
    runs after the ordered list, so it is not part of the list.
  * Heads (token sources): every vertex of a cycle or TDS-cycle constraint,
    both terminals of a path constraint, and the repeated-label vertices of a
    TDS-path constraint (token generation paragraph).
  * Order (ordering heuristics): path and cycle constraints first, by
    (edge count, cycles before paths, generation index), then TDS-cycle, then
    TDS-path constraints, each by (edge count, generation index).
"""
from __future__ import annotations

import dataclasses
from collections import Counter, deque
from typing import List, Sequence, Tuple

MAX_CYCLES = 32

CC, PC, TDS_CC, TDS_PC = 0, 1, 2, 3
KIND_NAMES = {CC: "CC", PC: "PC", TDS_CC: "TDS_CC", TDS_PC: "TDS_PC"}


@dataclasses.dataclass
class Constraint:
    kind: int
    edges: Tuple[Tuple[int, int], ...]   # sorted (a < b)
    heads: int                           # bit mask over V0
    gen_index: int

    @property
    def vertices(self) -> int:
        vm = 0
        for a, b in self.edges:
            vm |= (1 << a) | (1 << b)
        return vm

    def key(self):
        return (self.kind, self.edges, self.heads)


def _adj(n0: int, edges: Sequence[Tuple[int, int]]) -> List[List[int]]:
    adj = [[] for _ in range(n0)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    for x in adj:
        x.sort()
    return adj


def _norm(a, b):
    return (a, b) if a < b else (b, a)


MAX_CYCLES_PER_LENGTH = 100000


def simple_cycles(n0: int, edges: Sequence[Tuple[int, int]], allowed: int) -> List[Tuple[int, ...]]:
    """Simple cycles (length >= 3) of the subgraph induced on `allowed`, by
    increasing length; enumeration stops after the first length at which at
    least MAX_CYCLES cycles have been found (only the first MAX_CYCLES in
    (length, sequence) order are used)."""
    adj = _adj(n0, [e for e in edges if (allowed >> e[0]) & 1 and (allowed >> e[1]) & 1])
    out = []
    for length in range(3, n0 + 1):
        found = []
        for s in range(n0):
            if not (allowed >> s) & 1:
                continue
            path = [s]
            on = {s}

            def dfs(x):
                for y in adj[x]:
                    if len(path) == length:
                        if y == s and path[1] < path[-1]:
                            found.append(tuple(path))
                            if len(found) > MAX_CYCLES_PER_LENGTH:
                                raise ValueError("too many cycles in template")
                    elif y > s and y not in on:
                        path.append(y); on.add(y)
                        dfs(y)
                        path.pop(); on.discard(y)
            dfs(s)
        found.sort()
        out += found
        if len(out) >= MAX_CYCLES:
            break
    return out

def shortest_path(n0: int, edges, src: int, dst: int) -> List[int]:
    adj = _adj(n0, edges)
    parent = [-1] * n0
    seen = [False] * n0
    seen[src] = True
    dq = deque([src])
    while dq:
        x = dq.popleft()
        for y in adj[x]:
            if not seen[y]:
                seen[y] = True
                parent[y] = x
                dq.append(y)
    if not seen[dst]:
        return []
    path = [dst]
    while path[-1] != src:
        path.append(parent[path[-1]])
    return path[::-1]


def _merge(items: List[frozenset], need_edge: bool) -> List[Tuple[frozenset, int]]:
    """TDS_CONSTRAINTS merge loop; returns (edge set, member count) groups in
    the order of their first member."""
    groups = [(set(e), 1) for e in items]
    changed = True
    while changed:
        changed = False
        i = 0
        while i < len(groups):
            j = i + 1
            while j < len(groups):
                ei, ej = groups[i][0], groups[j][0]
                vi = {x for e in ei for x in e}
                vj = {x for e in ej for x in e}
                if vi & vj and ((ei & ej) or not need_edge):
                    groups[i] = (ei | ej, groups[i][1] + groups[j][1])
                    del groups[j]
                    changed = True
                    j = i + 1
                else:
                    j += 1
            i += 1
    return [(frozenset(g), c) for g, c in groups]


def spanning_tree(edges: frozenset) -> Tuple[Tuple[int, int], ...]:
    verts = sorted({x for e in edges for x in e})
    n0 = max(verts) + 1
    adj = _adj(n0, list(edges))
    root = verts[0]
    seen = {root}
    dq = deque([root])
    out = []
    while dq:
        x = dq.popleft()
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                out.append(_norm(x, y))
                dq.append(y)
    return tuple(sorted(out))


def non_local_constraints(labels: Sequence[int], edges: Sequence[Tuple[int, int]]) -> List[Constraint]:
    """Ordered constraint list K0 for template (labels, edges)."""
    n0 = len(labels)
    edges = [_norm(int(a), int(b)) for a, b in edges]
    adj = _adj(n0, edges)
    cnt = Counter(labels)
    # Step 1: leaves with unique labels are left to LCC
    v_u = [q for q in range(n0) if cnt[labels[q]] == 1]
    v_ul = {q for q in v_u if len(adj[q]) == 1}
    allowed = 0
    for q in range(n0):
        if q not in v_ul:
            allowed |= 1 << q
    # Step 2: vertices with repeated labels
    v_d = [q for q in range(n0) if cnt[labels[q]] > 1]
    # Step 3: cycle constraints
    cycles = simple_cycles(n0, edges, allowed)[:MAX_CYCLES]
    cc = []
    for c in cycles:
        es = tuple(sorted(_norm(c[i], c[(i + 1) % len(c)]) for i in range(len(c))))
        m = 0
        for x in c:
            m |= 1 << x
        cc.append(Constraint(CC, es, m, len(cc)))
    # Step 4: path constraints
    pc = []
    for i in range(len(v_d)):
        for j in range(i + 1, len(v_d)):
            qi, qj = v_d[i], v_d[j]
            if labels[qi] != labels[qj]:
                continue
            path = shortest_path(n0, edges, qi, qj)
            if len(path) - 1 < 3:
                continue
            es = tuple(sorted(_norm(path[k], path[k + 1]) for k in range(len(path) - 1)))
            if any(set(es) <= set(c.edges) for c in cc):
                continue
            pc.append(Constraint(PC, es, (1 << qi) | (1 << qj), len(pc)))
    # Step 5(1): unions of cycles that share an edge
    tds_cc = []
    for es, members in _merge([frozenset(c.edges) for c in cc], need_edge=True):
        if members < 2:
            continue
        vm = 0
        for a, b in es:
            vm |= (1 << a) | (1 << b)
        tds_cc.append(Constraint(TDS_CC, tuple(sorted(es)), vm, len(tds_cc)))
    # Step 5(2): unions of paths that share a vertex, reduced to a spanning tree
    tds_pc = []
    dup_mask = 0
    for q in v_d:
        dup_mask |= 1 << q
    for es, members in _merge([frozenset(p.edges) for p in pc], need_edge=False):
        if members < 2:
            continue
        tree = spanning_tree(es)
        vm = 0
        for a, b in tree:
            vm |= (1 << a) | (1 << b)
        tds_pc.append(Constraint(TDS_PC, tree, vm & dup_mask, len(tds_pc)))
    # ordering heuristics
    first = sorted(cc + pc, key=lambda c: (len(c.edges), 0 if c.kind == CC else 1, c.gen_index))
    second = sorted(tds_cc, key=lambda c: (len(c.edges), c.gen_index))
    third = sorted(tds_pc, key=lambda c: (len(c.edges), c.gen_index))
    return first + second + third


def is_acyclic_unique(labels: Sequence[int], edges) -> bool:
    """Acyclic template with pairwise distinct labels: LCC alone is exact."""
    n0 = len(labels)
    return len(set(labels)) == n0 and len(edges) == n0 - 1
