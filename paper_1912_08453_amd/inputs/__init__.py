"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module generates background graphs, vertex labels and search templates.
It holds none of the pruning method's arithmetic: both the HIP path and the
CPU oracle consume what it produces, and neither is imported here.

Graph recipe: the paper's synthetic R-MAT graphs (Graph500 parameters
(0.57, 0.19, 0.19, 0.05), edge factor 16, undirected) with degree-derived
labels ceil(log2(d + 1)) (synthetic-graph setup and the R-MAT degree
sensitivity study), or uniform random labels as used for the paper's
unlabeled graphs (Twitter / UK Web setup).  The paper's real datasets are not
available; these synthetic graphs stand in for them.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmgen.so")
_lib = None

GRAPH500_ABC = (0.57, 0.19, 0.19)
CHAKRABARTI_ABC = (0.45, 0.15, 0.15)
UNIFORM_ABC = (0.25, 0.25, 0.25)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"input generator library missing: {LIB_PATH}; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    lib.pmgen_rmat_build.restype = ctypes.c_void_p
    lib.pmgen_rmat_build.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                     ctypes.c_int]
    lib.pmgen_graph_n.restype = ctypes.c_int64
    lib.pmgen_graph_n.argtypes = [ctypes.c_void_p]
    lib.pmgen_graph_m.restype = ctypes.c_int64
    lib.pmgen_graph_m.argtypes = [ctypes.c_void_p]
    lib.pmgen_graph_export.restype = None
    lib.pmgen_graph_export.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.pmgen_graph_free.restype = None
    lib.pmgen_graph_free.argtypes = [ctypes.c_void_p]
    lib.pmgen_labels_uniform.restype = None
    lib.pmgen_labels_uniform.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_uint64,
                                         ctypes.c_void_p]
    lib.pmgen_labels_log2deg.restype = None
    lib.pmgen_labels_log2deg.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    lib.pmgen_philox4x32_10.restype = None
    lib.pmgen_philox4x32_10.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.pmgen_perm.restype = ctypes.c_uint64
    lib.pmgen_perm.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> Tuple[int, int, int, int]:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().pmgen_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return tuple(int(x) for x in out)


def _thr(x: float) -> int:
    return max(0, min(int(round(x * 2.0 ** 32)), 2 ** 32 - 1))


@dataclasses.dataclass
class Graph:
    """Symmetric CSR: row_ptr int64[n+1], col int32[m] (sorted rows, no loops,
    no duplicate entries), labels uint8/uint16[n]."""
    row_ptr: np.ndarray
    col: np.ndarray
    labels: np.ndarray
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def rmat_csr(scale: int, edge_factor: int = 16, abc=GRAPH500_ABC, seed: int = 1,
             permute: bool = True) -> Tuple[np.ndarray, np.ndarray]:
    """R-MAT graph with 2^scale vertices and edge_factor * 2^scale samples,
    symmetrised, self-loops and duplicates dropped, rows sorted."""
    lib = _load()
    a, b, c = abc
    nsamples = edge_factor * (1 << scale)
    h = lib.pmgen_rmat_build(scale, nsamples, _thr(a), _thr(a + b), _thr(a + b + c),
                             seed & 0xFFFFFFFFFFFFFFFF, 1 if permute else 0)
    if not h:
        raise MemoryError("R-MAT build failed")
    try:
        n = lib.pmgen_graph_n(h)
        m = lib.pmgen_graph_m(h)
        row_ptr = np.empty(n + 1, dtype=np.int64)
        col = np.empty(max(m, 1), dtype=np.int32)[:m]
        lib.pmgen_graph_export(h, _ptr(row_ptr), _ptr(col) if m else None)
    finally:
        lib.pmgen_graph_free(h)
    return row_ptr, col


def labels_uniform(n: int, nlabels: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint8)
    _load().pmgen_labels_uniform(n, nlabels, seed & 0xFFFFFFFFFFFFFFFF, _ptr(out))
    return out


def labels_log2deg(row_ptr: np.ndarray) -> np.ndarray:
    n = row_ptr.shape[0] - 1
    out = np.empty(n, dtype=np.uint8)
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    _load().pmgen_labels_log2deg(n, _ptr(rp), _ptr(out))
    return out


def csr_from_edges(n: int, edges: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Symmetric sorted CSR from an undirected edge list (pairs), dropping
    loops and duplicates.  For small hand-built and random test graphs."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    e = e[e[:, 0] != e[:, 1]]
    both = np.concatenate([e, e[:, ::-1]], axis=0)
    if both.shape[0]:
        key = np.unique(both[:, 0] * n + both[:, 1])
        src, dst = key // n, key % n
    else:
        src = dst = np.zeros(0, dtype=np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr.astype(np.int64), dst.astype(np.int32)


def random_graph(n: int, p: float, nlabels: int, seed: int) -> Graph:
    """Erdos-Renyi G(n, p) with uniform labels, for tiny exhaustive tests."""
    rng = np.random.Generator(np.random.Philox(seed))
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.shape[0]) < p
    row_ptr, col = csr_from_edges(n, np.stack([iu[keep], ju[keep]], axis=1))
    labels = rng.integers(0, nlabels, size=n).astype(np.uint8)
    return Graph(row_ptr, col, labels, name=f"gnp{n}_{p}_{seed}")


# --------------------------------------------------------------------------
# templates
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Template:
    """Search template G0: labels[q] for q in 0..n0-1, undirected edges.
    The vertex order defines the bit order of the role masks."""
    labels: List[int]
    edges: List[Tuple[int, int]]
    name: str = ""

    @property
    def n0(self) -> int:
        return len(self.labels)

    @property
    def m0(self) -> int:
        return len(self.edges)

    def adjacency(self) -> List[set]:
        adj = [set() for _ in range(self.n0)]
        for a, b in self.edges:
            adj[a].add(b)
            adj[b].add(a)
        return adj


def template_square_pendant() -> Template:
    """4-cycle q0(0)-q1(1)-q2(2)-q3(3)-q0 plus a pendant q4(4) on q0."""
    return Template([0, 1, 2, 3, 4], [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4)], "sq+pendant")


def _feasible_labels(label_hist: np.ndarray, tdeg: int) -> np.ndarray:
    """Labels whose log2-degree class admits template degree tdeg:
    a vertex of label L has degree at most 2^L - 1."""
    labs = np.arange(label_hist.shape[0])
    ok = (label_hist > 0) & (labs >= 1) & ((2 ** labs.astype(np.float64) - 1) >= tdeg)
    return labs[ok]


def draw_labels(rng: np.random.Generator, tdegs: Sequence[int], label_hist: np.ndarray,
                repeat_pairs: Sequence[Tuple[int, int]] = (), distinct: bool = True) -> List[int]:
    """Draw template labels weighted by background label frequency among
    degree-feasible labels; vertices in repeat_pairs share a label."""
    n0 = len(tdegs)
    group = list(range(n0))
    for a, b in repeat_pairs:
        group[b] = group[a]
    labels = [-1] * n0
    used = set()
    for q in range(n0):
        if group[q] != q:
            continue
        members = [x for x in range(n0) if group[x] == q]
        need = max(tdegs[x] for x in members)
        cand = _feasible_labels(label_hist, need)
        if distinct:
            cand = np.array([c for c in cand if c not in used], dtype=np.int64)
        if cand.shape[0] == 0:
            cand = _feasible_labels(label_hist, need)
        w = label_hist[cand].astype(np.float64)
        lab = int(rng.choice(cand, p=w / w.sum()))
        used.add(lab)
        for x in members:
            labels[x] = lab
    return labels


def _degrees(n0: int, edges) -> List[int]:
    d = [0] * n0
    for a, b in edges:
        d[a] += 1
        d[b] += 1
    return d


TRI_SQUARE_EDGES = [(0, 1), (1, 2), (0, 2), (1, 3), (3, 4), (4, 0), (3, 5)]


def template_tri_square(graph: "Graph", seed: int) -> Template:
    """Triangle (q0,q1,q2) and 4-cycle (q0,q1,q3,q4) sharing edge q0-q1, a
    pendant q5 on q3, and the repeated label l(q5) = l(q2); the labels are
    those of an occurrence of this shape found from a seeded random start
    vertex, so the template has at least one match."""
    return extract_template(graph, 6, TRI_SQUARE_EDGES, seed, repeat_pairs=[(2, 5)],
                            name=f"tri+sq+pendant/s{seed}")


def frequent_labels(labels: np.ndarray, frac: float = 0.01) -> List[int]:
    """Labels carried by at least `frac` of the non-isolated vertices (label 0
    is the isolated class of degree labels).  The paper's R-MAT templates use
    labels among the most frequent in the graph."""
    h = label_histogram(labels)
    nz = int(h[1:].sum())
    return [L for L in range(1, h.shape[0]) if h[L] >= frac * nz]


def extract_template(graph: "Graph", n0: int, edges, seed: int, repeat_pairs=(),
                     allowed_labels=None, name: str = "", max_attempts: int = 20000,
                     fanout: int = 24, budget: int = 4000, distinct: bool = True) -> Template:
    """Labels for a template shape taken from one occurrence of the shape in
    the background graph (query generation by seeded random search, as is
    usual for subgraph-matching workloads).  Vertices in repeat_pairs share a
    label; all other template vertices get pairwise distinct labels.

    The search proposes, from a random start vertex, images for the shape's
    vertices in breadth-first order, each among a random sample of at most
    `fanout` neighbours of its parent's image, checking injectivity, the
    shape's other edges and the label pattern; it gives up on a start after
    `budget` proposals.  If allowed_labels is given, only vertices with those
    labels are used.  With distinct=False the labels are whatever the
    occurrence carries (repeats allowed anywhere)."""
    rng = np.random.Generator(np.random.Philox(seed))
    rp, col, lab = graph.row_ptr, graph.col, graph.labels
    ok_lab = np.ones(int(lab.max()) + 1 if lab.size else 1, dtype=bool)
    if allowed_labels is not None:
        ok_lab[:] = False
        ok_lab[list(allowed_labels)] = True
    adj = [[] for _ in range(n0)]
    for a, b in edges:
        adj[a].append(b); adj[b].append(a)
    tdeg = [len(x) for x in adj]
    order, parent = [0], {0: -1}
    for x in order:
        for y in sorted(adj[x]):
            if y not in parent:
                parent[y] = x; order.append(y)
    pos = {q: i for i, q in enumerate(order)}
    same = {}
    for a, b in repeat_pairs:
        same.setdefault(a, set()).add(b); same.setdefault(b, set()).add(a)
    deg = np.diff(rp)
    starts = np.nonzero((deg >= tdeg[0]) & ok_lab[lab])[0]
    if starts.shape[0] == 0:
        raise ValueError("no start vertex of sufficient degree")

    def has_edge(u, w):
        row = col[rp[u]:rp[u + 1]]
        i = np.searchsorted(row, w)
        return i < row.shape[0] and row[i] == w

    for _ in range(max_attempts):
        img = {0: int(starts[rng.integers(0, starts.shape[0])])}
        work = [0]

        def extend(i):
            if i == n0:
                return True
            q = order[i]
            p = img[parent[q]]
            row = col[rp[p]:rp[p + 1]]
            if row.shape[0] > fanout:
                row = row[rng.choice(row.shape[0], size=fanout, replace=False)]
            else:
                row = row[rng.permutation(row.shape[0])]
            used = set(img.values())
            for x in row.tolist():
                work[0] += 1
                if work[0] > budget:
                    return False
                if x in used or deg[x] < tdeg[q] or not ok_lab[lab[x]]:
                    continue
                ok = True
                for r, v in img.items():
                    if r in adj[q] and r != parent[q] and not has_edge(x, v):
                        ok = False; break
                    eq = lab[x] == lab[v]
                    if distinct and (r in same.get(q, ())) != eq:
                        ok = False; break
                if not ok:
                    continue
                img[q] = x
                if extend(i + 1):
                    return True
                del img[q]
            return False

        if extend(1):
            labels = [int(lab[img[q]]) for q in range(n0)]
            return Template(labels, [tuple(e) for e in edges], name)
    raise RuntimeError("no occurrence found for template shape")


def _prufer_tree(rng, n0):
    if n0 == 1:
        return []
    if n0 == 2:
        return [(0, 1)]
    seq = list(rng.integers(0, n0, size=n0 - 2))
    deg = [1] * n0
    for x in seq:
        deg[x] += 1
    edges = []
    for x in seq:
        leaf = min(i for i in range(n0) if deg[i] == 1)
        edges.append((leaf, int(x)))
        deg[leaf] -= 1
        deg[x] -= 1
    u, w = [i for i in range(n0) if deg[i] == 1]
    edges.append((u, w))
    return edges


def _attach_tree(rng, base_n: int, edges: list, n0: int) -> list:
    """Attach vertices base_n..n0-1 one at a time to a random earlier vertex."""
    edges = list(edges)
    for v in range(base_n, n0):
        edges.append((int(rng.integers(0, v)), v))
    return edges


def _norm_edges(edges):
    out = set()
    for a, b in edges:
        a, b = int(a), int(b)
        if a != b:
            out.add((min(a, b), max(a, b)))
    return sorted(out)


def shape_tree(rng, n0):
    return _norm_edges(_prufer_tree(rng, n0))


def shape_one_cycle(rng, n0):
    k = int(rng.integers(3, n0 + 1))
    cyc = [(i, (i + 1) % k) for i in range(k)]
    return _norm_edges(_attach_tree(rng, k, cyc, n0))


def shape_two_cycles(rng, n0):
    """Two cycles sharing a vertex or an edge, then tree vertices."""
    share_edge = bool(rng.integers(0, 2)) and n0 >= 4
    if share_edge:
        # theta graph: two paths of lengths p1, p2 >= 2 between vertices 0 and 1
        # plus the chord 0-1
        room = n0 - 2
        p1 = int(rng.integers(1, max(1, room) + 1)) if room >= 2 else 1
        p1 = min(p1, room - 1) if room >= 2 else 1
        p2 = int(rng.integers(1, room - p1 + 1)) if room - p1 >= 1 else 0
        edges = [(0, 1)]
        nxt = 2
        prev = 0
        for _ in range(p1):
            edges.append((prev, nxt)); prev = nxt; nxt += 1
        edges.append((prev, 1))
        if p2 >= 1:
            prev = 0
            for _ in range(p2):
                edges.append((prev, nxt)); prev = nxt; nxt += 1
            edges.append((prev, 1))
        else:
            return shape_one_cycle(rng, n0)
        return _norm_edges(_attach_tree(rng, nxt, edges, n0))
    # bowtie-like: two cycles through vertex 0
    if n0 < 5:
        return shape_one_cycle(rng, n0)
    k1 = int(rng.integers(3, n0 - 1))
    k1 = min(k1, n0 - 2)
    k2 = int(rng.integers(3, n0 - k1 + 2))
    edges = [(i, (i + 1) % k1) for i in range(k1)]
    ring = [0] + list(range(k1, k1 + k2 - 1))
    for i in range(len(ring)):
        edges.append((ring[i], ring[(i + 1) % len(ring)]))
    return _norm_edges(_attach_tree(rng, k1 + k2 - 1, edges, n0))


def shape_k4(rng, n0):
    edges = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    return _norm_edges(_attach_tree(rng, 4, edges, n0))


def _repeat_pair(rng, n0, edges, min_hops=1):
    """Pick a vertex pair at least min_hops apart to share a label."""
    import itertools
    dist = _all_pairs_hops(n0, edges)
    pairs = [(a, b) for a, b in itertools.combinations(range(n0), 2) if dist[a][b] >= min_hops]
    if not pairs:
        return []
    a, b = pairs[int(rng.integers(0, len(pairs)))]
    return [(a, b)]


def _all_pairs_hops(n0, edges):
    adj = [[] for _ in range(n0)]
    for a, b in edges:
        adj[a].append(b); adj[b].append(a)
    inf = 1 << 30
    dist = [[inf] * n0 for _ in range(n0)]
    for s in range(n0):
        dist[s][s] = 0
        frontier = [s]
        while frontier:
            nxt = []
            for x in frontier:
                for y in adj[x]:
                    if dist[s][y] == inf:
                        dist[s][y] = dist[s][x] + 1
                        nxt.append(y)
            frontier = nxt
    return dist


def templates_batch(graph: "Graph", seed: int, count: int = 64) -> List[Template]:
    """Mixed batch: 1/4 paths/trees, 3/8 one cycle, 1/4 two cycles, 1/8
    4-cliques (16/24/16/8 of 64), 3..8 vertices, ~20% with one repeated-label
    pair (at least 2 hops apart); labels from an occurrence in the graph."""
    rng = np.random.Generator(np.random.Philox(seed))
    kinds = (["tree"] * (count // 4) + ["one"] * (3 * count // 8) + ["two"] * (count // 4))
    kinds += ["k4"] * (count - len(kinds))
    n_rep = int(round(0.2 * count))
    rep_idx = set(int(x) for x in rng.choice(count, size=n_rep, replace=False))
    out = []
    for i, kind in enumerate(kinds):
        for attempt in range(50):
            if kind == "tree":
                n0 = int(rng.integers(3, 9)); edges = shape_tree(rng, n0)
            elif kind == "one":
                n0 = int(rng.integers(3, 9)); edges = shape_one_cycle(rng, n0)
            elif kind == "two":
                n0 = int(rng.integers(5, 9)); edges = shape_two_cycles(rng, n0)
            else:
                n0 = int(rng.integers(4, 9)); edges = shape_k4(rng, n0)
            rep = _repeat_pair(rng, n0, edges, 2) if i in rep_idx else []
            try:
                t = extract_template(graph, n0, edges, int(rng.integers(0, 2 ** 62)),
                                     repeat_pairs=rep, name=f"{kind}{n0}/{i}",
                                     max_attempts=400)
            except RuntimeError:
                continue
            out.append(t)
            break
        else:
            raise RuntimeError(f"could not draw template {i} ({kind})")
    return out


def templates_multicycle(graph: "Graph", seed: int, count: int = 64) -> List[Template]:
    """7-8 vertex templates with cyclomatic number >= 2, labels from an
    occurrence in the graph; about 30% carry one repeated-label pair."""
    rng = np.random.Generator(np.random.Philox(seed))
    out = []
    while len(out) < count:
        n0 = int(rng.integers(7, 9))
        edges = shape_two_cycles(rng, n0)
        if rng.random() < 0.5:
            a, b = (int(x) for x in rng.choice(n0, size=2, replace=False))
            edges = _norm_edges(edges + [(a, b)])
        if len(edges) - n0 + 1 < 2:
            continue
        rep = _repeat_pair(rng, n0, edges, 2) if rng.random() < 0.3 else []
        try:
            t = extract_template(graph, n0, edges, int(rng.integers(0, 2 ** 62)),
                                 repeat_pairs=rep, name=f"mc{n0}/{len(out)}",
                                 max_attempts=400)
        except RuntimeError:
            continue
        out.append(t)
    return out


def label_histogram(labels: np.ndarray) -> np.ndarray:
    return np.bincount(labels.astype(np.int64), minlength=int(labels.max()) + 1 if labels.size else 1)


def model_params(seed: int, n_params: int = 5122, fan_ins=((768, 12), (64, 0), (4096, 64),
                                                            (64, 0), (128, 64), (2, 0))):
    """Seeded initial parameters of the ordering model, packed block by block
    (weights uniform in +-sqrt(6 / fan_in), biases 0.01), float32."""
    rng = np.random.Generator(np.random.Philox(seed))
    parts = []
    for size, fan_in in fan_ins:
        if fan_in:
            b = float(np.sqrt(6.0 / fan_in))
            parts.append(rng.uniform(-b, b, size))
        else:
            parts.append(np.full(size, 0.01))
    w = np.concatenate(parts).astype(np.float32)
    assert w.shape[0] == n_params
    return w


# Large exploratory workload: an 8-vertex theta graph (edge q0-q1, path
# q1-q2-q3-q4-q0 of length 4, path q1-q5-q6-q0 of length 3; cyclomatic number
# 2) with a pendant q7 on q6, and one repeated label on q3 and q7, which are
# 4 hops apart (q7-q6-q0-q4-q3), so the constraint list holds a path
# constraint of length 4.
THETA8_EDGES = [(0, 1), (1, 2), (2, 3), (3, 4), (0, 4), (1, 5), (5, 6), (0, 6), (6, 7)]
THETA8_REPEAT = (3, 7)


def template_theta8(graph: "Graph", seed: int) -> Template:
    """The 8-vertex two-cycle base template with labels from an occurrence
    in the graph (so it has at least one match)."""
    return extract_template(graph, 8, THETA8_EDGES, seed, repeat_pairs=[THETA8_REPEAT],
                            name=f"theta8+pendant/s{seed}")


def _connected(n0: int, edges) -> bool:
    adj = [[] for _ in range(n0)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    seen, stack = {0}, [0]
    while stack:
        x = stack.pop()
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                stack.append(y)
    return len(seen) == n0


def _canonical(labels, edges):
    """Smallest sorted edge list over the label-preserving relabellings of
    the vertices (vertices ordered by label, ties permuted)."""
    import itertools
    n0 = len(labels)
    groups = {}
    for q in range(n0):
        groups.setdefault(labels[q], []).append(q)
    keys = sorted(groups)
    slots = []
    for L in keys:
        slots += [L] * len(groups[L])
    best = None
    for choice in itertools.product(*[itertools.permutations(groups[L]) for L in keys]):
        order = [q for grp in choice for q in grp]
        pos = {q: i for i, q in enumerate(order)}
        es = tuple(sorted(tuple(sorted((pos[a], pos[b]))) for a, b in edges))
        if best is None or es < best:
            best = es
    return tuple(slots), best


def relaxations(t: Template, max_deletions: int = 2) -> List[Template]:
    """The template and every variant with 1..max_deletions edges deleted
    that still spans all template vertices connectedly, deduplicated up to
    label-preserving isomorphism; base first, then by deletion count and
    deleted-edge indices."""
    import itertools
    out = [t]
    seen = {_canonical(t.labels, t.edges)}
    m0 = len(t.edges)
    for d in range(1, max_deletions + 1):
        for dels in itertools.combinations(range(m0), d):
            es = [e for i, e in enumerate(t.edges) if i not in dels]
            if not _connected(len(t.labels), es):
                continue
            key = _canonical(t.labels, es)
            if key in seen:
                continue
            seen.add(key)
            out.append(Template(list(t.labels), es,
                                f"{t.name}-del{'.'.join(str(i) for i in dels)}"))
    return out
