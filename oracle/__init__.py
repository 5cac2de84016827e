"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Plain CPU reference for the constraint-checking pruner.  Only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import this package;
the library never does, and the two share no code.

`prune` runs the paper's main constraint-checking loop (generate the
non-local constraints, initialise vertex state, LCC to a fixpoint, then for
each constraint NLCC followed by LCC when anything changed) and finishes with
the full-template search that makes the result exact.  `bruteforce` computes
the plain definition of the output (union of all exact matches,
Definition 1) by enumeration, and pins `prune` on small inputs;
`enumerate_maps` lists those matches (counting and enumeration on the
reduced graph).  `candidate_set` is the local-only superset of the complete
sets of every edge-deleted variant of a template (interactive incremental
search).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
import time
from typing import List, Optional, Sequence

import numpy as np

from . import constraints as _cons

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle's C library with gcc (OpenMP)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-Wno-unused-function", src, "-o", tmp])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I64, I32 = ctypes.c_int64, ctypes.c_int
    lib.orc_init_roles.restype = I32
    lib.orc_init_roles.argtypes = [I64, P, I32, I32, P, P, P]
    lib.orc_lcc.restype = I64
    lib.orc_lcc.argtypes = [I64, P, P, P, I32, I32, P, P, P, I64]
    lib.orc_embed_exists.restype = I32
    lib.orc_embed_exists.argtypes = [I64, P, P, P, I32, P, I32, ctypes.c_int32, I32,
                                     ctypes.c_int32]
    lib.orc_nlcc.restype = I64
    lib.orc_nlcc.argtypes = [I64, P, P, P, I32, P, ctypes.c_uint64]
    lib.orc_exact.restype = I32
    lib.orc_exact.argtypes = [I64, P, P, P, I32, I32, P, P, P, P]
    lib.orc_bruteforce.restype = I64
    lib.orc_bruteforce.argtypes = [I64, P, P, P, I32, I32, P, P, P, P]
    lib.orc_active_edges.restype = I32
    lib.orc_active_edges.argtypes = [I64, P, P, P, I32, I32, P, P, P]
    lib.orc_exact_subset.restype = I64
    lib.orc_exact_subset.argtypes = [I64, P, P, P, I32, I32, P, P, P, I64]
    lib.orc_exact_sample.restype = I64
    lib.orc_exact_sample.argtypes = [I64, P, P, P, I32, I32, P, P, P, I64, P, P, P]
    lib.orc_enumerate.restype = I64
    lib.orc_enumerate.argtypes = [I64, P, P, P, I32, I32, P, P, P, I64]
    lib.orc_lcc_sample.restype = I64
    lib.orc_lcc_sample.argtypes = [I64, P, P, P, I32, I32, P, P, P, P, I64, P]
    lib.orc_num_threads.restype = I32
    lib.orc_set_threads.restype = None
    lib.orc_set_threads.argtypes = [I32]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(t: int) -> None:
    _load().orc_set_threads(int(t))


class _G:
    """Contiguous views of a graph in the oracle's argument types."""

    def __init__(self, row_ptr, col, labels):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.labels = np.ascontiguousarray(labels, dtype=np.int32)
        self.n = self.row_ptr.shape[0] - 1
        self.m = int(self.row_ptr[-1])
        if self.col.shape[0] == 0:
            self.col = np.zeros(1, dtype=np.int32)


class _T:
    def __init__(self, labels, edges):
        self.labels = np.ascontiguousarray(labels, dtype=np.int32)
        e = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
        self.edges = np.ascontiguousarray(e if e.size else np.zeros((1, 2), np.int32))
        self.n0 = len(labels)
        self.m0 = int(e.shape[0])
        self.edge_list = [(int(a), int(b)) for a, b in e]
        self.label_list = [int(x) for x in labels]


def nwords(m: int) -> int:
    return (m + 63) // 64


def init_roles(g: _G, t: _T) -> np.ndarray:
    om = np.zeros(max(g.n, 1), dtype=np.uint64)
    rc = _load().orc_init_roles(g.n, _p(g.labels), t.n0, t.m0, _p(t.labels), _p(t.edges), _p(om))
    if rc:
        raise ValueError("bad template")
    return om[:g.n]


def lcc(g: _G, t: _T, omega: np.ndarray, max_sweeps: int = -1) -> int:
    sweeps = _load().orc_lcc(g.n, _p(g.row_ptr), _p(g.col), _p(g.labels), t.n0, t.m0,
                             _p(t.labels), _p(t.edges), _p(omega), max_sweeps)
    if sweeps < 0:
        raise ValueError("bad template")
    return int(sweeps)


def nlcc(g: _G, omega: np.ndarray, c: _cons.Constraint) -> int:
    se = np.ascontiguousarray(np.asarray(c.edges, dtype=np.int32).reshape(-1, 2))
    ch = _load().orc_nlcc(g.n, _p(g.row_ptr), _p(g.col), _p(omega), se.shape[0], _p(se),
                          ctypes.c_uint64(c.heads))
    if ch < 0:
        raise ValueError("bad constraint")
    return int(ch)


def exact(g: _G, t: _T, omega: np.ndarray):
    role = np.zeros(max(g.n, 1), dtype=np.uint64)
    edge = np.zeros(max(nwords(g.m), 1), dtype=np.uint64)
    rc = _load().orc_exact(g.n, _p(g.row_ptr), _p(g.col), _p(omega), t.n0, t.m0,
                           _p(t.labels), _p(t.edges), _p(role), _p(edge))
    if rc:
        raise ValueError("bad template")
    return role[:g.n], edge[:nwords(g.m)]


def lcc_sample(g: _G, t: _T, omega: np.ndarray, verts: np.ndarray):
    """One LCC sweep evaluated for the given vertices only: (new role masks
    of those vertices, CSR entries their rows hold).  Timing samples."""
    vs = np.ascontiguousarray(verts, dtype=np.int32)
    out = np.zeros(max(vs.shape[0], 1), dtype=np.uint64)
    om = np.ascontiguousarray(omega, dtype=np.uint64)
    e = _load().orc_lcc_sample(g.n, _p(g.row_ptr), _p(g.col), _p(g.labels), t.n0, t.m0,
                               _p(t.labels), _p(t.edges), _p(om), _p(vs), vs.shape[0], _p(out))
    if e < 0:
        raise ValueError("bad template")
    return out[:vs.shape[0]], int(e)


def exact_subset(g: _G, t: _T, omega: np.ndarray, verts: np.ndarray) -> int:
    """The exact step's searches for the given vertices only (timing samples)."""
    vs = np.ascontiguousarray(verts, dtype=np.int32)
    r = _load().orc_exact_subset(g.n, _p(g.row_ptr), _p(g.col), _p(omega), t.n0, t.m0,
                                 _p(t.labels), _p(t.edges), _p(vs), vs.shape[0])
    if r < 0:
        raise ValueError("bad template")
    return int(r)


def exact_sample(g: _G, t: _T, omega: np.ndarray, verts: np.ndarray):
    """Exact-step results for the given vertices: (role masks uint64[len],
    per-entry membership uint8 over the concatenated rows of the vertices,
    row offsets int64[len + 1]).  omega: any sound state (superset of the
    complete set)."""
    vs = np.ascontiguousarray(verts, dtype=np.int32)
    deg = (g.row_ptr[vs.astype(np.int64) + 1] - g.row_ptr[vs]) if vs.size else np.zeros(0, np.int64)
    off = np.zeros(vs.shape[0] + 1, dtype=np.int64)
    np.cumsum(deg, out=off[1:])
    role = np.zeros(max(vs.shape[0], 1), dtype=np.uint64)
    inc = np.zeros(max(int(off[-1]), 1), dtype=np.uint8)
    om = np.ascontiguousarray(omega, dtype=np.uint64)
    r = _load().orc_exact_sample(g.n, _p(g.row_ptr), _p(g.col), _p(om), t.n0, t.m0,
                                 _p(t.labels), _p(t.edges), _p(vs), vs.shape[0], _p(role),
                                 _p(off), _p(inc))
    if r < 0:
        raise ValueError("bad template")
    return role[:vs.shape[0]], inc[:int(off[-1])], off


def state(row_ptr, col, labels, t_labels, t_edges, order=None):
    """omega after the first LCC fixpoint and every non-local constraint
    (the constraint loop of `prune` without the exact step)."""
    g = _G(row_ptr, col, labels)
    t = _T(t_labels, t_edges)
    K0 = constraints_for(t.label_list, t.edge_list)
    seq = list(range(len(K0))) if order is None else list(order)
    omega = init_roles(g, t)
    lcc(g, t, omega)
    for ci in seq:
        if nlcc(g, omega, K0[ci]):
            lcc(g, t, omega)
    return omega


def active_edges(g: _G, t: _T, omega: np.ndarray) -> np.ndarray:
    edge = np.zeros(max(nwords(g.m), 1), dtype=np.uint64)
    _load().orc_active_edges(g.n, _p(g.row_ptr), _p(g.col), _p(omega), t.n0, t.m0,
                             _p(t.labels), _p(t.edges), _p(edge))
    return edge[:nwords(g.m)]


def embed_exists(row_ptr, col, omega, sub_edges, qa, va, qb=-1, vb=-1) -> bool:
    g = _G(row_ptr, col, np.zeros(len(row_ptr) - 1, np.int32))
    om = np.ascontiguousarray(omega, dtype=np.uint64)
    se = np.ascontiguousarray(np.asarray(sub_edges, dtype=np.int32).reshape(-1, 2))
    if se.size == 0:
        se = np.zeros((1, 2), np.int32)
        me = 0
    else:
        me = se.shape[0]
    return bool(_load().orc_embed_exists(g.n, _p(g.row_ptr), _p(g.col), _p(om), me, _p(se),
                                         qa, va, qb, vb))


@dataclasses.dataclass
class Result:
    role_mask: np.ndarray          # uint64[n]
    edge_bits: np.ndarray          # uint64[ceil(m/64)]
    lcc_sweeps: List[int]          # Jacobi sweeps per LCC call
    constraint_changes: List[int]  # vertices shrunk by each constraint
    order: List[int]
    seconds: float = 0.0


def constraints_for(labels, edges) -> List[_cons.Constraint]:
    return _cons.non_local_constraints(list(labels), [tuple(e) for e in edges])


def prune(row_ptr, col, labels, t_labels, t_edges, order: Optional[Sequence[int]] = None,
          stop_after: Optional[int] = None) -> Result:
    """Main constraint-checking loop plus the exact final step.

    order: permutation of the constraint list (default: generated order).
    stop_after: if given, stop after that many constraints (0 = after the
    first LCC fixpoint) and return omega with the derived edge state instead
    of running the exact step.
    """
    t0 = time.perf_counter()
    g = _G(row_ptr, col, labels)
    t = _T(t_labels, t_edges)
    K0 = constraints_for(t.label_list, t.edge_list)
    seq = list(range(len(K0))) if order is None else list(order)
    omega = init_roles(g, t)
    sweeps = [lcc(g, t, omega)]
    changes = []
    for k, ci in enumerate(seq):
        if stop_after is not None and k >= stop_after:
            break
        ch = nlcc(g, omega, K0[ci])
        changes.append(ch)
        if ch:
            sweeps.append(lcc(g, t, omega))
    if stop_after is not None:
        role, edge = omega.copy(), active_edges(g, t, omega)
    else:
        role, edge = exact(g, t, omega)
    return Result(role, edge, sweeps, changes, seq, time.perf_counter() - t0)


def bruteforce(row_ptr, col, labels, t_labels, t_edges):
    """Union of all exact matches (Definition 1) by enumeration.
    Returns (role_mask uint64[n], edge_bits uint64[ceil(m/64)], n_maps)."""
    g = _G(row_ptr, col, labels)
    t = _T(t_labels, t_edges)
    role = np.zeros(max(g.n, 1), dtype=np.uint64)
    edge = np.zeros(max(nwords(g.m), 1), dtype=np.uint64)
    cnt = _load().orc_bruteforce(g.n, _p(g.row_ptr), _p(g.col), _p(g.labels), t.n0, t.m0,
                                 _p(t.labels), _p(t.edges), _p(role), _p(edge))
    if cnt < 0:
        raise ValueError("bad or disconnected template")
    return role[:g.n], edge[:nwords(g.m)], int(cnt)


def enumerate_maps(row_ptr, col, labels, t_labels, t_edges, cap: int = 1 << 20):
    """Every match as a map (Definition 1): (count, maps int32[min(count,
    cap)][n0], rows sorted).  Plain enumeration, tiny inputs only."""
    g = _G(row_ptr, col, labels)
    t = _T(t_labels, t_edges)
    maps = np.zeros((max(cap, 1), t.n0), dtype=np.int32)
    cnt = _load().orc_enumerate(g.n, _p(g.row_ptr), _p(g.col), _p(g.labels), t.n0, t.m0,
                                _p(t.labels), _p(t.edges), _p(maps), cap)
    if cnt < 0:
        raise ValueError("bad or disconnected template")
    k = min(int(cnt), cap)
    out = maps[:k]
    if k:
        out = out[np.lexsort(out.T[::-1])]
    return int(cnt), out


def candidate_set(row_ptr, col, labels, t_labels, t_edges):
    """Candidate set of the interactive incremental search: role sets after
    local checking to a fixpoint with the rule every connected template
    obtained by deleting edges satisfies -- role q of v stays while some
    neighbour of v holds a role adjacent to q in G0 (synchronous sweeps,
    each reading only the previous sweep's state).  Returns (omega
    uint64[n], derived edge bits)."""
    g = _G(row_ptr, col, labels)
    t = _T(t_labels, t_edges)
    om = init_roles(g, t)
    if t.n0 > 1 and g.n > 0:
        adj = [0] * t.n0
        for a, b in t.edge_list:
            adj[a] |= 1 << b
            adj[b] |= 1 << a
        src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        while True:
            cover = np.zeros(g.n, dtype=np.uint64)
            if g.m:
                np.bitwise_or.at(cover, src, om[g.col[:g.m]])
            new = np.zeros_like(om)
            for q in range(t.n0):
                bit = np.uint64(1 << q)
                keep = ((om & bit) != 0) & ((cover & np.uint64(adj[q])) != 0)
                new |= np.where(keep, bit, np.uint64(0))
            if np.array_equal(new, om):
                break
            om = new
    return om, active_edges(g, t, om)
