"""Python binding of libpm (argument marshalling only).

Every step of the pruning runs in libpm's HIP kernels; this module only
turns torch tensors into device pointers, fills the option and template
structs and checks status codes.  PyTorch provides device memory and the
stream.  There is no fallback: if libpm.so is missing or fails to load, the
constructor raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpm.so")

PM_OK = 0
PM_HOST_PTRS = 1
PM_VALIDATE = 2
PM_ORDER_FIXED = 0
PM_ORDER_GIVEN = 1
PM_ORDER_LEARNED = 2
PM_MODE_FULL = 0
PM_MODE_CANDIDATE = 1
PM_ABLATE_EDGE_ELIMINATION = 1
PM_ABLATE_WORK_AGGREGATION = 2
NOALLOC_SCRATCH_BYTES = 64 << 20
MAX_CONSTRAINTS = 64
MLP_FEATURES = 12
MLP_OUTPUTS = 2
MLP_PARAMS = 5122

ERRORS = {
    -1: "PM_ERR_INVALID_ARG", -2: "PM_ERR_HIP", -3: "PM_ERR_GRAPH", -4: "PM_ERR_TEMPLATE",
    -5: "PM_ERR_NO_GRAPH", -6: "PM_ERR_CAPACITY", -7: "PM_ERR_OOM", -8: "PM_ERR_NOT_FOUND",
    -9: "PM_ERR_MODEL", -10: "PM_ERR_WORKSPACE",
}

# exported symbols declared in include/pm.h
SYMBOLS = ["pm_last_error", "pm_version", "pm_create", "pm_destroy", "pm_load_graph",
           "pm_unload_graph", "pm_load_templates", "pm_template_constraints",
           "pm_inspect_template", "pm_prune", "pm_load_model", "pm_mlp_forward", "pm_mlp_grad",
           "pm_mlp_train", "pm_set_param", "pm_get_param", "pm_export_state",
           "pm_import_state", "pm_workspace_size", "pm_set_workspace", "pm_prune_noalloc",
           "pm_count_matches", "pm_build_count_index", "pm_graph_info", "pm_build_pair_index"]


class PMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class pm_template(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_uint32), ("m0", ctypes.c_uint32),
                ("labels", ctypes.POINTER(ctypes.c_uint16)),
                ("edges", ctypes.POINTER(ctypes.c_uint32))]


class pm_trace_entry(ctypes.Structure):
    _fields_ = [("constraint", ctypes.c_int32), ("changed", ctypes.c_int32),
                ("roles_before", ctypes.c_int64), ("roles_after", ctypes.c_int64),
                ("active_before", ctypes.c_int64), ("ms", ctypes.c_float),
                ("score", ctypes.c_float), ("predicted", ctypes.c_float * MLP_OUTPUTS),
                ("features", ctypes.c_float * MLP_FEATURES)]

    def as_dict(self):
        return {"constraint": self.constraint, "changed": self.changed,
                "roles_before": self.roles_before, "roles_after": self.roles_after,
                "active_before": self.active_before, "ms": self.ms, "score": self.score,
                "predicted": list(self.predicted), "features": list(self.features)}


class pm_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("ms_total", "ms_init", "ms_lcc", "ms_compact", "ms_nlcc", "ms_exact",
                 "ms_first_sweep", "ms_sweep_kernel", "wave_ms_vq_pos", "wave_ms_vq_neg",
                 "wave_ms_eq_pos", "wave_ms_eq_neg", "wave_ms_certify", "wave_ms_expand")] + \
               [(k, ctypes.c_int64) for k in
                ("lcc_sweeps", "constraints", "first_sweep_vertices", "first_sweep_entries",
                 "candidate_entries", "vertex_queries", "edge_queries", "result_vertices",
                 "edge_candidates", "vq_pos", "vq_neg", "eq_pos", "eq_neg", "trace_entries", "expand_scans",
                 "expand_candidates", "expand_valid", "first_sweep_bytes", "witness_edges",
                 "split_tasks")] + \
               [("done_mask", ctypes.c_uint64), ("workspace_bytes", ctypes.c_int64),
                ("join_edges", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class pm_options(ctypes.Structure):
    _fields_ = [("order_mode", ctypes.c_int32), ("n_order", ctypes.c_int32),
                ("order", ctypes.c_int32 * MAX_CONSTRAINTS), ("stop_after", ctypes.c_int32),
                ("batch_streams", ctypes.c_int32), ("learned_min_score", ctypes.c_float),
                ("learned_stop", ctypes.c_int32), ("trace_cap", ctypes.c_int32),
                ("trace", ctypes.POINTER(pm_trace_entry)), ("mode", ctypes.c_int32),
                ("ablate", ctypes.c_uint32), ("init_state", ctypes.c_void_p),
                ("skip_mask", ctypes.c_uint64), ("known_roles", ctypes.c_void_p),
                ("known_edges", ctypes.c_void_p), ("shared_inputs", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("union_roles", ctypes.c_void_p),
                ("union_edges", ctypes.c_void_p),
                ("per_template", ctypes.POINTER(pm_stats)), ("limit_checks", ctypes.c_int32),
                ("max_checks", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


class pm_graph_info_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("label_bytes", ctypes.c_int32),
                ("index_labels", ctypes.c_int32), ("index_bytes", ctypes.c_int64),
                ("hubs", ctypes.c_int64), ("hub_segments", ctypes.c_int64),
                ("ms_count_index", ctypes.c_double), ("pair_entries", ctypes.c_int64),
                ("ms_pair_index", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class pm_match_count(ctypes.Structure):
    _fields_ = [("maps", ctypes.c_uint64), ("automorphisms", ctypes.c_uint64),
                ("subgraphs", ctypes.c_uint64), ("written", ctypes.c_int64),
                ("roots", ctypes.c_int64), ("ms_total", ctypes.c_double),
                ("complete", ctypes.c_int32), ("pad_", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library():
    """Load the in-tree libpm.so; raises if it is missing (no CPU fallback
    exists)."""
    global _lib
    if _lib is not None:
        return _lib
    path = LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"libpm.so not built at {path}; run __graft_entry__.build()")
    # torch ships its own HIP runtime; loading it first makes libpm bind to
    # that same runtime (matched by soname), so one process has one runtime
    # and libpm can use torch's streams and allocations.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.pm_last_error.restype = ctypes.c_char_p
    lib.pm_version.restype = ctypes.c_char_p
    lib.pm_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, P]
    lib.pm_destroy.argtypes = [P]
    lib.pm_load_graph.argtypes = [P, I64, I64, P, P, P, ctypes.c_int, ctypes.c_uint32]
    lib.pm_unload_graph.argtypes = [P]
    lib.pm_load_templates.argtypes = [P, I32, ctypes.POINTER(pm_template), ctypes.POINTER(I32)]
    lib.pm_template_constraints.argtypes = [P, I32, ctypes.POINTER(I32), P, P, P, P]
    lib.pm_inspect_template.argtypes = [ctypes.POINTER(pm_template), ctypes.POINTER(I32), P, P,
                                        P, P]
    lib.pm_prune.argtypes = [P, I32, I32, P, P, ctypes.POINTER(pm_options),
                             ctypes.POINTER(pm_stats)]
    lib.pm_load_model.argtypes = [P, P, ctypes.c_size_t]
    lib.pm_set_param.argtypes = [P, ctypes.c_char_p, I64]
    lib.pm_get_param.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(I64)]
    lib.pm_mlp_forward.argtypes = [P, P, P, I64, P]
    lib.pm_mlp_grad.argtypes = [P, P, P, P, I64, P, P]
    lib.pm_mlp_train.argtypes = [P, P, P, P, I64, I32, ctypes.c_float, P]
    lib.pm_export_state.argtypes = [P, I32, I32, ctypes.POINTER(pm_options), P,
                                    ctypes.POINTER(ctypes.c_uint64)]
    lib.pm_import_state.argtypes = [P, I32, P, ctypes.c_uint64, P, P, ctypes.POINTER(pm_options),
                                    ctypes.POINTER(pm_stats)]
    lib.pm_workspace_size.argtypes = [P, I32, I32, ctypes.POINTER(pm_options),
                                      ctypes.POINTER(ctypes.c_size_t)]
    lib.pm_set_workspace.argtypes = [P, P, ctypes.c_size_t]
    lib.pm_prune_noalloc.argtypes = [P, I32, P, P, ctypes.POINTER(pm_options),
                                     ctypes.POINTER(pm_stats)]
    lib.pm_count_matches.argtypes = [P, I32, P, P, I64, ctypes.c_uint64,
                                     ctypes.POINTER(pm_match_count)]
    lib.pm_build_count_index.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
    lib.pm_build_pair_index.argtypes = [P, I32, I32, ctypes.POINTER(ctypes.c_double)]
    lib.pm_graph_info.argtypes = [P, ctypes.POINTER(pm_graph_info_t)]
    for name in SYMBOLS[2:]:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(lib, rc: int):
    if rc != PM_OK:
        raise PMError(rc, lib.pm_last_error().decode())


class PM:
    """One libpm context on a CUDA (HIP) device and torch stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(self.lib, self.lib.pm_create(ctypes.byref(h), device,
                                            ctypes.c_void_p(stream.cuda_stream)))
        self.h = h
        self.n = 0
        self.m = 0
        self._graph_refs = None
        self.templates: List = []

    def close(self):
        if getattr(self, "h", None):
            self.lib.pm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- graph
    def load_graph(self, row_ptr, col, labels, validate: bool = False):
        """row_ptr int64[n+1], col int32[m], labels uint8/int16-as-uint16[n]:
        torch tensors on the context's device (borrowed), or numpy arrays
        (copied by the library)."""
        torch = self.torch
        flags = PM_VALIDATE if validate else 0
        if isinstance(row_ptr, np.ndarray):
            rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
            cl = np.ascontiguousarray(col, dtype=np.int32)
            lb = np.ascontiguousarray(labels)
            lbytes = lb.dtype.itemsize
            flags |= PM_HOST_PTRS
            ptrs = [a.ctypes.data if a.size else 0 for a in (rp, cl, lb)]
            refs = (rp, cl, lb)
        else:
            rp, cl, lb = row_ptr, col, labels
            assert rp.dtype == torch.int64 and cl.dtype == torch.int32
            assert rp.is_contiguous() and cl.is_contiguous() and lb.is_contiguous()
            lbytes = lb.element_size()
            ptrs = [t.data_ptr() for t in (rp, cl, lb)]
            refs = (rp, cl, lb)
        n = int(rp.shape[0]) - 1
        m = int(cl.shape[0])
        _check(self.lib, self.lib.pm_load_graph(self.h, n, m, ctypes.c_void_p(ptrs[0]),
                                                ctypes.c_void_p(ptrs[1]), ctypes.c_void_p(ptrs[2]),
                                                lbytes, flags))
        self.n, self.m = n, m
        self._graph_refs = refs if not (flags & PM_HOST_PTRS) else None

    def build_count_index(self) -> float:
        """Rebuild the neighbour-label count index; returns its device ms."""
        ms = ctypes.c_double()
        _check(self.lib, self.lib.pm_build_count_index(self.h, ctypes.byref(ms)))
        return float(ms.value)

    def build_pair_index(self, first_id: int, count: int = 1) -> float:
        """Build the label-pair subgraph for templates [first_id,
        first_id + count) (count 0 frees it); returns its device ms."""
        ms = ctypes.c_double()
        _check(self.lib, self.lib.pm_build_pair_index(self.h, int(first_id), int(count),
                                                      ctypes.byref(ms)))
        return float(ms.value)

    def graph_info(self) -> dict:
        g = pm_graph_info_t()
        _check(self.lib, self.lib.pm_graph_info(self.h, ctypes.byref(g)))
        return g.as_dict()

    # --------------------------------------------------------- templates
    def load_templates(self, templates: Sequence) -> int:
        """templates: objects with .labels (list[int]) and .edges (list of
        pairs).  Returns the id of the first."""
        arr = (pm_template * len(templates))()
        keep = []
        for i, t in enumerate(templates):
            lab = np.ascontiguousarray(np.asarray(t.labels, dtype=np.uint16))
            e = np.ascontiguousarray(np.asarray(t.edges, dtype=np.uint32).reshape(-1))
            if e.size == 0:
                e = np.zeros(2, dtype=np.uint32)
            keep += [lab, e]
            arr[i].n0 = len(t.labels)
            arr[i].m0 = len(t.edges)
            arr[i].labels = lab.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16))
            arr[i].edges = e.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        first = ctypes.c_int32()
        _check(self.lib, self.lib.pm_load_templates(self.h, len(templates), arr,
                                                    ctypes.byref(first)))
        self.templates += list(templates)
        return int(first.value)

    def constraints(self, tid: int):
        """[(kind, edges tuple, heads mask)] in generation order."""
        cnt = ctypes.c_int32()
        kinds = np.zeros(MAX_CONSTRAINTS, np.int32)
        ne = np.zeros(MAX_CONSTRAINTS, np.int32)
        heads = np.zeros(MAX_CONSTRAINTS, np.uint64)
        edges = np.zeros(MAX_CONSTRAINTS * 128, np.uint32)
        _check(self.lib, self.lib.pm_template_constraints(
            self.h, tid, ctypes.byref(cnt), kinds.ctypes.data_as(ctypes.c_void_p),
            ne.ctypes.data_as(ctypes.c_void_p), heads.ctypes.data_as(ctypes.c_void_p),
            edges.ctypes.data_as(ctypes.c_void_p)))
        return _unpack_constraints(cnt.value, kinds, ne, heads, edges)

    # ------------------------------------------------------------- prune
    def _options(self, order=None, stop_after=-1, batch_streams=0, learned_min_score=None,
                 mode=PM_MODE_FULL, ablate=0, init_state=None, skip_mask=0, known_roles=None,
                 known_edges=None, shared_inputs=False, union_roles=None, union_edges=None,
                 max_checks=None):
        opt = pm_options()
        opt.stop_after = stop_after
        opt.batch_streams = batch_streams
        opt.mode = int(mode)
        opt.ablate = int(ablate)
        if isinstance(order, str):
            if order != "learned":
                raise ValueError("order must be None, 'learned' or a permutation")
            opt.order_mode = PM_ORDER_LEARNED
        elif order is not None:
            opt.order_mode = PM_ORDER_GIVEN
            opt.n_order = len(order)
            for i, k in enumerate(order):
                opt.order[i] = int(k)
        if learned_min_score is not None:
            opt.learned_stop = 1
            opt.learned_min_score = float(learned_min_score)
        opt.shared_inputs = 1 if shared_inputs else 0
        if max_checks is not None:
            opt.limit_checks = 1
            opt.max_checks = int(max_checks)
        for name, t in (("init_state", init_state), ("known_roles", known_roles),
                        ("known_edges", known_edges), ("union_roles", union_roles),
                        ("union_edges", union_edges)):
            if t is not None:
                self._check_device_i64(t, name)
                setattr(opt, name, t.data_ptr())
        opt.skip_mask = int(skip_mask) & 0xFFFFFFFFFFFFFFFF
        return opt

    def _check_device_i64(self, t, name):
        torch = self.torch
        if not (isinstance(t, torch.Tensor) and t.dtype == torch.int64 and t.is_contiguous()
                and t.device == self.device):
            raise ValueError(f"{name} must be a contiguous int64 tensor on {self.device}")

    def prune(self, first_id: int, count: int = 1, order=None,
              stop_after: int = -1, role_mask=None, edge_bits=None, batch_streams: int = 0,
              learned_min_score: Optional[float] = None, trace: bool = False,
              mode: int = PM_MODE_FULL, ablate: int = 0, init_state=None, skip_mask: int = 0,
              known_roles=None, known_edges=None, shared_inputs: bool = False,
              union_roles=None, union_edges=None, per_template: bool = False,
              max_checks: Optional[int] = None):
        """Returns (role_mask uint64-as-int64 tensor [count, n], edge_bits
        [count, ceil(m/64)], stats dict); with trace=True the stats dict also
        holds "trace", the list of per-step records.  order: None (fixed),
        "learned" (greedy by the loaded model), or a permutation.  mode:
        PM_MODE_FULL or PM_MODE_CANDIDATE; ablate: PM_ABLATE_* bits;
        init_state / known_roles [count, n] and known_edges [count, words]:
        device int64 tensors (one [n] / [words] array for all templates with
        shared_inputs); union_roles [n] / union_edges [words]: device int64
        tensors every template's output is ORed into (see pm.h).  With
        per_template the stats dict holds "per_template", one dict per
        template.  max_checks: check at most that many non-local constraints
        before the final search (output unchanged)."""
        torch = self.torch
        words = (self.m + 63) // 64
        if role_mask is None:
            role_mask = torch.empty((count, max(self.n, 1)), dtype=torch.int64, device=self.device)
        if edge_bits is None:
            edge_bits = torch.empty((count, max(words, 1)), dtype=torch.int64, device=self.device)
        opt = self._options(order, stop_after, batch_streams, learned_min_score, mode, ablate,
                            init_state, skip_mask, known_roles, known_edges, shared_inputs,
                            union_roles, union_edges, max_checks)
        per = None
        if per_template:
            per = (pm_stats * count)()
            opt.per_template = ctypes.cast(per, ctypes.POINTER(pm_stats))
        tr = None
        if trace:
            tr = (pm_trace_entry * (MAX_CONSTRAINTS + 1))()
            opt.trace_cap = MAX_CONSTRAINTS + 1
            opt.trace = ctypes.cast(tr, ctypes.POINTER(pm_trace_entry))
        st = pm_stats()
        _check(self.lib, self.lib.pm_prune(self.h, first_id, count,
                                           ctypes.c_void_p(role_mask.data_ptr()),
                                           ctypes.c_void_p(edge_bits.data_ptr()),
                                           ctypes.byref(opt), ctypes.byref(st)))
        out = st.as_dict()
        if per is not None:
            out["per_template"] = [per[i].as_dict() for i in range(count)]
        if tr is not None:
            out["trace"] = [tr[i].as_dict() for i in range(int(st.trace_entries))]
        return role_mask[:, :self.n], edge_bits[:, :words], out

    # ------------------------------------------------------ state, counting
    def export_state(self, tid: int, stop_after: int = -1, order=None, learned_min_score=None,
                     state=None):
        """(state int64 tensor [n] on the device, done_mask) after the first
        LCC fixpoint and stop_after constraints (< 0: all)."""
        torch = self.torch
        if state is None:
            state = torch.empty(max(self.n, 1), dtype=torch.int64, device=self.device)
        opt = self._options(order, stop_after, 0, learned_min_score)
        done = ctypes.c_uint64()
        _check(self.lib, self.lib.pm_export_state(self.h, tid, int(stop_after), ctypes.byref(opt),
                                                  ctypes.c_void_p(state.data_ptr()),
                                                  ctypes.byref(done)))
        return state[:self.n], int(done.value)

    def import_state(self, tid: int, state, done_mask: int, order=None, stop_after: int = -1,
                     learned_min_score=None, role_mask=None, edge_bits=None):
        """Resume from an exported state; returns (role_mask [1, n],
        edge_bits [1, words], stats)."""
        torch = self.torch
        words = (self.m + 63) // 64
        self._check_device_i64(state, "state")
        if role_mask is None:
            role_mask = torch.empty((1, max(self.n, 1)), dtype=torch.int64, device=self.device)
        if edge_bits is None:
            edge_bits = torch.empty((1, max(words, 1)), dtype=torch.int64, device=self.device)
        opt = self._options(order, stop_after, 0, learned_min_score)
        st = pm_stats()
        _check(self.lib, self.lib.pm_import_state(
            self.h, tid, ctypes.c_void_p(state.data_ptr()), ctypes.c_uint64(done_mask & 0xFFFFFFFFFFFFFFFF),
            ctypes.c_void_p(role_mask.data_ptr()), ctypes.c_void_p(edge_bits.data_ptr()),
            ctypes.byref(opt), ctypes.byref(st)))
        return role_mask[:, :self.n], edge_bits[:, :words], st.as_dict()

    def workspace_size(self, first_id: int, count: int = 1, batch_streams: int = 0) -> int:
        opt = self._options(batch_streams=batch_streams)
        b = ctypes.c_size_t()
        _check(self.lib, self.lib.pm_workspace_size(self.h, first_id, count, ctypes.byref(opt),
                                                    ctypes.byref(b)))
        return int(b.value)

    def set_workspace(self, ws) -> None:
        """Use the device tensor ws (any dtype, contiguous; kept alive by
        this object) for all scratch; None returns to library-owned
        scratch."""
        if ws is None:
            _check(self.lib, self.lib.pm_set_workspace(self.h, None, 0))
            self._ws = None
            return
        _check(self.lib, self.lib.pm_set_workspace(self.h, ctypes.c_void_p(ws.data_ptr()),
                                                   ws.numel() * ws.element_size()))
        self._ws = ws

    def prune_noalloc(self, tid: int, role_mask, edge_bits, order=None, stop_after: int = -1,
                      learned_min_score=None):
        """pm_prune_noalloc: outputs are caller-owned device tensors
        [1, n] / [1, words]; returns the stats dict."""
        opt = self._options(order, stop_after, 0, learned_min_score)
        st = pm_stats()
        _check(self.lib, self.lib.pm_prune_noalloc(self.h, tid,
                                                   ctypes.c_void_p(role_mask.data_ptr()),
                                                   ctypes.c_void_p(edge_bits.data_ptr()),
                                                   ctypes.byref(opt), ctypes.byref(st)))
        return st.as_dict()

    def count_matches(self, tid: int, state=None, cap: int = 0, max_maps: int = 0):
        """Match count of template tid within state ([n] or [1, n] device
        int64 role masks, None: label roles).  With cap > 0 also returns up
        to cap maps as an int32 tensor [k, n0]; max_maps > 0 stops counting
        soon after that many (then "complete" is 0)."""
        torch = self.torch
        n0 = len(self.templates[tid].labels)
        sp = None
        if state is not None:
            st_t = state.reshape(-1)
            self._check_device_i64(st_t, "state")
            sp = ctypes.c_void_p(st_t.data_ptr())
        maps = None
        mp = None
        if cap > 0:
            maps = torch.empty((cap, n0), dtype=torch.int32, device=self.device)
            mp = ctypes.c_void_p(maps.data_ptr())
        out = pm_match_count()
        _check(self.lib, self.lib.pm_count_matches(self.h, tid, sp, mp, int(cap),
                                                   ctypes.c_uint64(int(max_maps)),
                                                   ctypes.byref(out)))
        res = out.as_dict()
        if maps is not None:
            res["maps_out"] = maps[:out.written]
        return res

    # ------------------------------------------------------------ tuning
    TUNING = ("expand", "expand_edges", "expand_max", "witness", "tree_exact", "relist", "edge_chunk",
              "edge_stripes",
              "search_grid", "search_grid_solo", "split_budget", "edge_tail", "expand_table_log2",
              "split_capacity", "read_first", "lcc_bin_small", "lcc_bin_mid")

    def set_param(self, name: str, value: int) -> None:
        _check(self.lib, self.lib.pm_set_param(self.h, name.encode(), int(value)))

    def get_param(self, name: str) -> int:
        v = ctypes.c_int64()
        _check(self.lib, self.lib.pm_get_param(self.h, name.encode(), ctypes.byref(v)))
        return int(v.value)

    def params(self) -> dict:
        return {k: self.get_param(k) for k in self.TUNING}

    # ----------------------------------------------------- ordering model
    def load_model(self, w) -> None:
        """Load the ordering model (MLP_PARAMS float32 values, host)."""
        a = np.ascontiguousarray(np.asarray(w, dtype=np.float32).reshape(-1))
        _check(self.lib, self.lib.pm_load_model(self.h, a.ctypes.data_as(ctypes.c_void_p),
                                                a.shape[0]))

    def _f32(self, a, shape):
        t = self.torch.as_tensor(a, dtype=self.torch.float32, device=self.device)
        return t.reshape(shape).contiguous()

    def mlp_forward(self, w, x):
        """Model outputs [N][2] for inputs [N][12] (device kernel)."""
        wd = self._f32(w, (MLP_PARAMS,))
        xd = self._f32(x, (-1, MLP_FEATURES))
        y = self.torch.empty((xd.shape[0], MLP_OUTPUTS), dtype=self.torch.float32,
                             device=self.device)
        _check(self.lib, self.lib.pm_mlp_forward(self.h, ctypes.c_void_p(wd.data_ptr()),
                                                 ctypes.c_void_p(xd.data_ptr()), xd.shape[0],
                                                 ctypes.c_void_p(y.data_ptr())))
        return y

    def mlp_grad(self, w, x, t):
        """(loss, gradient [MLP_PARAMS]) of the halved mean squared error."""
        wd = self._f32(w, (MLP_PARAMS,))
        xd = self._f32(x, (-1, MLP_FEATURES))
        td = self._f32(t, (-1, MLP_OUTPUTS))
        g = self.torch.empty(MLP_PARAMS, dtype=self.torch.float32, device=self.device)
        loss = self.torch.empty(1, dtype=self.torch.float32, device=self.device)
        _check(self.lib, self.lib.pm_mlp_grad(self.h, ctypes.c_void_p(wd.data_ptr()),
                                              ctypes.c_void_p(xd.data_ptr()),
                                              ctypes.c_void_p(td.data_ptr()), xd.shape[0],
                                              ctypes.c_void_p(g.data_ptr()),
                                              ctypes.c_void_p(loss.data_ptr())))
        return float(loss.item()), g

    def mlp_train(self, w, x, t, steps: int, lr: float):
        """Full-batch Adam on the device; returns (parameters, loss history)."""
        wd = self._f32(w, (MLP_PARAMS,)).clone()
        xd = self._f32(x, (-1, MLP_FEATURES))
        td = self._f32(t, (-1, MLP_OUTPUTS))
        hist = np.zeros(max(steps, 1), dtype=np.float32)
        _check(self.lib, self.lib.pm_mlp_train(self.h, ctypes.c_void_p(wd.data_ptr()),
                                               ctypes.c_void_p(xd.data_ptr()),
                                               ctypes.c_void_p(td.data_ptr()), xd.shape[0],
                                               int(steps), float(lr),
                                               hist.ctypes.data_as(ctypes.c_void_p)))
        return wd, hist[:steps]


def _unpack_constraints(cnt, kinds, ne, heads, edges):
    out = []
    for i in range(cnt):
        es = tuple((int(edges[i * 128 + 2 * j]), int(edges[i * 128 + 2 * j + 1]))
                   for j in range(int(ne[i])))
        out.append((int(kinds[i]), es, int(heads[i])))
    return out


def inspect_template(t):
    """Constraint list of a template compiled on the host only (no device):
    [(kind, edges tuple, heads mask)] in generation order."""
    lib = load_library()
    lab = np.ascontiguousarray(np.asarray(t.labels, dtype=np.uint16))
    e = np.ascontiguousarray(np.asarray(t.edges, dtype=np.uint32).reshape(-1))
    if e.size == 0:
        e = np.zeros(2, dtype=np.uint32)
    tt = pm_template(len(t.labels), len(t.edges),
                     lab.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                     e.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    cnt = ctypes.c_int32()
    kinds = np.zeros(MAX_CONSTRAINTS, np.int32)
    ne = np.zeros(MAX_CONSTRAINTS, np.int32)
    heads = np.zeros(MAX_CONSTRAINTS, np.uint64)
    edges = np.zeros(MAX_CONSTRAINTS * 128, np.uint32)
    _check(lib, lib.pm_inspect_template(ctypes.byref(tt), ctypes.byref(cnt),
                                        kinds.ctypes.data_as(ctypes.c_void_p),
                                        ne.ctypes.data_as(ctypes.c_void_p),
                                        heads.ctypes.data_as(ctypes.c_void_p),
                                        edges.ctypes.data_as(ctypes.c_void_p)))
    return _unpack_constraints(cnt.value, kinds, ne, heads, edges)


def to_u64(t) -> np.ndarray:
    """Device int64 tensor -> host uint64 numpy view."""
    return t.detach().cpu().numpy().view(np.uint64)
