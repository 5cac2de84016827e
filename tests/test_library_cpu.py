"""Host-side checks of libpm that need no GPU: the library loads, exports
every symbol declared in include/pm.h, and its template compiler produces
the same ordered non-local constraint list as the oracle's independent
generator (Steps 1-5 of constraint generation, TDS generation, ordering
heuristics) and rejects invalid templates."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import constraints as C
from paper_1912_08453_amd import _build
from paper_1912_08453_amd import inputs as I
from paper_1912_08453_amd import pm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pm.LIB_PATH):
        _build.build_pm()
    return pm.load_library()


def header_functions():
    src = open(os.path.join(ROOT, "include", "pm.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(pm_\w+)\(", src, re.M)))


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(pm.SYMBOLS)
    assert lib.pm_version().startswith(b"pm ")


def oracle_list(t):
    return [(c.kind, c.edges, c.heads) for c in C.non_local_constraints(t.labels, t.edges)]


def shapes(seed):
    rng = np.random.Generator(np.random.Philox(seed))
    kind = seed % 5
    n0 = int(rng.integers(2, 9))
    if kind == 0:
        edges = I.shape_tree(rng, n0)
    elif kind == 1:
        edges = I.shape_one_cycle(rng, max(n0, 3))
    elif kind == 2:
        edges = I.shape_two_cycles(rng, max(n0, 5))
    elif kind == 3:
        edges = I.shape_k4(rng, max(n0, 4))
    else:
        edges = I.shape_two_cycles(rng, max(n0, 6))
        a, b = (int(x) for x in rng.choice(max(n0, 6), size=2, replace=False))
        edges = sorted(set(edges) | {(min(a, b), max(a, b))})
    n0 = max(max(e) for e in edges) + 1
    nl = int(rng.integers(1, n0 + 1))
    labels = [int(x) for x in rng.integers(0, nl, size=n0)]
    return I.Template(labels, edges)


@pytest.mark.parametrize("seed", range(300))
def test_constraint_lists_match_oracle(lib, seed):
    t = shapes(seed)
    assert pm.inspect_template(t) == oracle_list(t)


def test_constraint_list_named_shapes(lib):
    for t in [I.template_square_pendant(), I.Template([10, 11, 12, 13, 14, 12], I.TRI_SQUARE_EDGES),
              I.Template([0] * 4, [(a, b) for a in range(4) for b in range(a + 1, 4)]),
              I.Template([0, 1, 2, 0, 1, 2, 3], [(i, i + 1) for i in range(6)]),
              I.Template([0] * 6, [(i, (i + 1) % 6) for i in range(6)]),
              I.Template([3], [])]:
        assert pm.inspect_template(t) == oracle_list(t)


@pytest.mark.parametrize("labels,edges,why", [
    ([0, 1, 2], [(0, 1)], "disconnected"),
    ([0, 1], [(0, 0)], "self-loop"),
    ([0, 1], [(0, 1), (1, 0)], "duplicate"),
    ([0, 1], [(0, 2)], "range"),
    ([], [], "empty"),
    ([0] * 65, [(i, i + 1) for i in range(64)], "too large"),
])
def test_invalid_templates_rejected(lib, labels, edges, why):
    with pytest.raises(pm.PMError) as ei:
        pm.inspect_template(I.Template(labels, edges))
    assert ei.value.code == -4, why


def test_count_rule_limit(lib):
    """A 40-vertex single-label path has 38 distinct-count rules (> 32)."""
    with pytest.raises(pm.PMError) as ei:
        pm.inspect_template(I.Template([0] * 40, [(i, i + 1) for i in range(39)]))
    assert ei.value.code == -4


def test_cycle_rich_template_bounded(lib):
    """K_{6,6}: cycle enumeration stops after the 4-cycles (225 of them)."""
    k = 6
    t = I.Template([0] * k + [1] * k, [(a, k + b) for a in range(k) for b in range(k)])
    got = pm.inspect_template(t)
    assert got == oracle_list(t)
    assert sum(1 for c in got if c[0] == C.CC) == 32


def _c_layout(tmp_path):
    """sizeof/offsetof of the ABI structs as the C compiler lays them out."""
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stddef.h>
#include <stdio.h>
#include "pm.h"
#define F(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void) {
    printf("pm_options %zu\n", sizeof(pm_options));
    printf("pm_trace_entry %zu\n", sizeof(pm_trace_entry));
    printf("pm_stats %zu\n", sizeof(pm_stats));
    printf("pm_template %zu\n", sizeof(pm_template));
    F(pm_options, stop_after); F(pm_options, batch_streams); F(pm_options, learned_min_score);
    F(pm_options, learned_stop); F(pm_options, trace_cap); F(pm_options, trace);
    F(pm_options, mode); F(pm_options, ablate); F(pm_options, init_state);
    F(pm_options, skip_mask); F(pm_options, known_roles); F(pm_options, known_edges);
    F(pm_options, shared_inputs); F(pm_options, union_roles); F(pm_options, union_edges);
    F(pm_options, per_template); F(pm_options, limit_checks); F(pm_options, max_checks);
    F(pm_options, reserved);
    F(pm_trace_entry, roles_before); F(pm_trace_entry, ms); F(pm_trace_entry, score);
    F(pm_trace_entry, predicted); F(pm_trace_entry, features);
    F(pm_stats, lcc_sweeps); F(pm_stats, trace_entries); F(pm_stats, split_tasks);
    F(pm_stats, done_mask); F(pm_stats, workspace_bytes); F(pm_stats, join_edges);
    printf("pm_match_count %zu\n", sizeof(pm_match_count));
    printf("pm_graph_info_t %zu\n", sizeof(pm_graph_info_t));
    F(pm_graph_info_t, index_labels); F(pm_graph_info_t, index_bytes); F(pm_graph_info_t, ms_count_index);
    F(pm_graph_info_t, pair_entries); F(pm_graph_info_t, ms_pair_index);
    F(pm_match_count, maps); F(pm_match_count, automorphisms); F(pm_match_count, subgraphs);
    F(pm_match_count, written); F(pm_match_count, roots); F(pm_match_count, ms_total);
    F(pm_match_count, complete);
    return 0;
}
''')
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    return dict(line.rsplit(" ", 1) for line in out if line)


def test_ctypes_structs_match_the_c_layout(tmp_path):
    c = {k: int(v) for k, v in _c_layout(tmp_path).items()}
    assert c["pm_options"] == ctypes.sizeof(pm.pm_options)
    assert c["pm_trace_entry"] == ctypes.sizeof(pm.pm_trace_entry)
    assert c["pm_stats"] == ctypes.sizeof(pm.pm_stats)
    assert c["pm_template"] == ctypes.sizeof(pm.pm_template)
    assert c["pm_match_count"] == ctypes.sizeof(pm.pm_match_count)
    assert c["pm_graph_info_t"] == ctypes.sizeof(pm.pm_graph_info_t)
    for key, v in c.items():
        if "." in key:
            struct, field = key.split(".")
            assert getattr(getattr(pm, struct), field).offset == v, key
