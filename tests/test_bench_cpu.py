"""Host-side checks of the benchmark's measurement helpers: the refusal of
more than one GPU, the algorithmic bytes of the label-pair subgraph pass
(counted here entry by entry on a small graph), and the counter records
under profiles/ (used only while every source they name is unchanged)."""
import hashlib
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1912_08453_amd import inputs as I  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


class _Ctx:
    def __init__(self, pair_entries):
        self.pe = pair_entries

    def graph_info(self):
        return {"pair_entries": self.pe}


def test_pair_bytes_counts_rows_of_template_edge_labels():
    rp, col = I.rmat_csr(9, seed=5)
    g = I.Graph(rp, col, I.labels_log2deg(rp))
    ts = [I.Template([1, 2, 3], [(0, 1), (1, 2)]), I.Template([2, 4], [(0, 1)])]
    labs = {1, 2, 3, 4}
    pairs = {(1, 2), (2, 1), (2, 3), (3, 2), (2, 4), (4, 2)}
    n_a = m_a = m_p = 0
    for v in range(g.n):
        if int(g.labels[v]) not in labs:
            continue
        n_a += 1
        for k in range(int(rp[v]), int(rp[v + 1])):
            m_a += 1
            if (int(g.labels[v]), int(g.labels[col[k]])) in pairs:
                m_p += 1
    b, sizes = bench.pair_bytes(g, ts, _Ctx(m_p))
    assert sizes == {"n_a": n_a, "m_a": m_a, "m_p": m_p}
    nlab = int(g.labels.max()) + 1
    padded = (g.n + 255) // 256 * 256
    assert b == (g.n + 8 * n_a + 4 * m_a + n_a + 8 * (g.n + 1) + 8 * m_p + nlab * padded)


def _record(root, name, srcs, shas):
    os.makedirs(os.path.join(root, "profiles"), exist_ok=True)
    with open(os.path.join(root, "profiles", name), "w") as f:
        f.write("# comment line\n")
        f.write("source=" + ",".join(srcs) + "\n")
        f.write("source_sha1=" + ",".join(shas) + "\n")
        f.write("fetch_kib_per_dispatch=100.0\nwrite_kib_per_dispatch=10.0\n")
        f.write("fetch_scale=2.0\nwrite_scale=1.0\n")


def test_recorded_traffic_follows_the_sources(tmp_path, monkeypatch):
    root = str(tmp_path)
    monkeypatch.setattr(bench, "ROOT", root)
    for name, text in (("a.hip", "kernel a\n"), ("b.cpp", "driver b\n")):
        with open(os.path.join(root, name), "w") as f:
            f.write(text)
    sha = lambda name: hashlib.sha1(open(os.path.join(root, name), "rb").read()).hexdigest()
    _record(root, "rec.txt", ["a.hip", "b.cpp"], [sha("a.hip"), sha("b.cpp")])
    assert bench.recorded_traffic("rec.txt") == int(100.0 * 1024 * 2.0 + 10.0 * 1024 * 1.0)
    assert bench.recorded_traffic("missing.txt") is None
    _record(root, "short.txt", ["a.hip", "b.cpp"], [sha("a.hip")])
    assert bench.recorded_traffic("short.txt") is None
    with open(os.path.join(root, "b.cpp"), "a") as f:
        f.write("// changed\n")
    assert bench.recorded_traffic("rec.txt") is None


def test_committed_records_name_existing_sources():
    for name in ("pair_subgraph_theta8_rmat26.txt", "label_count_rmat22_log2deg.txt"):
        rec = {}
        for line in open(os.path.join(ROOT, "profiles", name)):
            if "=" in line and not line.startswith("#"):
                k, v = line.strip().split("=", 1)
                rec[k] = v
        for src in rec["source"].split(","):
            assert os.path.exists(os.path.join(ROOT, src)), src
        assert float(rec["fetch_kib_per_dispatch"]) > 0 and float(rec["write_kib_per_dispatch"]) > 0
