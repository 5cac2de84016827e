// Template compiler: validation, local-rule tables, non-local constraint
// generation and search plans.  Host code.
//
// Constraint generation follows the paper's constraint-generation table
// (Step 1: unique-label leaves are left to LCC; Step 2: repeated-label
// vertices; Step 3: one cycle constraint per cycle of G'0; Step 4: one
// shortest path of >= 3 hops per repeated-label pair, unless a single cycle
// constraint contains it; Step 5: TDS unions of cycles sharing an edge and
// of paths sharing a vertex, the latter reduced to a spanning tree), the TDS
// constraint generation algorithm, and the ordering heuristics (paths and
// cycles first by walk length, TDS after).  Where the paper leaves a choice
// open the same deterministic reading is used throughout the library:
//   * cycles: simple cycles of G'0 as vertex sequences starting at the
//     smallest vertex with second vertex < last vertex, sorted by (length,
//     sequence), at most 32, enumerated length by length;
//   * shortest path: breadth-first search, neighbours in ascending index,
//     first discoverer is the parent;
//   * merge: repeat while some pair qualifies (cycles: common edge; paths:
//     common vertex); groups keep their first member's position and only
//     groups of two or more members become new constraints; spanning tree:
//     breadth-first from the lowest vertex, neighbours ascending;
//   * heads: all vertices of cycle and TDS-cycle constraints, both ends of a
//     path constraint, repeated-label vertices of a TDS-path constraint;
//   * order: (edges, cycle before path, index) over cycles and paths, then
//     TDS-cycle, then TDS-path constraints by (edges, index);
//   * the mandatory full-template search (Step 5(3)) is the final exact step.

#include <algorithm>
#include <deque>
#include <map>
#include <set>

#include "pm_internal.h"

namespace pm {
namespace {

using Edge = std::pair<int, int>;

Edge norm(int a, int b) { return a < b ? Edge(a, b) : Edge(b, a); }

std::vector<std::vector<int>> adjacency(int n0, const std::vector<Edge> &edges) {
    std::vector<std::vector<int>> adj(n0);
    for (auto &e : edges) {
        adj[e.first].push_back(e.second);
        adj[e.second].push_back(e.first);
    }
    for (auto &a : adj) std::sort(a.begin(), a.end());
    return adj;
}

// Simple cycles of the subgraph induced on `allowed`, canonical form, by
// increasing length; stops after the first length at which at least
// `keep` cycles exist.  Returns false if one length has more than
// `per_length_limit` cycles.
bool find_cycles(int n0, const std::vector<Edge> &edges, uint64_t allowed, size_t keep,
                 size_t per_length_limit, std::vector<std::vector<int>> &out) {
    std::vector<Edge> sub;
    for (auto &e : edges)
        if (((allowed >> e.first) & 1) && ((allowed >> e.second) & 1)) sub.push_back(e);
    auto adj = adjacency(n0, sub);
    for (int length = 3; length <= n0; ++length) {
        std::vector<std::vector<int>> found;
        for (int s = 0; s < n0; ++s) {
            if (!((allowed >> s) & 1)) continue;
            std::vector<int> path{s};
            uint64_t on = 1ull << s;
            std::vector<size_t> cur{0};
            while (!cur.empty()) {
                int x = path.back();
                size_t &i = cur.back();
                if (i >= adj[x].size()) {
                    on &= ~(1ull << x);
                    path.pop_back();
                    cur.pop_back();
                    continue;
                }
                int y = adj[x][i++];
                if ((int)path.size() == length) {
                    if (y == s && path[1] < path.back()) {
                        found.push_back(path);
                        if (found.size() > per_length_limit) return false;
                    }
                } else if (y > s && !((on >> y) & 1)) {
                    path.push_back(y);
                    on |= 1ull << y;
                    cur.push_back(0);
                }
            }
        }
        std::sort(found.begin(), found.end());
        out.insert(out.end(), found.begin(), found.end());
        if (out.size() >= keep) break;
    }
    return true;
}

std::vector<int> bfs_path(int n0, const std::vector<Edge> &edges, int src, int dst) {
    auto adj = adjacency(n0, edges);
    std::vector<int> parent(n0, -1);
    std::vector<char> seen(n0, 0);
    std::deque<int> dq{src};
    seen[src] = 1;
    while (!dq.empty()) {
        int x = dq.front();
        dq.pop_front();
        for (int y : adj[x])
            if (!seen[y]) {
                seen[y] = 1;
                parent[y] = x;
                dq.push_back(y);
            }
    }
    if (!seen[dst]) return {};
    std::vector<int> p{dst};
    while (p.back() != src) p.push_back(parent[p.back()]);
    std::reverse(p.begin(), p.end());
    return p;
}

struct Group {
    std::set<Edge> edges;
    int members;
};

uint64_t vertex_mask(const std::set<Edge> &es) {
    uint64_t m = 0;
    for (auto &e : es) m |= (1ull << e.first) | (1ull << e.second);
    return m;
}

std::vector<Group> merge_groups(const std::vector<std::set<Edge>> &items, bool need_edge) {
    std::vector<Group> g;
    for (auto &it : items) g.push_back({it, 1});
    bool changed = true;
    while (changed) {
        changed = false;
        for (size_t i = 0; i < g.size(); ++i) {
            for (size_t j = i + 1; j < g.size();) {
                bool share_v = (vertex_mask(g[i].edges) & vertex_mask(g[j].edges)) != 0;
                bool share_e = false;
                for (auto &e : g[j].edges)
                    if (g[i].edges.count(e)) { share_e = true; break; }
                if (share_v && (share_e || !need_edge)) {
                    g[i].edges.insert(g[j].edges.begin(), g[j].edges.end());
                    g[i].members += g[j].members;
                    g.erase(g.begin() + (long)j);
                    changed = true;
                    j = i + 1;
                } else {
                    ++j;
                }
            }
        }
    }
    return g;
}

std::vector<Edge> bfs_spanning_tree(const std::set<Edge> &es) {
    uint64_t vm = vertex_mask(es);
    int root = __builtin_ctzll(vm);
    int n0 = 64 - __builtin_clzll(vm);
    auto adj = adjacency(n0, std::vector<Edge>(es.begin(), es.end()));
    std::vector<char> seen(n0, 0);
    std::deque<int> dq{root};
    seen[root] = 1;
    std::vector<Edge> out;
    while (!dq.empty()) {
        int x = dq.front();
        dq.pop_front();
        for (int y : adj[x])
            if (!seen[y]) {
                seen[y] = 1;
                out.push_back(norm(x, y));
                dq.push_back(y);
            }
    }
    std::sort(out.begin(), out.end());
    return out;
}

// Search plan over the substructure `sub` (edge list) pinned at qa (and qb).
SearchPlan make_plan(const std::vector<Edge> &sub, const std::vector<int32_t> &labels, int qa,
                     int qb, uint64_t certify) {
    SearchPlan P{};
    uint64_t vm = 0;
    for (auto &e : sub) {
        P.adj[e.first] |= 1ull << e.second;
        P.adj[e.second] |= 1ull << e.first;
        vm |= (1ull << e.first) | (1ull << e.second);
    }
    if (sub.empty()) vm = 1ull << qa;
    P.vmask = vm;
    P.k = __builtin_popcountll(vm);
    P.pin[0] = qa;
    P.pin[1] = qb;
    P.npin = qb >= 0 ? 2 : 1;
    for (int q = 0; q < kMaxK; ++q) {
        if (!((vm >> q) & 1)) continue;
        for (int r = 0; r < kMaxK; ++r)
            if (r != q && ((vm >> r) & 1) && labels[r] == labels[q]) P.samelab[q] |= 1ull << r;
    }
    P.certify = certify;
    return P;
}

}  // namespace

std::string compile_template(int n0, int m0, const uint16_t *labels, const uint32_t *edges,
                             const std::vector<int64_t> &label_freq, CompiledTemplate &T) {
    if (n0 < 1 || n0 > kMaxK) return "template must have 1..64 vertices";
    if (m0 < 0 || (m0 > 0 && !edges) || !labels) return "null template arrays";
    T = CompiledTemplate{};
    T.n0 = n0;
    T.m0 = m0;
    T.labels.assign(labels, labels + n0);
    std::set<Edge> seen;
    for (int i = 0; i < m0; ++i) {
        uint32_t a = edges[2 * i], b = edges[2 * i + 1];
        if (a >= (uint32_t)n0 || b >= (uint32_t)n0) return "template edge vertex out of range";
        if (a == b) return "template self-loop";
        Edge e = norm((int)a, (int)b);
        if (!seen.insert(e).second) return "duplicate template edge";
        T.edges.push_back(e);
    }
    // connectivity (Preliminaries: G0 is connected)
    {
        auto adj = adjacency(n0, T.edges);
        std::vector<char> vis(n0, 0);
        std::deque<int> dq{0};
        vis[0] = 1;
        int cnt = 1;
        while (!dq.empty()) {
            int x = dq.front();
            dq.pop_front();
            for (int y : adj[x])
                if (!vis[y]) { vis[y] = 1; ++cnt; dq.push_back(y); }
        }
        if (cnt != n0) return "template is not connected";
    }
    T.mask_bytes = n0 <= 8 ? 1 : n0 <= 16 ? 2 : n0 <= 32 ? 4 : 8;
    std::map<int, int> lab_count;
    for (int q = 0; q < n0; ++q) lab_count[T.labels[q]]++;
    bool unique = (int)lab_count.size() == n0;
    T.acyclic_unique = unique && m0 == n0 - 1;
    // acyclic, one label on two vertices a, b, every other label on one:
    // the path a .. b and, off it, every vertex's neighbour towards it
    T.tree_pair = false;
    if (m0 == n0 - 1 && n0 >= 2 && (int)lab_count.size() == n0 - 1) {
        int a = -1, b = -1;
        for (int q = 0; q < n0 && b < 0; ++q)
            for (int r = q + 1; r < n0; ++r)
                if (T.labels[q] == T.labels[r]) { a = q; b = r; break; }
        auto adj = adjacency(n0, T.edges);
        std::vector<int> from(n0, -1);
        std::deque<int> dq{a};
        from[a] = a;
        while (!dq.empty()) {
            int x = dq.front();
            dq.pop_front();
            for (int y : adj[x])
                if (from[y] < 0) { from[y] = x; dq.push_back(y); }
        }
        std::vector<int> path;
        for (int x = b; x != a; x = from[x]) path.push_back(x);
        path.push_back(a);
        std::reverse(path.begin(), path.end());
        TreePlan &tp = T.tree;
        tp = TreePlan{};
        tp.k = (int)path.size() - 1;
        tp.m0 = m0;
        for (int q = 0; q < n0; ++q) { tp.pos[q] = -1; tp.par[q] = -1; }
        for (int i = 0; i <= tp.k; ++i) {
            tp.path[i] = (int8_t)path[(size_t)i];
            tp.pos[path[(size_t)i]] = (int8_t)i;
        }
        // distances from the path (breadth first from all its vertices)
        std::vector<int> dist(n0, -1);
        for (int x : path) { dist[x] = 0; dq.push_back(x); }
        while (!dq.empty()) {
            int x = dq.front();
            dq.pop_front();
            for (int y : adj[x])
                if (dist[y] < 0) {
                    dist[y] = dist[x] + 1;
                    tp.par[y] = (int8_t)x;
                    tp.depmask[dist[y]] |= 1ull << y;
                    tp.depth = std::max(tp.depth, dist[y]);
                    dq.push_back(y);
                }
        }
        for (int j = 0; j < m0; ++j) {
            tp.ea[j] = (int8_t)T.edges[(size_t)j].first;
            tp.eb[j] = (int8_t)T.edges[(size_t)j].second;
        }
        T.tree_pair = true;
    }
    for (int q = 0; q < n0; ++q) {
        T.label_mask_of[q] = 0;
        for (int r = 0; r < n0; ++r)
            if (T.labels[r] == T.labels[q]) T.label_mask_of[q] |= 1ull << r;
    }

    // ---- local rule tables --------------------------------------------------
    LccTable &L = T.lcc;
    L = LccTable{};
    L.n0 = n0;
    for (auto &e : T.edges) {
        L.adj[e.first] |= 1ull << e.second;
        L.adj[e.second] |= 1ull << e.first;
    }
    T.need_off.assign(1, 0);
    T.need_lab.clear();
    T.need_min.clear();
    T.need_labmask.assign((size_t)n0, 0);
    for (int q = 0; q < n0; ++q) {
        std::map<int, uint64_t> by_label;
        for (int r = 0; r < n0; ++r)
            if ((L.adj[q] >> r) & 1) by_label[T.labels[r]] |= 1ull << r;
        // first-sweep needs of q: every neighbour label with its multiplicity
        for (auto &kv : by_label) {
            T.need_lab.push_back(kv.first);
            T.need_min.push_back(__builtin_popcountll(kv.second));
            if (kv.first < 64) T.need_labmask[(size_t)q] |= 1ull << kv.first;
        }
        T.need_off.push_back((int32_t)T.need_lab.size());
        for (auto &kv : by_label) {
            int need = __builtin_popcountll(kv.second);
            if (need < 2) continue;
            if (L.ncount >= kMaxCount) return "too many distinct-count rules (limit 32)";
            L.cq[L.ncount] = q;
            L.cmask[L.ncount] = kv.second;
            L.cneed[L.ncount] = need;
            L.ncount++;
        }
    }

    // ---- non-local constraints ---------------------------------------------
    auto adj = adjacency(n0, T.edges);
    uint64_t allowed = 0;   // V'0: all but unique-label leaves (Step 1)
    for (int q = 0; q < n0; ++q) {
        bool uniq = lab_count[T.labels[q]] == 1;
        if (!(uniq && adj[q].size() == 1)) allowed |= 1ull << q;
    }
    std::vector<int> vd;    // repeated-label vertices (Step 2)
    for (int q = 0; q < n0; ++q)
        if (lab_count[T.labels[q]] > 1) vd.push_back(q);
    uint64_t vd_mask = 0;
    for (int q : vd) vd_mask |= 1ull << q;

    std::vector<std::vector<int>> cycles;
    if (!find_cycles(n0, T.edges, allowed, 32, 100000, cycles))
        return "too many cycles in template";
    if (cycles.size() > 32) cycles.resize(32);
    std::vector<Constraint> cc, pcs;
    for (auto &c : cycles) {
        Constraint k;
        k.kind = 0;
        k.gen_index = (int)cc.size();
        k.vmask = 0;
        std::set<Edge> es;
        for (size_t i = 0; i < c.size(); ++i) {
            es.insert(norm(c[i], c[(i + 1) % c.size()]));
            k.vmask |= 1ull << c[i];
        }
        k.edges.assign(es.begin(), es.end());
        k.heads = k.vmask;
        cc.push_back(k);
    }
    for (size_t i = 0; i < vd.size(); ++i)
        for (size_t j = i + 1; j < vd.size(); ++j) {
            int qi = vd[i], qj = vd[j];
            if (T.labels[qi] != T.labels[qj]) continue;
            auto p = bfs_path(n0, T.edges, qi, qj);
            if (p.size() < 4) continue;  // fewer than 3 hops: LCC covers it
            std::set<Edge> es;
            for (size_t k = 0; k + 1 < p.size(); ++k) es.insert(norm(p[k], p[k + 1]));
            bool inside = false;
            for (auto &c : cc) {
                std::set<Edge> ce(c.edges.begin(), c.edges.end());
                if (std::includes(ce.begin(), ce.end(), es.begin(), es.end())) { inside = true; break; }
            }
            if (inside) continue;
            Constraint k;
            k.kind = 1;
            k.gen_index = (int)pcs.size();
            k.edges.assign(es.begin(), es.end());
            k.vmask = vertex_mask(es);
            k.heads = (1ull << qi) | (1ull << qj);
            pcs.push_back(k);
        }
    std::vector<Constraint> tcc, tpc;
    {
        std::vector<std::set<Edge>> items;
        for (auto &c : cc) items.emplace_back(c.edges.begin(), c.edges.end());
        for (auto &g : merge_groups(items, true)) {
            if (g.members < 2) continue;
            Constraint k;
            k.kind = 2;
            k.gen_index = (int)tcc.size();
            k.edges.assign(g.edges.begin(), g.edges.end());
            k.vmask = vertex_mask(g.edges);
            k.heads = k.vmask;
            tcc.push_back(k);
        }
    }
    {
        std::vector<std::set<Edge>> items;
        for (auto &c : pcs) items.emplace_back(c.edges.begin(), c.edges.end());
        for (auto &g : merge_groups(items, false)) {
            if (g.members < 2) continue;
            Constraint k;
            k.kind = 3;
            k.gen_index = (int)tpc.size();
            k.edges = bfs_spanning_tree(g.edges);
            std::set<Edge> es(k.edges.begin(), k.edges.end());
            k.vmask = vertex_mask(es);
            k.heads = k.vmask & vd_mask;
            tpc.push_back(k);
        }
    }
    std::vector<Constraint> first;
    first.insert(first.end(), cc.begin(), cc.end());
    first.insert(first.end(), pcs.begin(), pcs.end());
    std::stable_sort(first.begin(), first.end(), [](const Constraint &a, const Constraint &b) {
        if (a.edges.size() != b.edges.size()) return a.edges.size() < b.edges.size();
        if (a.kind != b.kind) return a.kind < b.kind;
        return a.gen_index < b.gen_index;
    });
    auto by_len = [](const Constraint &a, const Constraint &b) {
        if (a.edges.size() != b.edges.size()) return a.edges.size() < b.edges.size();
        return a.gen_index < b.gen_index;
    };
    std::stable_sort(tcc.begin(), tcc.end(), by_len);
    std::stable_sort(tpc.begin(), tpc.end(), by_len);
    T.constraints = first;
    T.constraints.insert(T.constraints.end(), tcc.begin(), tcc.end());
    T.constraints.insert(T.constraints.end(), tpc.begin(), tpc.end());
    if ((int)T.constraints.size() > 64) return "too many non-local constraints (limit 64)";

    // ---- search plans ---------------------------------------------------------
    uint64_t all = n0 == 64 ? ~0ull : ((1ull << n0) - 1ull);
    for (auto &c : T.constraints) {
        for (int h = 0; h < kMaxK; ++h) c.plan_of_head[h] = -1;
        c.plan_base = (int)T.plans.size();
        for (int h = 0; h < n0; ++h) {
            if (!((c.heads >> h) & 1)) continue;
            c.plan_of_head[h] = (int)T.plans.size();
            T.plans.push_back(make_plan(c.edges, T.labels, h, -1, c.heads));
        }
    }
    for (int q = 0; q < kMaxK; ++q) T.vertex_plan[q] = -1;
    for (int q = 0; q < n0; ++q) {
        T.vertex_plan[q] = (int)T.plans.size();
        T.plans.push_back(make_plan(T.edges, T.labels, q, -1, all));
    }
    for (auto &e : T.edges) {
        T.edge_plans.push_back((int)T.plans.size());
        T.plans.push_back(make_plan(T.edges, T.labels, e.first, e.second, all));
        T.edge_plans.push_back((int)T.plans.size());
        T.plans.push_back(make_plan(T.edges, T.labels, e.second, e.first, all));
    }
    return "";
}

}  // namespace pm
