// Non-local constraint checking and the exact final step on gfx950.
//
// Every non-local constraint (cycle, path, TDS) asks, for each vertex v and
// head role h, whether the constraint's substructure of G0 embeds
// injectively in the current candidate graph with h at v, every vertex
// taking a role it still holds and every substructure edge on an edge of G
// (NLCC algorithm and visitor: a token walks the constraint; its history
// enforces repeated and distinct identities; work aggregation stops
// duplicate walks).  The walk is realised as a depth-first search run by
// one wavefront per query: at each step the 64 lanes scan 64 neighbours of
// the already-placed vertex with the smallest candidate adjacency, test role,
// identity and the other required edges (binary search in the sorted
// candidate rows), and ballot the survivors; the search descends into the
// first and backtracks through the rest.  All checks of one constraint read
// the role sets as they were before the constraint (all tokens finish
// before the barrier), so the result of a check does not depend on the
// order of the searches.  A search that succeeds certifies every head role
// on its path at once, which stops later searches for those roles (the
// shared-memory counterpart of work aggregation).
//
// The final step is the full-template search (Step 5(3) of constraint
// generation, Remark on template-driven search): first from every surviving
// (vertex, role) pair, giving the exact role sets; then from every candidate
// edge not yet covered by a found match, giving the exact edge set.  Every
// match found certifies all its roles and edges.
#include "device_util.h"
#include "pm_internal.h"

namespace pm {

constexpr int kSearchBlock = 256;
constexpr int kTaskChunk = 4;

// Depth-first search of plan P with positions 0 (and 1) pinned at v0 (v1).
// Lane-distributed state: lane i holds the image of position i and the scan
// state of level i.  Returns true with img_r holding a full embedding.
template <typename M>
__device__ bool dfs_search(const SearchArgs &a, const SearchPlan *__restrict__ P,
                           const M *__restrict__ om, int32_t v0, int32_t v1, int32_t &img_r) {
    const int lane = lane_id();
    const int k = P->k;
    const int npin = P->npin;
    int64_t cur_r = 0, end_r = 0, base_r = 0;
    uint64_t pend_r = 0;
    int32_t par_r = 0;
    img_r = lane == 0 ? v0 : (lane == 1 ? v1 : -1);
    if (k <= npin) return true;
    const int64_t *__restrict__ crp = a.c_rp;
    const int32_t *__restrict__ ccol = a.c_col;

    int lvl = npin;
    auto setup = [&](int l) {
        const uint64_t back = P->back[l];
        int best = -1;
        int64_t bd = INT64_MAX;
        for (uint64_t m = back; m; m &= m - 1) {
            const int j = __builtin_ctzll(m);
            const int32_t y = read_lane32(img_r, j);
            const int64_t d = crp[y + 1] - crp[y];
            if (d < bd) {
                bd = d;
                best = j;
            }
        }
        int64_t s = 0, e = 0;
        if (best >= 0) {
            const int32_t y = read_lane32(img_r, best);
            s = crp[y];
            e = crp[y + 1];
        }
        if (lane == l) {
            cur_r = s;
            end_r = e;
            pend_r = 0;
            par_r = best < 0 ? 0 : best;
        }
    };
    setup(lvl);
    for (;;) {
        uint64_t pend = read_lane_u64(pend_r, lvl);
        if (pend == 0) {
            const int64_t cur = read_lane64(cur_r, lvl);
            const int64_t end = read_lane64(end_r, lvl);
            if (cur >= end) {
                if (--lvl < npin) return false;
                continue;
            }
            const int q = P->q[lvl];
            const uint64_t same = P->same[lvl];
            const uint64_t back = P->back[lvl] & ~(1ull << read_lane32(par_r, lvl));
            const int64_t kk = cur + lane;
            const bool in_range = kk < end;
            const int32_t x = in_range ? ccol[kk] : -1;
            bool ok = in_range && (((uint64_t)om[x] >> q) & 1ull);
            for (uint64_t m = same; m; m &= m - 1) {
                const int32_t y = read_lane32(img_r, __builtin_ctzll(m));
                ok = ok && (y != x);
            }
            for (uint64_t m = back; m; m &= m - 1) {
                const int32_t y = read_lane32(img_r, __builtin_ctzll(m));
                const int64_t ys = crp[y], ye = crp[y + 1];
                if (ok) ok = find_sorted(ccol, ys, ye, x) >= 0;
            }
            const uint64_t b = ballot64(ok);
            if (lane == lvl) {
                pend_r = b;
                base_r = cur;
                cur_r = cur + kWave;
            }
            continue;
        }
        const int j = __builtin_ctzll(pend);
        pend &= pend - 1;
        const int64_t base = read_lane64(base_r, lvl);
        const int32_t x = ccol[base + j];
        if (lane == lvl) {
            pend_r = pend;
            img_r = x;
        }
        if (lvl == k - 1) return true;
        ++lvl;
        setup(lvl);
    }
}

// Certify the roles (and, for full-template plans, the edges) of a found
// embedding.
template <typename M>
__device__ void certify(const SearchArgs &a, const SearchPlan *__restrict__ P, int plan_idx,
                        int32_t img_r, M *sat, bool edges) {
    const int lane = lane_id();
    const int k = P->k;
    if (lane < k) {
        const int q = P->q[lane];
        if ((P->certify >> q) & 1ull) atomic_or_elem<M>(sat, img_r, 1ull << q);
    }
    if (!edges) return;
    for (int base = 0; base < a.m0; base += kWave) {
        const int i = base + lane;
        int pa = 0, pb = 0;
        if (i < a.m0) {
            pa = a.plan_edges[(int64_t)plan_idx * a.m0 + i].pa;
            pb = a.plan_edges[(int64_t)plan_idx * a.m0 + i].pb;
        }
        const int32_t u = __shfl(img_r, pa);
        const int32_t w = __shfl(img_r, pb);
        if (i < a.m0) {
            const int64_t e1 = find_sorted(a.col, a.rp[u], a.rp[u + 1], w);
            const int64_t e2 = find_sorted(a.col, a.rp[w], a.rp[w + 1], u);
            if (e1 >= 0) set_bit(a.edge_bits, e1);
            if (e2 >= 0) set_bit(a.edge_bits, e2);
        }
    }
}

template <typename M>
__device__ __forceinline__ uint64_t load_fresh(const M *p) {
    return (uint64_t)__atomic_load_n(p, __ATOMIC_RELAXED);
}

template <typename M>
__global__ __launch_bounds__(kSearchBlock) void vertex_search_kernel(const int32_t *tasks,
                                                                     int64_t n_tasks, const M *om,
                                                                     M *sat, SearchArgs a) {
    const int lane = lane_id();
    unsigned long long queries = 0;
    for (;;) {
        int t0 = 0;
        if (lane == 0) t0 = atomicAdd(a.task_counter, kTaskChunk);
        t0 = __shfl(t0, 0);
        if ((int64_t)t0 >= n_tasks) break;
        const int64_t t1 = (int64_t)t0 + kTaskChunk < n_tasks ? (int64_t)t0 + kTaskChunk : n_tasks;
        for (int64_t t = t0; t < t1; ++t) {
            const int32_t v = tasks[t];
            uint64_t cand = (uint64_t)om[v] & a.heads & ~load_fresh(sat + v);
            while (cand) {
                const int h = __builtin_ctzll(cand);
                cand &= cand - 1;
                if ((load_fresh(sat + v) >> h) & 1ull) continue;
                const int pidx = a.plan_of_head[h];
                const SearchPlan *P = a.plans + pidx;
                int32_t img = 0;
                ++queries;
                if (dfs_search<M>(a, P, om, v, -1, img)) certify<M>(a, P, pidx, img, sat, a.mode == 1);
            }
        }
    }
    if (lane == 0 && queries) atomicAdd(a.n_queries, queries);
}

template <typename M>
void launch_vertex_search(hipStream_t s, const int32_t *tasks, int64_t n_tasks, const M *omega,
                          M *sat, const SearchArgs &a, int grid) {
    if (n_tasks <= 0) return;
    hipLaunchKernelGGL(vertex_search_kernel<M>, dim3(grid), dim3(kSearchBlock), 0, s, tasks,
                       n_tasks, omega, sat, a);
}

// ---------------------------------------------------------- NLCC apply
// Remove the head roles that no embedding supported (NLCC algorithm's
// elimination of unsatisfied token sources), clear the certificates.
template <typename M>
__global__ void apply_kernel(const int32_t *tasks, int64_t n_tasks, M *omega, M *sat,
                             uint64_t heads, int32_t *changed) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool ch = false;
    if (t < n_tasks) {
        const int32_t v = tasks[t];
        const uint64_t w = (uint64_t)omega[v];
        const uint64_t nw = w & (~heads | (uint64_t)sat[v]);
        sat[v] = 0;
        if (nw != w) {
            omega[v] = (M)nw;
            ch = true;
        }
    }
    if (ballot64(ch) && lane_id() == 0) atomicAdd(changed, 1);
}

template <typename M>
void launch_apply(hipStream_t s, const int32_t *tasks, int64_t n_tasks, M *omega, M *sat,
                  uint64_t heads, int32_t *changed) {
    if (n_tasks <= 0) return;
    hipLaunchKernelGGL(apply_kernel<M>, dim3((unsigned)((n_tasks + 255) / 256)), dim3(256), 0, s,
                       tasks, n_tasks, omega, sat, heads, changed);
}

// ------------------------------------------------ exact step: edge part
template <typename M>
__device__ __forceinline__ uint64_t reach_mask(uint64_t w, const LccTable &tab) {
    uint64_t r = 0;
    for (int q = 0; q < tab.n0; ++q)
        if ((w >> q) & 1ull) r |= tab.adj[q];
    return r;
}

// Candidate edges: u < w in the compacted subgraph, certified roles of u and
// w adjacent in G0, edge bit not set by an earlier witness.
template <typename M>
__global__ __launch_bounds__(kSearchBlock) void edge_candidates_kernel(
    const int32_t *tasks, int64_t n_tasks, const int64_t *c_rp, const int32_t *c_col,
    const int32_t *c_off, const int64_t *rp, const M *cert, LccTable tab,
    const uint64_t *edge_bits, int32_t *eu, int32_t *ew, int64_t *e_idx, int32_t *n_out,
    int64_t cap) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t t = wave; t < n_tasks; t += nwaves) {
        const int32_t u = tasks[t];
        const uint64_t cu = (uint64_t)cert[u];
        if (!cu) continue;
        const uint64_t reach = reach_mask<M>(cu, tab);
        const int64_t s = c_rp[u], e = c_rp[u + 1], r0 = rp[u];
        for (int64_t base = s; base < e; base += kWave) {
            const int64_t k = base + lane;
            bool p = false;
            int32_t w = 0;
            int64_t orig = 0;
            if (k < e) {
                w = c_col[k];
                orig = r0 + c_off[k];
                p = w > u && ((uint64_t)cert[w] & reach) != 0ull &&
                    !((edge_bits[orig >> 6] >> (orig & 63)) & 1ull);
            }
            const uint64_t m = ballot64(p);
            if (!m) continue;
            int pos = 0;
            if (lane == 0) pos = atomicAdd(n_out, __popcll(m));
            pos = __shfl(pos, 0);
            if (p) {
                const int64_t o = pos + __popcll(m & lanemask_lt());
                if (o < cap) {
                    eu[o] = u;
                    ew[o] = w;
                    e_idx[o] = orig;
                }
            }
        }
    }
}

template <typename M>
void launch_edge_candidates(hipStream_t s, const int32_t *tasks, int64_t n_tasks,
                            const int64_t *c_rp, const int32_t *c_col, const int32_t *c_off,
                            const int64_t *rp, const M *cert, const LccTable &tab,
                            const uint64_t *edge_bits, int32_t *eu, int32_t *ew, int64_t *e_idx,
                            int32_t *n_out, int64_t cap) {
    if (n_tasks <= 0) return;
    int64_t grid = (n_tasks * kWave + kSearchBlock - 1) / kSearchBlock;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(edge_candidates_kernel<M>, dim3((unsigned)grid), dim3(kSearchBlock), 0, s,
                       tasks, n_tasks, c_rp, c_col, c_off, rp, cert, tab, edge_bits, eu, ew,
                       e_idx, n_out, cap);
}

template <typename M>
__global__ __launch_bounds__(kSearchBlock) void edge_search_kernel(
    const int32_t *eu, const int32_t *ew, const int64_t *e_idx, int64_t n_edges, const M *om,
    M *cert, const int32_t *edge_plan, int32_t n_edge_plans, SearchArgs a) {
    const int lane = lane_id();
    unsigned long long queries = 0;
    for (;;) {
        int t0 = 0;
        if (lane == 0) t0 = atomicAdd(a.task_counter, kTaskChunk);
        t0 = __shfl(t0, 0);
        if ((int64_t)t0 >= n_edges) break;
        const int64_t t1 = (int64_t)t0 + kTaskChunk < n_edges ? (int64_t)t0 + kTaskChunk : n_edges;
        for (int64_t t = t0; t < t1; ++t) {
            const int32_t u = eu[t], w = ew[t];
            const int64_t e = e_idx[t];
            const uint64_t cu = (uint64_t)om[u], cw = (uint64_t)om[w];
            for (int i = 0; i < n_edge_plans; ++i) {
                if ((load_fresh(a.edge_bits + (e >> 6)) >> (e & 63)) & 1ull) break;
                const int pidx = edge_plan[i];
                const SearchPlan *P = a.plans + pidx;
                if (!((cu >> P->q[0]) & 1ull) || !((cw >> P->q[1]) & 1ull)) continue;
                int32_t img = 0;
                ++queries;
                if (dfs_search<M>(a, P, om, u, w, img)) {
                    certify<M>(a, P, pidx, img, cert, true);
                    break;
                }
            }
        }
    }
    if (lane == 0 && queries) atomicAdd(a.n_queries, queries);
}

template <typename M>
void launch_edge_search(hipStream_t s, const int32_t *eu, const int32_t *ew,
                        const int64_t *e_idx, int64_t n_edges, const M *omega, M *cert,
                        const int32_t *edge_plan_dev, int32_t n_edge_plans, const SearchArgs &a,
                        int grid) {
    if (n_edges <= 0) return;
    hipLaunchKernelGGL(edge_search_kernel<M>, dim3(grid), dim3(kSearchBlock), 0, s, eu, ew,
                       e_idx, n_edges, omega, cert, edge_plan_dev, n_edge_plans, a);
}

// Edge state implied by role sets (edge elimination rule): bit of entry
// u->w set iff omega(w) meets the roles adjacent to omega(u).
template <typename M>
__global__ __launch_bounds__(kSearchBlock) void active_edges_kernel(
    const int32_t *tasks, int64_t n_tasks, const int64_t *c_rp, const int32_t *c_col,
    const int32_t *c_off, const int64_t *rp, const M *om, LccTable tab, uint64_t *edge_bits) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t t = wave; t < n_tasks; t += nwaves) {
        const int32_t u = tasks[t];
        const uint64_t reach = reach_mask<M>((uint64_t)om[u], tab);
        if (!reach) continue;
        const int64_t s = c_rp[u], e = c_rp[u + 1], r0 = rp[u];
        for (int64_t k = s + lane; k < e; k += kWave)
            if ((uint64_t)om[c_col[k]] & reach) set_bit(edge_bits, r0 + c_off[k]);
    }
}

template <typename M>
void launch_active_edges(hipStream_t s, const int32_t *tasks, int64_t n_tasks,
                         const int64_t *c_rp, const int32_t *c_col, const int32_t *c_off,
                         const int64_t *rp, const M *omega, const LccTable &tab,
                         uint64_t *edge_bits) {
    if (n_tasks <= 0) return;
    int64_t grid = (n_tasks * kWave + kSearchBlock - 1) / kSearchBlock;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(active_edges_kernel<M>, dim3((unsigned)grid), dim3(kSearchBlock), 0, s,
                       tasks, n_tasks, c_rp, c_col, c_off, rp, omega, tab, edge_bits);
}

#define PM_INSTANTIATE_SEARCH(M)                                                                  \
    template void launch_vertex_search<M>(hipStream_t, const int32_t *, int64_t, const M *, M *,  \
                                          const SearchArgs &, int);                               \
    template void launch_apply<M>(hipStream_t, const int32_t *, int64_t, M *, M *, uint64_t,      \
                                  int32_t *);                                                     \
    template void launch_edge_candidates<M>(hipStream_t, const int32_t *, int64_t,                \
                                            const int64_t *, const int32_t *, const int32_t *,    \
                                            const int64_t *, const M *, const LccTable &,         \
                                            const uint64_t *, int32_t *, int32_t *, int64_t *,    \
                                            int32_t *, int64_t);                                  \
    template void launch_edge_search<M>(hipStream_t, const int32_t *, const int32_t *,            \
                                        const int64_t *, int64_t, const M *, M *,                 \
                                        const int32_t *, int32_t, const SearchArgs &, int);       \
    template void launch_active_edges<M>(hipStream_t, const int32_t *, int64_t, const int64_t *,  \
                                         const int32_t *, const int32_t *, const int64_t *,       \
                                         const M *, const LccTable &, uint64_t *);

PM_INSTANTIATE_SEARCH(uint8_t)
PM_INSTANTIATE_SEARCH(uint16_t)
PM_INSTANTIATE_SEARCH(uint32_t)
PM_INSTANTIATE_SEARCH(uint64_t)

}  // namespace pm
