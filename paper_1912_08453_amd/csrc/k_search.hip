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

// Estimated number of candidates for template vertex p next to the image y
// of a placed neighbour: neighbours of y holding role p (role counts), or
// y's candidate degree when no counts are available.
__device__ __forceinline__ int64_t cand_estimate(const SearchArgs &a, int32_t y, int p) {
    if (a.rcnt) return (int64_t)a.rcnt[(int64_t)y * a.rcnt_stride + p];
    return a.c_rp[y + 1] - a.c_rp[y];
}

// Depth-first search for an embedding of plan P's substructure with the
// pinned template vertices at v0 (and v1).  Lane-distributed state: lane q
// holds the image of template vertex q; lane l holds the scan state of
// search level l (which template vertex it places, the placed neighbour
// whose candidate row it scans, the row cursor and the ballot of surviving
// candidates of the current 64-entry chunk).  At each new level the
// unplaced vertex with the fewest estimated candidates is placed next (the
// paper's constraint optimisation visits rare labels first; here the
// estimate is per partial match).  Returns true with img_r holding a full
// embedding.
template <typename M>
__device__ bool dfs_search(const SearchArgs &a, const SearchPlan *__restrict__ P,
                           const M *__restrict__ om, int32_t v0, int32_t v1, int32_t &img_r) {
    const int lane = lane_id();
    const int k = P->k;
    const int npin = P->npin;
    const uint64_t vmask = P->vmask;
    const int p0 = P->pin[0], p1 = P->pin[1];
    img_r = lane == p0 ? v0 : ((npin == 2 && lane == p1) ? v1 : -1);
    uint64_t placed = (1ull << p0) | (npin == 2 ? (1ull << p1) : 0ull);
    if (k <= npin) return true;
    const int64_t *__restrict__ crp = a.c_rp;
    const int32_t *__restrict__ ccol = a.c_col;
    int64_t cur_r = 0, end_r = 0, base_r = 0;
    uint64_t pend_r = 0;
    int32_t pv_r = 0, par_r = 0;

    auto select = [&](int l) {
        int bp = -1, bj = -1;
        int64_t bs = INT64_MAX;
        for (uint64_t mp = vmask & ~placed; mp; mp &= mp - 1) {
            const int p = __builtin_ctzll(mp);
            for (uint64_t mj = P->adj[p] & placed; mj; mj &= mj - 1) {
                const int j = __builtin_ctzll(mj);
                const int64_t sc = cand_estimate(a, read_lane32(img_r, j), p);
                if (sc < bs) {
                    bs = sc;
                    bp = p;
                    bj = j;
                }
            }
        }
        int64_t s = 0, e = 0;
        if (bj >= 0) {
            const int32_t y = read_lane32(img_r, bj);
            s = crp[y];
            e = crp[y + 1];
        }
        if (lane == l) {
            cur_r = s;
            end_r = e;
            pend_r = 0;
            pv_r = bp < 0 ? 0 : bp;
            par_r = bj < 0 ? 0 : bj;
        }
    };
    int lvl = npin;
    select(lvl);
    for (;;) {
        uint64_t pend = read_lane_u64(pend_r, lvl);
        if (pend == 0) {
            const int64_t cur = read_lane64(cur_r, lvl);
            const int64_t end = read_lane64(end_r, lvl);
            if (cur >= end) {
                if (--lvl < npin) return false;
                placed &= ~(1ull << read_lane32(pv_r, lvl));
                continue;
            }
            const int q = read_lane32(pv_r, lvl);
            const int par = read_lane32(par_r, lvl);
            const uint64_t same = P->samelab[q] & placed;
            const uint64_t back = P->adj[q] & placed & ~(1ull << par);
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
        const int q = read_lane32(pv_r, lvl);
        if (lane == lvl) pend_r = pend;
        if (lane == q) img_r = x;
        placed |= 1ull << q;
        if (lvl == k - 1) return true;
        ++lvl;
        select(lvl);
    }
}

// Certify the head roles of a found embedding (NLCC).
template <typename M>
__device__ void certify_roles(const SearchPlan *__restrict__ P, int32_t img_r, M *sat) {
    const int lane = lane_id();
    if ((P->vmask >> lane) & 1ull)
        if ((P->certify >> lane) & 1ull) atomic_or_elem<M>(sat, img_r, 1ull << lane);
}

__device__ __forceinline__ bool test_bit(const uint64_t *bits, int64_t k) {
    return (bits[k >> 6] >> (k & 63)) & 1ull;
}

// Certify a full match: every role, and every template edge as an entry of
// the compacted subgraph (one direction; the output ORs in the reverse).
template <typename M>
__device__ void certify_match(const SearchArgs &a, const SearchPlan *__restrict__ P,
                              int32_t img_r, M *cert) {
    const int lane = lane_id();
    if ((P->vmask >> lane) & 1ull) atomic_or_elem<M>(cert, img_r, 1ull << lane);
    for (int base = 0; base < a.m0; base += kWave) {
        const int i = base + lane;
        int ta = 0, tb = 0;
        if (i < a.m0) {
            ta = a.tedges[2 * i];
            tb = a.tedges[2 * i + 1];
        }
        const int32_t u = __shfl(img_r, ta);
        const int32_t w = __shfl(img_r, tb);
        if (i < a.m0) {
            const int64_t k = find_sorted(a.c_col, a.c_rp[u], a.c_rp[u + 1], w);
            if (k >= 0) set_bit(a.c_cert, k);
        }
    }
}

// Single-vertex swaps of a found match: for each template vertex q, every x
// that can replace phi(q) with all other images fixed (role q, adjacent to
// the images of all template neighbours of q, distinct from the images of
// same-label vertices) gives another match, whose role (x, q) and edges at
// x are certified.  Purely a saving: anything it misses is queried later.
template <typename M>
__device__ void expand_match(const SearchArgs &a, const SearchPlan *__restrict__ P,
                             int32_t img_r, const M *__restrict__ om, M *cert) {
    const int lane = lane_id();
    const int64_t *__restrict__ crp = a.c_rp;
    const int32_t *__restrict__ ccol = a.c_col;
    for (uint64_t mq = P->vmask; mq; mq &= mq - 1) {
        const int q = __builtin_ctzll(mq);
        const uint64_t nb = P->adj[q];
        if (!nb) continue;
        int js = -1;
        int64_t bd = INT64_MAX;
        for (uint64_t m = nb; m; m &= m - 1) {
            const int j = __builtin_ctzll(m);
            const int64_t d = cand_estimate(a, read_lane32(img_r, j), q);
            if (d < bd) {
                bd = d;
                js = j;
            }
        }
        const int32_t ys = read_lane32(img_r, js);
        if (__popcll(nb) == 1) {
            // a pendant vertex depends (up to identity checks) only on its
            // neighbour's image: expand it once per (vertex, role)
            unsigned long long old = 0;
            if (lane == 0) old = atomicOr((unsigned long long *)&a.exp_done[ys], 1ull << q);
            old = __shfl(old, 0);
            if ((old >> q) & 1ull) continue;
        }
        const uint64_t others = nb & ~(1ull << js);
        const uint64_t same = P->samelab[q];
        const int64_t s = crp[ys], e = crp[ys + 1];
        for (int64_t base = s; base < e; base += kWave) {
            const int64_t kk = base + lane;
            const bool in = kk < e;
            const int32_t x = in ? ccol[kk] : -1;
            bool ok = in && (((uint64_t)om[x] >> q) & 1ull);
            for (uint64_t m = same; m; m &= m - 1) {
                const int32_t y = read_lane32(img_r, __builtin_ctzll(m));
                ok = ok && (x != y);
            }
            for (uint64_t m = others; m; m &= m - 1) {
                const int32_t y = read_lane32(img_r, __builtin_ctzll(m));
                const int64_t y0 = crp[y], y1 = crp[y + 1];
                if (ok) ok = find_sorted(ccol, y0, y1, x) >= 0;
            }
            if (ok) {
                atomic_or_elem<M>(cert, x, 1ull << q);
                set_bit(a.c_cert, kk);
                for (uint64_t m = others; m; m &= m - 1) {
                    const int32_t y = read_lane32(img_r, __builtin_ctzll(m));
                    const int64_t kj = find_sorted(ccol, crp[y], crp[y + 1], x);
                    if (kj >= 0) set_bit(a.c_cert, kj);
                }
            }
        }
    }
}

// Role counts of the vertices in tasks (one wavefront per vertex; per-wave
// counters in LDS).
template <typename M>
__global__ __launch_bounds__(kSearchBlock) void role_counts_kernel(
    const int32_t *tasks, int64_t n_tasks, const int64_t *c_rp, const int32_t *c_col,
    const M *omega, int n0, uint16_t *rcnt) {
    __shared__ unsigned int acc[kSearchBlock / kWave][kMaxK];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t t = wave; t < n_tasks; t += nwaves) {
        const int32_t v = tasks[t];
        if (lane < kMaxK) acc[wib][lane] = 0;
        __builtin_amdgcn_wave_barrier();
        const int64_t s = c_rp[v], e = c_rp[v + 1];
        for (int64_t k = s + lane; k < e; k += kWave) {
            uint64_t w = (uint64_t)omega[c_col[k]];
            while (w) {
                const int q = __builtin_ctzll(w);
                w &= w - 1;
                atomicAdd(&acc[wib][q], 1u);
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (lane < n0) {
            const unsigned int c = acc[wib][lane];
            rcnt[(int64_t)v * n0 + lane] = (uint16_t)(c > 65535u ? 65535u : c);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

template <typename M>
void launch_role_counts(hipStream_t s, const int32_t *tasks, int64_t n_tasks, const int64_t *c_rp,
                        const int32_t *c_col, const M *omega, int n0, uint16_t *rcnt) {
    if (n_tasks <= 0) return;
    int64_t grid = (n_tasks * kWave + kSearchBlock - 1) / kSearchBlock;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(role_counts_kernel<M>, dim3((unsigned)grid), dim3(kSearchBlock), 0, s,
                       tasks, n_tasks, c_rp, c_col, omega, n0, rcnt);
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
    unsigned long long queries = 0, npos = 0, tpos = 0, tneg = 0;
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
                const uint64_t c0 = wall_clock64();
                const bool found = dfs_search<M>(a, P, om, v, -1, img);
                const uint64_t dt = wall_clock64() - c0;
                if (found) {
                    ++npos;
                    tpos += dt;
                    if (a.mode == 1) {
                        certify_match<M>(a, P, img, sat);
                        if (a.expand) expand_match<M>(a, P, img, om, sat);
                    } else {
                        certify_roles<M>(P, img, sat);
                    }
                } else {
                    tneg += dt;
                }
            }
        }
    }
    if (lane == 0 && queries) {
        atomicAdd(a.n_queries, queries);
        if (a.qstats) {
            atomicAdd(a.qstats + 0, npos);
            atomicAdd(a.qstats + 1, queries - npos);
            atomicAdd(a.qstats + 2, tpos);
            atomicAdd(a.qstats + 3, tneg);
        }
    }
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

// Candidate edges: entries a -> b (a < b) of the compacted subgraph whose
// certified roles are adjacent in G0 and that no found match certified yet.
template <typename M>
__global__ __launch_bounds__(kSearchBlock) void edge_candidates_kernel(
    const int32_t *tasks, int64_t n_tasks, const int64_t *c_rp, const int32_t *c_col,
    const int32_t *c_rev, const M *cert, LccTable tab, const uint64_t *c_cert, int32_t *eu,
    int32_t *ew, int64_t *e_idx, int32_t *n_out, int64_t cap) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t t = wave; t < n_tasks; t += nwaves) {
        const int32_t u = tasks[t];
        const uint64_t cu = (uint64_t)cert[u];
        if (!cu) continue;
        const uint64_t reach = reach_mask<M>(cu, tab);
        const int64_t s = c_rp[u], e = c_rp[u + 1];
        for (int64_t base = s; base < e; base += kWave) {
            const int64_t k = base + lane;
            bool p = false;
            int32_t w = 0;
            if (k < e) {
                w = c_col[k];
                p = w > u && ((uint64_t)cert[w] & reach) != 0ull && !test_bit(c_cert, k) &&
                    !test_bit(c_cert, c_rev[k]);
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
                    e_idx[o] = k;
                }
            }
        }
    }
}

template <typename M>
void launch_edge_candidates(hipStream_t s, const int32_t *tasks, int64_t n_tasks,
                            const int64_t *c_rp, const int32_t *c_col, const int32_t *c_rev,
                            const M *cert, const LccTable &tab, const uint64_t *c_cert,
                            int32_t *eu, int32_t *ew, int64_t *e_idx, int32_t *n_out,
                            int64_t cap) {
    if (n_tasks <= 0) return;
    int64_t grid = (n_tasks * kWave + kSearchBlock - 1) / kSearchBlock;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(edge_candidates_kernel<M>, dim3((unsigned)grid), dim3(kSearchBlock), 0, s,
                       tasks, n_tasks, c_rp, c_col, c_rev, cert, tab, c_cert, eu, ew, e_idx,
                       n_out, cap);
}

template <typename M>
__global__ __launch_bounds__(kSearchBlock) void edge_search_kernel(
    const int32_t *eu, const int32_t *ew, const int64_t *e_idx, int64_t n_edges, const M *om,
    M *cert, const int32_t *edge_plan, int32_t n_edge_plans, SearchArgs a) {
    const int lane = lane_id();
    unsigned long long queries = 0, npos = 0, tpos = 0, tneg = 0;
    for (;;) {
        int t0 = 0;
        if (lane == 0) t0 = atomicAdd(a.task_counter, kTaskChunk);
        t0 = __shfl(t0, 0);
        if ((int64_t)t0 >= n_edges) break;
        const int64_t t1 = (int64_t)t0 + kTaskChunk < n_edges ? (int64_t)t0 + kTaskChunk : n_edges;
        for (int64_t t = t0; t < t1; ++t) {
            const int32_t u = eu[t], w = ew[t];
            const int64_t k = e_idx[t];
            const int64_t kr = a.c_rev[k];
            const uint64_t cu = (uint64_t)om[u], cw = (uint64_t)om[w];
            for (int i = 0; i < n_edge_plans; ++i) {
                if (((load_fresh(a.c_cert + (k >> 6)) >> (k & 63)) & 1ull) ||
                    ((load_fresh(a.c_cert + (kr >> 6)) >> (kr & 63)) & 1ull))
                    break;
                const int pidx = edge_plan[i];
                const SearchPlan *P = a.plans + pidx;
                if (!((cu >> P->pin[0]) & 1ull) || !((cw >> P->pin[1]) & 1ull)) continue;
                int32_t img = 0;
                ++queries;
                const uint64_t c0 = wall_clock64();
                const bool found = dfs_search<M>(a, P, om, u, w, img);
                const uint64_t dt = wall_clock64() - c0;
                if (found) {
                    ++npos;
                    tpos += dt;
                    certify_match<M>(a, P, img, cert);
                    if (a.expand) expand_match<M>(a, P, img, om, cert);
                    break;
                }
                tneg += dt;
            }
        }
    }
    if (lane == 0 && queries) {
        atomicAdd(a.n_queries, queries);
        if (a.qstats) {
            atomicAdd(a.qstats + 4, npos);
            atomicAdd(a.qstats + 5, queries - npos);
            atomicAdd(a.qstats + 6, tpos);
            atomicAdd(a.qstats + 7, tneg);
        }
    }
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

__global__ __launch_bounds__(kSearchBlock) void reverse_index_kernel(
    const int32_t *tasks, int64_t n_tasks, const int64_t *c_rp, const int32_t *c_col,
    int32_t *c_rev) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t t = wave; t < n_tasks; t += nwaves) {
        const int32_t u = tasks[t];
        const int64_t s = c_rp[u], e = c_rp[u + 1];
        for (int64_t k = s + lane; k < e; k += kWave) {
            const int32_t w = c_col[k];
            c_rev[k] = (int32_t)find_sorted(c_col, c_rp[w], c_rp[w + 1], u);
        }
    }
}

void launch_reverse_index(hipStream_t s, const int32_t *tasks, int64_t n_tasks,
                          const int64_t *c_rp, const int32_t *c_col, int32_t *c_rev) {
    if (n_tasks <= 0) return;
    int64_t grid = (n_tasks * kWave + kSearchBlock - 1) / kSearchBlock;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(reverse_index_kernel, dim3((unsigned)grid), dim3(kSearchBlock), 0, s,
                       tasks, n_tasks, c_rp, c_col, c_rev);
}

__global__ __launch_bounds__(kSearchBlock) void edges_from_cert_kernel(
    const int32_t *tasks, int64_t n_tasks, const int64_t *c_rp, const int32_t *c_off,
    const int32_t *c_rev, const int64_t *rp, const uint64_t *c_cert, uint64_t *edge_bits) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t t = wave; t < n_tasks; t += nwaves) {
        const int32_t u = tasks[t];
        const int64_t s = c_rp[u], e = c_rp[u + 1], r0 = rp[u];
        for (int64_t k = s + lane; k < e; k += kWave)
            if (test_bit(c_cert, k) || test_bit(c_cert, c_rev[k])) set_bit(edge_bits, r0 + c_off[k]);
    }
}

void launch_edges_from_cert(hipStream_t s, const int32_t *tasks, int64_t n_tasks,
                            const int64_t *c_rp, const int32_t *c_off, const int32_t *c_rev,
                            const int64_t *rp, const uint64_t *c_cert, uint64_t *edge_bits) {
    if (n_tasks <= 0) return;
    int64_t grid = (n_tasks * kWave + kSearchBlock - 1) / kSearchBlock;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(edges_from_cert_kernel, dim3((unsigned)grid), dim3(kSearchBlock), 0, s,
                       tasks, n_tasks, c_rp, c_off, c_rev, rp, c_cert, edge_bits);
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
                                            const M *, const LccTable &, const uint64_t *,        \
                                            int32_t *, int32_t *, int64_t *, int32_t *, int64_t); \
    template void launch_edge_search<M>(hipStream_t, const int32_t *, const int32_t *,            \
                                        const int64_t *, int64_t, const M *, M *,                 \
                                        const int32_t *, int32_t, const SearchArgs &, int);       \
    template void launch_role_counts<M>(hipStream_t, const int32_t *, int64_t, const int64_t *,   \
                                        const int32_t *, const M *, int, uint16_t *);             \
    template void launch_active_edges<M>(hipStream_t, const int32_t *, int64_t, const int64_t *,  \
                                         const int32_t *, const int32_t *, const int64_t *,       \
                                         const M *, const LccTable &, uint64_t *);

PM_INSTANTIATE_SEARCH(uint8_t)
PM_INSTANTIATE_SEARCH(uint16_t)
PM_INSTANTIATE_SEARCH(uint32_t)
PM_INSTANTIATE_SEARCH(uint64_t)

}  // namespace pm
