// Non-local constraint checking and the exact final step on gfx950.
//
// Every non-local constraint (cycle, path, TDS) asks, for each vertex v and
// head role h, whether the constraint's substructure of G0 embeds
// injectively in the current candidate graph with h at v, every vertex
// taking a role it still holds and every substructure edge on an edge of G
// (NLCC algorithm and visitor: a token walks the constraint; its history
// enforces repeated and distinct identities; work aggregation stops
// duplicate walks).  The walk is realised as a depth-first search run by
// one wavefront per query: at each step the 64 lanes scan 64 candidates from
// the role list of an already placed vertex, test identity and the other
// required edges (binary search in sorted role lists), and ballot the
// survivors; the search descends into the first and backtracks through the
// rest.  All checks of one constraint read the role sets as they were
// before the constraint (all tokens finish before the barrier), so the
// result of a check does not depend on the order of the searches.  A search
// that succeeds certifies every head role on its path at once, which stops
// later searches for those roles (the shared-memory counterpart of work
// aggregation).
//
// Role lists: for every active vertex u and role q, the sorted list of the
// neighbours of u (in the compacted candidate subgraph) whose role set holds
// q.  Scans then touch only candidates of the right role, and an adjacency
// test "x next to y, x in role q" searches only y's q-list.
//
// The final step is the full-template search (Step 5(3) of constraint
// generation, Remark on template-driven search): first from every surviving
// (vertex, role) pair, giving the exact role sets; then from every candidate
// edge not yet covered by a found match, giving the exact edge set.  Every
// match found certifies all its roles and edges, and every single-vertex
// swap of it that is again a match.  An edge-rooted search that runs long
// hands the untried candidates of its shallowest open level to other
// wavefronts (split tasks, searched by the next launch), so one hard query
// does not hold the GPU while a single wavefront works on it.
#include "device_util.h"
#include "pm_internal.h"

namespace pm {

constexpr int kSearchBlock = 256;

__device__ __forceinline__ bool test_bit(const uint64_t *bits, int64_t k) {
    return (bits[k >> 6] >> (k & 63)) & 1ull;
}

template <typename M>
__device__ __forceinline__ uint64_t load_fresh(const M *p) {
    return (uint64_t)__atomic_load_n(p, __ATOMIC_RELAXED);
}


template <typename M>
__device__ __forceinline__ uint64_t reach_mask(uint64_t w, const LccTable &tab) {
    uint64_t r = 0;
    for (int q = 0; q < tab.n0; ++q)
        if ((w >> q) & 1ull) r |= tab.adj[q];
    return r;
}

// ------------------------------------------------------------ role lists
// Pass 1: per (vertex, role) counts, one wavefront per vertex with per-wave
// counters in LDS.
template <typename M>
__global__ __launch_bounds__(kSearchBlock) void role_count_kernel(
    const int32_t *tasks, int64_t n_tasks, const int64_t *c_rp, const int32_t *c_col,
    const M *omega, int n0, int64_t *cnt, int32_t *pos_of) {
    __shared__ unsigned int acc[kSearchBlock / kWave][kMaxK];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t t = wave; t < n_tasks; t += nwaves) {
        const int32_t v = tasks[t];
        acc[wib][lane] = 0;
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
        if (lane < n0) cnt[t * n0 + lane] = acc[wib][lane];
        if (lane == 0) pos_of[v] = (int32_t)t;
        __builtin_amdgcn_wave_barrier();
    }
}

// Pass 2: fill the lists in row order (so each list is sorted), one ballot
// per role and 64-entry chunk; lane q keeps the write cursor of role q.
// rl_ent receives the compacted entry index of every list entry.
template <typename M>
__global__ __launch_bounds__(kSearchBlock) void role_fill_kernel(
    const int32_t *tasks, int64_t n_tasks, const int64_t *c_rp, const int32_t *c_col,
    const M *omega, int n0, const int64_t *rl_off, int32_t *rl_col, int32_t *rl_ent) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t t = wave; t < n_tasks; t += nwaves) {
        const int32_t v = tasks[t];
        int64_t run = lane < n0 ? rl_off[t * n0 + lane] : 0;
        const int64_t s = c_rp[v], e = c_rp[v + 1];
        for (int64_t base = s; base < e; base += kWave) {
            const int64_t k = base + lane;
            const int32_t w = k < e ? c_col[k] : -1;
            const uint64_t bits = k < e ? (uint64_t)omega[w] : 0ull;
            for (int q = 0; q < n0; ++q) {
                const bool has = (bits >> q) & 1ull;
                const uint64_t m = ballot64(has);
                if (!m) continue;
                const int64_t at = read_lane64(run, q);
                if (has) {
                    const int64_t o = at + __popcll(m & lanemask_lt());
                    rl_col[o] = w;
                    rl_ent[o] = (int32_t)k;
                }
                if (lane == q) run += __popcll(m);
            }
        }
    }
}

template <typename M>
void launch_role_count(hipStream_t s, const int32_t *tasks, int64_t n_tasks, const int64_t *c_rp,
                       const int32_t *c_col, const M *omega, int n0, int64_t *cnt,
                       int32_t *pos_of) {
    if (n_tasks <= 0) return;
    int64_t grid = (n_tasks * kWave + kSearchBlock - 1) / kSearchBlock;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(role_count_kernel<M>, dim3((unsigned)grid), dim3(kSearchBlock), 0, s,
                       tasks, n_tasks, c_rp, c_col, omega, n0, cnt, pos_of);
}

template <typename M>
void launch_role_fill(hipStream_t s, const int32_t *tasks, int64_t n_tasks, const int64_t *c_rp,
                      const int32_t *c_col, const M *omega, int n0, const int64_t *rl_off,
                      int32_t *rl_col, int32_t *rl_ent) {
    if (n_tasks <= 0) return;
    int64_t grid = (n_tasks * kWave + kSearchBlock - 1) / kSearchBlock;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(role_fill_kernel<M>, dim3((unsigned)grid), dim3(kSearchBlock), 0, s,
                       tasks, n_tasks, c_rp, c_col, omega, n0, rl_off, rl_col, rl_ent);
}

// Per-vertex copy of the list bounds: rl_v[v * (n0 + 1) + q] = start of
// v's role-q list (q = n0: end of its last list), so a search reaches a
// vertex's lists from its id without the task-position lookup.
__global__ __launch_bounds__(kSearchBlock) void role_rows_kernel(const int32_t *tasks,
                                                                 int64_t n_tasks, int n0,
                                                                 const int64_t *rl_off,
                                                                 int32_t *rl_v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w = n0 + 1;
    if (i >= n_tasks * w) return;
    const int64_t t = i / w;
    const int64_t q = i - t * w;
    rl_v[(int64_t)tasks[t] * w + q] = (int32_t)rl_off[t * n0 + q];
}

void launch_role_rows(hipStream_t s, const int32_t *tasks, int64_t n_tasks, int n0,
                      const int64_t *rl_off, int32_t *rl_v) {
    const int64_t total = n_tasks * (n0 + 1);
    if (total <= 0) return;
    hipLaunchKernelGGL(role_rows_kernel, dim3((unsigned)((total + kSearchBlock - 1) / kSearchBlock)),
                       dim3(kSearchBlock), 0, s, tasks, n_tasks, n0, rl_off, rl_v);
}

// ----------------------------------------------------- sorted-list search
// Membership of each lane's key x in one sorted list col[lo, hi) shared by
// the whole wavefront (all lanes call with the same bounds; lanes with
// !want get -1).  One coalesced load fetches 64 evenly spaced samples of
// the list (the whole list when it is at most 64 long); each lane finds its
// segment among them through lane shuffles and finishes with a binary
// search of that segment only, so a list of length L costs one load plus
// log2(L / 64) dependent loads instead of log2(L).  Returns the position of
// x or -1.
__device__ __forceinline__ int64_t wave_find(const int32_t *__restrict__ col, int64_t lo,
                                             int64_t hi, int32_t x, bool want) {
    const int lane = lane_id();
    const int64_t len = hi - lo;
    if (len <= 0) return -1;
    const bool small = len <= kWave;
    const int64_t sp = small ? lo + lane : lo + ((len * lane) >> 6);
    const int32_t sv = (!small || lane < len) ? col[sp] : INT32_MAX;
    // largest sample index i with sample_i <= x (upper bound - 1); samples
    // are non-decreasing over the lanes
    int lo_i = 0, cnt = kWave;
#pragma unroll
    for (int st = 0; st < 6; ++st) {
        const int half = cnt >> 1;
        const int mid = lo_i + half;
        const int32_t mv = __shfl(sv, mid);
        if (mv <= x) {
            lo_i = mid;
            cnt -= half;
        } else {
            cnt = half;
        }
    }
    // lo_i: the last sample <= x, or 0 with sample_0 > x
    // every lane takes part in the shuffles before any lane leaves
    const int32_t v0 = __shfl(sv, lo_i);
    const int64_t p0 = __shfl(sp, lo_i);
    const int64_t p1 = __shfl(sp, lo_i + 1 < kWave ? lo_i + 1 : lo_i);
    if (!want || v0 > x) return -1;
    if (v0 == x) return p0;
    if (small) return -1;
    return find_sorted(col, p0 + 1, lo_i == kWave - 1 ? hi : p1, x);
}

// ---------------------------------------------------------------- search
// Every vertex a search reaches holds a role, so it is in the task list the
// role lists were built from and has a list position.
__device__ __forceinline__ int64_t rl_begin(const SearchArgs &a, int32_t y, int q) {
    return a.rl_v[(int64_t)y * (a.n0 + 1) + q];
}
__device__ __forceinline__ int64_t rl_end(const SearchArgs &a, int32_t y, int q) {
    return a.rl_v[(int64_t)y * (a.n0 + 1) + q + 1];
}

// Depth-first search for an embedding of plan P's substructure with the
// pinned template vertices at v0 (and v1).  Lane-distributed state: lane q
// holds the image of template vertex q and the start of that image's row of
// role-list offsets (rb_r); lane l holds the scan state of search level l
// (the template vertex it places, the placed neighbour whose role list it
// scans, the list cursor and the ballot of surviving candidates of the
// current 64-entry chunk).  At each new level the unplaced vertex with the
// shortest candidate list is placed next (the paper's constraint
// optimisation visits rare labels first; here the choice is made per
// partial match from exact list lengths): every open template vertex's lane
// reads its list lengths under the placed neighbours in parallel and a
// wavefront minimum picks the shortest (ties: lowest vertex, then lowest
// neighbour).
//
// With rt set the search is a split task: rt's prefix vertices are placed
// as well and the first level scans rt's candidate range.  With `split`,
// every a.split_budget steps (chunk scans and descents) the search hands
// the untried candidates of its shallowest open level -- the largest
// subtrees left -- to other wavefronts as split tasks (the vertices placed
// above that level, and a piece of its candidate range) and carries on
// with the rest.  The handed-on pieces and what the search keeps partition
// its tree, so together they find a match if there is one; a miss here
// only says that this search's own part holds none.
//
// Counting mode (kCount, match counting and enumeration): the search does
// not stop at a match.  At the last level every candidate that passes the
// checks completes a match; their number is added to cs->n (and their maps
// written to cs->maps while room is left) instead of descending into them,
// and the search ends when its tree is exhausted.  Splitting partitions the
// tree in this mode too, so every map is counted exactly once.
enum { kSearchMiss = 0, kSearchFound = 1 };

struct CountSink {
    unsigned long long n = 0;           // maps counted by this wavefront, not yet added
    int32_t *maps = nullptr;            // [cap][n0] or null
    int64_t cap = 0;
    unsigned long long *written = nullptr;
    unsigned long long *total = nullptr;   // device total of all wavefronts
    unsigned long long limit = 0;       // > 0: stop every search once total >= limit
    int32_t *stop = nullptr;            // set when the limit is reached
    int since = 0;
};

// Counting with a limit: every kCountPoll steps the wavefront adds its
// count to the total and polls the stop flag.  Returns true to stop.
constexpr int kCountPoll = 1024;
__device__ __forceinline__ bool count_poll(CountSink *cs) {
    if (!cs->limit || ++cs->since < kCountPoll) return false;
    cs->since = 0;
    int st = 0;
    if (lane_id() == 0) {
        const unsigned long long before = atomicAdd(cs->total, cs->n);
        if (before + cs->n >= cs->limit) atomicExch(cs->stop, 1);
        st = __hip_atomic_load(cs->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    cs->n = 0;
    return __shfl(st, 0) != 0;
}

// Write the maps completed at the last level: the placed images, with
// template vertex q at each passing candidate x.
__device__ __forceinline__ void emit_maps(const SearchArgs &a, CountSink *cs, int32_t img_r,
                                          int q, int32_t x, bool ok, uint64_t b) {
    const int lane = lane_id();
    unsigned long long at = 0;
    if (lane == 0) at = atomicAdd(cs->written, (unsigned long long)__popcll(b));
    at = __shfl(at, 0);
    if ((int64_t)at >= cs->cap) return;
    const int64_t o = (int64_t)at + __popcll(b & lanemask_lt());
    const bool w = ok && o < cs->cap;
    for (int p = 0; p < a.n0; ++p) {
        const int32_t y = read_lane32(img_r, p);
        if (w) cs->maps[o * a.n0 + p] = p == q ? x : y;
    }
}

template <typename M, bool kCount = false>
__device__ int dfs_search(const SearchArgs &a, const SearchPlan *__restrict__ P,
                          const M *__restrict__ om, int32_t v0, int32_t v1,
                          const SplitTask *__restrict__ rt, int64_t task, int plan, bool split,
                          int32_t &img_r, int32_t &rb_r, CountSink *cs = nullptr) {
    const int lane = lane_id();
    const int k = P->k;
    const int npin = P->npin;
    const uint64_t vmask = P->vmask;
    const int p0 = P->pin[0], p1 = P->pin[1];
    img_r = lane == p0 ? v0 : ((npin == 2 && lane == p1) ? v1 : -1);
    uint64_t placed = (1ull << p0) | (npin == 2 ? (1ull << p1) : 0ull);
    const int rt_np = rt ? (int)rt->np : 0;
    for (int i = 0; i < rt_np; ++i) {
        const int q = rt->pq[i];
        if (lane == q) img_r = rt->px[i];
        placed |= 1ull << q;
    }
    rb_r = img_r >= 0 ? img_r : 0;
    const int base_lvl = npin + rt_np;
    if (!rt && k <= npin) {
        if constexpr (kCount) {
            cs->n += 1;
            if (cs->maps) emit_maps(a, cs, img_r, -1, 0, lane == 0, 1ull);
        }
        return kSearchFound;
    }
    const int32_t *__restrict__ rlc = a.rl_col;
    // role-list bounds of vertex x: rlv[x * (n0 + 1) + q .. + q + 1]
    const int32_t *__restrict__ rlv = a.rl_v;
    const int64_t stride = a.n0 + 1;
    // role-list positions fit in 32 bits (checked when the lists are built)
    int32_t cur_r = 0, end_r = 0, base_r = 0;
    uint64_t pend_r = 0;
    int32_t pv_r = 0, par_r = 0;

    auto select = [&](int l) {
        const uint64_t nbr = ((vmask & ~placed) >> lane) & 1ull ? (P->adj[lane] & placed) : 0ull;
        uint64_t key = ~0ull;
        for (uint64_t mj = placed; mj; mj &= mj - 1) {
            const int j = __builtin_ctzll(mj);
            const int64_t rowj = (int64_t)read_lane32(rb_r, j) * stride;
            if ((nbr >> j) & 1ull) {
                const int64_t len = rlv[rowj + lane + 1] - rlv[rowj + lane];
                const uint64_t kv = ((uint64_t)len << 12) | ((uint64_t)lane << 6) | (uint64_t)j;
                if (kv < key) key = kv;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t o = shfl_xor_u64(key, off, kWave);
            if (o < key) key = o;
        }
        int bp = 0, bj = 0;
        int32_t bb = 0, be = 0;
        if (key != ~0ull) {
            bp = (int)((key >> 6) & 63ull);
            bj = (int)(key & 63ull);
            bb = rlv[(int64_t)read_lane32(rb_r, bj) * stride + bp];
            be = bb + (int32_t)(key >> 12);
        }
        if (lane == l) {
            cur_r = bb;
            end_r = be;
            pend_r = 0;
            pv_r = bp;
            par_r = bj;
        }
    };

    // Hand on the rest of the shallowest level l < lvl that still has
    // candidates to try, cut into up to kSplitPieces tasks of near-equal
    // length, and drop it from this search.  Only levels above the current
    // one qualify: their placed candidate's subtree stays here, so every
    // handed-on task covers strictly less than this search (a search never
    // hands on all of its own work, and the rounds of split tasks end).
    // Returns false if nothing could be handed on for want of room.
    auto hand_off = [&](int lvl) -> bool {
        int l = base_lvl;
        int32_t r0 = 0, len = 0;
        for (; l < lvl; ++l) {
            const uint64_t pend = read_lane_u64(pend_r, l);
            r0 = pend ? read_lane32(base_r, l) + __builtin_ctzll(pend) : read_lane32(cur_r, l);
            len = read_lane32(end_r, l) - r0;
            if (len > 0) break;
        }
        if (l >= lvl) return true;      // nothing left above the current level
        const int np = rt_np + (l - base_lvl);
        if (np > kSplitPrefix) return false;
        const int pieces = len < kSplitPieces ? len : kSplitPieces;
        int32_t first = -1;
        if (lane == 0) {
            int32_t old = __hip_atomic_load(a.split_n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (;;) {
                if ((int64_t)old + pieces > a.split_cap) break;
                const int32_t prev = atomicCAS(a.split_n, old, old + pieces);
                if (prev == old) {
                    first = old;
                    break;
                }
                old = prev;
            }
        }
        first = __shfl(first, 0);
        if (first < 0) return false;
        const int qv = read_lane32(pv_r, l), pv = read_lane32(par_r, l);
        // lane i < np: prefix vertex i (the task's own prefix, then the
        // vertices placed at levels base_lvl .. l-1) and its image
        int pq_l = 0;
        if (lane < rt_np) pq_l = rt->pq[lane];
        for (int i = rt_np; i < np; ++i) {
            const int q = read_lane32(pv_r, base_lvl + (i - rt_np));
            if (lane == i) pq_l = q;
        }
        const int32_t px_l = __shfl(img_r, pq_l);
        for (int p = 0; p < pieces; ++p) {
            SplitTask *o = a.split_out + first + p;
            if (lane == 0) {
                o->t = task;
                o->r0 = r0 + (int32_t)((int64_t)len * p / pieces);
                o->r1 = r0 + (int32_t)((int64_t)len * (p + 1) / pieces);
                o->plan = (int16_t)plan;
                o->q = (uint8_t)qv;
                o->par = (uint8_t)pv;
                o->np = (uint8_t)np;
            }
            if (lane < np) {
                o->pq[lane] = (uint8_t)pq_l;
                o->px[lane] = px_l;
            }
        }
        if (lane == l) {
            pend_r = 0;
            cur_r = end_r;
        }
        return true;
    };

    int lvl = base_lvl;
    if (rt) {
        if (lane == lvl) {
            cur_r = rt->r0;
            end_r = rt->r1;
            pend_r = 0;
            pv_r = rt->q;
            par_r = rt->par;
        }
    } else {
        select(lvl);
    }
    int64_t steps = 0;
    for (;;) {
        if constexpr (kCount) {
            if (count_poll(cs)) return kSearchMiss;
        }
        if (split && ++steps > a.split_budget) {
            steps = 0;
            split = hand_off(lvl);
        }
        uint64_t pend = read_lane_u64(pend_r, lvl);
        if (pend == 0) {
            const int32_t cur = read_lane32(cur_r, lvl);
            const int32_t end = read_lane32(end_r, lvl);
            if (cur >= end) {
                if (--lvl < base_lvl) return kSearchMiss;
                placed &= ~(1ull << read_lane32(pv_r, lvl));
                continue;
            }
            const int q = read_lane32(pv_r, lvl);
            const int par = read_lane32(par_r, lvl);
            const uint64_t same = P->samelab[q] & placed;
            const uint64_t back = P->adj[q] & placed & ~(1ull << par);
            const int32_t kk = cur + lane;
            const bool in_range = kk < end;
            const int32_t x = in_range ? rlc[kk] : -1;
            bool ok = in_range && (!a.check_om || (((uint64_t)om[x] >> q) & 1ull));
            for (uint64_t m = same; m; m &= m - 1) {
                const int32_t y = read_lane32(img_r, __builtin_ctzll(m));
                ok = ok && (y != x);
            }
            for (uint64_t m = back; m; m &= m - 1) {
                if (!ballot64(ok)) break;
                const int64_t rowj = (int64_t)read_lane32(rb_r, __builtin_ctzll(m)) * stride;
                ok = wave_find(rlc, rlv[rowj + q], rlv[rowj + q + 1], x, ok) >= 0;
            }
            const uint64_t b = ballot64(ok);
            if constexpr (kCount) {
                if (lvl == k - 1) {
                    // every passing candidate completes a map
                    cs->n += (unsigned long long)__popcll(b);
                    if (cs->maps && b) emit_maps(a, cs, img_r, q, x, ok, b);
                    if (lane == lvl) cur_r = cur + kWave;
                    continue;
                }
            }
            if (lane == lvl) {
                pend_r = b;
                base_r = cur;
                cur_r = cur + kWave;
            }
            continue;
        }
        const int j = __builtin_ctzll(pend);
        pend &= pend - 1;
        const int32_t base = read_lane32(base_r, lvl);
        const int32_t x = rlc[base + j];
        const int q = read_lane32(pv_r, lvl);
        if (lane == lvl) pend_r = pend;
        if (lane == q) {
            img_r = x;
            rb_r = x;
        }
        placed |= 1ull << q;
        if (lvl == k - 1) return kSearchFound;
        ++lvl;
        select(lvl);
    }
}

// Certify the head roles of a found embedding (NLCC); with work aggregation
// off, only the root's role.
template <typename M>
__device__ void certify_roles(const SearchArgs &a, const SearchPlan *__restrict__ P,
                              int32_t img_r, M *sat) {
    const int lane = lane_id();
    const bool mine = a.aggregate ? (((P->vmask >> lane) & 1ull) && ((P->certify >> lane) & 1ull))
                                  : lane == P->pin[0];
    if (mine) atomic_or_elem<M>(sat, img_r, 1ull << lane);
}

// An edge is certified through the bit of either of its two compacted
// entries (certify_match uses the one from the smaller to the larger vertex
// id; swaps use the entry whose position they already hold).  By default a
// plain atomic without a return value, which the wavefront does not wait
// for; with a.read_first the word is read first (workgroup scope, may be
// stale: a stale read only costs a redundant atomic) and the atomic skipped
// when the bit is already set -- fewer atomics, but a load to wait for.
template <typename M>
__device__ __forceinline__ uint64_t load_hint(const M *p) {
    return (uint64_t)__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void set_entry(const SearchArgs &a, int64_t rl_index) {
    const int64_t e = a.rl_ent[rl_index];
    if (a.read_first && ((load_hint(a.c_cert + (e >> 6)) >> (e & 63)) & 1ull)) return;
    set_bit(a.c_cert, e);
}

template <typename M>
__device__ __forceinline__ void certify_role(const SearchArgs &a, M *cert, int32_t x, int q) {
    if (a.read_first && ((load_hint(cert + x) >> q) & 1ull)) return;
    atomic_or_elem<M>(cert, x, 1ull << q);
}

// Certify edge {u, w} where u holds role qu and w role qw in the match: the
// entry min -> max is found in the role list of the smaller vertex for the
// role of the larger.
__device__ __forceinline__ void certify_pair(const SearchArgs &a, int32_t u, int qu, int32_t w,
                                             int qw) {
    if (u > w) {
        const int32_t t = u; u = w; w = t;
        const int tq = qu; qu = qw; qw = tq;
    }
    const int64_t p = find_sorted(a.rl_col, rl_begin(a, u, qw), rl_end(a, u, qw), w);
    if (p >= 0) set_entry(a, p);
}

// Record the match (images img_r, with x in place of template vertex q
// when q >= 0) as the witness of (lane's vertex, lane's role) for every
// lane with `claim` whose (vertex, role) has none yet.
// pos_v: the role-list position of the witnessed vertex (loaded by the
// caller, early, so that its latency overlaps the caller's other loads).
__device__ void record_witness(const SearchArgs &a, uint64_t vmask, int32_t img_r, bool claim,
                               int32_t pos_v, int role, int q, int32_t x) {
    const int64_t idx = (int64_t)pos_v * a.n0 + role;
    if (claim) claim = atomicCAS(a.wit_flag + idx, 0u, 1u) == 0u;
    for (uint64_t m = vmask; m; m &= m - 1) {
        const int p = __builtin_ctzll(m);
        const int32_t y = p == q ? x : read_lane32(img_r, p);
        if (claim) a.wit[idx * a.n0 + p] = y;
    }
}

// Certify a full match: every role and every template edge.
template <typename M>
__device__ void certify_match(const SearchArgs &a, const SearchPlan *__restrict__ P,
                              int32_t img_r, M *cert) {
    const int lane = lane_id();
    if ((P->vmask >> lane) & 1ull) atomic_or_elem<M>(cert, img_r, 1ull << lane);
    if (a.wit_on) {
        const bool mine = (P->vmask >> lane) & 1ull;
        record_witness(a, P->vmask, img_r, mine, mine ? a.rl_pos[img_r] : 0, lane, -1, 0);
    }
    for (int base = 0; base < a.m0; base += kWave) {
        const int i = base + lane;
        int ta = 0, tb = 0;
        if (i < a.m0) {
            ta = a.tedges[2 * i];
            tb = a.tedges[2 * i + 1];
        }
        const int32_t u = __shfl(img_r, ta);
        const int32_t w = __shfl(img_r, tb);
        if (i < a.m0) certify_pair(a, u, ta, w, tb);
    }
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Single-vertex swaps of a found match: for each template vertex q, every x
// that can replace phi(q) with all other images fixed (role q, adjacent to
// the images of all template neighbours of q, distinct from the images of
// same-label vertices) gives another match, whose role (x, q) and edges at
// x are certified.  Purely a saving: anything it misses is queried later.
// The candidates depend (up to the identity checks) only on q and the
// images of q's template neighbours, so each such key is scanned once: a
// hash of the key is exchanged into a table, and a scan whose hash is
// already there is skipped (a collision or an overwritten slot only skips
// or repeats a scan, neither of which affects the result).
struct ExpandCount {
    unsigned long long scans = 0, cands = 0, valid = 0;
};

template <typename M>
__device__ void expand_match(const SearchArgs &a, const SearchPlan *__restrict__ P,
                             int32_t img_r, int32_t rb_r, const M *__restrict__ om, M *cert,
                             ExpandCount &ec) {
    const int lane = lane_id();
    const int32_t *__restrict__ rlc = a.rl_col;
    for (uint64_t mq = P->vmask; mq; mq &= mq - 1) {
        const int q = __builtin_ctzll(mq);
        const uint64_t nb = P->adj[q];
        if (!nb) continue;
        // lane j (a template neighbour of q) holds the bounds of the q-list
        // of its image
        int32_t lb_r = 0, le_r = 0;
        if ((nb >> lane) & 1ull) {
            const int64_t row = (int64_t)rb_r * (a.n0 + 1);
            lb_r = a.rl_v[row + q];
            le_r = a.rl_v[row + q + 1];
        }
        // scan the shortest list; test the others shortest first (the most
        // selective), at most kOrd of them in that order, the rest by index
        constexpr int kOrd = 10;
        int js = -1;
        int64_t bd = INT64_MAX;
        for (uint64_t m = nb; m; m &= m - 1) {
            const int j = __builtin_ctzll(m);
            const int64_t len = read_lane32(le_r, j) - read_lane32(lb_r, j);
            if (len < bd) {
                bd = len;
                js = j;
            }
        }
        const int32_t s = read_lane32(lb_r, js), e = read_lane32(le_r, js);
        if (e - s > a.expand_max) continue;
        {
            uint64_t h = mix64((uint64_t)q + 1ull);
            for (uint64_t m = nb; m; m &= m - 1)
                h = mix64(h ^ (uint64_t)(uint32_t)read_lane32(img_r, __builtin_ctzll(m)));
            h |= 1ull;
            unsigned long long old = 0;
            if (lane == 0) old = atomicExch(a.exp_seen + (h >> (64 - a.exp_log2)),
                                            (unsigned long long)h);
            old = __shfl(old, 0);
            if (old == h) continue;
        }
        uint64_t rest = nb & ~(1ull << js);
        uint64_t ordc = 0;
        int nord = 0;
        while (rest && nord < kOrd) {
            int bj = -1;
            int64_t bl = INT64_MAX;
            for (uint64_t m = rest; m; m &= m - 1) {
                const int j = __builtin_ctzll(m);
                const int64_t len = read_lane32(le_r, j) - read_lane32(lb_r, j);
                if (len < bl) {
                    bl = len;
                    bj = j;
                }
            }
            ordc |= (uint64_t)bj << (6 * nord);
            ++nord;
            rest &= ~(1ull << bj);
        }
        const uint64_t same = P->samelab[q];
        ++ec.scans;
        ec.cands += (unsigned long long)(e - s);
        for (int32_t base = s; base < e; base += kWave) {
            const int32_t kk = base + lane;
            const bool in = kk < e;
            const int32_t x = in ? rlc[kk] : -1;
            // x's list position for its witness, loaded before the tests
            const int32_t px = (a.wit_on && in) ? a.rl_pos[x] : 0;
            bool ok = in && (!a.check_om || (((uint64_t)om[x] >> q) & 1ull));
            for (uint64_t m = same; m; m &= m - 1) {
                const int32_t y = read_lane32(img_r, __builtin_ctzll(m));
                ok = ok && (x != y);
            }
            // adjacency to the other neighbours' images; positions kept for
            // the first three (certification of entries y -> x, y < x)
            int32_t p0 = -1, p1 = -1, p2 = -1;
            for (int i = 0; i < nord; ++i) {
                if (!ballot64(ok)) break;
                const int j = (int)((ordc >> (6 * i)) & 63ull);
                const int32_t y0 = read_lane32(lb_r, j), y1 = read_lane32(le_r, j);
                const int32_t p = (int32_t)wave_find(rlc, y0, y1, x, ok);
                ok = p >= 0;
                if (i == 0) p0 = p;
                else if (i == 1) p1 = p;
                else if (i == 2) p2 = p;
            }
            for (uint64_t m = rest; m; m &= m - 1) {
                if (!ballot64(ok)) break;
                const int j = __builtin_ctzll(m);
                const int32_t y0 = read_lane32(lb_r, j), y1 = read_lane32(le_r, j);
                ok = wave_find(rlc, y0, y1, x, ok) >= 0;
            }
            ec.valid += (unsigned long long)__popcll(ballot64(ok));
            if (a.wit_on) record_witness(a, P->vmask, img_r, ok, px, q, q, x);
            if (ok) {
                certify_role<M>(a, cert, x, q);
                // every edge at x is certified through its entry y -> x in
                // y's list of role-q vertices: the scanned list holds it at
                // kk, the tested lists at the positions found above
                set_entry(a, kk);
                for (int i = 0; i < nord; ++i) {
                    const int j = (int)((ordc >> (6 * i)) & 63ull);
                    int64_t p = i == 0 ? p0 : (i == 1 ? p1 : (i == 2 ? p2 : -1));
                    if (p < 0)
                        p = find_sorted(rlc, read_lane32(lb_r, j), read_lane32(le_r, j), x);
                    if (p >= 0) set_entry(a, p);
                }
                for (uint64_t m = rest; m; m &= m - 1) {
                    const int j = __builtin_ctzll(m);
                    const int64_t p =
                        find_sorted(rlc, read_lane32(lb_r, j), read_lane32(le_r, j), x);
                    if (p >= 0) set_entry(a, p);
                }
            }
        }
    }
}

template <typename M>
__global__ __launch_bounds__(kSearchBlock) void vertex_search_kernel(const int32_t *tasks,
                                                                     int64_t n_tasks, const M *om,
                                                                     M *sat, SearchArgs a) {
    const int lane = lane_id();
    unsigned long long queries = 0, npos = 0, tpos = 0, tneg = 0, tcert = 0, texp = 0;
    ExpandCount ec;
    for (;;) {
        int t0 = 0;
        if (lane == 0) t0 = atomicAdd(a.task_counter, a.task_chunk);
        t0 = __shfl(t0, 0);
        if ((int64_t)t0 >= n_tasks) break;
        const int64_t t1 = (int64_t)t0 + a.task_chunk < n_tasks ? (int64_t)t0 + a.task_chunk : n_tasks;
        for (int64_t t = t0; t < t1; ++t) {
            const int32_t v = tasks[t];
            uint64_t cand = (uint64_t)om[v] & a.heads & ~load_fresh(sat + v);
            while (cand) {
                const int h = __builtin_ctzll(cand);
                cand &= cand - 1;
                if ((load_fresh(sat + v) >> h) & 1ull) continue;
                const SearchPlan *P = a.plans + a.plan_of_head[h];
                int32_t img = 0;
                int32_t rb = 0;
                ++queries;
                const uint64_t c0 = wall_clock64();
                const bool found =
                    dfs_search<M>(a, P, om, v, -1, nullptr, 0, 0, false, img, rb) == kSearchFound;
                const uint64_t c1 = wall_clock64();
                if (found) {
                    ++npos;
                    tpos += c1 - c0;
                    if (a.mode == 1 && !a.aggregate) {
                        if (lane == h) atomic_or_elem<M>(sat, img, 1ull << h);
                    } else if (a.mode == 1) {
                        certify_match<M>(a, P, img, sat);
                        if (a.expand) {
                            const uint64_t c2 = wall_clock64();
                            expand_match<M>(a, P, img, rb, om, sat, ec);
                            texp += wall_clock64() - c2;
                        }
                    } else {
                        certify_roles<M>(a, P, img, sat);
                    }
                    tcert += wall_clock64() - c1;
                } else {
                    tneg += c1 - c0;
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
            atomicAdd(a.qstats + 8, tcert);
            atomicAdd(a.qstats + 10, texp);
            atomicAdd(a.qstats + 11, ec.scans);
            atomicAdd(a.qstats + 12, ec.cands);
            atomicAdd(a.qstats + 13, ec.valid);
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
    const uint64_t b = ballot64(ch);
    if (b && lane_id() == 0) atomicAdd(changed, (int32_t)__popcll(b));
}

template <typename M>
void launch_apply(hipStream_t s, const int32_t *tasks, int64_t n_tasks, M *omega, M *sat,
                  uint64_t heads, int32_t *changed) {
    if (n_tasks <= 0) return;
    hipLaunchKernelGGL(apply_kernel<M>, dim3((unsigned)((n_tasks + 255) / 256)), dim3(256), 0, s,
                       tasks, n_tasks, omega, sat, heads, changed);
}

// ------------------------------------------------ exact step: edge part
// Does the witness of (v, qv) stay a match when template vertex qx moves to
// x?  x holds role qx and is adjacent to v; it must differ from the other
// images and be adjacent to the images of qx's other template neighbours.
__device__ bool try_swap(const SearchArgs &a, const LccTable &tab, int32_t v, int qv, int32_t x,
                         int qx) {
    const int64_t idx = (int64_t)a.rl_pos[v] * a.n0 + qv;
    if (!__atomic_load_n(a.wit_flag + idx, __ATOMIC_RELAXED)) return false;
    const int32_t *W = a.wit + idx * a.n0;
    if (W[qx] == x) return true;
    for (int p = 0; p < a.n0; ++p)
        if (p != qx && W[p] == x) return false;
    for (uint64_t m = tab.adj[qx] & ~(1ull << qv); m; m &= m - 1) {
        const int p = __builtin_ctzll(m);
        const int32_t y = W[p];
        if (find_sorted(a.rl_col, rl_begin(a, y, qx), rl_end(a, y, qx), x) < 0) return false;
    }
    return true;
}

// Some match uses edge {u, w}: a recorded witness of u or w becomes one by
// moving a single template vertex onto the other end.
__device__ bool witness_swap(const SearchArgs &a, const LccTable &tab, uint64_t cu, uint64_t cw,
                             int32_t u, int32_t w) {
    for (int i = 0; i < a.m0; ++i) {
        const int ta = a.tedges[2 * i], tb = a.tedges[2 * i + 1];
        for (int o = 0; o < 2; ++o) {
            const int qa = o ? tb : ta, qb = o ? ta : tb;
            if (!((cu >> qa) & 1ull) || !((cw >> qb) & 1ull)) continue;
            if (try_swap(a, tab, u, qa, w, qb)) return true;
            if (try_swap(a, tab, w, qb, u, qa)) return true;
        }
    }
    return false;
}

// Some match uses edge {u, w} through a bridge of G0: the recorded witness
// of (u, qa) on qa's side of bridge (qa, qb), that of (w, qb) on the other
// side, and the edge between them form a match unless a vertex of one side
// and one of the same label on the other side share an image (every edge
// of G0 lies within one side or is the bridge itself, so it is kept).
__device__ bool join_at(const SearchArgs &a, int32_t u, int qa, int32_t w, int qb,
                        uint64_t side_u) {
    const int64_t iu = (int64_t)a.rl_pos[u] * a.n0 + qa;
    const int64_t iw = (int64_t)a.rl_pos[w] * a.n0 + qb;
    if (!__atomic_load_n(a.wit_flag + iu, __ATOMIC_RELAXED) ||
        !__atomic_load_n(a.wit_flag + iw, __ATOMIC_RELAXED))
        return false;
    const int32_t *Wu = a.wit + iu * a.n0;
    const int32_t *Ww = a.wit + iw * a.n0;
    for (uint64_t m = side_u; m; m &= m - 1) {
        const int p = __builtin_ctzll(m);
        const uint64_t other = a.tsame[p] & ~side_u;
        if (!other) continue;
        const int32_t x = Wu[p];
        for (uint64_t mo = other; mo; mo &= mo - 1)
            if (Ww[__builtin_ctzll(mo)] == x) return false;
    }
    return true;
}

__device__ bool witness_join(const SearchArgs &a, uint64_t cu, uint64_t cw, int32_t u,
                             int32_t w, uint64_t vmask) {
    for (int i = 0; i < a.m0; ++i) {
        const uint64_t side = a.tside[i];
        if (!side) continue;
        const int ta = a.tedges[2 * i], tb = a.tedges[2 * i + 1];
        if (((cu >> ta) & 1ull) && ((cw >> tb) & 1ull) && join_at(a, u, ta, w, tb, side))
            return true;
        if (((cu >> tb) & 1ull) && ((cw >> ta) & 1ull) && join_at(a, u, tb, w, ta, vmask & ~side))
            return true;
    }
    return false;
}

// Candidate edges: entries a -> b (a < b) of the compacted subgraph whose
// certified roles are adjacent in G0 and that no found match certified yet
// (neither the bit of this entry nor that of its reverse b -> a is set; the
// reverse entry's index goes with the task, e_idx holding both); those a
// witness swap or a witness join across a bridge of G0 certifies are
// certified here instead.  One thread per
// compacted entry (c_own gives its row), so hub rows do not serialise on
// one wavefront.
template <typename M>
__global__ __launch_bounds__(kSearchBlock) void edge_candidates_kernel(
    int64_t c_m, const int64_t *__restrict__ c_rp, const int32_t *__restrict__ c_own,
    const int32_t *__restrict__ c_col, const M *cert, LccTable tab, uint64_t *c_cert, int32_t *eu,
    int32_t *ew, int64_t *e_idx, int32_t *n_out, int64_t cap, SearchArgs a) {
    const int lane = lane_id();
    unsigned long long swapped = 0, joined = 0;
    const uint64_t vmask = a.n0 == 64 ? ~0ull : ((1ull << a.n0) - 1ull);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // the loop bound is uniform over the block, so ballots see every lane
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < c_m; base += stride) {
        const int64_t k = base + threadIdx.x;
        bool p = false;
        int32_t u = 0, w = 0;
        int64_t kr = -1;
        if (k < c_m) {
            u = c_own[k];
            w = c_col[k];
            if (w > u) {
                const uint64_t cu = (uint64_t)cert[u];
                const uint64_t cw = cu ? (uint64_t)cert[w] : 0ull;
                p = cw != 0ull && (cw & reach_mask<M>(cu, tab)) != 0ull && !test_bit(c_cert, k);
                // the edge may be certified through its reverse entry
                if (p) {
                    kr = find_sorted(c_col, c_rp[w], c_rp[w + 1], u);
                    p = kr < 0 || !test_bit(c_cert, kr);
                }
                if (p && a.wit_on && witness_swap(a, tab, cu, cw, u, w)) {
                    set_bit(c_cert, k);
                    ++swapped;
                    p = false;
                }
                if (p && a.wit_on && witness_join(a, cu, cw, u, w, vmask)) {
                    set_bit(c_cert, k);
                    ++joined;
                    p = false;
                }
            }
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
                e_idx[2 * o] = k;
                e_idx[2 * o + 1] = kr;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        swapped += __shfl_xor(swapped, off, 64);
        joined += __shfl_xor(joined, off, 64);
    }
    if (lane == 0 && swapped && a.qstats) atomicAdd(a.qstats + 14, swapped);
    if (lane == 0 && joined && a.qstats) atomicAdd(a.qstats + 15, joined);
}

template <typename M>
void launch_edge_candidates(hipStream_t s, int64_t c_m, const int64_t *c_rp,
                            const int32_t *c_own, const int32_t *c_col, const M *cert,
                            const LccTable &tab, uint64_t *c_cert, int32_t *eu, int32_t *ew,
                            int64_t *e_idx, int32_t *n_out, int64_t cap, const SearchArgs &a) {
    if (c_m <= 0) return;
    int64_t grid = (c_m + kSearchBlock - 1) / kSearchBlock;
    if (grid > 16384) grid = 16384;
    hipLaunchKernelGGL(edge_candidates_kernel<M>, dim3((unsigned)grid), dim3(kSearchBlock), 0, s,
                       c_m, c_rp, c_own, c_col, cert, tab, c_cert, eu, ew, e_idx, n_out, cap, a);
}

// One edge-rooted query (plan P with its pins at u, w; or split task rt):
// a found match certifies its roles and edges and its single-vertex swaps.
struct QueryCount {
    unsigned long long queries = 0, npos = 0, tpos = 0, tneg = 0, tcert = 0, texp = 0;
    ExpandCount ec;
};

template <typename M, bool kExpand = true>
__device__ bool edge_query(const SearchArgs &a, const SearchPlan *__restrict__ P,
                           const M *__restrict__ om, M *cert, int32_t u, int32_t w,
                           const SplitTask *rt, int64_t t, int plan, QueryCount &qc) {
    int32_t img = 0;
    int32_t rb = 0;
    ++qc.queries;
    const uint64_t c0 = wall_clock64();
    const int r = dfs_search<M>(a, P, om, u, w, rt, t, plan, a.split_budget > 0, img, rb);
    const uint64_t c1 = wall_clock64();
    if (r != kSearchFound) {
        qc.tneg += c1 - c0;
        return false;
    }
    ++qc.npos;
    qc.tpos += c1 - c0;
    if (!a.aggregate) {
        // only the edge this query was asked about
        if (lane_id() == 0) certify_pair(a, u, P->pin[0], w, P->pin[1]);
        qc.tcert += wall_clock64() - c1;
        return true;
    }
    certify_match<M>(a, P, img, cert);
    if (kExpand && a.expand) {
        const uint64_t c2 = wall_clock64();
        expand_match<M>(a, P, img, rb, om, cert, qc.ec);
        qc.texp += wall_clock64() - c2;
    }
    qc.tcert += wall_clock64() - c1;
    return true;
}

__device__ __forceinline__ void flush_edge_stats(const SearchArgs &a, const QueryCount &qc) {
    if (lane_id() == 0 && qc.queries) {
        atomicAdd(a.n_queries, qc.queries);
        if (a.qstats) {
            atomicAdd(a.qstats + 4, qc.npos);
            atomicAdd(a.qstats + 5, qc.queries - qc.npos);
            atomicAdd(a.qstats + 6, qc.tpos);
            atomicAdd(a.qstats + 7, qc.tneg);
            atomicAdd(a.qstats + 9, qc.tcert);
            atomicAdd(a.qstats + 10, qc.texp);
            atomicAdd(a.qstats + 11, qc.ec.scans);
            atomicAdd(a.qstats + 12, qc.ec.cands);
            atomicAdd(a.qstats + 13, qc.ec.valid);
        }
    }
}

// Is the edge of task t certified (through either of its entries)?  The
// reverse entry's word is read even when there is none (k's word again),
// so both loads are issued together.
__device__ __forceinline__ bool edge_certified(const SearchArgs &a, const int64_t *e_idx,
                                               int64_t t) {
    const int64_t k = e_idx[2 * t], kr = e_idx[2 * t + 1];
    const int64_t kq = kr >= 0 ? kr : k;
    const uint64_t wk = load_fresh(a.c_cert + (k >> 6));
    const uint64_t wq = load_fresh(a.c_cert + (kq >> 6));
    return ((wk >> (k & 63)) | (wq >> (kq & 63))) & 1ull;
}

// kExpand false: compiled without the swap scans (the edge-rooted phase
// runs without them by default), which frees enough registers for five
// wavefronts per SIMD instead of four.
template <typename M, bool kExpand>
__global__ __launch_bounds__(kSearchBlock) __attribute__((amdgpu_waves_per_eu(kExpand ? 1 : 5)))
void edge_search_kernel(
    const int32_t *eu, const int32_t *ew, const int64_t *e_idx, int64_t n_edges, const M *om,
    M *cert, const int32_t *edge_plan, int32_t n_edge_plans, SearchArgs a) {
    const int lane = lane_id();
    QueryCount qc;
    // chunks of task_chunk consecutive candidates are handed out in striped
    // order: chunk c is the (c / S)-th chunk of stripe c % S, so waves
    // running at the same time work on distant parts of the list (other
    // vertices) and later chunks of a vertex find more of its edges already
    // certified.  The last tail_single candidates follow one at a time, so
    // the waves finish close together.
    const int64_t n_single = a.tail_single < n_edges ? a.tail_single : n_edges;
    const int64_t n_head = n_edges - n_single;
    const int64_t n_chunks = (n_head + a.task_chunk - 1) / a.task_chunk;
    const int64_t S = a.stripes > 1 ? a.stripes : 1;
    const int64_t R = (n_chunks + S - 1) / S;
    for (;;) {
        int c = 0;
        if (lane == 0) c = atomicAdd(a.task_counter, 1);
        c = __shfl(c, 0);
        int64_t t0, t1;
        if ((int64_t)c < S * R) {
            const int64_t pc = ((int64_t)c % S) * R + (int64_t)c / S;
            if (pc >= n_chunks) continue;
            t0 = pc * a.task_chunk;
            t1 = t0 + a.task_chunk < n_head ? t0 + a.task_chunk : n_head;
        } else {
            t0 = n_head + ((int64_t)c - S * R);
            if (t0 >= n_edges) break;
            t1 = t0 + 1;
        }
        for (int64_t t = t0; t < t1; ++t) {
            const int32_t u = eu[t], w = ew[t];
            const uint64_t cu = (uint64_t)om[u], cw = (uint64_t)om[w];
            // a plan whose search splits is finished by its split tasks;
            // the next plans are tried meanwhile
            for (int i = 0; i < n_edge_plans; ++i) {
                if (edge_certified(a, e_idx, t)) break;
                const SearchPlan *P = a.plans + edge_plan[i];
                if (!((cu >> P->pin[0]) & 1ull) || !((cw >> P->pin[1]) & 1ull)) continue;
                if (edge_query<M, kExpand>(a, P, om, cert, u, w, nullptr, t, i, qc)) break;
            }
        }
    }
    flush_edge_stats(a, qc);
}

template <typename M>
void launch_edge_search(hipStream_t s, const int32_t *eu, const int32_t *ew,
                        const int64_t *e_idx, int64_t n_edges, const M *omega, M *cert,
                        const int32_t *edge_plan_dev, int32_t n_edge_plans, const SearchArgs &a,
                        int grid) {
    if (n_edges <= 0) return;
    if (a.expand)
        hipLaunchKernelGGL((edge_search_kernel<M, true>), dim3(grid), dim3(kSearchBlock), 0, s, eu, ew,
                           e_idx, n_edges, omega, cert, edge_plan_dev, n_edge_plans, a);
    else
        hipLaunchKernelGGL((edge_search_kernel<M, false>), dim3(grid), dim3(kSearchBlock), 0, s, eu, ew,
                           e_idx, n_edges, omega, cert, edge_plan_dev, n_edge_plans, a);
}

// Split tasks, one per fetch (each is a long search); skipped once their
// edge is certified.
template <typename M>
__global__ __launch_bounds__(kSearchBlock) void split_search_kernel(
    const SplitTask *tasks, int64_t n_tasks, const int32_t *eu, const int32_t *ew,
    const int64_t *e_idx, const M *om, M *cert, const int32_t *edge_plan, SearchArgs a) {
    const int lane = lane_id();
    QueryCount qc;
    for (;;) {
        int i = 0;
        if (lane == 0) i = atomicAdd(a.task_counter, 1);
        i = __shfl(i, 0);
        if ((int64_t)i >= n_tasks) break;
        const SplitTask *rt = tasks + i;
        const int64_t t = rt->t;
        if (edge_certified(a, e_idx, t)) continue;
        const int plan = rt->plan;
        edge_query<M>(a, a.plans + edge_plan[plan], om, cert, eu[t], ew[t], rt, t, plan, qc);
    }
    flush_edge_stats(a, qc);
}

template <typename M>
void launch_split_search(hipStream_t s, const SplitTask *tasks, int64_t n_tasks,
                         const int32_t *eu, const int32_t *ew, const int64_t *e_idx,
                         const M *omega, M *cert, const int32_t *edge_plan, const SearchArgs &a,
                         int grid) {
    if (n_tasks <= 0) return;
    int64_t g = (n_tasks * kWave + kSearchBlock - 1) / kSearchBlock;
    if (g > grid) g = grid;
    hipLaunchKernelGGL(split_search_kernel<M>, dim3((unsigned)g), dim3(kSearchBlock), 0, s, tasks,
                       n_tasks, eu, ew, e_idx, omega, cert, edge_plan, a);
}

// Output edge bits from certified compacted entries (a certified edge holds
// the bit of one or both of its entries).  One thread per entry u -> w:
// entries not certified are skipped after one coalesced read of their
// certificate word; a certified one sets its own CSR entry's bit and, found
// by a search of w's compacted row, that of its reverse entry.  The searches
// scale with the certified entries, not with the candidate subgraph.
// Entries go by wavefront-aligned chunks: the own bits of a chunk ascend
// (rows in vertex order), so they take one atomic per output word.
__global__ __launch_bounds__(kSearchBlock) void edges_from_cert_kernel(
    int64_t c_m, const int64_t *c_rp, const int32_t *c_col, const int32_t *c_own,
    const int32_t *c_off, const int64_t *rp, const uint64_t *c_cert, uint64_t *edge_bits) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < c_m;
         base += stride) {
        const int64_t k = base + lane_id();
        const bool cert = k < c_m && test_bit(c_cert, k);
        int64_t own = 0;
        if (cert) {
            const int32_t u = c_own[k], w = c_col[k];
            own = rp[u] + c_off[k];
            const int64_t kr = find_sorted(c_col, c_rp[w], c_rp[w + 1], u);
            if (kr >= 0) set_bit(edge_bits, rp[w] + c_off[kr]);
        }
        set_bits_wave(edge_bits, own, cert);
    }
}

void launch_edges_from_cert(hipStream_t s, int64_t c_m, const int64_t *c_rp, const int32_t *c_col,
                            const int32_t *c_own, const int32_t *c_off, const int64_t *rp,
                            const uint64_t *c_cert, uint64_t *edge_bits) {
    if (c_m <= 0) return;
    int64_t grid = (c_m + kSearchBlock - 1) / kSearchBlock;
    if (grid > 16384) grid = 16384;
    hipLaunchKernelGGL(edges_from_cert_kernel, dim3((unsigned)grid), dim3(kSearchBlock), 0, s,
                       c_m, c_rp, c_col, c_own, c_off, rp, c_cert, edge_bits);
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
        // the row's entries go 64 at a time (bounds uniform over the
        // wavefront): one atomic per output word
        for (int64_t k0 = s; k0 < e; k0 += kWave) {
            const int64_t k = k0 + lane;
            const bool on = k < e && ((uint64_t)om[c_col[k]] & reach);
            set_bits_wave(edge_bits, on ? r0 + c_off[k] : 0, on);
        }
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

// ---------------------------------------------- match counting/enumeration
// Count tasks: compacted entries u -> w whose ends hold the pinned roles
// (qa at u, qb at w).  Every map puts its template edge (qa, qb) on exactly
// one such entry, so counting from each task once counts every map once.
template <typename M>
__global__ __launch_bounds__(kSearchBlock) void count_tasks_kernel(
    int64_t c_m, const int32_t *__restrict__ c_own, const int32_t *__restrict__ c_col,
    const M *__restrict__ om, int qa, int qb, int32_t *eu, int32_t *ew, int32_t *n_out,
    int64_t cap) {
    const int lane = lane_id();
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < c_m;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = base + threadIdx.x;
        bool p = false;
        int32_t u = 0, w = 0;
        if (k < c_m) {
            u = c_own[k];
            w = c_col[k];
            p = (((uint64_t)om[u] >> qa) & 1ull) && (((uint64_t)om[w] >> qb) & 1ull);
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
            }
        }
    }
}

template <typename M>
void launch_count_tasks(hipStream_t s, int64_t c_m, const int32_t *c_own, const int32_t *c_col,
                        const M *omega, int qa, int qb, int32_t *eu, int32_t *ew, int32_t *n_out,
                        int64_t cap) {
    if (c_m <= 0) return;
    int64_t grid = (c_m + kSearchBlock - 1) / kSearchBlock;
    if (grid > 16384) grid = 16384;
    hipLaunchKernelGGL(count_tasks_kernel<M>, dim3((unsigned)grid), dim3(kSearchBlock), 0, s, c_m,
                       c_own, c_col, omega, qa, qb, eu, ew, n_out, cap);
}

// One wavefront per task (chunks of a.task_chunk per fetch), the full
// template pinned at the task's entry; searches past the step budget hand
// on parts of their tree as split tasks (a.split_out).
__device__ __forceinline__ bool count_stopped(const CountSink &cs) {
    int st = 0;
    if (cs.limit && lane_id() == 0)
        st = __hip_atomic_load(cs.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __shfl(st, 0) != 0;
}

template <typename M>
__global__ __launch_bounds__(kSearchBlock) void count_search_kernel(
    const int32_t *eu, const int32_t *ew, int64_t n_tasks, const M *om, const int32_t *plan_id,
    SearchArgs a, int32_t *maps, int64_t cap, unsigned long long *written,
    unsigned long long *total, unsigned long long limit, int32_t *stop) {
    const int lane = lane_id();
    CountSink cs;
    cs.maps = maps;
    cs.cap = cap;
    cs.written = written;
    cs.total = total;
    cs.limit = limit;
    cs.stop = stop;
    const SearchPlan *P = a.plans + plan_id[0];
    for (;;) {
        if (count_stopped(cs)) break;
        int t0 = 0;
        if (lane == 0) t0 = atomicAdd(a.task_counter, a.task_chunk);
        t0 = __shfl(t0, 0);
        if ((int64_t)t0 >= n_tasks) break;
        const int64_t t1 =
            (int64_t)t0 + a.task_chunk < n_tasks ? (int64_t)t0 + a.task_chunk : n_tasks;
        for (int64_t t = t0; t < t1; ++t) {
            int32_t img = 0, rb = 0;
            dfs_search<M, true>(a, P, om, eu[t], ew[t], nullptr, t, 0, a.split_budget > 0, img,
                                rb, &cs);
        }
    }
    if (lane == 0 && cs.n) atomicAdd(total, cs.n);
}

template <typename M>
__global__ __launch_bounds__(kSearchBlock) void count_split_kernel(
    const SplitTask *tasks, int64_t n_tasks, const int32_t *eu, const int32_t *ew, const M *om,
    const int32_t *plan_id, SearchArgs a, int32_t *maps, int64_t cap,
    unsigned long long *written, unsigned long long *total, unsigned long long limit,
    int32_t *stop) {
    const int lane = lane_id();
    CountSink cs;
    cs.maps = maps;
    cs.cap = cap;
    cs.written = written;
    cs.total = total;
    cs.limit = limit;
    cs.stop = stop;
    const SearchPlan *P = a.plans + plan_id[0];
    for (;;) {
        if (count_stopped(cs)) break;
        int i = 0;
        if (lane == 0) i = atomicAdd(a.task_counter, 1);
        i = __shfl(i, 0);
        if ((int64_t)i >= n_tasks) break;
        const SplitTask *rt = tasks + i;
        const int64_t t = rt->t;
        int32_t img = 0, rb = 0;
        dfs_search<M, true>(a, P, om, eu[t], ew[t], rt, t, 0, a.split_budget > 0, img, rb, &cs);
    }
    if (lane == 0 && cs.n) atomicAdd(total, cs.n);
}

template <typename M>
void launch_count_search(hipStream_t s, const int32_t *eu, const int32_t *ew, int64_t n_tasks,
                         const M *omega, const int32_t *plan_id, const SearchArgs &a,
                         int32_t *maps, int64_t cap, unsigned long long *written,
                         unsigned long long *total, unsigned long long limit, int32_t *stop,
                         int grid) {
    if (n_tasks <= 0) return;
    hipLaunchKernelGGL(count_search_kernel<M>, dim3(grid), dim3(kSearchBlock), 0, s, eu, ew,
                       n_tasks, omega, plan_id, a, maps, cap, written, total, limit, stop);
}

template <typename M>
void launch_count_split(hipStream_t s, const SplitTask *tasks, int64_t n_tasks, const int32_t *eu,
                        const int32_t *ew, const M *omega, const int32_t *plan_id,
                        const SearchArgs &a, int32_t *maps, int64_t cap,
                        unsigned long long *written, unsigned long long *total,
                        unsigned long long limit, int32_t *stop, int grid) {
    if (n_tasks <= 0) return;
    int64_t g = (n_tasks * kWave + kSearchBlock - 1) / kSearchBlock;
    if (g > grid) g = grid;
    hipLaunchKernelGGL(count_split_kernel<M>, dim3((unsigned)g), dim3(kSearchBlock), 0, s, tasks,
                       n_tasks, eu, ew, omega, plan_id, a, maps, cap, written, total, limit,
                       stop);
}

#define PM_INSTANTIATE_SEARCH(M)                                                                  \
    template void launch_role_count<M>(hipStream_t, const int32_t *, int64_t, const int64_t *,    \
                                       const int32_t *, const M *, int, int64_t *, int32_t *);    \
    template void launch_role_fill<M>(hipStream_t, const int32_t *, int64_t, const int64_t *,     \
                                      const int32_t *, const M *, int, const int64_t *,           \
                                      int32_t *, int32_t *);                                      \
    template void launch_vertex_search<M>(hipStream_t, const int32_t *, int64_t, const M *, M *,  \
                                          const SearchArgs &, int);                               \
    template void launch_apply<M>(hipStream_t, const int32_t *, int64_t, M *, M *, uint64_t,      \
                                  int32_t *);                                                     \
    template void launch_edge_candidates<M>(hipStream_t, int64_t, const int64_t *,                \
                                            const int32_t *, const int32_t *, const M *,          \
                                            const LccTable &,                                     \
                                            uint64_t *, int32_t *, int32_t *, int64_t *,          \
                                            int32_t *, int64_t, const SearchArgs &);              \
    template void launch_split_search<M>(hipStream_t, const SplitTask *, int64_t,                 \
                                         const int32_t *, const int32_t *, const int64_t *,       \
                                         const M *, M *, const int32_t *, const SearchArgs &,     \
                                         int);                                                    \
    template void launch_edge_search<M>(hipStream_t, const int32_t *, const int32_t *,            \
                                        const int64_t *, int64_t, const M *, M *,                 \
                                        const int32_t *, int32_t, const SearchArgs &, int);       \
    template void launch_active_edges<M>(hipStream_t, const int32_t *, int64_t, const int64_t *,  \
                                         const int32_t *, const int32_t *, const int64_t *,       \
                                         const M *, const LccTable &, uint64_t *);                \
    template void launch_count_tasks<M>(hipStream_t, int64_t, const int32_t *, const int32_t *,   \
                                        const M *, int, int, int32_t *, int32_t *, int32_t *,     \
                                        int64_t);                                                 \
    template void launch_count_search<M>(hipStream_t, const int32_t *, const int32_t *, int64_t, \
                                         const M *, const int32_t *, const SearchArgs &,          \
                                         int32_t *, int64_t, unsigned long long *,                \
                                         unsigned long long *, unsigned long long, int32_t *,     \
                                         int);                                                    \
    template void launch_count_split<M>(hipStream_t, const SplitTask *, int64_t, const int32_t *, \
                                        const int32_t *, const M *, const int32_t *,              \
                                        const SearchArgs &, int32_t *, int64_t,                   \
                                        unsigned long long *, unsigned long long *,               \
                                        unsigned long long, int32_t *, int);

PM_INSTANTIATE_SEARCH(uint8_t)
PM_INSTANTIATE_SEARCH(uint16_t)
PM_INSTANTIATE_SEARCH(uint32_t)
PM_INSTANTIATE_SEARCH(uint64_t)

}  // namespace pm
