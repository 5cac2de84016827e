// Host engine and C ABI of libpm: context, graph and template loading, and
// the pruning driver (main constraint-checking loop of the paper: generate
// the non-local constraints, initialise vertex state, LCC to a fixpoint,
// then for each constraint NLCC and, when it changed anything, LCC again;
// finally the full-template search that certifies roles and edges).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <tuple>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "pm.h"
#include "pm_internal.h"

namespace pm {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

static thread_local std::string g_last_error;

#define PM_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t _e = (call);                                                               \
        if (_e != hipSuccess)                                                                 \
            throw Error(_e == hipErrorOutOfMemory ? PM_ERR_OOM : PM_ERR_HIP,                  \
                        std::string(#call) + ": " + hipGetErrorString(_e));                  \
    } while (0)

// Caller-owned device memory that a worker's buffers are carved from (bump
// allocation, 256-byte aligned); reset at the start of every template.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0, peak = 0;
    void *take(size_t want) {
        const size_t off = (used + 255) & ~(size_t)255;
        if (off > cap || want > cap - off)
            throw Error(PM_ERR_WORKSPACE, "workspace too small: needs more than " +
                                              std::to_string(cap) + " bytes (" +
                                              std::to_string(off + want) + " requested so far)");
        used = off + want;
        peak = std::max(peak, used);
        return base + off;
    }
};

// Grow-only device buffer: library-owned (hipMalloc) unless it draws from an
// arena, where growing takes a new block and abandons the old one.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    Arena *arena = nullptr;
    void ensure(size_t want) {
        if (want <= bytes) return;
        size_t alloc = std::max<size_t>(want, 256);
        if (arena) {
            p = arena->take(alloc);
            bytes = alloc;
            return;
        }
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        PM_HIP(hipMalloc(&p, alloc));
        bytes = alloc;
    }
    void release() {
        if (p && !arena) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

struct Timer {
    hipEvent_t a{}, b{};
    hipStream_t s{};
    explicit Timer(hipStream_t st) : s(st) {
        PM_HIP(hipEventCreate(&a));
        PM_HIP(hipEventCreate(&b));
        PM_HIP(hipEventRecord(a, s));
    }
    double stop() {
        PM_HIP(hipEventRecord(b, s));
        PM_HIP(hipEventSynchronize(b));
        float ms = 0;
        PM_HIP(hipEventElapsedTime(&ms, a, b));
        return ms;
    }
    ~Timer() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
};

// Phase timing without waits: each span records an event pair on the
// stream, and the pairs are read once the prune has finished, so timing a
// phase never stalls the host between launches.
struct TimeLog {
    struct Ent {
        hipEvent_t a, b;
        double *dst, *dst2;
        double sign;
    };
    std::vector<Ent> ents;
    std::vector<hipEvent_t> pool;
    hipEvent_t take() {
        hipEvent_t e{};
        if (pool.empty()) {
            PM_HIP(hipEventCreate(&e));
        } else {
            e = pool.back();
            pool.pop_back();
        }
        return e;
    }
    // Adds every recorded span to its destinations (waits for the last).
    void resolve() {
        for (Ent &x : ents) {
            PM_HIP(hipEventSynchronize(x.b));
            float ms = 0;
            PM_HIP(hipEventElapsedTime(&ms, x.a, x.b));
            *x.dst += x.sign * ms;
            if (x.dst2) *x.dst2 += x.sign * ms;
            pool.push_back(x.a);
            pool.push_back(x.b);
        }
        ents.clear();
    }
    ~TimeLog() {
        for (Ent &x : ents) {
            (void)hipEventDestroy(x.a);
            (void)hipEventDestroy(x.b);
        }
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

struct Span {
    TimeLog &log;
    hipStream_t s;
    hipEvent_t a;
    bool done = false;
    Span(TimeLog &l, hipStream_t st) : log(l), s(st), a(l.take()) { PM_HIP(hipEventRecord(a, s)); }
    // The span's device time is added (times sign) to dst, and to *dst2,
    // when the log resolves.
    void stop(double &dst, double *dst2 = nullptr, double sign = 1.0) {
        hipEvent_t b = log.take();
        PM_HIP(hipEventRecord(b, s));
        log.ents.push_back(TimeLog::Ent{a, b, &dst, dst2, sign});
        done = true;
    }
    ~Span() {
        if (!done) log.pool.push_back(a);
    }
};

// Device scratch of one pruning worker (one template at a time) and the
// stream its kernels run on.
struct Scratch {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Arena arena;
    bool in_arena = false;
    DevBuf omega, sat, alist[2], bins, counters, hub, cdeg, crp, ccol, coff, cown, crp2, ccol2,
        coff2, cown2,
        segcnt, segscan, segbits, scan_scratch;
    DevBuf eu, ew, eidx, edge_plan_ids, ccert, expseen, wit, witflag, rlcnt, rloff, rlpos, rlcol, rlent, rlscan,
        rlv, actbits, ord, afilt, split[2], tsum;
    std::vector<DevBuf *> all() {
        return {&omega, &sat, &alist[0], &alist[1], &bins, &counters, &hub, &cdeg, &crp,
                &ccol, &coff, &cown, &crp2, &ccol2, &coff2, &cown2, &segcnt, &segscan, &segbits,
                &scan_scratch, &eu, &ew, &eidx, &edge_plan_ids, &ccert, &expseen, &wit, &witflag,
                &rlcnt, &rloff, &rlpos, &rlcol, &rlent, &rlscan, &rlv, &actbits, &ord,
                &afilt, &split[0], &split[1], &tsum};
    }
    // Draw every buffer from [base, base + cap) from now on (library-owned
    // buffers are freed first), or, with base == nullptr, return to
    // library-owned buffers.
    void use_arena(char *base, size_t cap) {
        for (DevBuf *b : all()) {
            b->release();
            b->arena = base ? &arena : nullptr;
        }
        arena = Arena{};
        arena.base = base;
        arena.cap = cap;
        in_arena = base != nullptr;
    }
    // Start of a template's prune in arena mode: every buffer is taken
    // again from the start of the arena.
    void reset_arena() {
        if (!in_arena) return;
        for (DevBuf *b : all()) b->release();
        arena.used = 0;
        arena.peak = 0;
    }
    size_t bytes_held() {
        if (in_arena) return arena.peak;
        size_t t = 0;
        for (DevBuf *b : all()) t += b->bytes;
        return t;
    }
    void release() {
        for (DevBuf *b : all()) b->release();
        if (own_stream && stream) (void)hipStreamDestroy(stream);
        stream = nullptr;
        own_stream = false;
    }
    ~Scratch() { release(); }
};

}  // namespace pm

using namespace pm;

struct pm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // graph
    bool has_graph = false;
    int64_t n = 0, m = 0;
    const int64_t *rp = nullptr;
    const int32_t *col = nullptr;
    const void *labels = nullptr;
    int label_bytes = 1;
    DevBuf own_rp, own_col, own_labels;
    std::vector<int64_t> label_freq;
    std::vector<int64_t> label_degsum;   // sum of degrees per label
    // neighbour-label count index (uint8 labels below kCountLabels): count
    // of neighbours of v with label L at lab_cnt[L * n + v]; nlab = 0: none
    DevBuf lab_cnt;
    int nlab = 0;
    int index_nlab = 0;                  // labels the index would cover (0: not eligible)
    DevBuf idx_hub_v, idx_seg_slot, idx_seg_b, idx_seg_e, idx_hub_cnt;
    int64_t idx_hubs = 0, idx_segs = 0;
    int64_t cnt_stride = 0;
    double ms_count_index = 0.0;
    // label-pair subgraph: the entries u -> x of the loaded graph whose label
    // pair (label(u), label(x)) is that of a template edge of the templates
    // it was built for (pair_adj[la * pair_nl + lb], labels < pair_nl);
    // pair_off holds each entry's offset in its original row.  pair_m < 0:
    // none.
    DevBuf pair_rp, pair_col, pair_off;
    int64_t pair_m = -1;
    int pair_nl = 0;
    std::vector<uint8_t> pair_adj;
    // count index of the label-pair subgraph (same layout as lab_cnt; for
    // a label pair of the subgraph its counts are those of the graph);
    // pair_cnt_nlab = 0: none
    DevBuf pair_cnt;
    int pair_cnt_nlab = 0;
    int64_t pair_cnt_stride = 0;
    double ms_pair_index = 0.0;
    int64_t hub_cap = 0, seg_cap = 0;
    // templates
    std::vector<std::unique_ptr<CompiledTemplate>> templates;
    // per-worker scratch; worker 0 runs on the context stream
    std::vector<std::unique_ptr<pm::Scratch>> scratch;
    int grid_search = 2048;
    // blocks shared by the searches that run at once (0: every search
    // launch takes grid_search); `searching` counts the workers whose last
    // search launch the host has not yet seen finish
    int grid_search_solo = 0;
    std::atomic<int> searching{0};
    int expand = 1;
    int expand_edges = 1;   // swap scans after edge-rooted finds too
    int tree_exact = 1;     // final step of one-repeated-pair trees by path sweeps
    int64_t expand_max = 4096;
    int witness = 0;
    int edge_chunk = 16;
    int relist = 1;
    int edge_stripes = 64;
    int64_t split_budget = 8192;
    int64_t edge_tail = 0;
    int exp_log2 = kExpSeenLog2;
    int64_t split_cap = kSplitCap;
    int read_first = 0;
    int64_t bin_small = kBinSmallMaxDeg;   // LCC degree-bin bounds (settings)
    int64_t bin_mid = kBinMidMaxDeg;
    int64_t wall_khz = 0;
    // caller-owned workspace (pm_set_workspace); null: library-owned scratch
    char *ws = nullptr;
    size_t ws_bytes = 0;
    void *noalloc = nullptr;             // this device's static scratch array
    // learned-order model and the workspace of its training kernels
    DevBuf model;
    bool has_model = false;
    DevBuf mlp_partial, mlp_ploss, mlp_grad, mlp_m, mlp_v, mlp_loss;
};

namespace {

void set_device(pm_ctx *c) { PM_HIP(hipSetDevice(c->device)); }

// Blocks for one search launch, held from the launch until the host has
// seen the search finish.  A search launched while k workers of a batch
// search (itself included) takes search_grid_solo / k blocks, never fewer
// than search_grid: a search that runs alone, or at the tail of a batch,
// fills the GPU, and concurrent ones split it.  The search kernels pull
// their tasks from a counter, so any grid gives the same result.
struct SearchShare {
    pm_ctx *c;
    int grid;
    explicit SearchShare(pm_ctx *cc) : c(cc) {
        const int k = ++c->searching;
        grid = c->grid_search;
        if (c->grid_search_solo > grid) grid = std::max(grid, c->grid_search_solo / k);
    }
    ~SearchShare() { --c->searching; }
    SearchShare(const SearchShare &) = delete;
    SearchShare &operator=(const SearchShare &) = delete;
};

template <typename T>
void d2h(hipStream_t s, T *dst, const T *src, size_t count) {
    PM_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
}

// Counter block layout (int32 unless noted).
enum : int {
    C_BINS = 0,        // [4]
    C_NSEG = 4,
    C_CHANGED = 5,
    C_TASK = 6,
    C_ACTIVE = 7,
    C_NOUT = 8,
    C_SPLIT = 9,       // split tasks appended
    C_QUERIES_U64 = 16,   // byte offset 64: unsigned long long
    C_ENTRIES_U64 = 18,   // byte offset 72: unsigned long long
    C_COUNT_U64 = 64,     // byte offset 256: maps counted (unsigned long long)
    C_WRITTEN_U64 = 66,   // byte offset 264: maps written
    C_STOP = 68,          // byte offset 272: counting stopped at its limit
    C_TOTAL_BYTES = 512,      // bytes 128..255: query statistics [16]
};

struct Graph {
    const int64_t *rp;
    const int32_t *col;
};

template <typename M>
struct Pruner {
    pm_ctx *c;
    Scratch *w;
    const CompiledTemplate &T;
    hipStream_t s;
    M *om;
    M *sat;
    int32_t *A;              // active list
    int32_t *Aalt;
    int64_t nA = 0;
    Worklists wl{};
    int32_t *ctr;
    unsigned long long *queries;
    unsigned long long *qstats;
    int64_t hc[4] = {0, 0, 0, 0};
    int64_t nseg = 0;
    // compacted candidate subgraph
    int64_t *c_rp = nullptr;
    int32_t *c_col = nullptr;
    int32_t *c_off = nullptr;
    int32_t *c_own = nullptr;
    int64_t c_m = 0;
    pm_stats st{};
    // per-call options and the state brought in with them
    const pm_options *opt = nullptr;
    LccTable lcc;                   // the template's local rule, per mode
    bool candidate = false;         // PM_MODE_CANDIDATE
    uint32_t ablate = 0;
    const uint64_t *init_state = nullptr;
    uint64_t skip_mask = 0;
    const uint64_t *known_roles = nullptr;
    const uint64_t *known_edges = nullptr;
    uint64_t done_mask = 0;
    int exp_log2;
    int64_t split_cap;
    TimeLog tl;                     // phase times, read when the prune ends

    Pruner(pm_ctx *ctx, Scratch *scr, const CompiledTemplate &t, const pm_options *o = nullptr)
        : c(ctx), w(scr), T(t), s(scr->stream), opt(o), lcc(t.lcc), exp_log2(ctx->exp_log2),
          split_cap(ctx->split_cap) {
        if (opt) {
            candidate = opt->mode == PM_MODE_CANDIDATE;
            ablate = opt->ablate;
        }
        if (candidate) {
            lcc.any = 1;
            lcc.ncount = 0;
        }
        if (ablate & PM_ABLATE_EDGE_ELIMINATION) lcc.keep_all = 1;
        const int64_t n = c->n;
        w->omega.ensure(sizeof(M) * (size_t)std::max<int64_t>(n, 1));
        w->sat.ensure(sizeof(M) * (size_t)std::max<int64_t>(n, 1));
        w->alist[0].ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1));
        w->alist[1].ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1));
        w->bins.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1) * kNumBins);
        w->counters.ensure(C_TOTAL_BYTES);
        const int64_t hubs = std::max<int64_t>(c->hub_cap, 1), segs = std::max<int64_t>(c->seg_cap, 1);
        size_t hub_bytes = (size_t)segs * (4 + 8 + 8 + 4) + (size_t)hubs * (4 + 4 + 8 + 4 * kMaxCount + 4);
        w->hub.ensure(hub_bytes + 256);
        w->segcnt.ensure(sizeof(int64_t) * (size_t)segs);
        w->segscan.ensure(sizeof(int64_t) * (size_t)(segs + 1));
        w->segbits.ensure(sizeof(uint64_t) * (size_t)segs * (kHubSegment / kWave));
        om = w->omega.as<M>();
        sat = w->sat.as<M>();
        A = w->alist[0].as<int32_t>();
        Aalt = w->alist[1].as<int32_t>();
        ctr = w->counters.as<int32_t>();
        queries = reinterpret_cast<unsigned long long *>(w->counters.as<char>() + 64);
        qstats = reinterpret_cast<unsigned long long *>(w->counters.as<char>() + 128);
        for (int b = 0; b < kNumBins; ++b) wl.list[b] = w->bins.as<int32_t>() + (size_t)b * n;
        wl.count = ctr + C_BINS;
        wl.entries = reinterpret_cast<unsigned long long *>(w->counters.as<char>() + 72);
        wl.n_seg = ctr + C_NSEG;
        char *h = w->hub.as<char>();
        wl.hub_seg_begin = reinterpret_cast<int64_t *>(h); h += 8 * (size_t)segs;
        wl.hub_seg_end = reinterpret_cast<int64_t *>(h); h += 8 * (size_t)segs;
        wl.hub_cover = reinterpret_cast<uint64_t *>(h); h += 8 * (size_t)hubs;
        wl.hub_seg_v = reinterpret_cast<int32_t *>(h); h += 4 * (size_t)segs;
        wl.hub_seg_slot = reinterpret_cast<int32_t *>(h); h += 4 * (size_t)segs;
        wl.hub_nseg = reinterpret_cast<int32_t *>(h); h += 4 * (size_t)hubs;
        wl.hub_seg_first = reinterpret_cast<int32_t *>(h); h += 4 * (size_t)hubs;
        wl.hub_ticket = reinterpret_cast<int32_t *>(h); h += 4 * (size_t)hubs;
        wl.hub_count = reinterpret_cast<int32_t *>(h);
        wl.capacity = n;
        wl.hub_capacity = hubs;
        wl.seg_capacity = segs;
        wl.bin_small = c->bin_small;
        wl.bin_mid = c->bin_mid;
    }

    void zero_counters() { PM_HIP(hipMemsetAsync(ctr, 0, C_TOTAL_BYTES, s)); }

    int32_t read_ctr(int idx) {
        int32_t v = 0;
        d2h(s, &v, ctr + idx, 1);
        return v;
    }

    // Active list <- vertices of the current list whose role set is non-empty.
    void collect(bool from_all) {
        PM_HIP(hipMemsetAsync(ctr + C_ACTIVE, 0, sizeof(int32_t), s));
        if (from_all) {
            launch_collect<M>(s, nullptr, c->n, om, A, ctr + C_ACTIVE);
        } else {
            launch_collect<M>(s, A, nA, om, Aalt, ctr + C_ACTIVE);
            std::swap(A, Aalt);
        }
        nA = read_ctr(C_ACTIVE);
    }

    // The loop-control words of the counter block (bins, hub segments,
    // change flag, active count, binned entries), read in one round trip.
    struct Ctl {
        int32_t w[C_ENTRIES_U64];
        unsigned long long entries;
    };
    Ctl read_control() {
        Ctl cb;
        d2h(s, reinterpret_cast<char *>(&cb), w->counters.as<char>(), sizeof(Ctl));
        return cb;
    }
    void take_bins(const Ctl &cb) {
        for (int b = 0; b < 4; ++b) hc[b] = cb.w[C_BINS + b];
        nseg = cb.w[C_NSEG];
        binned_entries = (int64_t)cb.entries;
        if (hc[3] > wl.hub_capacity || nseg > wl.seg_capacity)
            throw Error(PM_ERR_CAPACITY, "hub segment capacity exceeded");
    }
    // Bins (and hub segments) of the vertices of the active list that hold
    // a role in graph g; launched only, the counts are read with the next
    // control read.
    void launch_bins(const Graph &g) {
        PM_HIP(hipMemsetAsync(ctr + C_BINS, 0, sizeof(int32_t) * 5, s));
        PM_HIP(hipMemsetAsync(wl.entries, 0, sizeof(unsigned long long), s));
        launch_bin<M>(s, A, nA, g.rp, om, wl);
        launch_hub_segments(s, g.rp, wl, 0);
    }

    // Degree bins of the active list in graph g, hub segments, host counts.
    int64_t binned_entries = 0;
    void bin(const Graph &g) {
        launch_bins(g);
        take_bins(read_control());
    }

    int32_t sweep(const Graph &g, bool full = false) {
        PM_HIP(hipMemsetAsync(ctr + C_CHANGED, 0, sizeof(int32_t), s));
        if (full) {
            // device time of the sweep kernel alone (the HBM-bound step)
            Span k(tl, s);
            launch_lcc_sweep<M>(s, g.rp, g.col, om, wl, hc, nseg, lcc, ctr + C_CHANGED, true);
            k.stop(st.ms_sweep_kernel);
        } else {
            launch_lcc_sweep<M>(s, g.rp, g.col, om, wl, hc, nseg, lcc, ctr + C_CHANGED, false);
        }
        st.lcc_sweeps++;
        return read_ctr(C_CHANGED);
    }

    // LCC to the fixpoint on graph g, starting from the current active list.
    // LCC to the fixpoint on the candidate subgraph.  When the active set
    // has shrunk to under half of what it was at the last compaction and
    // the active rows still hold many entries, the candidate subgraph is
    // compacted again first (entries to eliminated vertices go), so later
    // sweeps and the role lists read only live entries.
    void lcc_fixpoint() {
        Span t(tl, s);
        Graph g{c_rp, c_col};
        bin(g);
        for (;;) {
            if (nA * 2 < nA_compact && binned_entries > kRecompactEntries &&
                binned_entries > 4 * nA) {
                Span rc(tl, s);   // counted as compaction, not LCC
                compact(true);
                rc.stop(st.ms_lcc, nullptr, -1.0);
                g = Graph{c_rp, c_col};
                bin(g);
            }
            // the sweep, then the next active list and its bins, whose
            // counts come back with the change flag in one round trip (if
            // nothing changed they are discarded: the set is the same)
            PM_HIP(hipMemsetAsync(ctr + C_CHANGED, 0, sizeof(int32_t), s));
            launch_lcc_sweep<M>(s, g.rp, g.col, om, wl, hc, nseg, lcc, ctr + C_CHANGED, false);
            st.lcc_sweeps++;
            PM_HIP(hipMemsetAsync(ctr + C_ACTIVE, 0, sizeof(int32_t), s));
            launch_collect<M>(s, A, nA, om, Aalt, ctr + C_ACTIVE);
            launch_bins(g);
            const Ctl cb = read_control();
            if (!cb.w[C_CHANGED]) {
                take_bins(cb);
                break;
            }
            std::swap(A, Aalt);
            nA = cb.w[C_ACTIVE];
            take_bins(cb);
            rl_valid = false;
            if (nA == 0) break;
        }
        t.stop(st.ms_lcc);
    }

    // Compacted candidate subgraph of the current state (edge elimination),
    // from the full graph or, once one exists, from the current candidate
    // subgraph (a superset of the new one; offsets into the original rows
    // are carried through c_off).  Two buffer sets alternate.
    int cbuf = 0;
    int64_t nA_compact = 0;   // active vertices when the subgraph was built
    static constexpr int64_t kRecompactEntries = 1 << 20;
    // The label-pair subgraph holds every entry a compaction of this
    // template can keep (a kept entry joins roles adjacent in G0, whose
    // labels are those of a template edge), unless edge elimination is
    // ablated.
    bool pairs_cover() const {
        if (c->pair_m < 0 || lcc.keep_all) return false;
        for (const auto &e : T.edges) {
            const int la = T.labels[(size_t)e.first], lb = T.labels[(size_t)e.second];
            if (la >= c->pair_nl || lb >= c->pair_nl ||
                !c->pair_adj[(size_t)la * (size_t)c->pair_nl + (size_t)lb])
                return false;
        }
        return true;
    }

    // Candidate subgraph: from the current one, else from the label-pair
    // subgraph when it covers the template, else from the loaded graph.
    void compact(bool from_candidate = false) {
        if (from_candidate)
            compact_from(c_rp, c_col, c_off, false);
        else if (pairs_cover())
            compact_from(c->pair_rp.as<int64_t>(), c->pair_col.as<int32_t>(),
                         c->pair_off.as<int32_t>(), true);
        else
            compact_from(c->rp, c->col, nullptr, true);
    }

    // The label-pair subgraph: with one role per label (T's vertices are the
    // labels, its local table their pair adjacency), initial roles from the
    // labels and one compaction of the loaded graph keep exactly the entries
    // whose label pair is adjacent.
    void label_pair_compaction() {
        const int64_t n = c->n;
        zero_counters();
        w->actbits.ensure(sizeof(uint64_t) * (size_t)std::max<int64_t>((n + 63) / 64, 1));
        wl.act_bits = w->actbits.as<uint64_t>();
        launch_init_roles<M>(s, n, c->labels, c->label_bytes, T.d_init_lut, T.init_lut_len, om,
                             w->actbits.as<uint64_t>());
        collect(true);
        compact_from(c->rp, c->col, nullptr, true);
    }

    // Compaction of src (row_ptr, col and, for a subgraph of the loaded
    // graph, every entry's offset in its original row; null: src is the
    // loaded graph).  first: the prune's first compaction (it builds the
    // coarse activity filter the later ones reuse).
    void compact_from(const int64_t *src_rp, const int32_t *src_col, const int32_t *base_off,
                      bool first) {
        Span t(tl, s);
        const int64_t n = c->n;
        Graph src{src_rp, src_col};
        bin(src);
        const int nb = first ? cbuf : 1 - cbuf;
        DevBuf &crp = nb ? w->crp2 : w->crp;
        DevBuf &ccol = nb ? w->ccol2 : w->ccol;
        DevBuf &coff = nb ? w->coff2 : w->coff;
        DevBuf &cown = nb ? w->cown2 : w->cown;
        // kept entries per row, 32-bit (a candidate subgraph holds under
        // 2^31 entries), scanned into the 64-bit row pointer
        w->cdeg.ensure(sizeof(int32_t) * (size_t)(n + 1));
        crp.ensure(sizeof(int64_t) * (size_t)(n + 1));
        int32_t *deg = w->cdeg.as<int32_t>();
        PM_HIP(hipMemsetAsync(deg, 0, sizeof(int32_t) * (size_t)(n + 1), s));
        if (first) {
            // coarse filter of the active set; it stays valid (a superset)
            // for later compactions of this prune, since role sets only shrink
            w->afilt.ensure(sizeof(uint32_t) * (size_t)std::max<int64_t>((n + 255) / 256, 1));
            launch_active_filter<M>(s, n, om, w->afilt.as<uint32_t>());
        }
        const uint32_t *filt = w->afilt.as<uint32_t>();
        launch_compact_count<M>(s, src_rp, src_col, om, wl, hc, nseg, lcc, filt, deg,
                                w->segcnt.as<int64_t>(), w->segbits.as<uint64_t>());
        int64_t sl = scan_scratch_len(std::max<int64_t>(n, nseg));
        w->scan_scratch.ensure(sizeof(int64_t) * (size_t)sl);
        int64_t *new_rp = crp.as<int64_t>();
        launch_exclusive_scan(s, deg, new_rp, n, w->scan_scratch.as<int64_t>(), sl);
        if (nseg > 0)
            launch_exclusive_scan(s, w->segcnt.as<int64_t>(), w->segscan.as<int64_t>(), nseg,
                                  w->scan_scratch.as<int64_t>(), sl);
        int64_t new_m = 0;
        d2h(s, &new_m, new_rp + n, 1);
        if (new_m > (int64_t)INT32_MAX)
            throw Error(PM_ERR_CAPACITY, "candidate subgraph has more than 2^31 - 1 entries");
        ccol.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(new_m, 1));
        coff.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(new_m, 1));
        cown.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(new_m, 1));
        launch_compact_fill<M>(s, src_rp, src_col, om, wl, hc, nseg, lcc, filt, new_rp,
                               w->segscan.as<int64_t>(), w->segbits.as<uint64_t>(), base_off,
                               ccol.as<int32_t>(), coff.as<int32_t>(), cown.as<int32_t>());
        c_rp = new_rp;
        c_col = ccol.as<int32_t>();
        c_off = coff.as<int32_t>();
        c_own = cown.as<int32_t>();
        c_m = new_m;
        cbuf = nb;
        nA_compact = nA;
        rl_valid = false;
        rl_graph_ok = false;
        st.candidate_entries = c_m;
        t.stop(st.ms_compact);
    }

    SearchArgs search_args(int mode, uint64_t heads, const int32_t *plan_of_head,
                           uint64_t *edge_bits) {
        SearchArgs a{};
        a.c_rp = c_rp;
        a.c_col = c_col;
        a.c_off = c_off;
        a.rp = c->rp;
        a.col = c->col;
        a.plans = T.d_plans;
        a.tedges = T.d_tedges;
        a.m0 = T.m0;
        a.rl_off = w->rloff.as<int64_t>();
        a.rl_v = w->rlv.as<int32_t>();
        a.rl_col = w->rlcol.as<int32_t>();
        a.rl_ent = w->rlent.as<int32_t>();
        a.rl_pos = w->rlpos.as<int32_t>();
        a.n0 = T.n0;
        a.mode = mode;
        a.heads = heads;
        for (int i = 0; i < kMaxK; ++i) a.plan_of_head[i] = plan_of_head[i];
        a.edge_bits = edge_bits;
        a.task_counter = ctr + C_TASK;
        a.task_chunk = 4;
        a.stripes = 1;
        a.tail_single = 0;
        a.n_queries = queries;
        a.c_cert = nullptr;
        a.exp_seen = nullptr;
        a.exp_log2 = 0;
        a.wit = nullptr;
        a.wit_flag = nullptr;
        a.wit_on = 0;
        a.qstats = nullptr;
        a.expand = 0;
        a.expand_max = c->expand_max;
        a.check_om = 0;
        a.split_budget = 0;
        a.read_first = c->read_first;
        a.split_out = nullptr;
        a.split_n = nullptr;
        a.split_cap = 0;
        a.aggregate = (ablate & PM_ABLATE_WORK_AGGREGATION) ? 0 : 1;
        a.tside = T.d_tjoin;
        a.tsame = T.d_tjoin + T.m0;
        return a;
    }

    // Role lists of the active vertices over the compacted subgraph, built
    // from the current role sets (the snapshot a constraint reads).  They
    // stay valid until the role sets, the active list or the subgraph
    // change (rl_valid), so a constraint that removed nothing lets the next
    // one reuse them.
    int64_t rl_total = 0;
    bool rl_valid = false;
    int64_t nA_lists = 0;       // tasks of the current lists (their positions)
    bool rl_graph_ok = false;   // the lists index the current candidate subgraph
    bool rl_stale = false;      // they may hold roles lost since: searches test omega
    void role_lists() {
        const int64_t nn = std::max<int64_t>(nA, 1) * T.n0;
        w->rlcnt.ensure(sizeof(int64_t) * (size_t)(nn + 1));
        w->rloff.ensure(sizeof(int64_t) * (size_t)(nn + 1));
        w->rlpos.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(c->n, 1));
        const int64_t sl = scan_scratch_len(nn);
        w->rlscan.ensure(sizeof(int64_t) * (size_t)sl);
        launch_role_count<M>(s, A, nA, c_rp, c_col, om, T.n0, w->rlcnt.as<int64_t>(),
                             w->rlpos.as<int32_t>());
        launch_exclusive_scan(s, w->rlcnt.as<int64_t>(), w->rloff.as<int64_t>(), nA * T.n0,
                              w->rlscan.as<int64_t>(), sl);
        rl_total = 0;
        d2h(s, &rl_total, w->rloff.as<int64_t>() + nA * T.n0, 1);
        // the searches keep role-list positions and row bases in 32 bits
        if (rl_total > (int64_t)INT32_MAX - 64 || nA * (int64_t)T.n0 > (int64_t)INT32_MAX - 64)
            throw Error(PM_ERR_CAPACITY, "role lists exceed 2^31 entries");
        w->rlcol.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(rl_total, 1));
        w->rlent.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(rl_total, 1));
        launch_role_fill<M>(s, A, nA, c_rp, c_col, om, T.n0, w->rloff.as<int64_t>(),
                            w->rlcol.as<int32_t>(), w->rlent.as<int32_t>());
        w->rlv.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(c->n, 1) * (size_t)(T.n0 + 1));
        launch_role_rows(s, A, nA, T.n0, w->rloff.as<int64_t>(), w->rlv.as<int32_t>());
        rl_valid = true;
        rl_stale = false;
        rl_graph_ok = true;
        nA_lists = nA;
    }

    // Lists for the next search: the current ones while valid; after role
    // sets shrank, still the current ones (a superset: the searches then
    // test every candidate's role set) if they index the current subgraph
    // and the active set has lost less than a quarter since they were
    // built; otherwise new ones.
    void ensure_lists() {
        if (rl_valid) return;
        if (rl_graph_ok && nA * 4 >= nA_lists * 3) {
            rl_valid = true;
            rl_stale = true;
            return;
        }
        role_lists();
    }

    // One non-local constraint (snapshot semantics); returns the vertices
    // changed, with the active list already updated.
    int32_t nlcc(const Constraint &k) {
        Span t(tl, s);
        ensure_lists();
        PM_HIP(hipMemsetAsync(ctr + C_TASK, 0, sizeof(int32_t), s));
        SearchArgs a = search_args(0, k.heads, k.plan_of_head, nullptr);
        a.check_om = rl_stale ? 1 : 0;
        SearchShare share(c);   // until read_control below
        launch_vertex_search<M>(s, A, nA, om, sat, a, share.grid);
        PM_HIP(hipMemsetAsync(ctr + C_CHANGED, 0, sizeof(int32_t), s));
        launch_apply<M>(s, A, nA, om, sat, k.heads, ctr + C_CHANGED);
        // the next active list comes back with the change count in one
        // round trip (discarded when nothing changed: the set is the same)
        PM_HIP(hipMemsetAsync(ctr + C_ACTIVE, 0, sizeof(int32_t), s));
        launch_collect<M>(s, A, nA, om, Aalt, ctr + C_ACTIVE);
        const Ctl cb = read_control();
        const int32_t ch = cb.w[C_CHANGED];
        if (ch) {
            rl_valid = false;
            std::swap(A, Aalt);
            nA = cb.w[C_ACTIVE];
        }
        st.constraints++;
        t.stop(st.ms_nlcc);
        return ch;
    }

    void exact(uint64_t *role_out, uint64_t *edge_out) {
        Span t(tl, s);
        const int64_t n = c->n;
        // certified roles live in sat (cleared by every apply and at start)
        const uint64_t all = T.n0 == 64 ? ~0ull : ((1ull << T.n0) - 1ull);
        unsigned long long q0 = 0, q1 = 0;
        const int64_t cwords = (c_m + 63) / 64;
        w->ccert.ensure(sizeof(uint64_t) * (size_t)std::max<int64_t>(cwords, 1));
        w->expseen.ensure(sizeof(uint64_t) << exp_log2);
        uint64_t *c_cert = w->ccert.as<uint64_t>();
        ensure_lists();
        launch_fill_u64(s, c_cert, cwords, 0ull);
        launch_fill_u64(s, w->expseen.as<uint64_t>(), 1ll << exp_log2, 0ull);
        // roles and edges known to be in the complete set count as
        // certified: no search is run for them
        if (known_roles) launch_known_roles<M>(s, A, nA, om, known_roles, sat);
        if (known_edges) launch_known_edges(s, c_m, c_own, c_off, c->rp, known_edges, c_cert);
        PM_HIP(hipMemsetAsync(qstats, 0, sizeof(unsigned long long) * 16, s));
        PM_HIP(hipMemsetAsync(ctr + C_TASK, 0, sizeof(int32_t), s));
        PM_HIP(hipMemsetAsync(queries, 0, sizeof(unsigned long long), s));
        SearchArgs a = search_args(1, all, T.vertex_plan, edge_out);
        a.check_om = rl_stale ? 1 : 0;
        a.c_cert = c_cert;
        a.exp_seen = w->expseen.as<unsigned long long>();
        a.exp_log2 = exp_log2;
        // witnesses of certified (vertex, role) pairs, for single-swap
        // certification of candidate edges (small templates only)
        // (indexed by list position: nA_lists slots)
        const int64_t wit_words = nA_lists * (int64_t)T.n0 * T.n0;
        if (c->witness && T.n0 <= 16 && nA > 0 && wit_words <= (int64_t)1 << 29) {
            w->wit.ensure(sizeof(int32_t) * (size_t)wit_words);
            w->witflag.ensure(sizeof(uint32_t) * (size_t)(nA_lists * T.n0));
            launch_fill_i32(s, w->witflag.as<int32_t>(), nA_lists * T.n0, 0);
            a.wit = w->wit.as<int32_t>();
            a.wit_flag = w->witflag.as<uint32_t>();
            a.wit_on = 1;
        }
        a.qstats = qstats;
        a.expand = a.aggregate ? c->expand : 0;
        {
            SearchShare share(c);
            launch_vertex_search<M>(s, A, nA, om, sat, a, share.grid);
            d2h(s, &q0, queries, 1);
        }
        // edge part over vertices with certified roles
        std::swap(om, sat);   // collect() reads `om`: use the certified sets
        collect(false);
        std::swap(om, sat);
        st.result_vertices = nA;
        const int64_t cap = c_m / 2 + 1;
        w->eu.ensure(sizeof(int32_t) * (size_t)cap);
        w->ew.ensure(sizeof(int32_t) * (size_t)cap);
        w->eidx.ensure(2 * sizeof(int64_t) * (size_t)cap);   // (entry, reverse entry)
        PM_HIP(hipMemsetAsync(ctr + C_NOUT, 0, sizeof(int32_t), s));
        launch_edge_candidates<M>(s, c_m, c_rp, c_own, c_col, sat, lcc, c_cert,
                                  w->eu.as<int32_t>(), w->ew.as<int32_t>(),
                                  w->eidx.as<int64_t>(), ctr + C_NOUT, cap, a);
        a.wit_on = 0;
        int64_t ne = read_ctr(C_NOUT);
        if (ne > cap) throw Error(PM_ERR_CAPACITY, "edge candidate capacity exceeded");
        st.edge_candidates = ne;
        if (ne > 0) {
            w->edge_plan_ids.ensure(sizeof(int32_t) * std::max<size_t>(T.edge_plans.size(), 1));
            PM_HIP(hipMemcpyAsync(w->edge_plan_ids.p, T.edge_plans.data(),
                                  sizeof(int32_t) * T.edge_plans.size(), hipMemcpyHostToDevice, s));
            if (c->relist) {
                // role lists over the certified role sets (the exact roles):
                // the edge searches then scan only vertices that can take
                // part in a match
                std::swap(om, sat);
                role_lists();
                std::swap(om, sat);
                rl_valid = false;   // lists of the certified sets, not of omega
                a.rl_off = w->rloff.as<int64_t>();
                a.rl_v = w->rlv.as<int32_t>();
                a.rl_col = w->rlcol.as<int32_t>();
                a.rl_ent = w->rlent.as<int32_t>();
                a.rl_pos = w->rlpos.as<int32_t>();
                a.check_om = 0;
            } else {
                // the edge searches read the certified role sets, a subset
                // of those the role lists were built from
                a.check_om = 1;
            }
            PM_HIP(hipMemsetAsync(ctr + C_TASK, 0, sizeof(int32_t), s));
            PM_HIP(hipMemsetAsync(queries, 0, sizeof(unsigned long long), s));
            // the dealing counter is 32-bit: it must stay below 2^31 after
            // every chunk and every wave's final fetch
            SearchShare share(c);   // until the split rounds are done
            int64_t chunk = c->edge_chunk;
            const int64_t waves = (int64_t)share.grid * 4;
            const int64_t tail = std::min<int64_t>(c->edge_tail, std::min<int64_t>(ne, 1 << 24));
            while ((ne + chunk - 1) / chunk + tail + c->edge_stripes + waves >= INT32_MAX)
                chunk *= 2;
            a.task_chunk = (int)chunk;
            a.stripes = c->edge_stripes;
            a.tail_single = tail;
            if (c->split_budget > 0) {
                // searches past the budget hand on their unexplored ranges,
                // which later launches (double-buffered lists) search
                for (DevBuf *b : {&w->split[0], &w->split[1]})
                    b->ensure(sizeof(SplitTask) * (size_t)split_cap);
                PM_HIP(hipMemsetAsync(ctr + C_SPLIT, 0, sizeof(int32_t), s));
                a.split_budget = c->split_budget;
                a.split_out = w->split[0].as<SplitTask>();
                a.split_n = ctr + C_SPLIT;
                a.split_cap = split_cap;
            }
            if (!c->expand_edges) a.expand = 0;
            launch_edge_search<M>(s, w->eu.as<int32_t>(), w->ew.as<int32_t>(),
                                  w->eidx.as<int64_t>(), ne, sat, sat,
                                  w->edge_plan_ids.as<int32_t>(), (int32_t)T.edge_plans.size(),
                                  a, share.grid);
            if (c->split_budget > 0) {
                int cur = 0;
                int64_t rounds = 0;
                for (int64_t nt = read_ctr(C_SPLIT); nt > 0; nt = read_ctr(C_SPLIT)) {
                    // every split task covers strictly less of its search
                    // than the search that made it; this bound only guards
                    // against a broken invariant
                    if (++rounds > (int64_t)1 << 20)
                        throw Error(PM_ERR_CAPACITY, "split searches did not finish");
                    st.split_tasks += nt;
                    // split tasks of later rounds are parts of searches
                    // already cut: a budget four times larger per round
                    // keeps them from being cut into ever smaller pieces
                    a.split_budget = std::min<int64_t>(a.split_budget * 4, (int64_t)1 << 40);
                    const SplitTask *in = w->split[cur].as<SplitTask>();
                    cur ^= 1;
                    a.split_out = w->split[cur].as<SplitTask>();
                    PM_HIP(hipMemsetAsync(ctr + C_SPLIT, 0, sizeof(int32_t), s));
                    PM_HIP(hipMemsetAsync(ctr + C_TASK, 0, sizeof(int32_t), s));
                    launch_split_search<M>(s, in, nt, w->eu.as<int32_t>(), w->ew.as<int32_t>(),
                                           w->eidx.as<int64_t>(), sat, sat,
                                           w->edge_plan_ids.as<int32_t>(), a, share.grid);
                }
                a.split_budget = 0;
            }
            d2h(s, &q1, queries, 1);
        }
        launch_edges_from_cert(s, c_m, c_rp, c_col, c_own, c_off, c->rp, c_cert, edge_out);
        launch_widen<M>(s, n, sat, role_out);
        unsigned long long qs[16];
        d2h(s, qs, qstats, 16);
        const double tick_ms = c->wall_khz > 0 ? 1.0 / (double)c->wall_khz : 0.0;
        st.vertex_queries += (int64_t)q0;
        st.edge_queries += (int64_t)q1;
        st.vq_pos += (int64_t)qs[0];
        st.vq_neg += (int64_t)qs[1];
        st.wave_ms_vq_pos += (double)qs[2] * tick_ms;
        st.wave_ms_vq_neg += (double)qs[3] * tick_ms;
        st.eq_pos += (int64_t)qs[4];
        st.eq_neg += (int64_t)qs[5];
        st.wave_ms_eq_pos += (double)qs[6] * tick_ms;
        st.wave_ms_eq_neg += (double)qs[7] * tick_ms;
        st.wave_ms_certify += (double)(qs[8] + qs[9]) * tick_ms;
        st.wave_ms_expand += (double)qs[10] * tick_ms;
        st.expand_scans += (int64_t)qs[11];
        st.expand_candidates += (int64_t)qs[12];
        st.expand_valid += (int64_t)qs[13];
        st.witness_edges += (int64_t)qs[14];
        st.join_edges += (int64_t)qs[15];
        t.stop(st.ms_exact);
    }

    // ---- constraint loop -----------------------------------------------------
    // Device block of the ordering state: counts [64], counts0 [64], pick.
    unsigned long long *ord_counts() { return w->ord.as<unsigned long long>(); }
    unsigned long long *ord_counts0() { return w->ord.as<unsigned long long>() + kMaxK; }
    OrderPick *ord_pick() {
        return reinterpret_cast<OrderPick *>(w->ord.as<unsigned long long>() + 2 * kMaxK);
    }

    void role_totals(unsigned long long *dst) {
        launch_fill_u64(s, reinterpret_cast<uint64_t *>(dst), kMaxK, 0ull);
        launch_role_totals<M>(s, A, nA, om, T.n0, dst);
    }

    // Features (and, with a model, scores) at the current state; forced >= 0
    // reports that constraint, otherwise the best remaining one is chosen.
    OrderPick pick(int forced, uint64_t remaining, int done) {
        role_totals(ord_counts());
        OrderArgs a{};
        a.counts = ord_counts();
        a.counts0 = ord_counts0();
        a.cons = T.d_cdesc;
        a.w = c->has_model ? c->model.as<float>() : nullptr;
        for (int q = 0; q < T.n0; ++q) {
            const int L = T.labels[(size_t)q];
            a.role_freq[q] = (size_t)L < c->label_freq.size() ? (uint64_t)c->label_freq[(size_t)L] : 0;
        }
        a.remaining = remaining;
        a.n_active = nA;
        a.n_cons = (int32_t)T.constraints.size();
        a.done = done;
        a.forced = forced;
        a.n0 = T.n0;
        launch_order_select(s, a, ord_pick());
        OrderPick p{};
        d2h(s, &p, ord_pick(), 1);
        return p;
    }

    int64_t roles_now() {
        role_totals(ord_counts());
        unsigned long long h[kMaxK];
        d2h(s, h, ord_counts(), kMaxK);
        int64_t r = 0;
        for (int q = 0; q < T.n0; ++q) r += (int64_t)h[q];
        return r;
    }

    // Main loop over the non-local constraints: NLCC, then LCC to the
    // fixpoint when anything changed.  In the learned mode the next
    // constraint is the remaining one of largest model score.  Constraints
    // in skip_mask (applied to an imported state already) are not checked
    // again but count as done.
    int64_t n_trace = 0;
    void constraint_loop(const std::vector<int> &order, bool learned, int stop_after) {
        const int K = (int)T.constraints.size();
        pm_trace_entry *trace = opt && opt->trace && opt->trace_cap > 0 ? opt->trace : nullptr;
        const int64_t cap = trace ? opt->trace_cap : 0;
        const bool featured = learned || trace;
        const uint64_t all = K == 64 ? ~0ull : ((1ull << K) - 1ull);
        const uint64_t skipped = skip_mask & all;
        done_mask = skipped;
        if (featured && K > 0) {
            w->ord.ensure(sizeof(unsigned long long) * 2 * kMaxK + sizeof(OrderPick) + 64);
            role_totals(ord_counts0());
        }
        uint64_t remaining = all & ~skipped;
        int done = __builtin_popcountll(skipped);
        size_t pos = 0;
        int64_t pending_after = -1;   // trace entry waiting for roles_after
        int checked = 0;
        const int limit = opt && opt->limit_checks ? std::max(0, opt->max_checks) : K + 1;
        while (done < K) {
            if (stop_after >= 0 && done >= stop_after) break;
            if (checked >= limit) break;
            if (nA == 0) break;
            OrderPick pk{};
            int k = -1;
            if (!learned) {
                while (pos < order.size() && ((skipped >> order[pos]) & 1ull)) ++pos;
                if (pos >= order.size()) break;
                k = order[pos++];
            }
            const int64_t active_before = nA;
            // the learned order has no choice to make for the last remaining
            // constraint (unless a threshold or the trace needs its score)
            const bool forced_last = learned && !trace && !(opt && opt->learned_stop) &&
                                     __builtin_popcountll(remaining) == 1;
            if (forced_last) {
                k = __builtin_ctzll(remaining);
            } else if (featured) {
                pk = pick(learned ? -1 : k, remaining, done);
                if (pending_after >= 0) {
                    trace[pending_after].roles_after = (int64_t)pk.roles;
                    pending_after = -1;
                }
                if (learned) {
                    k = pk.idx;
                    if (k < 0) break;
                    if (opt->learned_stop && !(pk.score >= opt->learned_min_score)) {
                        if (n_trace < cap) {
                            pm_trace_entry &e = trace[n_trace++];
                            e = pm_trace_entry{};
                            e.constraint = -1;
                            e.roles_before = e.roles_after = (int64_t)pk.roles;
                            e.active_before = active_before;
                            e.score = pk.score;
                            for (int i = 0; i < kMlpOut; ++i) e.predicted[i] = pk.pred[i];
                            for (int i = 0; i < kMlpIn; ++i) e.features[i] = pk.feat[i];
                        }
                        break;
                    }
                }
            }
            // per-step device time only for the trace (it waits)
            std::unique_ptr<Timer> tt;
            if (trace && n_trace < cap) tt.reset(new Timer(s));
            int32_t ch = nlcc(T.constraints[(size_t)k]);
            if (ch && nA > 0) lcc_fixpoint();
            const double ms = tt ? tt->stop() : 0.0;
            remaining &= ~(1ull << k);
            done_mask |= 1ull << k;
            ++done;
            ++checked;
            if (trace && n_trace < cap) {
                pm_trace_entry &e = trace[n_trace];
                e = pm_trace_entry{};
                e.constraint = k;
                e.changed = ch;
                e.roles_before = (int64_t)pk.roles;
                e.roles_after = -1;
                e.active_before = active_before;
                e.ms = (float)ms;
                e.score = pk.score;
                for (int i = 0; i < kMlpOut; ++i) e.predicted[i] = pk.pred[i];
                for (int i = 0; i < kMlpIn; ++i) e.features[i] = pk.feat[i];
                pending_after = n_trace++;
            }
        }
        if (pending_after >= 0) trace[pending_after].roles_after = nA > 0 ? roles_now() : 0;
        st.trace_entries = n_trace;
    }

    // Role initialisation (vertex state and initialisation algorithm) and,
    // from the neighbour-label count index when there is one, the first LCC
    // sweep; an imported state is intersected in; omega's active list.
    // Returns true when the first sweep has been applied.
    bool init_state_and_first_sweep(bool allow_counted) {
        const int64_t n = c->n;
        // the counts of the label-pair subgraph when it covers the template
        // (the sweep reads a vertex's counts only for labels of template
        // neighbours of its roles, pairs the subgraph keeps whole), else
        // the count index of the graph
        const bool from_pairs = c->pair_cnt_nlab > 0 && pairs_cover();
        const int cnl = from_pairs ? c->pair_cnt_nlab : c->nlab;
        const bool counted = allow_counted && cnl > 0 && T.n0 > 1 && !candidate;
        if (counted) {
            // first LCC sweep from the neighbour-label count index (it also
            // initialises omega)
            Span t(tl, s);
            Span k(tl, s);
            const int32_t *nd = T.d_need;
            launch_first_sweep_counts<M>(
                s, n, from_pairs ? c->pair_cnt_stride : c->cnt_stride, (const uint8_t *)c->labels,
                T.d_init_lut, (int)std::min<int64_t>(T.init_lut_len, 256),
                from_pairs ? c->pair_cnt.as<uint8_t>() : c->lab_cnt.as<uint8_t>(), cnl, nd,
                nd + T.n0 + 1, nd + T.n0 + 1 + T.need_lab.size(), T.n0, om);
            k.stop(st.ms_sweep_kernel);
            // compulsory bytes: every label, for each vertex the count bytes
            // of the labels its initial roles need (a function of its
            // label), and omega written
            int64_t reads = 0;
            for (size_t L = 0; L < c->label_freq.size() && L < 256; ++L) {
                uint64_t used = 0;
                for (int q = 0; q < T.n0; ++q)
                    if (T.labels[(size_t)q] == (int)L) used |= T.need_labmask[(size_t)q];
                const uint64_t in_index = cnl >= 64 ? ~0ull : ((1ull << cnl) - 1ull);
                reads += c->label_freq[L] * (int64_t)__builtin_popcountll(used & in_index);
            }
            st.first_sweep_vertices = n;
            st.first_sweep_entries = 0;
            st.first_sweep_bytes = n + reads + (int64_t)sizeof(M) * n;
            if (init_state) launch_and_state<M>(s, n, om, init_state);
            PM_HIP(hipMemsetAsync(sat, 0, sizeof(M) * (size_t)n, s));
            collect(true);
            t.stop(st.ms_first_sweep, &st.ms_lcc);
            st.lcc_sweeps++;
        } else {
            Span t(tl, s);
            w->actbits.ensure(sizeof(uint64_t) * (size_t)std::max<int64_t>((n + 63) / 64, 1));
            wl.act_bits = w->actbits.as<uint64_t>();
            launch_init_roles<M>(s, n, c->labels, c->label_bytes, T.d_init_lut, T.init_lut_len, om,
                                 w->actbits.as<uint64_t>());
            if (init_state) launch_and_state<M>(s, n, om, init_state);
            PM_HIP(hipMemsetAsync(sat, 0, sizeof(M) * (size_t)n, s));
            collect(true);
            t.stop(st.ms_init);
        }
        return counted;
    }

    // Final step of an acyclic template with one repeated-label pair: the
    // complete set from sweeps along the path between the pair over the
    // LCC fixpoint (launch_tree_exact), no searches.  The list positions
    // are overwritten, so the role lists are no longer valid.
    void tree_final(uint64_t *role_out, uint64_t *edge_out) {
        Span t(tl, s);
        const int64_t n = c->n;
        const TreePlan &tp = T.tree;
        w->rlpos.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1));
        w->tsum.ensure(sizeof(int2) * 2 * (size_t)(tp.k + 1) * (size_t)std::max<int64_t>(nA, 1));
        rl_valid = false;
        rl_graph_ok = false;
        PM_HIP(hipMemsetAsync(sat, 0, sizeof(M) * (size_t)n, s));
        launch_tree_exact<M>(s, A, nA, om, c_m, c_own, c_col, c_off, c->rp, tp,
                             w->rlpos.as<int32_t>(), w->tsum.as<int2>(), sat, edge_out);
        launch_widen<M>(s, n, sat, role_out);
        std::swap(om, sat);   // collect() reads `om`: count the vertices kept
        collect(false);
        std::swap(om, sat);
        st.result_vertices = nA;
        t.stop(st.ms_exact);
    }

    // Whole prune.  edge_out may be null (state export: no edge output).
    void run(uint64_t *role_out, uint64_t *edge_out) {
        Span total(tl, s);
        const int64_t n = c->n, m = c->m;
        if (opt) {
            init_state = opt->init_state;
            skip_mask = init_state ? opt->skip_mask : 0;
            known_roles = opt->known_roles;
            known_edges = opt->known_edges;
        }
        zero_counters();
        if (edge_out) launch_fill_u64(s, edge_out, (m + 63) / 64, 0ull);
        const bool counted = init_state_and_first_sweep(true);
        Graph full{c->rp, c->col};
        if (!counted && T.n0 > 1 && nA > 0) {
            // first sweep over the full graph
            Span t(tl, s);
            bin(full);
            st.first_sweep_vertices = nA;
            st.first_sweep_entries = binned_entries;
            int32_t ch = sweep(full, true);
            t.stop(st.ms_first_sweep, &st.ms_lcc);
            if (ch) collect(false);
        }
        // candidate subgraph (edge elimination) and the rest of LCC on it
        compact();
        if (T.n0 > 1 && nA > 0) lcc_fixpoint();
        int stop_after = opt ? opt->stop_after : -1;
        const int K = (int)T.constraints.size();
        const bool learned = opt && opt->order_mode == PM_ORDER_LEARNED;
        std::vector<int> order;
        if (opt && opt->order_mode == PM_ORDER_GIVEN) {
            if (opt->n_order != K)
                throw Error(PM_ERR_INVALID_ARG, "order length differs from the constraint count");
            std::vector<char> seen((size_t)K, 0);
            for (int i = 0; i < opt->n_order; ++i) {
                int k = opt->order[i];
                if (k < 0 || k >= K || seen[k])
                    throw Error(PM_ERR_INVALID_ARG, "order is not a permutation");
                seen[k] = 1;
                order.push_back(k);
            }
        } else {
            for (int i = 0; i < K; ++i) order.push_back(i);
        }
        // An acyclic template with one repeated-label pair a, b has at most
        // one non-local constraint, the path constraint between a and b
        // (heads at both ends; none when they are under three hops apart); the
        // path sweeps of tree_final are that token walk with the tokens at a
        // vertex aggregated to the smallest and largest origin, run at the
        // LCC fixpoint, and they give the complete set directly (a tree at
        // the fixpoint leaves injectivity as the only open condition).  So a
        // full prune of such a template goes from the LCC fixpoint straight
        // to the sweeps; a run that stops after some constraints (state
        // export, ablations) keeps the search-based loop.
        const bool swept = T.tree_pair && c->tree_exact && stop_after < 0 && !candidate &&
                           edge_out && !(opt && opt->limit_checks);
        if (!candidate && !swept) constraint_loop(order, learned, stop_after);
        if (candidate || stop_after >= 0 || T.acyclic_unique || T.n0 == 1 || !edge_out) {
            // omega and its implied edge state (exact for acyclic unique-label
            // templates: LCC alone suffices)
            launch_widen<M>(s, n, om, role_out);
            if (T.n0 > 1 && edge_out)
                launch_active_edges<M>(s, A, nA, c_rp, c_col, c_off, c->rp, om, lcc, edge_out);
            st.result_vertices = nA;
        } else if (T.tree_pair && c->tree_exact) {
            // the sweeps make k + depth + 2 passes of ~16 bytes per entry;
            // a compaction costs ~20 bytes per vertex of the graph (row
            // lengths cleared, counted, scanned into the row pointer) on
            // top of its own entries, so it can pay only when the entries
            // outweigh the vertices
            const int64_t passes = T.tree.k + T.tree.depth + 2;
            if (nA > 0 && nA * 4 < nA_compact * 3 && c_m * passes * 16 > c->n * 20)
                compact(true);
            tree_final(role_out, edge_out);
        } else {
            // a fresh candidate subgraph only when the active set has shrunk
            // by a quarter since the last one (any superset of the edges
            // between active vertices serves the final search; otherwise the
            // current one and its role lists are reused)
            if (nA > 0 && nA * 4 < nA_compact * 3) compact(true);
            exact(role_out, edge_out);
        }
        st.done_mask = done_mask;
        total.stop(st.ms_total);
        tl.resolve();
        st.workspace_bytes = (int64_t)w->bytes_held();
    }

    // ---- match counting (termination and output: enumeration/counting on
    // the pruned graph) ----------------------------------------------------
    // Maps of the full template within omega0 AND state, counted from every
    // compacted entry that can hold the chosen template edge.
    pm_match_count count_matches(const uint64_t *state, int32_t *maps_out, int64_t cap,
                                 uint64_t limit) {
        Span total(tl, s);
        pm_match_count r{};
        r.complete = 1;
        init_state = state;
        zero_counters();
        init_state_and_first_sweep(false);
        const int64_t n = c->n;
        (void)n;
        if (T.n0 == 1) {
            r.maps = (uint64_t)nA;
            r.roots = nA;
            const int64_t wr = std::min<int64_t>(std::max<int64_t>(cap, 0), nA);
            if (maps_out && wr > 0)
                PM_HIP(hipMemcpyAsync(maps_out, A, sizeof(int32_t) * (size_t)wr,
                                      hipMemcpyDeviceToDevice, s));
            r.written = maps_out ? wr : 0;
        } else if (nA > 0) {
            compact();
            role_lists();
            // root template edge: the one whose end roles are held by the
            // fewest vertices
            w->ord.ensure(sizeof(unsigned long long) * 2 * kMaxK + sizeof(OrderPick) + 64);
            role_totals(ord_counts());
            unsigned long long h[kMaxK];
            d2h(s, h, ord_counts(), kMaxK);
            int best = 0;
            unsigned long long bc = ~0ull;
            for (int i = 0; i < T.m0; ++i) {
                const unsigned long long cc = h[T.edges[(size_t)i].first] + h[T.edges[(size_t)i].second];
                if (cc < bc) {
                    bc = cc;
                    best = i;
                }
            }
            const int32_t plan = T.edge_plans[(size_t)(2 * best)];
            const SearchPlan &P = T.plans[(size_t)plan];
            w->edge_plan_ids.ensure(sizeof(int32_t));
            PM_HIP(hipMemcpyAsync(w->edge_plan_ids.p, &plan, sizeof(int32_t), hipMemcpyHostToDevice, s));
            const int64_t cap_t = std::max<int64_t>(c_m, 1);
            w->eu.ensure(sizeof(int32_t) * (size_t)cap_t);
            w->ew.ensure(sizeof(int32_t) * (size_t)cap_t);
            PM_HIP(hipMemsetAsync(ctr + C_NOUT, 0, sizeof(int32_t), s));
            launch_count_tasks<M>(s, c_m, c_own, c_col, om, P.pin[0], P.pin[1], w->eu.as<int32_t>(),
                                  w->ew.as<int32_t>(), ctr + C_NOUT, cap_t);
            const int64_t ne = read_ctr(C_NOUT);
            if (ne > cap_t) throw Error(PM_ERR_CAPACITY, "count task capacity exceeded");
            r.roots = ne;
            unsigned long long *tot = reinterpret_cast<unsigned long long *>(ctr + C_COUNT_U64);
            unsigned long long *wrt = reinterpret_cast<unsigned long long *>(ctr + C_WRITTEN_U64);
            if (ne > 0) {
                const uint64_t allr = T.n0 == 64 ? ~0ull : ((1ull << T.n0) - 1ull);
                SearchArgs a = search_args(1, allr, T.vertex_plan, nullptr);
                a.task_chunk = std::max(1, c->edge_chunk);
                PM_HIP(hipMemsetAsync(ctr + C_TASK, 0, sizeof(int32_t), s));
                if (c->split_budget > 0) {
                    for (DevBuf *b : {&w->split[0], &w->split[1]})
                        b->ensure(sizeof(SplitTask) * (size_t)split_cap);
                    PM_HIP(hipMemsetAsync(ctr + C_SPLIT, 0, sizeof(int32_t), s));
                    a.split_budget = c->split_budget;
                    a.split_out = w->split[0].as<SplitTask>();
                    a.split_n = ctr + C_SPLIT;
                    a.split_cap = split_cap;
                }
                SearchShare share(c);
                launch_count_search<M>(s, w->eu.as<int32_t>(), w->ew.as<int32_t>(), ne, om,
                                       w->edge_plan_ids.as<int32_t>(), a, maps_out,
                                       maps_out ? cap : 0, wrt, tot, limit, ctr + C_STOP,
                                       share.grid);
                if (c->split_budget > 0) {
                    int cur = 0;
                    int64_t rounds = 0;
                    for (int64_t nt = read_ctr(C_SPLIT); nt > 0; nt = read_ctr(C_SPLIT)) {
                        if (++rounds > (int64_t)1 << 20)
                            throw Error(PM_ERR_CAPACITY, "split searches did not finish");
                        st.split_tasks += nt;
                        a.split_budget = std::min<int64_t>(a.split_budget * 4, (int64_t)1 << 40);
                        const SplitTask *in = w->split[cur].as<SplitTask>();
                        cur ^= 1;
                        a.split_out = w->split[cur].as<SplitTask>();
                        PM_HIP(hipMemsetAsync(ctr + C_SPLIT, 0, sizeof(int32_t), s));
                        PM_HIP(hipMemsetAsync(ctr + C_TASK, 0, sizeof(int32_t), s));
                        launch_count_split<M>(s, in, nt, w->eu.as<int32_t>(), w->ew.as<int32_t>(),
                                              om, w->edge_plan_ids.as<int32_t>(), a, maps_out,
                                              maps_out ? cap : 0, wrt, tot, limit, ctr + C_STOP,
                                              share.grid);
                    }
                }
            }
            unsigned long long both[2] = {0, 0};
            d2h(s, both, tot, 2);
            r.complete = read_ctr(C_STOP) ? 0 : 1;
            r.maps = both[0];
            r.written = maps_out ? (int64_t)std::min<unsigned long long>(both[1], (unsigned long long)std::max<int64_t>(cap, 0)) : 0;
        }
        double ms_total = 0.0;
        total.stop(ms_total);
        tl.resolve();
        r.ms_total = ms_total;
        return r;
    }
};

void load_template_device(pm_ctx *c, CompiledTemplate &T) {
    PM_HIP(hipMalloc(&T.d_plans, sizeof(SearchPlan) * std::max<size_t>(T.plans.size(), 1)));
    PM_HIP(hipMemcpy(T.d_plans, T.plans.data(), sizeof(SearchPlan) * T.plans.size(),
                     hipMemcpyHostToDevice));
    std::vector<int32_t> te;
    for (auto &e : T.edges) {
        te.push_back(e.first);
        te.push_back(e.second);
    }
    PM_HIP(hipMalloc(&T.d_tedges, sizeof(int32_t) * std::max<size_t>(te.size(), 2)));
    if (!te.empty())
        PM_HIP(hipMemcpy(T.d_tedges, te.data(), sizeof(int32_t) * te.size(), hipMemcpyHostToDevice));
    // bridges of G0: edge i is one iff its ends fall apart without it; the
    // side of its first end is then kept (for joining two matches across it)
    std::vector<uint64_t> join((size_t)T.m0 + (size_t)T.n0, 0ull);
    for (int i = 0; i < T.m0; ++i) {
        uint64_t seen = 1ull << T.edges[i].first, grow = seen;
        while (grow) {
            uint64_t next = 0;
            for (int j = 0; j < T.m0; ++j) {
                if (j == i) continue;
                const uint64_t ea = 1ull << T.edges[j].first, eb = 1ull << T.edges[j].second;
                if ((grow & ea) && !(seen & eb)) next |= eb;
                if ((grow & eb) && !(seen & ea)) next |= ea;
            }
            seen |= next;
            grow = next;
        }
        if (!((seen >> T.edges[i].second) & 1ull)) join[(size_t)i] = seen;
    }
    for (int q = 0; q < T.n0; ++q) join[(size_t)T.m0 + q] = T.label_mask_of[q] & ~(1ull << q);
    PM_HIP(hipMalloc(&T.d_tjoin, sizeof(uint64_t) * std::max<size_t>(join.size(), 1)));
    if (!join.empty())
        PM_HIP(hipMemcpy(T.d_tjoin, join.data(), sizeof(uint64_t) * join.size(),
                         hipMemcpyHostToDevice));
    int maxl = 0;
    for (int q = 0; q < T.n0; ++q) maxl = std::max(maxl, T.labels[q]);
    std::vector<uint64_t> lut((size_t)maxl + 1, 0);
    for (int q = 0; q < T.n0; ++q) lut[T.labels[q]] |= 1ull << q;
    T.init_lut_len = (int64_t)lut.size();
    PM_HIP(hipMalloc(&T.d_init_lut, sizeof(uint64_t) * lut.size()));
    PM_HIP(hipMemcpy(T.d_init_lut, lut.data(), sizeof(uint64_t) * lut.size(), hipMemcpyHostToDevice));
    std::vector<int32_t> need(T.need_off);
    need.insert(need.end(), T.need_lab.begin(), T.need_lab.end());
    need.insert(need.end(), T.need_min.begin(), T.need_min.end());
    PM_HIP(hipMalloc(&T.d_need, sizeof(int32_t) * std::max<size_t>(need.size(), 1)));
    PM_HIP(hipMemcpy(T.d_need, need.data(), sizeof(int32_t) * need.size(), hipMemcpyHostToDevice));
    std::vector<ConstraintDesc> cd;
    for (const Constraint &k : T.constraints)
        cd.push_back(ConstraintDesc{k.vmask, k.heads, (int32_t)k.edges.size(), k.kind});
    PM_HIP(hipMalloc(&T.d_cdesc, sizeof(ConstraintDesc) * std::max<size_t>(cd.size(), 1)));
    if (!cd.empty())
        PM_HIP(hipMemcpy(T.d_cdesc, cd.data(), sizeof(ConstraintDesc) * cd.size(), hipMemcpyHostToDevice));
    (void)c;
}

void free_template_device(CompiledTemplate &T) {
    if (T.d_plans) (void)hipFree(T.d_plans);
    if (T.d_tedges) (void)hipFree(T.d_tedges);
    if (T.d_tjoin) (void)hipFree(T.d_tjoin);
    if (T.d_init_lut) (void)hipFree(T.d_init_lut);
    if (T.d_cdesc) (void)hipFree(T.d_cdesc);
    if (T.d_need) (void)hipFree(T.d_need);
    T.d_cdesc = nullptr;
    T.d_need = nullptr;
    T.d_plans = nullptr;
    T.d_tedges = nullptr;
    T.d_tjoin = nullptr;
    T.d_init_lut = nullptr;
}

void validate_graph(int64_t n, int64_t m, const int64_t *rp, const int32_t *col) {
    if (rp[0] != 0 || rp[n] != m) throw Error(PM_ERR_GRAPH, "row_ptr[0] must be 0 and row_ptr[n] = m");
    for (int64_t v = 0; v < n; ++v) {
        if (rp[v + 1] < rp[v]) throw Error(PM_ERR_GRAPH, "row_ptr not monotone");
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
            int32_t w = col[e];
            if (w < 0 || w >= n) throw Error(PM_ERR_GRAPH, "column index out of range");
            if (w == v) throw Error(PM_ERR_GRAPH, "self-loop");
            if (e > rp[v] && col[e - 1] >= w) throw Error(PM_ERR_GRAPH, "row not strictly sorted");
            // symmetric: v must appear in row w
            const int32_t *b = col + rp[w], *en = col + rp[w + 1];
            if (!std::binary_search(b, en, (int32_t)v)) throw Error(PM_ERR_GRAPH, "graph not symmetric");
        }
    }
}

template <typename F>
int guarded(F &&f) {
    try {
        f();
        g_last_error.clear();
        return PM_OK;
    } catch (const Error &e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return PM_ERR_OOM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return PM_ERR_HIP;
    }
}

// (Re)build the neighbour-label count index of the loaded graph (one pass
// over the CSR), timed with events on the context stream.
void build_count_index(pm_ctx *c) {
    const int nlab = c->index_nlab;
    const int64_t n = c->n;
    const int64_t np = (n + 255) / 256 * 256;
    c->lab_cnt.ensure((size_t)np * (size_t)nlab);
    c->cnt_stride = np;
    CountIndexHubs h;
    h.n_hubs = c->idx_hubs;
    h.n_segs = c->idx_segs;
    h.hub_v = c->idx_hub_v.as<int32_t>();
    h.seg_slot = c->idx_seg_slot.as<int32_t>();
    h.seg_b = c->idx_seg_b.as<int64_t>();
    h.seg_e = c->idx_seg_e.as<int64_t>();
    h.hub_cnt = c->idx_hub_cnt.as<uint32_t>();
    hipEvent_t a, b;
    PM_HIP(hipEventCreate(&a));
    PM_HIP(hipEventCreate(&b));
    PM_HIP(hipEventRecord(a, c->stream));
    launch_label_count(c->stream, n, np, c->rp, c->col, (const uint8_t *)c->labels, nlab,
                       c->lab_cnt.as<uint8_t>(), h);
    PM_HIP(hipGetLastError());
    PM_HIP(hipEventRecord(b, c->stream));
    PM_HIP(hipEventSynchronize(b));
    float ms = 0;
    PM_HIP(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    c->ms_count_index = ms;
    c->nlab = nlab;
}

int workers_for(const pm_options *opt, int32_t count) {
    int nw = 1;
    if (opt && opt->batch_streams > 1 && count > 1)
        nw = std::min<int>(std::min<int>(opt->batch_streams, 16), count);
    return nw;
}

void ensure_workers(pm_ctx *c, int nw) {
    while ((int)c->scratch.size() < nw) {
        auto sc = std::make_unique<Scratch>();
        if (c->scratch.empty()) {
            sc->stream = c->stream;
        } else {
            PM_HIP(hipStreamCreateWithFlags(&sc->stream, hipStreamNonBlocking));
            sc->own_stream = true;
        }
        c->scratch.push_back(std::move(sc));
    }
}

// Upper bound of the scratch one template's prune takes (see
// pm_workspace_size): every buffer at its largest, the compacted subgraph
// bounded by mt = the entries of the vertices whose label occurs in the
// template, the active vertices by nt = the vertices of those labels, the
// role lists by mt times the largest number of template vertices sharing a
// label.  Each buffer is rounded up to the arena's 256-byte alignment.
size_t workspace_bound(const pm_ctx *c, const CompiledTemplate &T, int exp_log2, int64_t split_cap) {
    const int64_t n = std::max<int64_t>(c->n, 1);
    int64_t mt = 0, nt = 0;
    std::vector<int> mult;
    for (int q = 0; q < T.n0; ++q) {
        const int L = T.labels[(size_t)q];
        bool seen = false;
        for (int r = 0; r < q; ++r)
            if (T.labels[(size_t)r] == L) seen = true;
        if (seen) continue;
        if ((size_t)L < c->label_degsum.size()) mt += c->label_degsum[(size_t)L];
        if ((size_t)L < c->label_freq.size()) nt += c->label_freq[(size_t)L];
    }
    int maxmult = 1;
    for (int q = 0; q < T.n0; ++q) {
        int k = 0;
        for (int r = 0; r < T.n0; ++r) k += T.labels[(size_t)r] == T.labels[(size_t)q];
        maxmult = std::max(maxmult, k);
    }
    mt = std::max<int64_t>(mt, 1);
    nt = std::max<int64_t>(nt, 1);
    const int64_t M = T.mask_bytes;
    const int64_t segs = std::max<int64_t>(c->seg_cap, 1), hubs = std::max<int64_t>(c->hub_cap, 1);
    const int64_t n0 = T.n0;
    size_t total = 0;
    auto add = [&](int64_t b) { total += (size_t)((std::max<int64_t>(b, 256) + 255) / 256 * 256); };
    add(M * n); add(M * n);                                   // omega, sat
    add(4 * n); add(4 * n);                                   // active lists
    add(4 * n * kNumBins);                                    // degree bins
    add(C_TOTAL_BYTES);                                       // counters
    add(segs * (4 + 8 + 8 + 4) + hubs * (4 + 4 + 8 + 4 * kMaxCount + 4) + 256);
    add(8 * segs); add(8 * (segs + 1)); add(8 * segs * (kHubSegment / kWave));
    add(4 * (n + 1)); add(8 * (n + 1)); add(8 * (n + 1));     // cdeg, crp, crp2
    add(8 * scan_scratch_len(std::max<int64_t>(n, segs)));
    for (int i = 0; i < 6; ++i) add(4 * mt);                  // two sets of c_col/c_off/c_own
    add(4 * ((n + 255) / 256));                               // active filter
    add(8 * ((n + 63) / 64));                                 // initial-role bitmap
    add(8 * ((mt + 63) / 64));                                // certified entries
    add((int64_t)sizeof(uint64_t) << exp_log2);               // swap-scan table
    add(4 * (mt / 2 + 1)); add(4 * (mt / 2 + 1)); add(16 * (mt / 2 + 1));   // edge tasks
    add(4 * std::max<int64_t>(2 * T.m0, 1));
    add(4 * std::max<int64_t>(mt, 1)); add(4 * std::max<int64_t>(mt, 1));    // count tasks
    if (c->witness && T.n0 <= 16) {
        add(4 * std::min<int64_t>(nt * n0 * n0, (int64_t)1 << 29));
        add(4 * nt * n0);
    }
    add(8 * (nt * n0 + 1)); add(8 * (nt * n0 + 1));           // role-list counts, offsets
    add(4 * n);                                               // list positions
    add(4 * n * (n0 + 1));                                    // list bounds by vertex
    add(4 * mt * maxmult); add(4 * mt * maxmult);             // role lists, entries
    add(8 * scan_scratch_len(nt * n0));
    add((int64_t)sizeof(unsigned long long) * 2 * kMaxK + (int64_t)sizeof(OrderPick) + 64);
    if (c->split_budget > 0) {
        add((int64_t)sizeof(SplitTask) * split_cap);
        add((int64_t)sizeof(SplitTask) * split_cap);
    }
    if (T.tree_pair) add(16 * n0 * nt);                       // path summaries
    return total;
}

// Label-preserving automorphisms of G0 (backtracking over images in vertex
// order, adjacency to every earlier vertex checked both ways); 0 when the
// count exceeds 2^40 or the search runs past 10^8 steps.
uint64_t count_automorphisms(const CompiledTemplate &T) {
    const int n0 = T.n0;
    std::vector<uint64_t> adj((size_t)n0, 0);
    for (auto &e : T.edges) {
        adj[(size_t)e.first] |= 1ull << e.second;
        adj[(size_t)e.second] |= 1ull << e.first;
    }
    std::vector<int> img((size_t)n0, -1);
    uint64_t used = 0, count = 0, steps = 0;
    bool abort = false;
    std::function<void(int)> rec = [&](int q) {
        if (abort) return;
        if (q == n0) {
            if (++count > (1ull << 40)) abort = true;
            return;
        }
        for (int r = 0; r < n0 && !abort; ++r) {
            if ((used >> r) & 1ull) continue;
            if (++steps > 100000000ull) { abort = true; return; }
            if (T.labels[(size_t)r] != T.labels[(size_t)q]) continue;
            if (__builtin_popcountll(adj[(size_t)r]) != __builtin_popcountll(adj[(size_t)q])) continue;
            bool ok = true;
            for (int j = 0; j < q && ok; ++j)
                ok = (((adj[(size_t)q] >> j) & 1ull) != 0) == (((adj[(size_t)r] >> img[(size_t)j]) & 1ull) != 0);
            if (!ok) continue;
            img[(size_t)q] = r;
            used |= 1ull << r;
            rec(q + 1);
            used &= ~(1ull << r);
        }
    };
    rec(0);
    return abort ? 0 : count;
}

// Scratch of the no-allocation prune: the static device array.
struct NoAlloc {
    char *base = nullptr;
    size_t bytes = 0;
};

// pm_prune's body.  With na, all scratch comes from the static array, one
// worker, and the swap-scan table and split lists are shrunk to fit.
void prune_impl(pm_ctx *c, int32_t first_id, int32_t count, uint64_t *role_mask,
                uint64_t *edge_bits, const pm_options *opt, pm_stats *stats, const NoAlloc *na) {
    if (!c->has_graph) throw Error(PM_ERR_NO_GRAPH, "no graph loaded");
    if (count <= 0 || first_id < 0 || first_id + count > (int32_t)c->templates.size())
        throw Error(PM_ERR_NOT_FOUND, "template id range out of bounds");
    if (!role_mask) throw Error(PM_ERR_INVALID_ARG, "null output");
    if (opt && (opt->order_mode < PM_ORDER_FIXED || opt->order_mode > PM_ORDER_LEARNED))
        throw Error(PM_ERR_INVALID_ARG, "unknown order mode");
    if (opt && (opt->mode != PM_MODE_FULL && opt->mode != PM_MODE_CANDIDATE))
        throw Error(PM_ERR_INVALID_ARG, "unknown mode");
    if (opt && (opt->ablate & ~(PM_ABLATE_EDGE_ELIMINATION | PM_ABLATE_WORK_AGGREGATION)))
        throw Error(PM_ERR_INVALID_ARG, "unknown ablation bit");
    if (opt && opt->order_mode == PM_ORDER_LEARNED && !c->has_model)
        throw Error(PM_ERR_MODEL, "learned order without a loaded model");
    if (opt && opt->trace && opt->trace_cap > 0 && count != 1)
        throw Error(PM_ERR_INVALID_ARG, "a trace records one template: count must be 1");
    set_device(c);
    const int64_t words = (c->m + 63) / 64;
    // workers: each prunes whole templates on its own stream with its own
    // scratch; worker 0 uses the context stream
    const int nw = na ? 1 : workers_for(opt, count);
    ensure_workers(c, nw);
    int na_exp = c->exp_log2;
    int64_t na_split = c->split_cap;
    if (na) {
        // work-saving tables sized for the static array
        na_exp = std::min(na_exp, 16);
        na_split = std::min<int64_t>(na_split, 4096);
        const CompiledTemplate &T = *c->templates[(size_t)first_id];
        const size_t need = workspace_bound(c, T, na_exp, na_split);
        if (need > na->bytes)
            throw Error(PM_ERR_WORKSPACE, "graph and template need up to " + std::to_string(need) +
                                              " bytes of scratch; the static array holds " +
                                              std::to_string(na->bytes));
        c->scratch[0]->use_arena(na->base, na->bytes);
    } else if (c->ws) {
        const size_t slice = (c->ws_bytes / (size_t)nw) & ~(size_t)255;
        for (int k = 0; k < nw; ++k)
            c->scratch[(size_t)k]->use_arena(c->ws + (size_t)k * slice, slice);
    } else {
        for (int k = 0; k < nw; ++k)
            if (c->scratch[(size_t)k]->in_arena) c->scratch[(size_t)k]->use_arena(nullptr, 0);
    }
    if (nw > 1) {
        // the caller's pending work on its stream precedes the workers
        PM_HIP(hipStreamSynchronize(c->stream));
    }
    std::vector<pm_stats> per((size_t)count);
    auto run_one = [&](Scratch *w, int32_t i) {
        const CompiledTemplate &T = *c->templates[(size_t)(first_id + i)];
        uint64_t *ro = role_mask + (size_t)i * (size_t)c->n;
        uint64_t *eo = edge_bits ? edge_bits + (size_t)i * (size_t)words : nullptr;
        pm_options o = opt ? *opt : pm_options{};
        if (!opt) o.stop_after = -1;
        if (!o.shared_inputs) {
            if (o.init_state) o.init_state += (size_t)i * (size_t)c->n;
            if (o.known_roles) o.known_roles += (size_t)i * (size_t)c->n;
            if (o.known_edges) o.known_edges += (size_t)i * (size_t)words;
        }
        w->reset_arena();
        auto go = [&](auto &p) {
            if (na) {
                p.exp_log2 = na_exp;
                p.split_cap = na_split;
            }
            p.run(ro, eo);
            per[(size_t)i] = p.st;
            if (o.union_roles) launch_or_into(w->stream, c->n, ro, o.union_roles);
            if (o.union_edges && eo) launch_or_into(w->stream, words, eo, o.union_edges);
        };
        switch (T.mask_bytes) {
        case 1: { Pruner<uint8_t> p(c, w, T, &o); go(p); break; }
        case 2: { Pruner<uint16_t> p(c, w, T, &o); go(p); break; }
        case 4: { Pruner<uint32_t> p(c, w, T, &o); go(p); break; }
        default: { Pruner<uint64_t> p(c, w, T, &o); go(p); break; }
        }
    };
    if (nw == 1) {
        for (int32_t i = 0; i < count; ++i) run_one(c->scratch[0].get(), i);
    } else {
        // the templates likely to take longest go first (more
        // independent cycles, then more edges and vertices), so the
        // long ones overlap each other and the short ones fill in at
        // the end instead of one long template running alone
        std::vector<int32_t> deal((size_t)count);
        for (int32_t i = 0; i < count; ++i) deal[(size_t)i] = i;
        auto cost = [&](int32_t i) {
            const CompiledTemplate &T = *c->templates[(size_t)(first_id + i)];
            return std::make_tuple(T.m0 - T.n0 + 1, T.m0, T.n0);
        };
        std::stable_sort(deal.begin(), deal.end(),
                         [&](int32_t x, int32_t y) { return cost(x) > cost(y); });
        std::atomic<int32_t> next{0};
        std::vector<std::string> errs((size_t)nw);
        std::vector<int> codes((size_t)nw, PM_OK);
        std::vector<std::thread> th;
        for (int k = 0; k < nw; ++k)
            th.emplace_back([&, k] {
                try {
                    PM_HIP(hipSetDevice(c->device));
                    for (;;) {
                        const int32_t j = next.fetch_add(1);
                        if (j >= count) break;
                        run_one(c->scratch[(size_t)k].get(), deal[(size_t)j]);
                    }
                    PM_HIP(hipStreamSynchronize(c->scratch[(size_t)k]->stream));
                } catch (const Error &e) {
                    errs[(size_t)k] = e.what();
                    codes[(size_t)k] = e.code;
                    next.store(count);
                } catch (const std::exception &e) {
                    errs[(size_t)k] = e.what();
                    codes[(size_t)k] = PM_ERR_HIP;
                    next.store(count);
                }
            });
        for (auto &t : th) t.join();
        for (int k = 0; k < nw; ++k)
            if (codes[(size_t)k] != PM_OK) throw Error(codes[(size_t)k], errs[(size_t)k]);
    }
    pm_stats total{};
    for (const pm_stats &st : per) {
        total.ms_total += st.ms_total;
        total.ms_init += st.ms_init;
        total.ms_lcc += st.ms_lcc;
        total.ms_compact += st.ms_compact;
        total.ms_nlcc += st.ms_nlcc;
        total.ms_exact += st.ms_exact;
        total.ms_first_sweep += st.ms_first_sweep;
        total.ms_sweep_kernel += st.ms_sweep_kernel;
        total.lcc_sweeps += st.lcc_sweeps;
        total.constraints += st.constraints;
        total.first_sweep_vertices += st.first_sweep_vertices;
        total.first_sweep_entries += st.first_sweep_entries;
        total.candidate_entries += st.candidate_entries;
        total.vertex_queries += st.vertex_queries;
        total.edge_queries += st.edge_queries;
        total.result_vertices += st.result_vertices;
        total.edge_candidates += st.edge_candidates;
        total.vq_pos += st.vq_pos;
        total.vq_neg += st.vq_neg;
        total.eq_pos += st.eq_pos;
        total.eq_neg += st.eq_neg;
        total.wave_ms_vq_pos += st.wave_ms_vq_pos;
        total.wave_ms_vq_neg += st.wave_ms_vq_neg;
        total.wave_ms_eq_pos += st.wave_ms_eq_pos;
        total.wave_ms_eq_neg += st.wave_ms_eq_neg;
        total.wave_ms_certify += st.wave_ms_certify;
        total.wave_ms_expand += st.wave_ms_expand;
        total.expand_scans += st.expand_scans;
        total.expand_candidates += st.expand_candidates;
        total.expand_valid += st.expand_valid;
        total.first_sweep_bytes += st.first_sweep_bytes;
        total.witness_edges += st.witness_edges;
        total.join_edges += st.join_edges;
        total.split_tasks += st.split_tasks;
        total.trace_entries += st.trace_entries;
        total.done_mask |= st.done_mask;
        total.workspace_bytes = std::max(total.workspace_bytes, st.workspace_bytes);
    }
    PM_HIP(hipStreamSynchronize(c->stream));
    if (na) c->scratch[0]->use_arena(nullptr, 0);
    if (stats) *stats = total;
    if (opt && opt->per_template)
        for (int32_t i = 0; i < count; ++i) opt->per_template[i] = per[(size_t)i];
}

// Label-pair subgraph for the label pairs of templates [first, first+count).
void build_pair_index(pm_ctx *c, int32_t first, int32_t count) {
    c->pair_m = -1;
    c->pair_nl = 0;
    c->pair_adj.clear();
    c->pair_cnt_nlab = 0;
    int maxl = -1;
    for (int32_t i = first; i < first + count; ++i)
        for (int l : c->templates[(size_t)i]->labels) maxl = std::max(maxl, l);
    const int nl = maxl + 1;
    std::vector<uint8_t> adj((size_t)nl * (size_t)std::max(nl, 0), 0);
    std::vector<int> role_of((size_t)std::max(nl, 1), -1);
    std::vector<int> labs;
    for (int32_t i = first; i < first + count; ++i) {
        const CompiledTemplate &T = *c->templates[(size_t)i];
        for (const auto &e : T.edges) {
            const int la = T.labels[(size_t)e.first], lb = T.labels[(size_t)e.second];
            adj[(size_t)la * nl + lb] = adj[(size_t)lb * nl + la] = 1;
            for (int l : {la, lb})
                if (role_of[(size_t)l] < 0) {
                    role_of[(size_t)l] = (int)labs.size();
                    labs.push_back(l);
                }
        }
    }
    if (labs.size() > (size_t)kMaxK)
        throw Error(PM_ERR_INVALID_ARG, "the templates' edges use more than 64 labels");
    // one role per label; its local table: the labels adjacent to it
    CompiledTemplate P;
    P.n0 = (int32_t)labs.size();
    P.labels = labs;
    P.mask_bytes = P.n0 <= 8 ? 1 : P.n0 <= 16 ? 2 : P.n0 <= 32 ? 4 : 8;
    P.lcc.n0 = P.n0;
    for (int i = 0; i < P.n0; ++i)
        for (int j = 0; j < P.n0; ++j)
            if (adj[(size_t)labs[(size_t)i] * nl + labs[(size_t)j]]) P.lcc.adj[i] |= 1ull << j;
    std::vector<uint64_t> lut((size_t)std::max(nl, 1), 0ull);
    for (int i = 0; i < P.n0; ++i) lut[(size_t)labs[(size_t)i]] = 1ull << i;
    DevBuf d_lut;
    d_lut.ensure(sizeof(uint64_t) * lut.size());
    PM_HIP(hipMemcpy(d_lut.p, lut.data(), sizeof(uint64_t) * lut.size(), hipMemcpyHostToDevice));
    P.d_init_lut = d_lut.as<uint64_t>();
    P.init_lut_len = (int64_t)lut.size();
    const int64_t n = c->n;
    Timer t(c->stream);
    Scratch tmp;
    tmp.stream = c->stream;
    auto go = [&](auto &p) {
        p.label_pair_compaction();
        c->pair_rp.ensure(sizeof(int64_t) * (size_t)(n + 1));
        c->pair_col.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(p.c_m, 1));
        c->pair_off.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(p.c_m, 1));
        PM_HIP(hipMemcpyAsync(c->pair_rp.p, p.c_rp, sizeof(int64_t) * (size_t)(n + 1),
                              hipMemcpyDeviceToDevice, c->stream));
        if (p.c_m > 0) {
            PM_HIP(hipMemcpyAsync(c->pair_col.p, p.c_col, sizeof(int32_t) * (size_t)p.c_m,
                                  hipMemcpyDeviceToDevice, c->stream));
            PM_HIP(hipMemcpyAsync(c->pair_off.p, p.c_off, sizeof(int32_t) * (size_t)p.c_m,
                                  hipMemcpyDeviceToDevice, c->stream));
        }
        c->pair_m = p.c_m;
        if (c->index_nlab > 0) {
            // its count index: one pass over its rows
            const int64_t np = (n + 255) / 256 * 256;
            c->pair_cnt.ensure((size_t)np * (size_t)c->index_nlab);
            launch_label_count_rows(c->stream, n, np, c->pair_rp.as<int64_t>(),
                                    c->pair_col.as<int32_t>(), (const uint8_t *)c->labels,
                                    c->index_nlab, c->pair_cnt.as<uint8_t>());
            PM_HIP(hipGetLastError());
            c->pair_cnt_stride = np;
            c->pair_cnt_nlab = c->index_nlab;
        }
    };
    switch (P.mask_bytes) {
    case 1: { Pruner<uint8_t> p(c, &tmp, P); go(p); break; }
    case 2: { Pruner<uint16_t> p(c, &tmp, P); go(p); break; }
    case 4: { Pruner<uint32_t> p(c, &tmp, P); go(p); break; }
    default: { Pruner<uint64_t> p(c, &tmp, P); go(p); break; }
    }
    c->ms_pair_index = t.stop();
    PM_HIP(hipStreamSynchronize(c->stream));
    P.d_init_lut = nullptr;
    c->pair_nl = nl;
    c->pair_adj = std::move(adj);
}

void drop_pair_index(pm_ctx *c) {
    c->pair_rp.release();
    c->pair_col.release();
    c->pair_off.release();
    c->pair_cnt.release();
    c->pair_cnt_nlab = 0;
    c->pair_m = -1;
    c->pair_nl = 0;
    c->pair_adj.clear();
}

}  // namespace

extern "C" {

const char *pm_last_error(void) { return g_last_error.c_str(); }

const char *pm_version(void) { return "pm 0.1 gfx950"; }

int pm_create(pm_ctx **out, int device, void *hip_stream) {
    return guarded([&] {
        if (!out) throw Error(PM_ERR_INVALID_ARG, "out is null");
        int ndev = 0;
        PM_HIP(hipGetDeviceCount(&ndev));
        if (device < 0 || device >= ndev) throw Error(PM_ERR_INVALID_ARG, "bad device index");
        auto *c = new pm_ctx();
        c->device = device;
        c->stream = (hipStream_t)hip_stream;
        try {
            set_device(c);
            // the no-allocation prune's static scratch of this device
            PM_HIP(noalloc_scratch(device, &c->noalloc));
            hipDeviceProp_t prop;
            PM_HIP(hipGetDeviceProperties(&prop, device));
            c->grid_search = std::max(256, prop.multiProcessorCount * 8);
            int khz = 0;
            if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess)
                c->wall_khz = khz;
            const char *ex = getenv("PM_EXPAND");
            if (ex) c->expand = atoi(ex);
            const char *ee = getenv("PM_EXPAND_EDGES");
            if (ee) c->expand_edges = atoi(ee) ? 1 : 0;
            const char *te = getenv("PM_TREE_EXACT");
            if (te) c->tree_exact = atoi(te) ? 1 : 0;
            const char *em = getenv("PM_EXPAND_MAX");
            if (em) c->expand_max = atoll(em);
            const char *wn = getenv("PM_WITNESS");
            if (wn) c->witness = atoi(wn);
            const char *rl = getenv("PM_RELIST");
            if (rl) c->relist = atoi(rl);
            const char *es = getenv("PM_EDGE_STRIPES");
            if (es) c->edge_stripes = std::min(1 << 16, std::max(1, atoi(es)));
            const char *sb = getenv("PM_SPLIT_BUDGET");
            if (sb) c->split_budget = std::max(0LL, atoll(sb));
            const char *et = getenv("PM_EDGE_TAIL");
            if (et) c->edge_tail = std::max(0LL, atoll(et));
            const char *xt = getenv("PM_EXPAND_TABLE_LOG2");
            if (xt) c->exp_log2 = std::min(30, std::max(10, atoi(xt)));
            const char *rf = getenv("PM_READ_FIRST");
            if (rf) c->read_first = atoi(rf) ? 1 : 0;
            const char *ec = getenv("PM_EDGE_CHUNK");
            if (ec) c->edge_chunk = std::min(1 << 16, std::max(1, atoi(ec)));
        } catch (...) {
            delete c;
            throw;
        }
        *out = c;
    });
}

int pm_destroy(pm_ctx *c) {
    return guarded([&] {
        if (!c) return;
        (void)hipSetDevice(c->device);
        for (auto &t : c->templates) free_template_device(*t);
        for (DevBuf *b : {&c->own_rp, &c->own_col, &c->own_labels, &c->lab_cnt, &c->idx_hub_v,
                          &c->idx_seg_slot, &c->idx_seg_b, &c->idx_seg_e, &c->idx_hub_cnt})
            b->release();
        drop_pair_index(c);
        c->scratch.clear();
        for (DevBuf *b : {&c->model, &c->mlp_partial, &c->mlp_ploss, &c->mlp_grad, &c->mlp_m,
                          &c->mlp_v, &c->mlp_loss})
            b->release();
        delete c;
    });
}

int pm_load_graph(pm_ctx *c, int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col,
                  const void *labels, int label_bytes, uint32_t flags) {
    return guarded([&] {
        if (!c) throw Error(PM_ERR_INVALID_ARG, "null context");
        if (n < 0 || m < 0 || n >= (int64_t)INT32_MAX) throw Error(PM_ERR_INVALID_ARG, "bad n or m");
        if (!row_ptr || (m > 0 && !col) || (n > 0 && !labels))
            throw Error(PM_ERR_INVALID_ARG, "null graph array");
        if (label_bytes != 1 && label_bytes != 2) throw Error(PM_ERR_INVALID_ARG, "label_bytes must be 1 or 2");
        set_device(c);
        const bool host = (flags & PM_HOST_PTRS) != 0;
        // host copy of row_ptr (hub sizing; validation)
        std::vector<int64_t> h_rp((size_t)n + 1);
        if (host) {
            std::memcpy(h_rp.data(), row_ptr, sizeof(int64_t) * (size_t)(n + 1));
        } else {
            PM_HIP(hipMemcpy(h_rp.data(), row_ptr, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyDeviceToHost));
        }
        if (h_rp[0] != 0 || h_rp[n] != m) throw Error(PM_ERR_GRAPH, "row_ptr[0] must be 0 and row_ptr[n] = m");
        if (flags & PM_VALIDATE) {
            std::vector<int32_t> h_col;
            const int32_t *hc = col;
            if (!host) {
                h_col.resize((size_t)std::max<int64_t>(m, 1));
                if (m) PM_HIP(hipMemcpy(h_col.data(), col, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToHost));
                hc = h_col.data();
            }
            validate_graph(n, m, h_rp.data(), hc);
        }
        c->has_graph = false;
        c->own_rp.release();
        c->own_col.release();
        c->own_labels.release();
        c->lab_cnt.release();
        drop_pair_index(c);
        for (DevBuf *b : {&c->idx_hub_v, &c->idx_seg_slot, &c->idx_seg_b, &c->idx_seg_e, &c->idx_hub_cnt})
            b->release();
        c->nlab = 0;
        c->index_nlab = 0;
        c->idx_hubs = c->idx_segs = 0;
        if (host) {
            c->own_rp.ensure(sizeof(int64_t) * (size_t)(n + 1));
            c->own_col.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1));
            c->own_labels.ensure((size_t)label_bytes * (size_t)std::max<int64_t>(n, 1));
            PM_HIP(hipMemcpy(c->own_rp.p, row_ptr, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyHostToDevice));
            if (m) PM_HIP(hipMemcpy(c->own_col.p, col, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice));
            if (n) PM_HIP(hipMemcpy(c->own_labels.p, labels, (size_t)label_bytes * (size_t)n, hipMemcpyHostToDevice));
            c->rp = c->own_rp.as<int64_t>();
            c->col = c->own_col.as<int32_t>();
            c->labels = c->own_labels.p;
        } else {
            c->rp = row_ptr;
            c->col = col;
            c->labels = labels;
        }
        c->n = n;
        c->m = m;
        c->label_bytes = label_bytes;
        // hub capacity for the LCC sweep and compaction
        int64_t hubs = 0, segs = 0;
        for (int64_t v = 0; v < n; ++v) {
            int64_t d = h_rp[v + 1] - h_rp[v];
            if (d > kBinWaveMaxDeg) {
                ++hubs;
                segs += (d + kHubSegment - 1) / kHubSegment;
            }
        }
        c->hub_cap = hubs;
        c->seg_cap = segs;
        // label frequencies (search-order heuristic)
        const int64_t hl = label_bytes == 1 ? 256 : 65536;
        DevBuf hist;
        hist.ensure(sizeof(unsigned long long) * (size_t)hl);
        PM_HIP(hipMemsetAsync(hist.p, 0, sizeof(unsigned long long) * (size_t)hl, c->stream));
        launch_label_hist(c->stream, n, c->labels, label_bytes, hist.as<unsigned long long>(), hl);
        std::vector<unsigned long long> h((size_t)hl);
        PM_HIP(hipMemcpyAsync(h.data(), hist.p, sizeof(unsigned long long) * (size_t)hl,
                              hipMemcpyDeviceToHost, c->stream));
        PM_HIP(hipStreamSynchronize(c->stream));
        c->label_freq.assign(h.begin(), h.end());
        // degree sums per label (scratch bounds of pm_workspace_size)
        PM_HIP(hipMemsetAsync(hist.p, 0, sizeof(unsigned long long) * (size_t)hl, c->stream));
        launch_label_degsum(c->stream, n, c->rp, c->labels, label_bytes,
                            hist.as<unsigned long long>(), hl);
        PM_HIP(hipMemcpyAsync(h.data(), hist.p, sizeof(unsigned long long) * (size_t)hl,
                              hipMemcpyDeviceToHost, c->stream));
        PM_HIP(hipStreamSynchronize(c->stream));
        c->label_degsum.assign(h.begin(), h.end());
        hist.release();
        // neighbour-label count index for the first LCC sweep (uint8 labels
        // below kCountLabels; tile offsets are 32-bit, so m < 2^32)
        int maxl = -1;
        for (int64_t L = 0; L < hl; ++L)
            if (h[(size_t)L]) maxl = (int)L;
        c->index_nlab = 0;
        if (label_bytes == 1 && maxl >= 0 && maxl < kCountLabels && n > 0 &&
            m < ((int64_t)1 << 32)) {
            c->index_nlab = maxl + 1;
            // hub rows and their segments, for the index's hub pass
            std::vector<int32_t> hv, ss;
            std::vector<int64_t> sb, se;
            for (int64_t v = 0; v < n; ++v) {
                const int64_t d = h_rp[(size_t)v + 1] - h_rp[(size_t)v];
                if (d <= kBinWaveMaxDeg) continue;
                for (int64_t b = h_rp[(size_t)v]; b < h_rp[(size_t)v + 1]; b += kHubSegment) {
                    ss.push_back((int32_t)hv.size());
                    sb.push_back(b);
                    se.push_back(std::min<int64_t>(b + kHubSegment, h_rp[(size_t)v + 1]));
                }
                hv.push_back((int32_t)v);
            }
            c->idx_hubs = (int64_t)hv.size();
            c->idx_segs = (int64_t)ss.size();
            if (!hv.empty()) {
                c->idx_hub_v.ensure(sizeof(int32_t) * hv.size());
                c->idx_seg_slot.ensure(sizeof(int32_t) * ss.size());
                c->idx_seg_b.ensure(sizeof(int64_t) * sb.size());
                c->idx_seg_e.ensure(sizeof(int64_t) * se.size());
                c->idx_hub_cnt.ensure(sizeof(uint32_t) * hv.size() * kCountLabels);
                PM_HIP(hipMemcpy(c->idx_hub_v.p, hv.data(), sizeof(int32_t) * hv.size(), hipMemcpyHostToDevice));
                PM_HIP(hipMemcpy(c->idx_seg_slot.p, ss.data(), sizeof(int32_t) * ss.size(), hipMemcpyHostToDevice));
                PM_HIP(hipMemcpy(c->idx_seg_b.p, sb.data(), sizeof(int64_t) * sb.size(), hipMemcpyHostToDevice));
                PM_HIP(hipMemcpy(c->idx_seg_e.p, se.data(), sizeof(int64_t) * se.size(), hipMemcpyHostToDevice));
            }
        }
        const char *noidx = getenv("PM_NO_COUNT_INDEX");
        if (c->index_nlab > 0 && !(noidx && atoi(noidx))) build_count_index(c);
        c->has_graph = true;
    });
}

int pm_build_pair_index(pm_ctx *c, int32_t first_id, int32_t count, double *ms) {
    return guarded([&] {
        if (!c || count < 0) throw Error(PM_ERR_INVALID_ARG, "bad arguments");
        if (!c->has_graph) throw Error(PM_ERR_NO_GRAPH, "no graph loaded");
        set_device(c);
        drop_pair_index(c);
        if (count == 0) {
            if (ms) *ms = 0.0;
            return;
        }
        if (first_id < 0 || (size_t)first_id + (size_t)count > c->templates.size())
            throw Error(PM_ERR_INVALID_ARG, "template id out of range");
        try {
            build_pair_index(c, first_id, count);
        } catch (...) {
            drop_pair_index(c);
            throw;
        }
        if (ms) *ms = c->ms_pair_index;
    });
}

int pm_build_count_index(pm_ctx *c, double *ms) {
    return guarded([&] {
        if (!c) throw Error(PM_ERR_INVALID_ARG, "null context");
        if (!c->has_graph) throw Error(PM_ERR_NO_GRAPH, "no graph loaded");
        if (c->index_nlab <= 0)
            throw Error(PM_ERR_INVALID_ARG, "graph not eligible for the count index "
                                            "(needs uint8 labels below 64 and m < 2^32)");
        set_device(c);
        build_count_index(c);
        if (ms) *ms = c->ms_count_index;
    });
}

int pm_graph_info(pm_ctx *c, pm_graph_info_t *out) {
    return guarded([&] {
        if (!c || !out) throw Error(PM_ERR_INVALID_ARG, "bad arguments");
        if (!c->has_graph) throw Error(PM_ERR_NO_GRAPH, "no graph loaded");
        pm_graph_info_t g{};
        g.n = c->n;
        g.m = c->m;
        g.label_bytes = c->label_bytes;
        g.index_labels = c->nlab;
        g.index_bytes = c->nlab > 0 ? c->cnt_stride * (int64_t)c->nlab : 0;
        g.hubs = c->idx_hubs;
        g.hub_segments = c->idx_segs;
        g.ms_count_index = c->ms_count_index;
        g.pair_entries = c->pair_m;
        g.ms_pair_index = c->pair_m >= 0 ? c->ms_pair_index : 0.0;
        *out = g;
    });
}

int pm_unload_graph(pm_ctx *c) {
    return guarded([&] {
        if (!c) throw Error(PM_ERR_INVALID_ARG, "null context");
        set_device(c);
        c->has_graph = false;
        c->own_rp.release();
        c->own_col.release();
        c->own_labels.release();
        c->lab_cnt.release();
        drop_pair_index(c);
        c->nlab = 0;
        c->rp = nullptr;
        c->col = nullptr;
        c->labels = nullptr;
    });
}

int pm_load_templates(pm_ctx *c, int32_t count, const pm_template *t, int32_t *first_id) {
    return guarded([&] {
        if (!c || !t || !first_id || count <= 0) throw Error(PM_ERR_INVALID_ARG, "bad arguments");
        set_device(c);
        std::vector<std::unique_ptr<CompiledTemplate>> made;
        for (int i = 0; i < count; ++i) {
            auto T = std::make_unique<CompiledTemplate>();
            std::string err = compile_template((int)t[i].n0, (int)t[i].m0, t[i].labels, t[i].edges,
                                               c->label_freq, *T);
            if (!err.empty()) {
                for (auto &x : made) free_template_device(*x);
                throw Error(PM_ERR_TEMPLATE, "template " + std::to_string(i) + ": " + err);
            }
            load_template_device(c, *T);
            made.push_back(std::move(T));
        }
        *first_id = (int32_t)c->templates.size();
        for (auto &x : made) c->templates.push_back(std::move(x));
    });
}

int pm_template_constraints(pm_ctx *c, int32_t id, int32_t *count, int32_t *kinds,
                            int32_t *n_edges, uint64_t *heads, uint32_t *edges_out) {
    return guarded([&] {
        if (!c || !count) throw Error(PM_ERR_INVALID_ARG, "bad arguments");
        if (id < 0 || id >= (int32_t)c->templates.size()) throw Error(PM_ERR_NOT_FOUND, "unknown template id");
        const CompiledTemplate &T = *c->templates[(size_t)id];
        *count = (int32_t)T.constraints.size();
        for (size_t i = 0; i < T.constraints.size(); ++i) {
            const Constraint &k = T.constraints[i];
            if (kinds) kinds[i] = k.kind;
            if (n_edges) n_edges[i] = (int32_t)k.edges.size();
            if (heads) heads[i] = k.heads;
            if (edges_out)
                for (size_t j = 0; j < k.edges.size() && j < 64; ++j) {
                    edges_out[i * 128 + 2 * j] = (uint32_t)k.edges[j].first;
                    edges_out[i * 128 + 2 * j + 1] = (uint32_t)k.edges[j].second;
                }
        }
    });
}

int pm_prune(pm_ctx *c, int32_t first_id, int32_t count, uint64_t *role_mask, uint64_t *edge_bits,
             const pm_options *opt, pm_stats *stats) {
    return guarded([&] {
        if (!c) throw Error(PM_ERR_INVALID_ARG, "null context");
        if (!role_mask || !edge_bits) throw Error(PM_ERR_INVALID_ARG, "null output");
        prune_impl(c, first_id, count, role_mask, edge_bits, opt, stats, nullptr);
    });
}

int pm_export_state(pm_ctx *c, int32_t id, int32_t stop_after, const pm_options *opt,
                    uint64_t *state, uint64_t *done_mask) {
    return guarded([&] {
        if (!c || !state || !done_mask) throw Error(PM_ERR_INVALID_ARG, "bad arguments");
        pm_options o = opt ? *opt : pm_options{};
        if (!opt) o.stop_after = -1;
        o.stop_after = stop_after < 0 ? PM_MAX_CONSTRAINTS : stop_after;
        o.mode = PM_MODE_FULL;
        o.known_roles = nullptr;
        o.known_edges = nullptr;
        pm_stats st{};
        prune_impl(c, id, 1, state, nullptr, &o, &st, nullptr);
        *done_mask = st.done_mask;
    });
}

int pm_import_state(pm_ctx *c, int32_t id, const uint64_t *state, uint64_t done_mask,
                    uint64_t *role_mask, uint64_t *edge_bits, const pm_options *opt,
                    pm_stats *stats) {
    return guarded([&] {
        if (!c || !state || !role_mask || !edge_bits) throw Error(PM_ERR_INVALID_ARG, "bad arguments");
        pm_options o = opt ? *opt : pm_options{};
        if (!opt) o.stop_after = -1;
        o.mode = PM_MODE_FULL;
        o.init_state = state;
        o.skip_mask = done_mask;
        prune_impl(c, id, 1, role_mask, edge_bits, &o, stats, nullptr);
    });
}

int pm_workspace_size(pm_ctx *c, int32_t first_id, int32_t count, const pm_options *opt,
                      size_t *bytes) {
    return guarded([&] {
        if (!c || !bytes) throw Error(PM_ERR_INVALID_ARG, "bad arguments");
        if (!c->has_graph) throw Error(PM_ERR_NO_GRAPH, "no graph loaded");
        if (count <= 0 || first_id < 0 || first_id + count > (int32_t)c->templates.size())
            throw Error(PM_ERR_NOT_FOUND, "template id range out of bounds");
        const int nw = workers_for(opt, count);
        size_t worst = 0;
        for (int32_t i = 0; i < count; ++i)
            worst = std::max(worst, workspace_bound(c, *c->templates[(size_t)(first_id + i)],
                                                    c->exp_log2, c->split_cap));
        *bytes = worst * (size_t)nw;
    });
}

int pm_set_workspace(pm_ctx *c, void *ws, size_t bytes) {
    return guarded([&] {
        if (!c) throw Error(PM_ERR_INVALID_ARG, "null context");
        if (ws && ((uintptr_t)ws & 255u))
            throw Error(PM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
        if (ws && bytes < 4096) throw Error(PM_ERR_WORKSPACE, "workspace smaller than 4 KiB");
        set_device(c);
        PM_HIP(hipStreamSynchronize(c->stream));
        for (auto &sc : c->scratch) {
            if (sc->stream) PM_HIP(hipStreamSynchronize(sc->stream));
            sc->use_arena(nullptr, 0);
        }
        c->ws = ws ? static_cast<char *>(ws) : nullptr;
        c->ws_bytes = ws ? bytes : 0;
    });
}

int pm_prune_noalloc(pm_ctx *c, int32_t id, uint64_t *role_mask, uint64_t *edge_bits,
                     const pm_options *opt, pm_stats *stats) {
    return guarded([&] {
        if (!c) throw Error(PM_ERR_INVALID_ARG, "null context");
        if (!role_mask || !edge_bits) throw Error(PM_ERR_INVALID_ARG, "null output");
        if (!c->noalloc) throw Error(PM_ERR_HIP, "no static scratch on this device");
        NoAlloc na;
        na.base = static_cast<char *>(c->noalloc);
        na.bytes = kNoAllocBytes;
        prune_impl(c, id, 1, role_mask, edge_bits, opt, stats, &na);
    });
}

int pm_count_matches(pm_ctx *c, int32_t id, const uint64_t *state, int32_t *maps_out,
                     int64_t cap, uint64_t max_maps, pm_match_count *out) {
    return guarded([&] {
        if (!c || !out) throw Error(PM_ERR_INVALID_ARG, "bad arguments");
        if (!c->has_graph) throw Error(PM_ERR_NO_GRAPH, "no graph loaded");
        if (id < 0 || id >= (int32_t)c->templates.size()) throw Error(PM_ERR_NOT_FOUND, "unknown template id");
        if (cap < 0 || (cap > 0 && !maps_out)) throw Error(PM_ERR_INVALID_ARG, "bad map output");
        set_device(c);
        ensure_workers(c, 1);
        Scratch *w = c->scratch[0].get();
        if (c->ws) {
            w->use_arena(c->ws, c->ws_bytes);
            w->reset_arena();
        } else if (w->in_arena) {
            w->use_arena(nullptr, 0);
        }
        const CompiledTemplate &T = *c->templates[(size_t)id];
        pm_match_count r{};
        switch (T.mask_bytes) {
        case 1: { Pruner<uint8_t> p(c, w, T); r = p.count_matches(state, maps_out, cap, max_maps); break; }
        case 2: { Pruner<uint16_t> p(c, w, T); r = p.count_matches(state, maps_out, cap, max_maps); break; }
        case 4: { Pruner<uint32_t> p(c, w, T); r = p.count_matches(state, maps_out, cap, max_maps); break; }
        default: { Pruner<uint64_t> p(c, w, T); r = p.count_matches(state, maps_out, cap, max_maps); break; }
        }
        r.automorphisms = count_automorphisms(T);
        r.subgraphs = r.automorphisms ? r.maps / r.automorphisms : 0;
        PM_HIP(hipStreamSynchronize(c->stream));
        *out = r;
    });
}

int pm_set_param(pm_ctx *c, const char *name, int64_t value) {
    return guarded([&] {
        if (!c || !name) throw Error(PM_ERR_INVALID_ARG, "bad arguments");
        const std::string k(name);
        if (k == "expand") c->expand = value ? 1 : 0;
        else if (k == "expand_max") c->expand_max = value < 0 ? INT64_MAX : value;
        else if (k == "expand_edges") c->expand_edges = value ? 1 : 0;
        else if (k == "tree_exact") c->tree_exact = value ? 1 : 0;
        else if (k == "witness") c->witness = value ? 1 : 0;
        else if (k == "relist") c->relist = value ? 1 : 0;
        else if (k == "edge_chunk" && value >= 1 && value <= (1 << 16)) c->edge_chunk = (int)value;
        else if (k == "edge_stripes" && value >= 1 && value <= (1 << 16)) c->edge_stripes = (int)value;
        else if (k == "search_grid" && value >= 1 && value <= (1 << 16)) c->grid_search = (int)value;
        else if (k == "search_grid_solo" && value >= 0 && value <= (1 << 16))
            c->grid_search_solo = (int)value;
        else if (k == "split_budget" && value >= 0) c->split_budget = value;
        else if (k == "edge_tail" && value >= 0) c->edge_tail = value;
        else if (k == "expand_table_log2" && value >= 10 && value <= 30) c->exp_log2 = (int)value;
        else if (k == "split_capacity" && value >= 1 && value <= ((int64_t)1 << 28)) c->split_cap = value;
        else if (k == "read_first") c->read_first = value ? 1 : 0;
        else if (k == "lcc_bin_small" && value >= 0 && value <= c->bin_mid) c->bin_small = value;
        else if (k == "lcc_bin_mid" && value >= c->bin_small && value <= kBinWaveMaxDeg)
            c->bin_mid = value;
        else throw Error(PM_ERR_INVALID_ARG, "unknown parameter or value out of range: " + k);
    });
}

int pm_get_param(pm_ctx *c, const char *name, int64_t *value) {
    return guarded([&] {
        if (!c || !name || !value) throw Error(PM_ERR_INVALID_ARG, "bad arguments");
        const std::string k(name);
        if (k == "expand") *value = c->expand;
        else if (k == "expand_max") *value = c->expand_max == INT64_MAX ? -1 : c->expand_max;
        else if (k == "expand_edges") *value = c->expand_edges;
        else if (k == "tree_exact") *value = c->tree_exact;
        else if (k == "witness") *value = c->witness;
        else if (k == "relist") *value = c->relist;
        else if (k == "edge_chunk") *value = c->edge_chunk;
        else if (k == "edge_stripes") *value = c->edge_stripes;
        else if (k == "search_grid") *value = c->grid_search;
        else if (k == "search_grid_solo") *value = c->grid_search_solo;
        else if (k == "split_budget") *value = c->split_budget;
        else if (k == "edge_tail") *value = c->edge_tail;
        else if (k == "expand_table_log2") *value = c->exp_log2;
        else if (k == "split_capacity") *value = c->split_cap;
        else if (k == "read_first") *value = c->read_first;
        else if (k == "lcc_bin_small") *value = c->bin_small;
        else if (k == "lcc_bin_mid") *value = c->bin_mid;
        else throw Error(PM_ERR_INVALID_ARG, "unknown parameter: " + k);
    });
}

int pm_load_model(pm_ctx *c, const float *w, size_t n) {
    return guarded([&] {
        if (!c || !w) throw Error(PM_ERR_INVALID_ARG, "bad arguments");
        if (n != (size_t)kMlpParams) throw Error(PM_ERR_INVALID_ARG, "model must have PM_MLP_PARAMS values");
        for (size_t i = 0; i < n; ++i)
            if (!std::isfinite(w[i])) throw Error(PM_ERR_MODEL, "model parameter is not finite");
        set_device(c);
        c->model.ensure(sizeof(float) * (size_t)kMlpParams);
        PM_HIP(hipMemcpyAsync(c->model.p, w, sizeof(float) * (size_t)kMlpParams,
                              hipMemcpyHostToDevice, c->stream));
        PM_HIP(hipStreamSynchronize(c->stream));
        c->has_model = true;
    });
}

int pm_mlp_forward(pm_ctx *c, const float *w, const float *x, int64_t n, float *y) {
    return guarded([&] {
        if (!c || n < 0 || (n > 0 && (!w || !x || !y))) throw Error(PM_ERR_INVALID_ARG, "bad arguments");
        set_device(c);
        launch_mlp_forward(c->stream, w, x, n, y);
        PM_HIP(hipGetLastError());
        PM_HIP(hipStreamSynchronize(c->stream));
    });
}

static void mlp_workspace(pm_ctx *c) {
    c->mlp_partial.ensure(sizeof(float) * (size_t)kMlpGradGrid * kMlpParams);
    c->mlp_ploss.ensure(sizeof(float) * kMlpGradGrid);
}

int pm_mlp_grad(pm_ctx *c, const float *w, const float *x, const float *t, int64_t n, float *grad,
                float *loss) {
    return guarded([&] {
        if (!c || n < 1 || !w || !x || !t || !grad || !loss)
            throw Error(PM_ERR_INVALID_ARG, "bad arguments");
        set_device(c);
        mlp_workspace(c);
        launch_mlp_grad(c->stream, w, x, t, n, c->mlp_partial.as<float>(), c->mlp_ploss.as<float>(),
                        grad, loss);
        PM_HIP(hipGetLastError());
        PM_HIP(hipStreamSynchronize(c->stream));
    });
}

int pm_mlp_train(pm_ctx *c, float *w, const float *x, const float *t, int64_t n, int32_t steps,
                 float lr, float *loss_history) {
    return guarded([&] {
        if (!c || n < 1 || steps < 0 || !w || !x || !t || !(lr > 0.0f))
            throw Error(PM_ERR_INVALID_ARG, "bad arguments");
        set_device(c);
        mlp_workspace(c);
        c->mlp_grad.ensure(sizeof(float) * kMlpParams);
        c->mlp_m.ensure(sizeof(float) * kMlpParams);
        c->mlp_v.ensure(sizeof(float) * kMlpParams);
        c->mlp_loss.ensure(sizeof(float) * (size_t)std::max(steps, 1));
        hipStream_t s = c->stream;
        launch_fill_i32(s, c->mlp_m.as<int32_t>(), kMlpParams, 0);
        launch_fill_i32(s, c->mlp_v.as<int32_t>(), kMlpParams, 0);
        double b1t = 1.0, b2t = 1.0;
        for (int32_t k = 1; k <= steps; ++k) {
            b1t *= 0.9;
            b2t *= 0.999;
            launch_mlp_grad(s, w, x, t, n, c->mlp_partial.as<float>(), c->mlp_ploss.as<float>(),
                            c->mlp_grad.as<float>(), c->mlp_loss.as<float>() + (k - 1));
            launch_adam(s, w, c->mlp_grad.as<float>(), c->mlp_m.as<float>(), c->mlp_v.as<float>(), lr,
                        (float)(1.0 - b1t), (float)(1.0 - b2t));
        }
        PM_HIP(hipGetLastError());
        if (loss_history && steps > 0) {
            PM_HIP(hipMemcpyAsync(loss_history, c->mlp_loss.p, sizeof(float) * (size_t)steps,
                                  hipMemcpyDeviceToHost, s));
        }
        PM_HIP(hipStreamSynchronize(s));
    });
}

}  // extern "C"

extern "C" int pm_inspect_template(const pm_template *t, int32_t *count, int32_t *kinds,
                                   int32_t *n_edges, uint64_t *heads, uint32_t *edges_out) {
    return guarded([&] {
        if (!t || !count) throw Error(PM_ERR_INVALID_ARG, "bad arguments");
        CompiledTemplate T;
        std::string err = compile_template((int)t->n0, (int)t->m0, t->labels, t->edges, {}, T);
        if (!err.empty()) throw Error(PM_ERR_TEMPLATE, err);
        *count = (int32_t)T.constraints.size();
        for (size_t i = 0; i < T.constraints.size(); ++i) {
            const Constraint &k = T.constraints[i];
            if (kinds) kinds[i] = k.kind;
            if (n_edges) n_edges[i] = (int32_t)k.edges.size();
            if (heads) heads[i] = k.heads;
            if (edges_out)
                for (size_t j = 0; j < k.edges.size() && j < 64; ++j) {
                    edges_out[i * 128 + 2 * j] = (uint32_t)k.edges[j].first;
                    edges_out[i * 128 + 2 * j + 1] = (uint32_t)k.edges[j].second;
                }
        }
    });
}
