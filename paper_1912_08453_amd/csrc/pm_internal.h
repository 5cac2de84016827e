// Internal declarations shared by the host engine and the HIP kernels of
// libpm.  Nothing here is part of the public ABI (include/pm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "pm.h"

namespace pm {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kMaxK = 64;            // template vertices
constexpr int kMaxCount = 32;        // distinct-count rules per template

// Degree bins of the LCC sweep: lanes cooperating on one vertex.
constexpr int kBinSmallMaxDeg = 8;   // 4 lanes per vertex
constexpr int kBinMidMaxDeg = 64;    // 16 lanes per vertex
constexpr int kBinWaveMaxDeg = 4096; // one wavefront per vertex
constexpr int kHubSegment = 4096;    // entries per wavefront for larger vertices
constexpr int kExpSeenLog2 = 22;     // default slots of the swap-scan table (32 MiB)
constexpr int kNumBins = 4;          // small, mid, wave, hub

// Local-rule tables of one template (LCC algorithm; distinct-count rule of
// the LCC description).  Passed by value as a kernel argument.
struct LccTable {
    int32_t n0;
    int32_t ncount;
    int32_t any;                    // candidate-set rule: q stays while SOME
                                    // template neighbour of q is covered
    int32_t keep_all;               // compaction keeps every entry of an
                                    // active row (edge elimination ablated)
    uint64_t adj[kMaxK];            // adj(q)
    uint64_t cmask[kMaxCount];      // adj(q) restricted to one label L
    int32_t cq[kMaxCount];          // q of the rule
    int32_t cneed[kMaxCount];       // |cmask| >= 2
};

// Acyclic template whose labels are unique except for one pair a, b: the
// path p_0 = a .. p_k = b between them and, off the path, each vertex's
// neighbour towards it.  Passed by value as a kernel argument.
struct TreePlan {
    int32_t k;                      // path length in edges (>= 1)
    int32_t depth;                  // largest distance of a vertex from the path
    int32_t m0;
    int8_t path[kMaxK];             // p_i
    int8_t pos[kMaxK];              // i for q = p_i, -1 off the path
    int8_t par[kMaxK];              // off the path: neighbour towards it; -1 on it
    int8_t ea[kMaxK], eb[kMaxK];    // template edges
    uint64_t depmask[kMaxK + 1];    // vertices at distance d from the path
};

// One search plan: a substructure of G0 (vertex set and its own edges) with
// one or two template vertices pinned (the head, or both ends of an edge).
// The search order is chosen per partial match at run time.
struct SearchPlan {
    int32_t k;                      // substructure vertices
    int32_t npin;                   // 1 or 2
    int32_t pin[2];                 // pinned template vertices
    uint64_t vmask;                 // substructure vertices
    uint64_t adj[kMaxK];            // substructure adjacency per template vertex
    uint64_t samelab[kMaxK];        // other substructure vertices of the same label
    uint64_t certify;               // roles certified by a successful search
};

// Compiled non-local constraint.
struct Constraint {
    int32_t kind;                   // 0 CC, 1 PC, 2 TDS_CC, 3 TDS_PC
    int32_t gen_index;
    uint64_t vmask;                 // substructure vertices
    uint64_t heads;                 // head roles (token sources)
    std::vector<std::pair<int, int>> edges;   // sorted (a < b)
    int32_t plan_base;              // index of the plan of its first head
    int32_t plan_of_head[kMaxK];    // -1 if not a head
};

// Learned constraint order: perceptron sizes and packed parameter offsets.
constexpr int kMlpIn = 12, kMlpHid = 64, kMlpOut = 2;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpHid * kMlpIn;      // 768
constexpr int kOffW2 = kOffB1 + kMlpHid;               // 832
constexpr int kOffB2 = kOffW2 + kMlpHid * kMlpHid;     // 4928
constexpr int kOffW3 = kOffB2 + kMlpHid;               // 4992
constexpr int kOffB3 = kOffW3 + kMlpOut * kMlpHid;     // 5120
constexpr int kMlpParams = kOffB3 + kMlpOut;           // 5122
constexpr int kMlpGradGrid = 128;                      // blocks of the gradient kernel

// Device descriptor of one constraint (features of the learned order).
struct ConstraintDesc {
    uint64_t vmask;
    uint64_t heads;
    int32_t n_edges;
    int32_t kind;
};

// Inputs of the feature/choice kernel (by value).
struct OrderArgs {
    const unsigned long long *counts;   // [64] active role counts now
    const unsigned long long *counts0;  // [64] at the first LCC fixpoint
    const ConstraintDesc *cons;         // [n_cons]
    const float *w;                     // model parameters, or null
    uint64_t role_freq[kMaxK];          // background vertices of q's label
    uint64_t remaining;                 // constraints not yet checked
    int64_t n_active;
    int32_t n_cons;
    int32_t done;
    int32_t forced;                     // >= 0: report this constraint
    int32_t n0;
};

// Output of the feature/choice kernel.
struct OrderPick {
    int32_t idx;                        // chosen (or forced) constraint, -1 none
    float score;
    float pred[kMlpOut];
    float feat[kMlpIn];
    unsigned long long roles;           // sum of counts
};

struct CompiledTemplate {
    int32_t n0 = 0, m0 = 0;
    std::vector<int32_t> labels;
    std::vector<std::pair<int, int>> edges;
    int mask_bytes = 1;             // 1, 2, 4 or 8
    bool acyclic_unique = false;    // LCC alone is exact
    LccTable lcc{};
    std::vector<Constraint> constraints;     // generation order
    std::vector<SearchPlan> plans;            // all plans of this template
    int32_t vertex_plan[kMaxK];               // full template, pinned at q
    std::vector<int32_t> edge_plans;          // 2*m0 plans: (a->b), (b->a)
    uint64_t label_mask_of[kMaxK];            // roles sharing q's label
    // device copies
    SearchPlan *d_plans = nullptr;
    int32_t *d_tedges = nullptr;              // [2*m0] template edges (a, b)
    // [m0] for a bridge (a, b) of G0 the vertices on a's side once it is
    // removed (0 for an edge on a cycle), then [n0] the other vertices of
    // q's label
    uint64_t *d_tjoin = nullptr;
    uint64_t *d_init_lut = nullptr;           // label -> initial roles
    int64_t init_lut_len = 0;
    ConstraintDesc *d_cdesc = nullptr;        // [constraints]
    // first-sweep needs: for role q, entries need_off[q] .. need_off[q+1] of
    // (label L, number of template neighbours of q with label L)
    std::vector<int32_t> need_off, need_lab, need_min;
    std::vector<uint64_t> need_labmask;       // labels < 64 that q needs
    int32_t *d_need = nullptr;                // need_off | need_lab | need_min
    // acyclic with exactly one pair of vertices sharing a label: the final
    // step can run as sweeps along the path between the pair (tree)
    bool tree_pair = false;
    TreePlan tree{};
};

// Template compiler (host).  Returns an empty string on success, otherwise
// the error message.  label_freq[L] is the number of background vertices of
// label L (may be empty), used only to order search positions.
std::string compile_template(int n0, int m0, const uint16_t *labels, const uint32_t *edges,
                             const std::vector<int64_t> &label_freq, CompiledTemplate &out);

// ---- kernel launchers (explicitly instantiated for M = uint8_t, uint16_t,
// uint32_t, uint64_t) ---------------------------------------------------------
struct Worklists {
    int32_t *list[kNumBins];        // vertex ids per degree bin
    int32_t *count;                 // [kNumBins] device counters
    int32_t *hub_seg_v;             // hub segments: vertex
    int64_t *hub_seg_begin;         // segment [begin, end)
    int64_t *hub_seg_end;
    int32_t *hub_seg_slot;          // accumulator slot of the vertex
    int32_t *hub_nseg;              // [n_hubs] segments per hub slot
    int32_t *hub_seg_first;         // [n_hubs] index of the slot's first segment
    uint64_t *hub_cover;            // [n_hubs]
    int32_t *hub_count;             // [n_hubs][kMaxCount]
    int32_t *hub_ticket;            // [n_hubs]
    int32_t *n_seg;                 // device scalar
    unsigned long long *entries;    // device scalar: CSR entries of binned vertices
    const uint64_t *act_bits;       // bit v: initial role set of v not empty
    int64_t capacity;               // per list
    int64_t hub_capacity;           // hub slots
    int64_t seg_capacity;
    int64_t bin_small;              // largest degree of the 4-lane bin
    int64_t bin_mid;                // largest degree of the 16-lane bin
};

// omega0(v) from the label LUT; bits (ceil(n/64) words, may be null)
// receives the bitmap of vertices with a non-empty initial role set.
template <typename M>
void launch_init_roles(hipStream_t s, int64_t n, const void *labels, int label_bytes,
                       const uint64_t *lut, int64_t lut_len, M *omega, uint64_t *bits);

// Active list: vertices of `in` (or 0..n_in-1 when in == nullptr) whose role
// set is not empty, appended to out via *counter (zeroed by the caller).
template <typename M>
void launch_collect(hipStream_t s, const int32_t *in, int64_t n_in, const M *omega,
                    int32_t *out, int32_t *counter);

// Bin the vertices of `in` (or 0..n-1 when in == nullptr) with omega != 0 by
// their degree in the CSR rp; counts go to wl.count (zeroed by the caller).
template <typename M>
void launch_bin(hipStream_t s, const int32_t *in, int64_t n_in, const int64_t *rp,
                const M *omega, Worklists &wl);

void launch_hub_segments(hipStream_t s, const int64_t *rp, Worklists &wl, int64_t n_hubs);

// One LCC sweep over the binned vertices, one kernel launch; changed
// (device int) is incremented once per wavefront that shrank at least one
// role set.  full selects the kernel symbol used for the first sweep over
// the whole graph.
template <typename M>
void launch_lcc_sweep(hipStream_t s, const int64_t *rp, const int32_t *col, M *omega,
                      const Worklists &wl, const int64_t *host_counts, int64_t n_seg,
                      const LccTable &tab, int32_t *changed, bool full);

// Candidate-subgraph compaction: keep the entries u->w of active u whose
// roles are adjacent (edge elimination).  Count pass writes deg_out[v]
// (32-bit: a compacted graph holds under 2^31 entries) for binned v
// (deg_out must be zeroed; hubs accumulate per segment into
// seg_count and store each segment's keep bits in seg_bits, kHubSegment/64
// words per segment), then an exclusive scan gives c_rp (n+1) and another
// one over seg_count gives seg_scan, then the fill pass writes c_col, c_own
// (the row's vertex) and c_off (offset of the entry within the original row: k - row start, or
// base_off[k] when the source is itself a compacted graph whose c_off is
// base_off).
template <typename M>
void launch_compact_count(hipStream_t s, const int64_t *rp, const int32_t *col, const M *omega,
                          const Worklists &wl, const int64_t *host_counts, int64_t n_seg,
                          const LccTable &tab, const uint32_t *filt, int32_t *deg_out,
                          int64_t *seg_count, uint64_t *seg_bits);
// Coarse filter of the active vertices (bit g: one of vertices 8g..8g+7
// has a non-empty role set), ceil(n / 256) 32-bit words, fully written.
template <typename M>
void launch_active_filter(hipStream_t s, int64_t n, const M *omega, uint32_t *filt);
// Exclusive scan of n values (T: int64_t, or int32_t) into 64-bit out[0, n),
// their sum to out[n]; scratch holds scan_scratch_len(n) values.
template <typename T>
void launch_exclusive_scan(hipStream_t s, const T *in, int64_t *out, int64_t n,
                           int64_t *scratch, int64_t scratch_len);
int64_t scan_scratch_len(int64_t n);
template <typename M>
void launch_compact_fill(hipStream_t s, const int64_t *rp, const int32_t *col, const M *omega,
                         const Worklists &wl, const int64_t *host_counts, int64_t n_seg,
                         const LccTable &tab, const uint32_t *filt, const int64_t *c_rp,
                         const int64_t *seg_scan,
                         const uint64_t *seg_bits, const int32_t *base_off, int32_t *c_col,
                         int32_t *c_off, int32_t *c_own);

// Vertex-rooted searches.  mode 0: NLCC (certify head roles into sat);
// mode 1: exact step (certify all roles into sat and edges into edge_bits).
// An unexplored part of an edge-rooted search, handed on when the search
// ran past its step budget: the plan's pins at the task's edge, np further
// placed vertices (pq[i] at image px[i]), and the candidates still to try
// for template vertex q at the next level, rl_col[r0, r1) (the role-q list
// of the image of the placed vertex par).
constexpr int kSplitPrefix = 8;
constexpr int kSplitPieces = 16;         // tasks per handed-on range, at most
constexpr int64_t kSplitCap = 1 << 18;   // default split tasks per launch (two lists)
struct alignas(16) SplitTask {
    int64_t t;                      // edge task index (eu / ew / e_idx)
    int32_t r0, r1;
    int16_t plan;                   // index into the edge plan list
    uint8_t q, par, np;
    uint8_t pq[kSplitPrefix];
    int32_t px[kSplitPrefix];
};

struct SearchArgs {
    const int64_t *c_rp;
    const int32_t *c_col;
    const int32_t *c_off;
    const int64_t *rp;              // original CSR (edge bit indices)
    const int32_t *col;
    const SearchPlan *plans;
    const int32_t *tedges;          // template edges (a, b) pairs
    int32_t m0;
    const int64_t *rl_off;          // role lists: [tasks * n0 + 1] offsets into rl_col
    const int32_t *rl_v;            // the same bounds by vertex id: [n * (n0 + 1)]
    const int32_t *rl_col;
    const int32_t *rl_ent;          // compacted entry index of each list entry
    const int32_t *rl_pos;          // list position (task index) of each listed vertex
    int32_t n0;
    int32_t mode;
    uint64_t heads;
    int32_t plan_of_head[kMaxK];
    uint64_t *edge_bits;
    int32_t *task_counter;
    int32_t task_chunk;             // consecutive tasks a wavefront takes per atomic
    int32_t stripes;                // edge searches: chunk order striped S ways
    int64_t tail_single;            // edge searches: trailing tasks dealt one at a time
    unsigned long long *n_queries;
    // exact step: certified edges of the compacted subgraph (bit k = entry k
    // = u -> w with u < w), the table of swap scans
    // already done (hashes of (role, images of its template neighbours);
    // exp_slots entries, a power of two), query statistics
    uint64_t *c_cert;
    unsigned long long *exp_seen;
    int32_t exp_log2;
    unsigned long long *qstats;     // [16]: vpos, vneg, vpos_t, vneg_t, epos, eneg, epos_t,
                                    // eneg_t, vcert_t, ecert_t, expand_t (wall-clock
                                    // ticks), expand scans, candidates, valid swaps
    int32_t expand;                 // run the single-vertex swap expansion
    // witnesses (exact step): for each certified (vertex, role) the first
    // match that certified it, wit[(pos * n0 + q) * n0 + p] = image of p,
    // valid once wit_flag[pos * n0 + q] is set; recorded while wit_on
    int32_t *wit;
    uint32_t *wit_flag;
    int32_t wit_on;
    int64_t expand_max;             // longest list a swap scan reads
    int32_t check_om;               // candidates' role sets may have shrunk since
                                    // the role lists were built: test them
    // splitting of long edge-rooted searches: one that takes more than
    // split_budget steps (0: never) stops and appends its unexplored
    // candidate ranges to split_out (capacity split_cap, count *split_n)
    int64_t split_budget;
    int32_t read_first;             // read certificate words before setting them
    SplitTask *split_out;
    int32_t *split_n;
    int64_t split_cap;
    int32_t aggregate;              // 0: a found embedding certifies only the
                                    // query it answers (work aggregation off)
    const uint64_t *tside;          // [m0] side masks of template bridges (0: none)
    const uint64_t *tsame;          // [n0] other template vertices of q's label
};

// Role lists of the vertices in tasks over the compacted subgraph: pass 1
// writes cnt[t * n0 + q] = neighbours of tasks[t] whose role set holds q and
// pos_of[tasks[t]] = t; an exclusive scan of cnt gives rl_off; pass 2 writes
// the sorted lists into rl_col.
template <typename M>
void launch_role_count(hipStream_t s, const int32_t *tasks, int64_t n_tasks, const int64_t *c_rp,
                       const int32_t *c_col, const M *omega, int n0, int64_t *cnt,
                       int32_t *pos_of);
template <typename M>
void launch_role_fill(hipStream_t s, const int32_t *tasks, int64_t n_tasks, const int64_t *c_rp,
                      const int32_t *c_col, const M *omega, int n0, const int64_t *rl_off,
                      int32_t *rl_col, int32_t *rl_ent);

// rl_v[tasks[t] * (n0 + 1) + q] = rl_off[t * n0 + q] for q <= n0.
void launch_role_rows(hipStream_t s, const int32_t *tasks, int64_t n_tasks, int n0,
                      const int64_t *rl_off, int32_t *rl_v);

// Output edge bits (both entries) from certified compacted entries; one
// thread per compacted entry (c_own gives each entry's row).
void launch_edges_from_cert(hipStream_t s, int64_t c_m, const int64_t *c_rp, const int32_t *c_col,
                            const int32_t *c_own, const int32_t *c_off, const int64_t *rp,
                            const uint64_t *c_cert, uint64_t *edge_bits);

template <typename M>
void launch_vertex_search(hipStream_t s, const int32_t *tasks, int64_t n_tasks, const M *omega,
                          M *sat, const SearchArgs &a, int grid);

// NLCC application: omega &= ~heads | sat; sat cleared; *changed += vertices
// whose role set shrank.
template <typename M>
void launch_apply(hipStream_t s, const int32_t *tasks, int64_t n_tasks, M *omega, M *sat,
                  uint64_t heads, int32_t *changed);

// Exact step, edge part: candidate edges u < w of the compacted subgraph
// with adjacent certified roles and no certified bit yet.
// Candidates whose edge a recorded witness certifies by one vertex swap are
// certified here instead of being listed (a.wit_on).
template <typename M>
void launch_edge_candidates(hipStream_t s, int64_t c_m, const int64_t *c_rp,
                            const int32_t *c_own, const int32_t *c_col, const M *cert,
                            const LccTable &tab, uint64_t *c_cert, int32_t *eu, int32_t *ew,
                            int64_t *e_idx, int32_t *n_out, int64_t cap, const SearchArgs &a);

// Searches of split tasks (edge-rooted searches handed on by a search
// that ran past its step budget); they may split again into a.split_out.
template <typename M>
void launch_split_search(hipStream_t s, const SplitTask *tasks, int64_t n_tasks,
                         const int32_t *eu, const int32_t *ew, const int64_t *e_idx,
                         const M *omega, M *cert, const int32_t *edge_plan, const SearchArgs &a,
                         int grid);

template <typename M>
void launch_edge_search(hipStream_t s, const int32_t *eu, const int32_t *ew,
                        const int64_t *e_idx, int64_t n_edges, const M *omega, M *cert,
                        const int32_t *edge_plan_dev, int32_t n_edge_plans, const SearchArgs &a,
                        int grid);

// Edge state implied by omega (acyclic unique-label templates and
// intermediate outputs): sets the bits of active entries, both directions.
template <typename M>
void launch_active_edges(hipStream_t s, const int32_t *tasks, int64_t n_tasks,
                         const int64_t *c_rp, const int32_t *c_col, const int32_t *c_off,
                         const int64_t *rp, const M *omega, const LccTable &tab,
                         uint64_t *edge_bits);

template <typename M>
void launch_widen(hipStream_t s, int64_t n, const M *src, uint64_t *dst);

// Final step of a template with a TreePlan (exact, no searches): sat
// (zeroed by the caller) receives the roles in some match, edge_bits (if
// not null) the entries that carry a template edge of one.  pos: int32[n]
// (overwritten: active-list positions); sum: int2[2 * (k + 1) * nA].
template <typename M>
void launch_tree_exact(hipStream_t s, const int32_t *A, int64_t nA, const M *om,
                       int64_t c_m, const int32_t *c_own, const int32_t *c_col,
                       const int32_t *c_off, const int64_t *rp, const TreePlan &tp,
                       int32_t *pos, int2 *sum, M *sat, uint64_t *edge_bits);

// Neighbour-label count index of a graph with uint8 labels below nlab:
// cnt[L * np + v] = min(255, neighbours of v with label L), np = n rounded
// up to a multiple of 256 (labels and omega must allow 4-byte accesses at
// multiples of 4: device allocations are aligned).
constexpr int kCountLabels = 64;
// Hub rows (more than kBinWaveMaxDeg entries) of the count index, counted by
// segments of kHubSegment entries: segment s covers entries [seg_b, seg_e)
// of hub slot seg_slot[s], whose vertex is hub_v[slot]; hub_cnt holds
// [n_hubs][kCountLabels] 32-bit counts (cleared by the launcher).
struct CountIndexHubs {
    int64_t n_hubs = 0, n_segs = 0;
    const int32_t *hub_v = nullptr;
    const int32_t *seg_slot = nullptr;
    const int64_t *seg_b = nullptr, *seg_e = nullptr;
    uint32_t *hub_cnt = nullptr;
};
void launch_label_count(hipStream_t s, int64_t n, int64_t np, const int64_t *rp,
                        const int32_t *col, const uint8_t *labels, int nlab, uint8_t *cnt,
                        const CountIndexHubs &h);
// The same counts for every row of a subgraph given as CSR over all n
// vertices (rows of up to 2^31 entries; counts saturate at 255), in one
// pass without a hub list.
void launch_label_count_rows(hipStream_t s, int64_t n, int64_t np, const int64_t *rp,
                             const int32_t *col, const uint8_t *labels, int nlab, uint8_t *cnt);

// First LCC sweep from the count index: omega(v) = roles q of label(v) with
// cnt[L][v] >= need for every (L, need) of q (need_off[q] .. need_off[q+1]
// in need_lab / need_min).
template <typename M>
void launch_first_sweep_counts(hipStream_t s, int64_t n, int64_t np, const uint8_t *labels,
                               const uint64_t *lut, int lut_len, const uint8_t *cnt, int nlab,
                               const int32_t *need_off, const int32_t *need_lab,
                               const int32_t *need_min, int n0, M *omega);

// ---- learned order ----------------------------------------------------------
// counts[q] += number of vertices of tasks whose role set holds q (counts
// zeroed by the caller).
template <typename M>
void launch_role_totals(hipStream_t s, const int32_t *tasks, int64_t n_tasks, const M *omega,
                        int n0, unsigned long long *counts);
// Features of the remaining constraints, model scores, greedy choice.
void launch_order_select(hipStream_t s, const OrderArgs &a, OrderPick *out);
void launch_mlp_forward(hipStream_t s, const float *w, const float *x, int64_t n, float *y);
// Per-block partial gradients [kMlpGradGrid][kMlpParams] and partial losses
// [kMlpGradGrid], then their fixed-order sums into grad and loss[0].
void launch_mlp_grad(hipStream_t s, const float *w, const float *x, const float *t, int64_t n,
                     float *partial, float *partial_loss, float *grad, float *loss);
void launch_adam(hipStream_t s, float *w, const float *grad, float *m, float *v, float lr,
                 float bc1, float bc2);

// ---- state import, reuse, no-allocation scratch -------------------------------
template <typename M>
void launch_and_state(hipStream_t s, int64_t n, M *omega, const uint64_t *state);
template <typename M>
void launch_known_roles(hipStream_t s, const int32_t *tasks, int64_t n_tasks, const M *omega,
                        const uint64_t *known, M *cert);
void launch_known_edges(hipStream_t s, int64_t c_m, const int32_t *c_own, const int32_t *c_off,
                        const int64_t *rp, const uint64_t *known, uint64_t *c_cert);
// dst[i] |= src[i] (atomic OR per 64-bit word), i < n.
void launch_or_into(hipStream_t s, int64_t n, const uint64_t *src, uint64_t *dst);
void launch_label_degsum(hipStream_t s, int64_t n, const int64_t *rp, const void *labels,
                         int label_bytes, unsigned long long *sum, int64_t hist_len);
constexpr size_t kNoAllocBytes = PM_NOALLOC_SCRATCH_BYTES;
// Device address of this device's static no-allocation scratch array
// (kNoAllocBytes bytes); the device must be current.
hipError_t noalloc_scratch(int device, void **ptr);

// ---- match counting ----------------------------------------------------------
// Count tasks: compacted entries u -> w with qa in omega(u) and qb in
// omega(w), appended to eu/ew via *n_out (zeroed by the caller; at most cap
// written).
template <typename M>
void launch_count_tasks(hipStream_t s, int64_t c_m, const int32_t *c_own, const int32_t *c_col,
                        const M *omega, int qa, int qb, int32_t *eu, int32_t *ew, int32_t *n_out,
                        int64_t cap);
// Every map of the full template with plan *plan_id's pins at (eu[t],
// ew[t]) (or within split task ranges) is counted into *total; up to cap
// of them are written to maps[cap][n0] through *written.
// limit > 0: searches stop once the total reaches limit (*stop is set;
// the total is then a lower bound of the maps).
template <typename M>
void launch_count_search(hipStream_t s, const int32_t *eu, const int32_t *ew, int64_t n_tasks,
                         const M *omega, const int32_t *plan_id, const SearchArgs &a,
                         int32_t *maps, int64_t cap, unsigned long long *written,
                         unsigned long long *total, unsigned long long limit, int32_t *stop,
                         int grid);
template <typename M>
void launch_count_split(hipStream_t s, const SplitTask *tasks, int64_t n_tasks, const int32_t *eu,
                        const int32_t *ew, const M *omega, const int32_t *plan_id,
                        const SearchArgs &a, int32_t *maps, int64_t cap,
                        unsigned long long *written, unsigned long long *total,
                        unsigned long long limit, int32_t *stop, int grid);

void launch_fill_u64(hipStream_t s, uint64_t *p, int64_t n, uint64_t v);
void launch_fill_i32(hipStream_t s, int32_t *p, int64_t n, int32_t v);
void launch_label_hist(hipStream_t s, int64_t n, const void *labels, int label_bytes,
                       unsigned long long *hist, int64_t hist_len);

}  // namespace pm
