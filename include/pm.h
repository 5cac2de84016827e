/*
 * pm.h -- C ABI of the constraint-checking pruner for AMD MI355X (gfx950).
 *
 * Problem (Preliminaries, Definition 1 of the paper): given a simple,
 * undirected, vertex-labeled background graph G(V, E) and a small connected
 * labeled template G0(V0, E0), compute the complete set: every (vertex,
 * template role) pair and every edge that takes part in at least one exact
 * match of G0 (an injective, label-preserving map phi of V0 into V that maps
 * every template edge onto an edge of G; non-induced).
 *
 * Method (main constraint-checking loop): initialise each vertex's candidate
 * roles omega(v) from its label (vertex state and initialisation algorithm),
 * run local constraint checking (LCC) to a fixpoint, then for each
 * non-local constraint (cycle, path and template-driven-search constraints
 * generated per the constraint-generation table) run non-local constraint
 * checking (NLCC) followed by LCC when anything changed, and finish with a
 * full-template search that certifies every surviving role and edge.  For
 * an acyclic template whose labels are unique except for one pair of
 * vertices the finish is exact without searches: at the LCC fixpoint a
 * role is in a match iff the homomorphisms of the template path between the
 * pair through it can put the pair on two different vertices, decided by
 * sweeps that carry the smallest and largest reachable end vertex along the
 * path (setting "tree_exact").
 *
 * Conventions
 *  - All functions return PM_OK (0) or a negative PM_ERR_* code; the message
 *    of the last error on the calling thread is returned by pm_last_error().
 *    No C++ exception crosses this boundary.
 *  - Device pointers are HIP device addresses on the context's device.
 *  - A context is bound to one device and one HIP stream and must not be used
 *    from two threads at once.  Calls on one context are serialised on its
 *    stream; pm_prune returns after its work has completed.
 *  - Role bit q of a role mask is template vertex q in the order given to
 *    pm_load_templates.  Edge bit e (bit e % 64 of word e / 64, least
 *    significant bit first) is CSR entry e of the loaded graph; the edge set
 *    is symmetric.
 *  - Environment variables read by pm_create (work-saving switches of the
 *    final search; none changes any result): PM_EXPAND=0 turns off the
 *    single-vertex swap scans of found matches, PM_EXPAND_EDGES=0 only
 *    those after edge-rooted finds, PM_EXPAND_MAX=k skips scans
 *    of lists longer than k (default 4096), PM_WITNESS=1 turns on certifying candidate
 *    edges by swaps of recorded witnesses (off by default: measured slower
 *    once the edge searches use relisted roles), PM_RELIST=0 keeps the edge
 *    searches on the pre-search role lists, PM_EDGE_CHUNK=k sets the edge
 *    tasks a wavefront takes at once (default 16), PM_EDGE_STRIPES=s the
 *    number of stripes the edge task list is dealt in (default 64),
 *    PM_SPLIT_BUDGET=s the steps after which an edge-rooted search hands
 *    its unexplored candidate ranges on (default 8192; 0 never),
 *    PM_EDGE_TAIL=k the trailing edge tasks dealt singly (default 0),
 *    PM_EXPAND_TABLE_LOG2=t the swap-scan table size (default 22),
 *    PM_READ_FIRST=1 reads certificate words before setting them,
 *    PM_TREE_EXACT=0 runs the search-based finish for one-repeated-pair
 *    trees too.  These seed
 *    the settings of pm_set_param.  Read by pm_load_graph:
 *    PM_NO_COUNT_INDEX=1 skips the neighbour-label count index (the first
 *    LCC sweep then gathers over the CSR).
 */
#ifndef PM_H
#define PM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PM_OK               0
#define PM_ERR_INVALID_ARG (-1)   /* null pointer, bad size or flag         */
#define PM_ERR_HIP         (-2)   /* a HIP runtime call failed              */
#define PM_ERR_GRAPH       (-3)   /* graph violates the CSR contract        */
#define PM_ERR_TEMPLATE    (-4)   /* template invalid or over the limits    */
#define PM_ERR_NO_GRAPH    (-5)   /* pm_prune before pm_load_graph          */
#define PM_ERR_CAPACITY    (-6)   /* an internal bound was exceeded         */
#define PM_ERR_OOM         (-7)   /* device memory exhausted                */
#define PM_ERR_NOT_FOUND   (-8)   /* unknown template id                    */
#define PM_ERR_MODEL       (-9)   /* no ordering model loaded, or bad one   */
#define PM_ERR_WORKSPACE  (-10)   /* caller workspace too small or misaligned */

/* ---- limits -------------------------------------------------------------- */
#define PM_MAX_TEMPLATE_VERTICES 64   /* role masks are 64-bit              */
#define PM_MAX_COUNT_RULES       32   /* per-label distinct-count rules     */
#define PM_MAX_CONSTRAINTS       64   /* non-local constraints per template */

/* ---- flags for pm_load_graph ---------------------------------------------- */
#define PM_HOST_PTRS  1u   /* row_ptr/col/labels are host memory: copied      */
#define PM_VALIDATE   2u   /* check the CSR contract (costs a host pass)      */

typedef struct pm_ctx pm_ctx;

/* Template: n0 vertices with labels[n0], m0 undirected edges given as
   edges[2*i], edges[2*i+1] (vertex indices < n0).  Host memory, copied. */
typedef struct {
    uint32_t n0;
    uint32_t m0;
    const uint16_t *labels;
    const uint32_t *edges;
} pm_template;

/* Order of the non-local constraints. */
#define PM_ORDER_FIXED   0   /* generation order (ordering heuristics)      */
#define PM_ORDER_GIVEN   1   /* options.order[] permutation                  */
#define PM_ORDER_LEARNED 2   /* greedy by the loaded model's score (below)   */

/* Learned ordering model (the paper leaves constraint selection and ordering
   by modelling open, conclusion): before each step the library computes
   PM_MLP_FEATURES features of every remaining constraint from the current
   state, runs a perceptron PM_MLP_FEATURES -> 64 -> 64 -> 2 (ReLU, fp32)
   that predicts y0 = log2(1 + role bits removed by the constraint and the
   LCC fixpoint after it) and y1 = log2(1 + microseconds both take), and
   checks the remaining constraint of largest score y0 - y1 (ties: lowest
   index).  Features of constraint k with vertex set Vk, edges Ek, heads
   Hk, at a state with active role counts c[q] (vertices whose role set
   holds q), counts c0[q] at the first LCC fixpoint, nA vertices with a
   non-empty role set, background label frequency F[q] of q's label, d of K
   constraints checked; lg(x) = log2(1 + x), min/mean/max over q in Vk:
     f0 |Ek|/8, f1 |Vk|/8, f2 cycle kind, f3 TDS kind, f4 |Hk|/|Vk|,
     f5 min lg(c)/16, f6 mean lg(c)/16, f7 max lg(c)/16, f8 lg(nA)/16,
     f9 mean lg(F)/16, f10 mean(lg(c0) - lg(c))/16, f11 d/K.
   Parameters (PM_MLP_PARAMS fp32, packed): W1[64][12], b1[64], W2[64][64],
   b2[64], W3[2][64], b3[2].  The final full-template search always runs,
   so the pruning output does not depend on the order or on the model. */
#define PM_MLP_FEATURES 12
#define PM_MLP_HIDDEN   64
#define PM_MLP_OUTPUTS  2
#define PM_MLP_PARAMS   5122

/* Pruning modes (pm_options.mode). */
#define PM_MODE_FULL      0   /* complete set of the template                */
#define PM_MODE_CANDIDATE 1   /* candidate set of the interactive incremental
                                 search: local constraints only, with the rule
                                 relaxed so that the result holds the complete
                                 set of EVERY connected template obtained from
                                 this one by deleting edges (role q of v stays
                                 while some neighbour of v holds a role
                                 adjacent to q in G0).  Outputs omega and the
                                 edge state it implies; no non-local
                                 constraint and no final search run.          */

/* Ablations of the paper's design decisions (pm_options.ablate bits), for
   measurement only: the output does not change. */
#define PM_ABLATE_EDGE_ELIMINATION 1u  /* the candidate subgraph keeps every
                                          entry of an active vertex's row
                                          (only vertex elimination prunes)   */
#define PM_ABLATE_WORK_AGGREGATION 2u  /* a found embedding certifies only the
                                          query it answers (its root role, or
                                          its root edge); no single-vertex
                                          swap expansion                     */

typedef struct pm_stats pm_stats;

/* One step of the constraint loop, recorded when options.trace is set. */
typedef struct {
    int32_t constraint;            /* generation index; -1: the learned loop
                                      stopped before this step (score below
                                      learned_min_score)                      */
    int32_t changed;               /* vertices whose role set the NLCC step
                                      shrank                                  */
    int64_t roles_before;          /* role bits over all vertices before     */
    int64_t roles_after;           /* after the step and its LCC fixpoint    */
    int64_t active_before;         /* vertices with a non-empty role set     */
    float ms;                      /* device time of the step and its LCC    */
    float score;                   /* model score (0 when no model loaded)   */
    float predicted[PM_MLP_OUTPUTS];
    float features[PM_MLP_FEATURES];
} pm_trace_entry;

typedef struct {
    int32_t order_mode;            /* PM_ORDER_FIXED, _GIVEN or _LEARNED      */
    int32_t n_order;               /* entries in order[] for PM_ORDER_GIVEN   */
    int32_t order[PM_MAX_CONSTRAINTS];
    int32_t stop_after;            /* -1: full prune.  k >= 0: stop after k
                                      constraints (0 = after the first LCC
                                      fixpoint); outputs are then omega and
                                      the edge state it implies, without the
                                      final search                            */
    int32_t batch_streams;         /* count > 1: prune up to this many
                                      templates concurrently, each on its own
                                      stream and scratch (0/1: one at a time).
                                      Templates are dealt longest-first by
                                      independent cycles, edges, vertices    */
    float learned_min_score;       /* PM_ORDER_LEARNED with learned_stop: end
                                      the constraint loop when the best
                                      remaining score is below this (the
                                      final search still runs)                */
    int32_t learned_stop;          /* nonzero: apply learned_min_score        */
    int32_t trace_cap;             /* entries available in trace[]            */
    pm_trace_entry *trace;         /* host array or NULL; count must be 1.
                                      stats.trace_entries receives the number
                                      written (at most trace_cap)            */
    int32_t mode;                  /* PM_MODE_FULL or PM_MODE_CANDIDATE      */
    uint32_t ablate;               /* PM_ABLATE_* bits                       */
    const uint64_t *init_state;    /* device uint64[count][n] or NULL: role
                                      masks known to hold the complete set of
                                      each template (an exported state, a
                                      candidate set, the complete set of a
                                      template this one adds edges to); the
                                      prune starts from omega0(v) AND
                                      init_state[v].  A state that is not a
                                      superset of the complete set gives a
                                      wrong (too small) result.              */
    uint64_t skip_mask;            /* with init_state: non-local constraints
                                      (bit = generation index) already applied
                                      to that state; they are not checked
                                      again and count towards stop_after     */
    const uint64_t *known_roles;   /* device uint64[count][n] or NULL: roles
                                      known to belong to the complete set
                                      (the complete set of a template this one
                                      deletes edges from); the final search
                                      takes them as certified.  Must be a
                                      subset of the complete set.             */
    const uint64_t *known_edges;   /* device uint64[count][ceil(m/64)] or
                                      NULL: edge bits known to belong to the
                                      complete set (same conditions)          */
    int32_t shared_inputs;         /* nonzero: init_state, known_roles and
                                      known_edges are ONE array ([n] or
                                      [ceil(m/64)]) used for every template of
                                      the call                                */
    int32_t pad_;
    uint64_t *union_roles;         /* device uint64[n] or NULL: every
                                      template's role masks are ORed into it
                                      (caller-initialised; atomic, so
                                      concurrent templates may share it)      */
    uint64_t *union_edges;         /* device uint64[ceil(m/64)] or NULL: the
                                      same for the edge bits                  */
    pm_stats *per_template;        /* host pm_stats[count] or NULL: each
                                      template's own statistics               */
    int32_t limit_checks;          /* nonzero: check at most max_checks
                                      non-local constraints (in the selected
                                      order), then run the final search as
                                      usual -- the output does not change     */
    int32_t max_checks;
    int32_t reserved[4];
} pm_options;

/* Per-call statistics (valid when pm_prune returns PM_OK). */
struct pm_stats {
    double ms_total;               /* whole prune, device time                */
    double ms_init;                /* role initialisation                     */
    double ms_lcc;                 /* all LCC sweeps                          */
    double ms_compact;             /* candidate-subgraph compaction           */
    double ms_nlcc;                /* all non-local constraint checks         */
    double ms_exact;               /* final full-template search              */
    double ms_first_sweep;         /* first LCC sweep over the full graph,
                                      including its binning                   */
    double ms_sweep_kernel;        /* the first sweep's kernel alone          */
    double wave_ms_vq_pos;         /* summed wavefront time of successful and */
    double wave_ms_vq_neg;         /* failed vertex-rooted searches, and of   */
    double wave_ms_eq_pos;         /* successful and failed edge-rooted       */
    double wave_ms_eq_neg;         /* searches (exact step)                   */
    double wave_ms_certify;        /* wavefront time certifying found matches
                                      and their single-vertex swaps           */
    double wave_ms_expand;         /* the single-vertex swaps alone           */
    int64_t lcc_sweeps;            /* LCC sweeps run                          */
    int64_t constraints;           /* non-local constraints checked           */
    int64_t first_sweep_vertices;  /* active vertices in the first sweep      */
    int64_t first_sweep_entries;   /* their CSR entries                       */
    int64_t candidate_entries;     /* entries of the compacted subgraph       */
    int64_t vertex_queries;        /* full-template searches from a vertex    */
    int64_t edge_queries;          /* full-template searches from an edge     */
    int64_t result_vertices;       /* vertices with a non-empty role mask     */
    int64_t edge_candidates;       /* edges left for edge-rooted searches     */
    int64_t vq_pos, vq_neg;        /* vertex-rooted searches found / failed   */
    int64_t eq_pos, eq_neg;        /* edge-rooted searches found / failed     */
    int64_t trace_entries;         /* pm_trace_entry records written          */
    int64_t expand_scans;          /* swap scans (found match, template vertex) */
    int64_t expand_candidates;     /* role-list entries those scans read      */
    int64_t expand_valid;          /* swaps that gave another match           */
    int64_t first_sweep_bytes;     /* compulsory bytes of the first LCC sweep
                                      when it runs from the neighbour-label
                                      count index (else 0)                     */
    int64_t witness_edges;         /* candidate edges certified by moving one
                                      template vertex of a recorded match      */
    int64_t split_tasks;           /* unexplored ranges handed on by edge-rooted
                                      searches that ran past their step budget */
    uint64_t done_mask;            /* non-local constraints applied to the
                                      final state (bit = generation index),
                                      including options.skip_mask; OR over the
                                      templates when count > 1               */
    int64_t workspace_bytes;       /* peak device scratch of one template's
                                      prune (largest over the templates)      */
    int64_t join_edges;            /* candidate edges certified by joining the
                                      recorded matches of their two ends
                                      across a bridge of the template         */
};

/* Returns the message for the last error on this thread ("" if none). */
const char *pm_last_error(void);

/* Library version string. */
const char *pm_version(void);

/* Create a context on HIP device `device` using `hip_stream` (a hipStream_t,
   NULL for the default stream).  *out receives the context. */
int pm_create(pm_ctx **out, int device, void *hip_stream);

/* Release the context and all device memory the library allocated. */
int pm_destroy(pm_ctx *ctx);

/* Load the background graph (Preliminaries: simple, undirected,
   vertex-labeled): n vertices, m CSR entries (both directions of every
   edge), row_ptr int64[n+1], col int32[m] with sorted rows, no self-loops
   and no duplicate entries, labels[n] of label_bytes (1 or 2) bytes each.
   The arrays are borrowed -- they must stay valid and unchanged until
   pm_unload_graph/pm_destroy -- unless PM_HOST_PTRS is set, in which case
   they are copied to device memory owned by the context.  PM_VALIDATE
   checks symmetry, ordering, loops and id range and returns PM_ERR_GRAPH on
   a violation.  For uint8 labels whose largest value is below 64 the call
   also builds a per-graph index, n * (largest label + 1) bytes of device
   memory owned by the context: the number of neighbours of each label at
   every vertex (saturated at 255), from which every prune evaluates its
   first LCC sweep without reading the adjacency lists. */
int pm_load_graph(pm_ctx *ctx, int64_t n, int64_t m, const int64_t *row_ptr,
                  const int32_t *col, const void *labels, int label_bytes, uint32_t flags);

/* (Re)build the neighbour-label count index of the loaded graph: one
   streaming pass over row_ptr and col that gathers every neighbour's label
   and writes cnt[L][v] (the counts the first LCC sweep of every template
   reads; vertex state and initialisation plus the LCC rule).  pm_load_graph
   builds it once; this call rebuilds it, e.g. to time the pass.  *ms (may
   be NULL) receives its device time (events on the context stream).
   PM_ERR_INVALID_ARG when the graph is not eligible (labels not uint8 below
   64, or m >= 2^32). */
int pm_build_count_index(pm_ctx *ctx, double *ms);

/* Build the label-pair subgraph of the loaded graph for the templates
   [first_id, first_id + count): the entries u -> x whose label pair
   (label(u), label(x)) is that of an edge of one of them, each with its
   offset in u's row (int64 row_ptr[n+1] plus two int32 arrays per entry,
   device memory owned by the context, replacing any earlier one; count = 0
   frees it).  An entry whose labels are not those of a template edge never
   joins two adjacent roles, so the edge elimination of the LCC description
   drops it in every prune: every later prune of a template whose edges'
   label pairs the subgraph holds starts its first compaction from it
   instead of from the whole graph (same results; with
   PM_ABLATE_EDGE_ELIMINATION the whole graph is used).  On a graph eligible
   for the count index, the call also counts the labels of every row of the
   subgraph (same layout as the count index, labels x n bytes): the first
   LCC sweep reads a vertex's counts only for labels of template neighbours
   of its roles, label pairs the subgraph keeps whole, so a template it
   covers takes its first sweep from these counts, with the same result as
   from the graph's index.  Meant for batches and sessions of templates over
   the same labels, e.g. a template and its relaxations.  *ms (may be NULL)
   receives its device time (subgraph and counts).
   PM_ERR_INVALID_ARG if the templates' edges use more than 64 labels or an
   id is out of range; PM_ERR_CAPACITY if the subgraph would have 2^31
   entries or more (no subgraph is kept then). */
int pm_build_pair_index(pm_ctx *ctx, int32_t first_id, int32_t count, double *ms);

/* Facts about the loaded graph. */
typedef struct {
    int64_t n, m;
    int32_t label_bytes;
    int32_t index_labels;      /* labels covered by the count index (0: none) */
    int64_t index_bytes;       /* bytes of the count index                    */
    int64_t hubs;              /* rows longer than 4096 entries               */
    int64_t hub_segments;      /* their 4096-entry segments                   */
    double ms_count_index;     /* device time of the last index build         */
    int64_t pair_entries;      /* entries of the label-pair subgraph (-1: none) */
    double ms_pair_index;      /* device time of its build                    */
} pm_graph_info_t;
int pm_graph_info(pm_ctx *ctx, pm_graph_info_t *out);

/* Forget the loaded graph (and free copies made under PM_HOST_PTRS). */
int pm_unload_graph(pm_ctx *ctx);

/* Compile `count` templates (constraint generation per the paper's table of
   Steps 1-5 and the TDS-generation algorithm; search plans; LCC tables).
   Templates must be connected (Preliminaries), have 1..64 vertices, no
   self-loops or duplicate edges, and at most PM_MAX_COUNT_RULES
   distinct-count rules.  *first_id receives the id of the first template;
   the others follow consecutively.  PM_ERR_TEMPLATE on a violation; no
   template is added then. */
int pm_load_templates(pm_ctx *ctx, int32_t count, const pm_template *t, int32_t *first_id);

/* Number of non-local constraints of template `id` and their kinds
   (0 cycle, 1 path, 2 TDS-cycle, 3 TDS-path), edge counts and head masks, in
   generation order.  Arrays must hold PM_MAX_CONSTRAINTS entries; edges_out
   receives, for constraint i, its edges at edges_out[i*2*64 ...] as pairs
   (a < b) sorted ascending, up to 64 pairs. */
int pm_template_constraints(pm_ctx *ctx, int32_t id, int32_t *count, int32_t *kinds,
                            int32_t *n_edges, uint64_t *heads, uint32_t *edges_out);

/* Same as pm_template_constraints for a template that is compiled on the
   host only (no context, no device): validation and constraint generation.
   Returns PM_ERR_TEMPLATE for an invalid template. */
int pm_inspect_template(const pm_template *t, int32_t *count, int32_t *kinds, int32_t *n_edges,
                        uint64_t *heads, uint32_t *edges_out);

/* Prune the loaded graph against templates first_id .. first_id+count-1.
   role_mask: device uint64[count][n]; edge_bits: device
   uint64[count][ceil(m/64)]; both caller-owned and fully overwritten.
   opt may be NULL (fixed order, full prune).  stats may be NULL; with count
   > 1 it receives the sums over the templates. */
int pm_prune(pm_ctx *ctx, int32_t first_id, int32_t count, uint64_t *role_mask,
             uint64_t *edge_bits, const pm_options *opt, pm_stats *stats);

/* ---- tuning parameters ---------------------------------------------------------
   Work-saving settings of the final search and the search launch; none
   changes any result.  Names and values:
     "expand"        1/0   single-vertex swap scans of found matches (1)
     "expand_max"    k     skip swap scans of lists longer than k; -1: none (4096)
     "expand_edges"  1/0   swap scans also after matches found by edge-rooted
                           searches (1; "expand" 0 turns off both)
     "witness"       1/0   certify candidate edges by witness swaps (0)
     "tree_exact"    1/0   finish acyclic templates with one repeated-label
                           pair by path sweeps instead of searches (1)
     "relist"        1/0   edge searches on role lists of the exact roles (1)
     "edge_chunk"    k     edge tasks a wavefront takes at once (16)
     "edge_stripes"  s     stripes the edge task list is dealt in (64)
     "search_grid"   b     blocks of the persistent search kernels (8 per CU)
     "search_grid_solo" b  blocks shared by the searches that run at once:
                           a search launched while k workers of a batch
                           search (itself included) takes max(search_grid,
                           b / k) blocks, so one searching alone or at the
                           tail of a batch can fill the GPU; 0: off (0)
     "split_budget"  s     steps after which an edge-rooted search hands its
                           unexplored candidate ranges on to other
                           wavefronts; 0: never (8192; four times more in
                           each later round of split tasks)
     "edge_tail"     k     trailing edge tasks dealt one at a time (0)
     "expand_table_log2" t log2 of the slots of the swap-scan table (22)
     "split_capacity" c    split tasks one launch may hand on; a search
                           that finds no room carries on unsplit (2^18)
     "read_first"    1/0   read certificate words before setting them (0)
     "lcc_bin_small" d     LCC sweeps and compaction: vertices of degree <= d
                           take 4 lanes (8; 0 <= d <= lcc_bin_mid)
     "lcc_bin_mid"   d     ... degree <= d take 16 lanes, larger ones up to
                           4096 a wavefront, hubs 4096-entry segments
                           (64; lcc_bin_small <= d <= 4096)
   The environment variables listed at the top seed these defaults when the
   context is created.  PM_ERR_INVALID_ARG for an unknown name or a value
   out of range. */
int pm_set_param(pm_ctx *ctx, const char *name, int64_t value);
int pm_get_param(pm_ctx *ctx, const char *name, int64_t *value);

/* ---- learned ordering model ------------------------------------------------
   The perceptron and its training run in the library's kernels; the
   features and model are defined above PM_MLP_PARAMS. */

/* Copy PM_MLP_PARAMS fp32 parameters from host memory `w` (n must equal
   PM_MLP_PARAMS) into the context; PM_ORDER_LEARNED uses them from then on.
   PM_ERR_MODEL if a value is not finite. */
int pm_load_model(pm_ctx *ctx, const float *w, size_t n);

/* Forward pass: y[N][2] = model(x[N][12]) with parameters w (device
   float[PM_MLP_PARAMS]); all device pointers, row-major.  N >= 0. */
int pm_mlp_forward(pm_ctx *ctx, const float *w, const float *x, int64_t N, float *y);

/* Loss L = sum over samples and outputs of (y - t)^2 / (2N) and its
   gradient with respect to the packed parameters (ReLU'(0) = 0).  x[N][12],
   t[N][2], grad[PM_MLP_PARAMS], loss[1]: device pointers.  N >= 1.  The
   sums over samples are taken in a fixed order: results are deterministic. */
int pm_mlp_grad(pm_ctx *ctx, const float *w, const float *x, const float *t, int64_t N,
                float *grad, float *loss);

/* Full-batch Adam (beta1 0.9, beta2 0.999, eps 1e-8, zero initial moments)
   for `steps` steps of learning rate lr on the loss above, updating the
   device parameters w in place.  loss_history: host float[steps] receiving
   the loss before each step, or NULL. */
int pm_mlp_train(pm_ctx *ctx, float *w, const float *x, const float *t, int64_t N,
                 int32_t steps, float lr, float *loss_history);

/* ---- pruning state: export and resume --------------------------------------
   The whole pruning state is the role-set array omega (the edge state is
   derived from it: an entry is active iff its ends hold roles adjacent in
   G0) plus the set of non-local constraints already applied.  Any state
   that holds the complete set is a valid starting point, which is what
   lets the paper's checkpoint-and-resume (load balancing subsection) and
   its incremental searches restart from a saved solution or candidate set. */

/* Run template `id` through its first LCC fixpoint and the first
   stop_after non-local constraints (in the order opt selects; opt may be
   NULL), then write omega widened to uint64 into state (device uint64[n],
   caller-owned) and the applied constraints (bit = generation index) into
   *done_mask (host).  stop_after < 0 applies every constraint; the final
   search does not run. */
int pm_export_state(pm_ctx *ctx, int32_t id, int32_t stop_after, const pm_options *opt,
                    uint64_t *state, uint64_t *done_mask);

/* Resume template `id` from an exported state: omega starts at
   omega0 AND state (device uint64[n]), the constraints in done_mask are not
   checked again, and the prune continues as pm_prune does (LCC fixpoint,
   the remaining constraints, the final search; opt->stop_after counts the
   skipped constraints too).  The state must hold the complete set (any
   state pm_export_state wrote for this template and graph does).  Outputs
   as pm_prune; opt->init_state and opt->skip_mask are ignored. */
int pm_import_state(pm_ctx *ctx, int32_t id, const uint64_t *state, uint64_t done_mask,
                    uint64_t *role_mask, uint64_t *edge_bits, const pm_options *opt,
                    pm_stats *stats);

/* ---- caller-owned workspace ----------------------------------------------------
   By default the library allocates its scratch (grow-only, kept until
   pm_destroy).  After pm_set_workspace every prune takes all its scratch
   from the caller's device buffer instead and allocates nothing: the buffer
   is split into batch_streams equal slices (one per concurrent template),
   each slice used from its start by every template the worker prunes.

   pm_workspace_size: an upper bound of the bytes pm_prune(first_id, count,
   opt) can need with the current graph and settings (the compacted
   subgraph bounded by the entries of the vertices whose label occurs in the
   template, the role lists by that times the largest number of template
   vertices sharing a label).  A smaller workspace works whenever the data
   allow it: pm_stats.workspace_bytes of an earlier prune is the peak one
   template actually used.  A prune that runs out fails with
   PM_ERR_WORKSPACE (outputs undefined) and leaves the context usable. */
int pm_workspace_size(pm_ctx *ctx, int32_t first_id, int32_t count, const pm_options *opt,
                      size_t *bytes);

/* Use ws (device memory of the context's device, 256-byte aligned,
   caller-owned; the library never frees it) of `bytes` bytes for all
   scratch from now on; ws = NULL returns to library-owned scratch.  The
   caller must keep the buffer alive and must not use it while a prune
   runs. */
int pm_set_workspace(pm_ctx *ctx, void *ws, size_t bytes);

/* ---- prune without allocation ---------------------------------------------------
   For callers that cannot allocate device memory (code under stream
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   prune as pm_prune with count = 1, with all scratch taken from a static
   device array of PM_NOALLOC_SCRATCH_BYTES bytes that the library holds on
   every device it runs on until the process ends.  No hipMalloc, hipFree or
   other allocating call is made.  The swap-scan table and the split-task
   lists use smaller sizes here (work-saving settings; results are the
   same).  PM_ERR_WORKSPACE when pm_workspace_size for this template exceeds
   the array.  All calls on one device share the array: calls that overlap
   on one device (two host threads, or two contexts on different streams)
   race and give undefined results; serialise them.  The array keeps the
   last call's contents; every call initialises what it reads. */
#define PM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int pm_prune_noalloc(pm_ctx *ctx, int32_t id, uint64_t *role_mask, uint64_t *edge_bits,
                     const pm_options *opt, pm_stats *stats);

/* ---- match counting and enumeration on the pruned graph --------------------
   Match enumeration and counting run on the reduced graph that pruning
   leaves (termination and output section): a full-template walk with
   aggregation off, every match verified.  Here: depth-first searches from
   every background CSR entry u -> w whose ends hold the roles of one chosen
   template edge (a, b), with a pinned at u and b at w, restricted to the
   role sets of `state`: every injective label-preserving map (Definition 1)
   puts (a, b) on exactly one entry, so each map is counted once. */
typedef struct {
    uint64_t maps;             /* matches as maps phi (Definition 1)            */
    uint64_t automorphisms;    /* label-preserving automorphisms of G0 (0 if
                                  more than 2^40 or too costly to count)        */
    uint64_t subgraphs;        /* maps / automorphisms: distinct matched
                                  subgraphs (0 when automorphisms is 0)         */
    int64_t written;           /* maps written to the output array            */
    int64_t roots;             /* edge-rooted searches run                    */
    double ms_total;           /* device time of the whole call               */
    int32_t complete;          /* 1: maps is the exact count; 0: the searches
                                  stopped at max_maps (maps is a lower bound) */
    int32_t pad_;
} pm_match_count;

/* Count (and optionally list) the matches of template `id` within state
   (device uint64[n]: role masks that hold the complete set -- the roles
   pm_prune returned for this template, an exported state -- or NULL for
   the label roles, which counts over the whole graph).  Role bits whose
   label differs from the vertex's are ignored.  maps_out: device
   int32[cap][n0] or NULL; receives min(cap, maps) maps (images of template
   vertices 0 .. n0-1), in no particular order.  max_maps > 0 stops the
   searches soon after that many maps are counted (out->complete = 0; the
   count of a template with very many matches grows with the matches, so a
   caller that only needs "at least" can bound the time).  Result in *out
   (host). */
int pm_count_matches(pm_ctx *ctx, int32_t id, const uint64_t *state, int32_t *maps_out,
                     int64_t cap, uint64_t max_maps, pm_match_count *out);

#ifdef __cplusplus
}
#endif

#endif /* PM_H */
