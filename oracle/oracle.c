/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct reference for the pruning computed by the
 * library.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load this file's library.  It shares no code, header or table
 * with the GPU path.
 *
 * Notation follows the paper: background graph G(V, E) in symmetric CSR
 * (row_ptr int64[n+1], col int32[m], sorted rows), labels l(v); template
 * G0(V0, E0) with n0 <= 64 vertices q, labels l(q); vertex match function
 * omega(v), a subset of V0 stored as a 64-bit mask (bit q = template vertex q),
 * as in the complexity section's bit-vector remark.
 *
 * Functions:
 *   orc_init_roles   -- INIT_VERTEX_STATE (vertex state and initialisation
 *                       algorithm): omega(v) = {q : l(q) = l(v)}.
 *   orc_lcc          -- LOCAL_CONSTRAINT_CHECKING (LCC algorithm and its
 *                       visitor), run synchronously (Jacobi): every sweep
 *                       reads only the previous sweep's state, as the barrier
 *                       after each traversal implies.  Local rule: role q of v
 *                       survives iff (coverage) every template neighbour of q
 *                       is a role of some neighbour of v, and (distinct count)
 *                       for each label L, at least as many distinct
 *                       neighbours u of label L carry a role adjacent to q as
 *                       q has template neighbours of label L (the LCC
 *                       description in the solution overview).
 *   orc_embed_exists -- the existence test behind every non-local constraint
 *                       and behind template-driven search (Remark on TDS):
 *                       an injective map of a substructure of G0 into G with
 *                       pinned images, label/role and edge checks at each
 *                       step.
 *   orc_nlcc         -- NON_LOCAL_CONSTRAINT_CHECKING for one constraint:
 *                       every (v, head role h) is checked against the state
 *                       before the constraint (all tokens finish before the
 *                       barrier), then unsatisfied head roles are removed.
 *   orc_exact        -- full-template search (Step 5(3) of constraint
 *                       generation, Remark on TDS) giving the exact role sets,
 *                       then for every edge the existence of a match that uses
 *                       it: the complete set of the problem statement.
 *   orc_bruteforce   -- the plain definition (exact match, Definition 1):
 *                       enumerate every injective, label-preserving map of V0
 *                       that maps E0 into E, and take the union of their
 *                       vertices (with roles) and edges.
 *   orc_lcc_sample   -- one LCC sweep (the rule above) evaluated for chosen
 *                       vertices only: timing samples of the CPU baseline.
 *   orc_enumerate    -- the same enumeration, writing every map phi out
 *                       (match enumeration and counting on the reduced
 *                       graph, termination and output section).
 *   orc_active_edges -- the edge state implied by omega during LCC/NLCC:
 *                       u->w is active iff some q in omega(u) and q' in
 *                       omega(w) are adjacent in G0 (edge elimination rule).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
    int64_t n;
    const int64_t *row_ptr;
    const int32_t *col;
    const int32_t *label;     /* l(v) */
} graph_t;

typedef struct {
    int n0, m0;
    int32_t label[64];        /* l(q) */
    uint64_t adj[64];         /* adj(q) as a mask over V0 */
    int32_t ea[64 * 64], eb[64 * 64];
} tmpl_t;

static int load_tmpl(tmpl_t *T, int n0, int m0, const int32_t *labels, const int32_t *edges) {
    if (n0 < 1 || n0 > 64 || m0 < 0 || m0 > 64 * 63 / 2) return -1;
    memset(T, 0, sizeof(*T));
    T->n0 = n0; T->m0 = m0;
    for (int q = 0; q < n0; ++q) T->label[q] = labels[q];
    for (int i = 0; i < m0; ++i) {
        int a = edges[2 * i], b = edges[2 * i + 1];
        if (a < 0 || b < 0 || a >= n0 || b >= n0 || a == b) return -1;
        T->ea[i] = a; T->eb[i] = b;
        T->adj[a] |= 1ull << b;
        T->adj[b] |= 1ull << a;
    }
    return 0;
}

static inline int popc(uint64_t x) { return __builtin_popcountll(x); }

/* binary search for w in the sorted adjacency of u; returns CSR index or -1 */
static int64_t find_edge(const graph_t *G, int32_t u, int32_t w) {
    int64_t lo = G->row_ptr[u], hi = G->row_ptr[u + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int32_t x = G->col[mid];
        if (x == w) return mid;
        if (x < w) lo = mid + 1; else hi = mid;
    }
    return -1;
}

/* ---- initial roles ----------------------------------------------------- */
int orc_init_roles(int64_t n, const int32_t *vlabel, int n0, int m0, const int32_t *tl,
                   const int32_t *te, uint64_t *omega) {
    tmpl_t T;
    if (load_tmpl(&T, n0, m0, tl, te)) return -1;
    #pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) {
        uint64_t w = 0;
        for (int q = 0; q < T.n0; ++q)
            if (T.label[q] == vlabel[v]) w |= 1ull << q;
        omega[v] = w;
    }
    return 0;
}

/* ---- LCC ---------------------------------------------------------------- */
/* One role q of v under the local rule, reading the neighbours' roles from
   `old`.  labmask[L] is the set of template vertices of label L. */
static int role_survives(const graph_t *G, const tmpl_t *T, const uint64_t *old, int64_t v,
                         int q, const uint64_t *labmask, int nlab) {
    const uint64_t need = T->adj[q];
    uint64_t cover = 0;
    for (int64_t e = G->row_ptr[v]; e < G->row_ptr[v + 1]; ++e) cover |= old[G->col[e]];
    if ((need & ~cover) != 0) return 0;                  /* adj(q) not covered */
    for (int L = 0; L < nlab; ++L) {
        uint64_t want = need & labmask[L];
        int mult = popc(want);
        if (mult < 2) continue;                           /* implied by coverage */
        int cnt = 0;
        for (int64_t e = G->row_ptr[v]; e < G->row_ptr[v + 1]; ++e)
            if (old[G->col[e]] & want) ++cnt;
        if (cnt < mult) return 0;                         /* too few distinct */
    }
    return 1;
}

/* Runs Jacobi sweeps to the fixpoint.  Returns the number of sweeps that
   changed at least one role (the last, unchanged sweep is not counted), or
   -1 on bad input. */
int64_t orc_lcc(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *vlabel,
                int n0, int m0, const int32_t *tl, const int32_t *te, uint64_t *omega,
                int64_t max_sweeps) {
    tmpl_t T;
    if (load_tmpl(&T, n0, m0, tl, te)) return -1;
    graph_t G = {n, row_ptr, col, vlabel};
    int nlab = 0;
    for (int q = 0; q < n0; ++q) if (T.label[q] + 1 > nlab) nlab = T.label[q] + 1;
    uint64_t *labmask = (uint64_t *)calloc((size_t)nlab + 1, sizeof(uint64_t));
    for (int q = 0; q < n0; ++q) labmask[T.label[q]] |= 1ull << q;
    uint64_t *old = (uint64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint64_t));
    int64_t sweeps = 0;
    for (;;) {
        if (max_sweeps >= 0 && sweeps >= max_sweeps) break;
        memcpy(old, omega, (size_t)n * sizeof(uint64_t));
        int64_t changed = 0;
        #pragma omp parallel for schedule(dynamic, 512) reduction(+:changed)
        for (int64_t v = 0; v < n; ++v) {
            uint64_t w = old[v];
            if (!w) continue;
            uint64_t nw = 0;
            for (int q = 0; q < T.n0; ++q)
                if (((w >> q) & 1) && role_survives(&G, &T, old, v, q, labmask, nlab))
                    nw |= 1ull << q;
            omega[v] = nw;
            if (nw != w) ++changed;
        }
        if (!changed) break;
        ++sweeps;
    }
    free(old); free(labmask);
    return sweeps;
}

/* ---- rooted injective embedding of a substructure ---------------------- */
typedef struct {
    int k;                 /* substructure vertices */
    int npin;              /* pinned prefix length (1 or 2) */
    int q[64];             /* template vertex at each search position */
    int parent[64];        /* earlier position adjacent to this one */
    uint64_t back[64];     /* earlier positions adjacent in the substructure */
} plan_t;

/* Search order: the pinned vertices first, then breadth-first over the
   substructure's edges, neighbours in ascending template index. */
static void make_plan(plan_t *P, uint64_t vmask, const uint64_t *sadj, int qa, int qb) {
    int pos_of[64];
    for (int i = 0; i < 64; ++i) pos_of[i] = -1;
    P->k = 0;
    P->q[P->k] = qa; P->parent[P->k] = -1; pos_of[qa] = P->k++;
    P->npin = 1;
    if (qb >= 0) { P->q[P->k] = qb; P->parent[P->k] = 0; pos_of[qb] = P->k++; P->npin = 2; }
    for (int head = 0; head < P->k; ++head) {
        int x = P->q[head];
        for (int y = 0; y < 64; ++y) {
            if (!((sadj[x] >> y) & 1) || !((vmask >> y) & 1) || pos_of[y] >= 0) continue;
            P->q[P->k] = y; P->parent[P->k] = head; pos_of[y] = P->k++;
        }
    }
    for (int i = 0; i < P->k; ++i) {
        P->back[i] = 0;
        for (int j = 0; j < i; ++j)
            if ((sadj[P->q[i]] >> P->q[j]) & 1) P->back[i] |= 1ull << j;
    }
}

/* Step `pos` proposes images for template vertex q[pos] among the neighbours
   of an already-mapped template neighbour's image -- the one with the
   fewest neighbours, which changes only how many proposals are made -- and
   accepts x if q[pos] is in omega(x) (so l(x) = l(q)), x is not yet used,
   and x is adjacent to the images of all mapped template neighbours. */
static int extend(const graph_t *G, const uint64_t *omega, const plan_t *P, int pos,
                  int32_t *img) {
    if (pos == P->k) return 1;
    const int q = P->q[pos];
    int32_t p = img[P->parent[pos]];
    for (int j = 0; j < pos; ++j)
        if (((P->back[pos] >> j) & 1) &&
            G->row_ptr[img[j] + 1] - G->row_ptr[img[j]] < G->row_ptr[p + 1] - G->row_ptr[p])
            p = img[j];
    for (int64_t e = G->row_ptr[p]; e < G->row_ptr[p + 1]; ++e) {
        const int32_t x = G->col[e];
        if (!((omega[x] >> q) & 1)) continue;            /* role / label check */
        int ok = 1;
        for (int j = 0; j < pos && ok; ++j) if (img[j] == x) ok = 0;   /* injective */
        for (int j = 0; j < pos && ok; ++j)
            if (((P->back[pos] >> j) & 1) && img[j] != p && find_edge(G, img[j], x) < 0) ok = 0;
        if (!ok) continue;
        img[pos] = x;
        if (extend(G, omega, P, pos + 1, img)) return 1;
    }
    return 0;
}

static uint64_t sub_adj_from_edges(uint64_t sadj[64], int me, const int32_t *se) {
    uint64_t vmask = 0;
    for (int i = 0; i < 64; ++i) sadj[i] = 0;
    for (int i = 0; i < me; ++i) {
        int a = se[2 * i], b = se[2 * i + 1];
        sadj[a] |= 1ull << b; sadj[b] |= 1ull << a;
        vmask |= (1ull << a) | (1ull << b);
    }
    return vmask;
}

/* Exported single query: does an injective embedding of the substructure
   (edge list se[2*me]) exist with qa -> va (and qb -> vb if qb >= 0)? */
int orc_embed_exists(int64_t n, const int64_t *row_ptr, const int32_t *col,
                     const uint64_t *omega, int me, const int32_t *se,
                     int qa, int32_t va, int qb, int32_t vb) {
    graph_t G = {n, row_ptr, col, NULL};
    uint64_t sadj[64];
    uint64_t vmask = sub_adj_from_edges(sadj, me, se);
    if (me == 0) vmask = 1ull << qa;
    if (!((omega[va] >> qa) & 1)) return 0;
    plan_t P;
    make_plan(&P, vmask, sadj, qa, qb);
    int32_t img[64];
    img[0] = va;
    if (qb >= 0) {
        if (!((omega[vb] >> qb) & 1) || vb == va) return 0;
        if (find_edge(&G, va, vb) < 0) return 0;
        img[1] = vb;
    }
    return extend(&G, omega, &P, P.npin, img);
}

/* ---- NLCC for one constraint (snapshot semantics) ---------------------- */
/* Returns the number of vertices whose role set shrank, or -1 on bad input. */
int64_t orc_nlcc(int64_t n, const int64_t *row_ptr, const int32_t *col, uint64_t *omega,
                 int me, const int32_t *se, uint64_t heads) {
    graph_t G = {n, row_ptr, col, NULL};
    uint64_t sadj[64];
    uint64_t vmask = sub_adj_from_edges(sadj, me, se);
    if (me <= 0 || (heads & ~vmask)) return -1;
    plan_t plans[64];
    for (int h = 0; h < 64; ++h)
        if ((heads >> h) & 1) make_plan(&plans[h], vmask, sadj, h, -1);
    uint64_t *sat = (uint64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t v = 0; v < n; ++v) {
        uint64_t cand = omega[v] & heads;
        for (int h = 0; h < 64; ++h) {
            if (!((cand >> h) & 1)) continue;
            int32_t img[64];
            img[0] = (int32_t)v;
            if (extend(&G, omega, &plans[h], 1, img)) sat[v] |= 1ull << h;
        }
    }
    int64_t changed = 0;
    for (int64_t v = 0; v < n; ++v) {
        uint64_t nw = omega[v] & (~heads | sat[v]);
        if (nw != omega[v]) { omega[v] = nw; ++changed; }
    }
    free(sat);
    return changed;
}

/* ---- exact step ---------------------------------------------------------- */
/* role_out[v] = roles of v that appear in some full match within the current
   candidate state; edge_out = CSR-entry bitmap (bit e%64 of word e/64) of
   entries u->w used by some match.  Returns 0, or -1 on bad input. */
int orc_exact(int64_t n, const int64_t *row_ptr, const int32_t *col, const uint64_t *omega,
              int n0, int m0, const int32_t *tl, const int32_t *te, uint64_t *role_out,
              uint64_t *edge_out) {
    tmpl_t T;
    if (load_tmpl(&T, n0, m0, tl, te)) return -1;
    graph_t G = {n, row_ptr, col, NULL};
    const int64_t m = row_ptr[n];
    memset(edge_out, 0, (size_t)((m + 63) / 64) * sizeof(uint64_t));
    if (n0 == 1) {
        for (int64_t v = 0; v < n; ++v) role_out[v] = omega[v] & 1ull;
        return 0;
    }
    uint64_t vmask = (n0 == 64) ? ~0ull : ((1ull << n0) - 1ull);
    plan_t vplan[64];
    for (int q = 0; q < n0; ++q) make_plan(&vplan[q], vmask, T.adj, q, -1);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t v = 0; v < n; ++v) {
        uint64_t r = 0;
        for (int q = 0; q < n0; ++q) {
            if (!((omega[v] >> q) & 1)) continue;
            int32_t img[64];
            img[0] = (int32_t)v;
            if (extend(&G, omega, &vplan[q], 1, img)) r |= 1ull << q;
        }
        role_out[v] = r;
    }
    /* oriented template edges: (a, b) and (b, a) */
    plan_t *eplan = (plan_t *)malloc(sizeof(plan_t) * (size_t)(2 * m0 > 0 ? 2 * m0 : 1));
    for (int i = 0; i < m0; ++i) {
        make_plan(&eplan[2 * i], vmask, T.adj, T.ea[i], T.eb[i]);
        make_plan(&eplan[2 * i + 1], vmask, T.adj, T.eb[i], T.ea[i]);
    }
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t u = 0; u < n; ++u) {
        if (!role_out[u]) continue;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            const int32_t w = col[e];
            if (!role_out[w]) continue;
            int used = 0;
            for (int k = 0; k < 2 * m0 && !used; ++k) {
                const plan_t *P = &eplan[k];
                if (!((role_out[u] >> P->q[0]) & 1) || !((role_out[w] >> P->q[1]) & 1)) continue;
                int32_t img[64];
                img[0] = (int32_t)u; img[1] = w;
                if (extend(&G, omega, P, 2, img)) used = 1;
            }
            if (used) {
                #pragma omp atomic
                edge_out[e >> 6] |= 1ull << (e & 63);
            }
        }
    }
    free(eplan);
    return 0;
}

/* ---- brute force: union of all exact matches --------------------------- */
typedef struct {
    const graph_t *G;
    const tmpl_t *T;
    plan_t P;
    uint64_t *role_out;
    uint64_t *edge_out;
    int64_t count;
    int64_t limit;
    int32_t *maps;           /* orc_enumerate: maps written here (or NULL) */
    int64_t cap, written;
} bf_t;

static void bf_record(bf_t *B, const int32_t *img) {
    const plan_t *P = &B->P;
    if (B->maps) {
        int64_t at;
        #pragma omp atomic capture
        at = B->written++;
        if (at < B->cap)
            for (int i = 0; i < P->k; ++i) B->maps[at * B->T->n0 + P->q[i]] = img[i];
    }
    for (int i = 0; i < P->k; ++i) {
        #pragma omp atomic
        B->role_out[img[i]] |= 1ull << P->q[i];
    }
    int pos_of[64];
    for (int i = 0; i < P->k; ++i) pos_of[P->q[i]] = i;
    for (int i = 0; i < B->T->m0; ++i) {
        int32_t a = img[pos_of[B->T->ea[i]]], b = img[pos_of[B->T->eb[i]]];
        int64_t e1 = find_edge(B->G, a, b), e2 = find_edge(B->G, b, a);
        #pragma omp atomic
        B->edge_out[e1 >> 6] |= 1ull << (e1 & 63);
        #pragma omp atomic
        B->edge_out[e2 >> 6] |= 1ull << (e2 & 63);
    }
}

/* Remark-1 search: step k proposes v_k adjacent to an earlier image, with
   the right label, unused, and adjacent to every earlier image that its
   template vertex is adjacent to. */
static void bf_extend(bf_t *B, int pos, int32_t *img, int64_t *local_count) {
    const plan_t *P = &B->P;
    if (pos == P->k) { bf_record(B, img); ++*local_count; return; }
    const int q = P->q[pos];
    const int32_t p = img[P->parent[pos]];
    const graph_t *G = B->G;
    for (int64_t e = G->row_ptr[p]; e < G->row_ptr[p + 1]; ++e) {
        const int32_t x = G->col[e];
        if (G->label[x] != B->T->label[q]) continue;
        int ok = 1;
        for (int j = 0; j < pos && ok; ++j) if (img[j] == x) ok = 0;
        for (int j = 0; j < pos && ok; ++j)
            if (((P->back[pos] >> j) & 1) && find_edge(G, x, img[j]) < 0) ok = 0;
        if (!ok) continue;
        img[pos] = x;
        bf_extend(B, pos + 1, img, local_count);
    }
}

/* Returns the number of injective maps phi enumerated (each subgraph H is
   counted once per automorphism of G0 that preserves labels), or -1. */
int64_t orc_bruteforce(int64_t n, const int64_t *row_ptr, const int32_t *col,
                       const int32_t *vlabel, int n0, int m0, const int32_t *tl,
                       const int32_t *te, uint64_t *role_out, uint64_t *edge_out) {
    tmpl_t T;
    if (load_tmpl(&T, n0, m0, tl, te)) return -1;
    graph_t G = {n, row_ptr, col, vlabel};
    const int64_t m = row_ptr[n];
    memset(role_out, 0, (size_t)n * sizeof(uint64_t));
    memset(edge_out, 0, (size_t)((m + 63) / 64) * sizeof(uint64_t));
    bf_t B;
    memset(&B, 0, sizeof(B));
    B.G = &G; B.T = &T; B.role_out = role_out; B.edge_out = edge_out;
    uint64_t vmask = (n0 == 64) ? ~0ull : ((1ull << n0) - 1ull);
    make_plan(&B.P, vmask, T.adj, 0, -1);
    if (B.P.k != n0) return -1;                        /* template disconnected */
    int64_t total = 0;
    #pragma omp parallel for schedule(dynamic, 64) reduction(+:total)
    for (int64_t v = 0; v < n; ++v) {
        if (vlabel[v] != T.label[0]) continue;
        int32_t img[64];
        img[0] = (int32_t)v;
        int64_t c = 0;
        bf_extend(&B, 1, img, &c);
        total += c;
    }
    return total;
}

/* ---- derived edge state -------------------------------------------------- */
int orc_active_edges(int64_t n, const int64_t *row_ptr, const int32_t *col,
                     const uint64_t *omega, int n0, int m0, const int32_t *tl,
                     const int32_t *te, uint64_t *edge_out) {
    tmpl_t T;
    if (load_tmpl(&T, n0, m0, tl, te)) return -1;
    const int64_t m = row_ptr[n];
    memset(edge_out, 0, (size_t)((m + 63) / 64) * sizeof(uint64_t));
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t u = 0; u < n; ++u) {
        uint64_t reach = 0;                     /* roles adjacent to omega(u) */
        for (int q = 0; q < n0; ++q) if ((omega[u] >> q) & 1) reach |= T.adj[q];
        if (!reach) continue;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
            if (omega[col[e]] & reach) {
                #pragma omp atomic
                edge_out[e >> 6] |= 1ull << (e & 63);
            }
    }
    return 0;
}

int orc_num_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int t) { if (t > 0) omp_set_num_threads(t); }

/* ---- exact step on a vertex subset (timing samples only) ---------------- */
/* Runs, for the given vertices only, the same searches orc_exact runs for
   them: one full-template search per candidate role, and one per candidate
   entry u->w and oriented template edge (w's candidate roles stand in for
   its exact roles).  Returns the number of searches run. */
int64_t orc_exact_subset(int64_t n, const int64_t *row_ptr, const int32_t *col,
                         const uint64_t *omega, int n0, int m0, const int32_t *tl,
                         const int32_t *te, const int32_t *verts, int64_t nverts) {
    tmpl_t T;
    if (load_tmpl(&T, n0, m0, tl, te)) return -1;
    graph_t G = {n, row_ptr, col, NULL};
    if (n0 == 1) return 0;
    uint64_t vmask = (n0 == 64) ? ~0ull : ((1ull << n0) - 1ull);
    plan_t vplan[64];
    for (int q = 0; q < n0; ++q) make_plan(&vplan[q], vmask, T.adj, q, -1);
    plan_t *eplan = (plan_t *)malloc(sizeof(plan_t) * (size_t)(2 * m0 > 0 ? 2 * m0 : 1));
    for (int i = 0; i < m0; ++i) {
        make_plan(&eplan[2 * i], vmask, T.adj, T.ea[i], T.eb[i]);
        make_plan(&eplan[2 * i + 1], vmask, T.adj, T.eb[i], T.ea[i]);
    }
    int64_t searches = 0;
    #pragma omp parallel for schedule(dynamic, 1) reduction(+:searches)
    for (int64_t i = 0; i < nverts; ++i) {
        const int32_t v = verts[i];
        uint64_t r = 0;
        for (int q = 0; q < n0; ++q) {
            if (!((omega[v] >> q) & 1)) continue;
            int32_t img[64];
            img[0] = v;
            ++searches;
            if (extend(&G, omega, &vplan[q], 1, img)) r |= 1ull << q;
        }
        if (!r) continue;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int32_t w = col[e];
            if (!omega[w]) continue;
            for (int k = 0; k < 2 * m0; ++k) {
                const plan_t *P = &eplan[k];
                if (!((r >> P->q[0]) & 1) || !((omega[w] >> P->q[1]) & 1)) continue;
                int32_t img[64];
                img[0] = v; img[1] = w;
                ++searches;
                if (extend(&G, omega, P, 2, img)) break;
            }
        }
    }
    free(eplan);
    return searches;
}

/* Exact-step results for sampled vertices only (parity checks at sizes the
 * full exact step cannot be run on the CPU): role_out[i] = the roles q in
 * omega(verts[i]) for which a full match with phi(q) = verts[i] exists, and
 * for the j-th CSR entry verts[i] -> w, inc_out[inc_off[i] + j] = 1 iff some
 * full match maps a template edge onto it (edge-pinned search over both
 * orientations of every template edge), else 0.  omega must be a sound
 * superset of the complete set (any state the constraint loop reaches).
 * Returns the number of searches, or -1 for a bad template. */
int64_t orc_exact_sample(int64_t n, const int64_t *row_ptr, const int32_t *col,
                         const uint64_t *omega, int n0, int m0, const int32_t *tl,
                         const int32_t *te, const int32_t *verts, int64_t nverts,
                         uint64_t *role_out, const int64_t *inc_off, uint8_t *inc_out) {
    tmpl_t T;
    if (load_tmpl(&T, n0, m0, tl, te)) return -1;
    graph_t G = {n, row_ptr, col, NULL};
    uint64_t vmask = (n0 == 64) ? ~0ull : ((1ull << n0) - 1ull);
    plan_t vplan[64];
    for (int q = 0; q < n0; ++q) make_plan(&vplan[q], vmask, T.adj, q, -1);
    plan_t *eplan = (plan_t *)malloc(sizeof(plan_t) * (size_t)(2 * m0 > 0 ? 2 * m0 : 1));
    for (int i = 0; i < m0; ++i) {
        make_plan(&eplan[2 * i], vmask, T.adj, T.ea[i], T.eb[i]);
        make_plan(&eplan[2 * i + 1], vmask, T.adj, T.eb[i], T.ea[i]);
    }
    int64_t searches = 0;
    #pragma omp parallel for schedule(dynamic, 1) reduction(+:searches)
    for (int64_t i = 0; i < nverts; ++i) {
        const int32_t v = verts[i];
        uint64_t r = 0;
        if (n0 == 1) {
            r = omega[v] & 1ull;
        } else {
            for (int q = 0; q < n0; ++q) {
                if (!((omega[v] >> q) & 1)) continue;
                int32_t img[64];
                img[0] = v;
                ++searches;
                if (extend(&G, omega, &vplan[q], 1, img)) r |= 1ull << q;
            }
        }
        role_out[i] = r;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            uint8_t hit = 0;
            const int32_t w = col[e];
            if (r && omega[w]) {
                for (int k = 0; k < 2 * m0 && !hit; ++k) {
                    const plan_t *P = &eplan[k];
                    if (!((r >> P->q[0]) & 1) || !((omega[w] >> P->q[1]) & 1)) continue;
                    int32_t img[64];
                    img[0] = v; img[1] = w;
                    ++searches;
                    if (extend(&G, omega, P, 2, img)) hit = 1;
                }
            }
            inc_out[inc_off[i] + (e - row_ptr[v])] = hit;
        }
    }
    free(eplan);
    return searches;
}

/* ---- enumeration (Definition 1 written out) ------------------------------- */
/* Every map phi of the brute force above, as n0 images in template-vertex
   order, the first `cap` of them written to maps[cap][n0] (in no fixed
   order: the vertex loop is parallel).  Returns the number of maps, or -1. */
int64_t orc_enumerate(int64_t n, const int64_t *row_ptr, const int32_t *col,
                      const int32_t *vlabel, int n0, int m0, const int32_t *tl,
                      const int32_t *te, int32_t *maps, int64_t cap) {
    const int64_t m = row_ptr[n];
    uint64_t *role = (uint64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
    uint64_t *edge = (uint64_t *)calloc((size_t)((m + 63) / 64 + 1), sizeof(uint64_t));
    tmpl_t T;
    if (load_tmpl(&T, n0, m0, tl, te)) { free(role); free(edge); return -1; }
    graph_t G = {n, row_ptr, col, vlabel};
    bf_t B;
    memset(&B, 0, sizeof(B));
    B.G = &G; B.T = &T; B.role_out = role; B.edge_out = edge;
    B.maps = maps; B.cap = cap;
    uint64_t vmask = (n0 == 64) ? ~0ull : ((1ull << n0) - 1ull);
    make_plan(&B.P, vmask, T.adj, 0, -1);
    if (B.P.k != n0) { free(role); free(edge); return -1; }
    int64_t total = 0;
    #pragma omp parallel for schedule(dynamic, 64) reduction(+:total)
    for (int64_t v = 0; v < n; ++v) {
        if (vlabel[v] != T.label[0]) continue;
        int32_t img[64];
        img[0] = (int32_t)v;
        int64_t c = 0;
        bf_extend(&B, 1, img, &c);
        total += c;
    }
    free(role); free(edge);
    return total;
}

/* ---- one LCC sweep on sampled vertices ------------------------------------ */
/* out[i] = the roles of verts[i] that survive one application of the local
   rule to the state `omega` (the vertex's own roles filtered by
   role_survives).  Returns the CSR entries the sampled rows hold, or -1. */
int64_t orc_lcc_sample(int64_t n, const int64_t *row_ptr, const int32_t *col,
                       const int32_t *vlabel, int n0, int m0, const int32_t *tl,
                       const int32_t *te, const uint64_t *omega, const int32_t *verts,
                       int64_t nv, uint64_t *out) {
    tmpl_t T;
    if (load_tmpl(&T, n0, m0, tl, te)) return -1;
    graph_t G = {n, row_ptr, col, vlabel};
    int nlab = 0;
    for (int q = 0; q < n0; ++q) if (T.label[q] + 1 > nlab) nlab = T.label[q] + 1;
    uint64_t *labmask = (uint64_t *)calloc((size_t)nlab + 1, sizeof(uint64_t));
    for (int q = 0; q < n0; ++q) labmask[T.label[q]] |= 1ull << q;
    int64_t entries = 0;
    #pragma omp parallel for schedule(dynamic, 256) reduction(+:entries)
    for (int64_t i = 0; i < nv; ++i) {
        const int64_t v = verts[i];
        const uint64_t w = omega[v];
        uint64_t nw = 0;
        for (int q = 0; q < T.n0; ++q)
            if (((w >> q) & 1) && role_survives(&G, &T, omega, v, q, labmask, nlab))
                nw |= 1ull << q;
        out[i] = nw;
        entries += row_ptr[v + 1] - row_ptr[v];
    }
    free(labmask);
    return entries;
}
