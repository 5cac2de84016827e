/*
 * Seeded synthetic inputs: R-MAT background graphs in symmetric CSR form and
 * vertex labels.  This module holds input generation only; nothing in it
 * computes any part of the pruning method.
 *
 * Graph recipe (the paper's synthetic-graph section and its R-MAT degree
 * sensitivity study): 2^S vertices, edge factor 16 samples per vertex, R-MAT
 * quadrant probabilities (A, B, C, D) (Graph500: 0.57, 0.19, 0.19, 0.05),
 * undirected (both directions stored), self-loops and duplicate edges
 * dropped, adjacency lists sorted ascending.  Vertex ids are scrambled by a
 * seeded bijection on [0, 2^S), as Graph500 does, so that hubs are not
 * clustered at low ids.
 *
 * Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC 2011), a counter-based
 * generator, so any sample can be regenerated independently and the
 * two-pass CSR build needs no sample buffer.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* ---- Philox4x32-10 ------------------------------------------------------ */
static inline void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

void pmgen_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(M0, c0, &hi0, &lo0);
        mulhilo32(M1, c2, &hi1, &lo1);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ---- seeded bijection on S-bit ids ------------------------------------- */
typedef struct { uint64_t mask; uint64_t m1, a1, m2, a2; int sh; } perm_t;

static perm_t make_perm(int scale, uint64_t seed) {
    perm_t p;
    p.mask = (scale >= 64) ? ~0ull : ((1ull << scale) - 1ull);
    uint32_t ctr[4] = {0u, 0u, 0u, 0xA5A5A5A5u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    pmgen_philox4x32_10(ctr, key, r);
    p.m1 = (((uint64_t)r[0] << 32) | r[1]) | 1ull;   /* odd multipliers are */
    p.m2 = (((uint64_t)r[2] << 32) | r[3]) | 1ull;   /* invertible mod 2^S  */
    ctr[0] = 1u;
    pmgen_philox4x32_10(ctr, key, r);
    p.a1 = ((uint64_t)r[0] << 32) | r[1];
    p.a2 = ((uint64_t)r[2] << 32) | r[3];
    p.sh = scale / 2 > 0 ? scale / 2 : 1;
    return p;
}

static inline uint64_t apply_perm(const perm_t *p, uint64_t x) {
    /* each step is a bijection of [0, 2^S): affine maps with odd multiplier,
       and x ^= x >> sh with sh >= 1 */
    x = (x * p->m1 + p->a1) & p->mask;
    x ^= x >> p->sh;
    x = (x * p->m2 + p->a2) & p->mask;
    x ^= x >> p->sh;
    x = (x * p->m1 + p->a2) & p->mask;
    return x;
}

uint64_t pmgen_perm(int scale, uint64_t seed, uint64_t x) {
    perm_t p = make_perm(scale, seed);
    return apply_perm(&p, x);
}

/* ---- one R-MAT sample --------------------------------------------------- */
typedef struct {
    int scale;
    uint32_t ta, tab, tabc;   /* cumulative thresholds scaled by 2^32 */
    uint32_t key[2];
    int permute;
    perm_t perm;
} rmat_t;

static inline void rmat_sample(const rmat_t *g, uint64_t i, uint64_t *src, uint64_t *dst) {
    uint64_t u = 0, v = 0;
    int level = 0;
    for (uint32_t blk = 0; level < g->scale; ++blk) {
        uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), blk, 0u};
        uint32_t r[4];
        pmgen_philox4x32_10(ctr, g->key, r);
        for (int k = 0; k < 4 && level < g->scale; ++k, ++level) {
            uint32_t x = r[k];
            int ub, vb;
            if (x < g->ta)        { ub = 0; vb = 0; }
            else if (x < g->tab)  { ub = 0; vb = 1; }
            else if (x < g->tabc) { ub = 1; vb = 0; }
            else                  { ub = 1; vb = 1; }
            u = (u << 1) | (uint64_t)ub;
            v = (v << 1) | (uint64_t)vb;
        }
    }
    if (g->permute) {
        u = apply_perm(&g->perm, u);
        v = apply_perm(&g->perm, v);
    }
    *src = u; *dst = v;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static void sort_i32(int32_t *a, int64_t len) {
    if (len < 24) {
        for (int64_t i = 1; i < len; ++i) {
            int32_t key = a[i];
            int64_t j = i - 1;
            while (j >= 0 && a[j] > key) { a[j + 1] = a[j]; --j; }
            a[j + 1] = key;
        }
    } else {
        qsort(a, (size_t)len, sizeof(int32_t), cmp_i32);
    }
}

/* Handle for a built graph; exported in a second call so that the caller
   owns the final arrays. */
typedef struct {
    int64_t n, m;
    int64_t *row_ptr;   /* n+1 */
    int32_t *col;       /* m   */
} pmgen_graph_t;

/*
 * Build the symmetric, sorted, duplicate- and loop-free CSR of an R-MAT
 * graph.  thr[0..2] are the cumulative quadrant thresholds A, A+B, A+B+C as
 * fractions of 2^32.  Returns NULL on allocation failure.
 */
void *pmgen_rmat_build(int scale, int64_t nsamples, uint32_t t_a, uint32_t t_ab,
                       uint32_t t_abc, uint64_t seed, int permute) {
    if (scale < 1 || scale > 31) return NULL;
    rmat_t g;
    g.scale = scale; g.ta = t_a; g.tab = t_ab; g.tabc = t_abc;
    g.key[0] = (uint32_t)seed; g.key[1] = (uint32_t)(seed >> 32);
    g.permute = permute;
    g.perm = make_perm(scale, seed ^ 0x5DEECE66Dull);
    const int64_t n = (int64_t)1 << scale;

    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return NULL;
    /* pass 1: raw degree of each endpoint (both directions) */
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nsamples; ++i) {
        uint64_t u, v;
        rmat_sample(&g, (uint64_t)i, &u, &v);
        if (u == v) continue;
        #pragma omp atomic
        cnt[u] += 1;
        #pragma omp atomic
        cnt[v] += 1;
    }
    int64_t *off = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!off) { free(cnt); return NULL; }
    off[0] = 0;
    for (int64_t v = 0; v < n; ++v) off[v + 1] = off[v] + cnt[v];
    const int64_t raw_m = off[n];
    int32_t *raw = (int32_t *)malloc((size_t)(raw_m > 0 ? raw_m : 1) * sizeof(int32_t));
    if (!raw) { free(cnt); free(off); return NULL; }
    memcpy(cnt, off, (size_t)n * sizeof(int64_t));   /* cnt becomes the fill cursor */
    /* pass 2: regenerate the same samples and scatter both directions */
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nsamples; ++i) {
        uint64_t u, v;
        rmat_sample(&g, (uint64_t)i, &u, &v);
        if (u == v) continue;
        int64_t pu, pv;
        #pragma omp atomic capture
        pu = cnt[u]++;
        #pragma omp atomic capture
        pv = cnt[v]++;
        raw[pu] = (int32_t)v;
        raw[pv] = (int32_t)u;
    }
    /* per-row sort and dedup (rows are independent) */
    int64_t *deg = cnt;
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t v = 0; v < n; ++v) {
        int32_t *row = raw + off[v];
        int64_t len = off[v + 1] - off[v];
        sort_i32(row, len);
        int64_t w = 0;
        for (int64_t k = 0; k < len; ++k)
            if (w == 0 || row[k] != row[w - 1]) row[w++] = row[k];
        deg[v] = w;
    }
    pmgen_graph_t *out = (pmgen_graph_t *)malloc(sizeof(pmgen_graph_t));
    if (!out) { free(cnt); free(off); free(raw); return NULL; }
    out->n = n;
    out->row_ptr = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!out->row_ptr) { free(out); free(cnt); free(off); free(raw); return NULL; }
    out->row_ptr[0] = 0;
    for (int64_t v = 0; v < n; ++v) out->row_ptr[v + 1] = out->row_ptr[v] + deg[v];
    out->m = out->row_ptr[n];
    out->col = (int32_t *)malloc((size_t)(out->m > 0 ? out->m : 1) * sizeof(int32_t));
    if (!out->col) { free(out->row_ptr); free(out); free(cnt); free(off); free(raw); return NULL; }
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < n; ++v)
        memcpy(out->col + out->row_ptr[v], raw + off[v], (size_t)deg[v] * sizeof(int32_t));
    free(raw); free(off); free(cnt);
    return out;
}

int64_t pmgen_graph_n(void *h) { return ((pmgen_graph_t *)h)->n; }
int64_t pmgen_graph_m(void *h) { return ((pmgen_graph_t *)h)->m; }

void pmgen_graph_export(void *h, int64_t *row_ptr, int32_t *col) {
    pmgen_graph_t *g = (pmgen_graph_t *)h;
    memcpy(row_ptr, g->row_ptr, ((size_t)g->n + 1) * sizeof(int64_t));
    /* large copies in parallel chunks */
    const int64_t chunk = (int64_t)1 << 22;
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < g->m; s += chunk) {
        int64_t e = s + chunk < g->m ? s + chunk : g->m;
        memcpy(col + s, g->col + s, (size_t)(e - s) * sizeof(int32_t));
    }
}

void pmgen_graph_free(void *h) {
    pmgen_graph_t *g = (pmgen_graph_t *)h;
    if (!g) return;
    free(g->row_ptr); free(g->col); free(g);
}

/* uniform labels in [0, nlabels): one Philox draw per vertex, scaled by a
   multiply-shift so the mapping is exact in integers */
void pmgen_labels_uniform(int64_t n, int nlabels, uint64_t seed, uint8_t *out) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    #pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) {
        uint32_t ctr[4] = {(uint32_t)v, (uint32_t)((uint64_t)v >> 32), 0u, 0x1AB31u};
        uint32_t r[4];
        pmgen_philox4x32_10(ctr, key, r);
        out[v] = (uint8_t)(((uint64_t)r[0] * (uint64_t)nlabels) >> 32);
    }
}

/* degree labels: ceil(log2(d + 1)), i.e. the bit length of d */
void pmgen_labels_log2deg(int64_t n, const int64_t *row_ptr, uint8_t *out) {
    #pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) {
        uint64_t d = (uint64_t)(row_ptr[v + 1] - row_ptr[v]);
        int b = 0;
        while (d) { ++b; d >>= 1; }
        out[v] = (uint8_t)b;
    }
}
