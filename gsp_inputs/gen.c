/*
 * gen.c - seeded synthetic graph generators shared by the tests, the bench
 * and the oracle's checks.  This file holds no arithmetic of the community
 * detection method: it only draws random graphs and writes them as a
 * symmetric CSR (int64 offsets, int32 columns, optional fp32 weights).
 *
 * Random numbers come from two published generators, written here from
 * their definitions:
 *   - SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), used for seeding and
 *     for the order-free edge-weight hash;
 *   - xoshiro256** (Blackman and Vigna, 2018), used for every stream.
 * G(n, p) blocks use the geometric skipping method of Batagelj and Brandes
 * (Phys. Rev. E 71, 2005).  R-MAT follows Chakrabarti, Zhan and Faloutsos
 * (SDM 2004): one quadrant draw per level.
 *
 * Conventions for every generator:
 *   - undirected graphs, stored with both directions of each edge;
 *   - self-loops dropped, duplicate edges dropped (not summed);
 *   - rows sorted by column;
 *   - optional random relabelling of the vertices (Graph500 convention);
 *   - weights either absent (unit) or w = lo + (hi-lo) * u rounded to fp32,
 *     with u = (h >> 40) / 2^24 and h = SplitMix64 hash of
 *     (min(u,v), max(u,v), seed), so both directions get the same weight.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct gen_graph {
    int64_t n, nnz;
    int64_t *off;  /* n+1 */
    int32_t *col;  /* nnz */
    float *w;      /* nnz, or NULL for unit weights */
    int64_t *block; /* planted block of each vertex (after relabelling), or NULL */
} gen_graph;

/* Progress lines on stderr for long generations (gen_set_verbose). */
#include <stdio.h>
static int gen_verbose = 0;
void gen_set_verbose(int v) { gen_verbose = v; }
static void progress(const char *what, int64_t count) {
    if (!gen_verbose) return;
    fprintf(stderr, "[gen] %s: %lld\n", what, (long long)count);
    fflush(stderr);
}

/* ---------------- PRNGs ---------------- */

static inline uint64_t splitmix64_next(uint64_t *x) {
    uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t splitmix64_hash(uint64_t v) {
    uint64_t x = v;
    return splitmix64_next(&x);
}

typedef struct { uint64_t s[4]; } xoshiro;

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static inline uint64_t xo_next(xoshiro *r) {
    uint64_t *s = r->s;
    uint64_t result = rotl64(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return result;
}

static void xo_seed(xoshiro *r, uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; i++) r->s[i] = splitmix64_next(&x);
}

/* uniform double in [0, 1) with 53 random bits */
static inline double xo_uniform(xoshiro *r) { return (double)(xo_next(r) >> 11) * 0x1.0p-53; }

/* ---------------- edge list ---------------- */

typedef struct { int64_t len, cap; int32_t *u, *v; } edge_list;

static int el_push(edge_list *e, int32_t u, int32_t v) {
    if (e->len == e->cap) {
        int64_t nc = e->cap ? e->cap * 2 : 1024;
        int32_t *nu = (int32_t *)realloc(e->u, (size_t)nc * sizeof(int32_t));
        if (!nu) return -1;
        e->u = nu;
        int32_t *nv = (int32_t *)realloc(e->v, (size_t)nc * sizeof(int32_t));
        if (!nv) return -1;
        e->v = nv;
        e->cap = nc;
    }
    e->u[e->len] = u;
    e->v[e->len] = v;
    e->len++;
    return 0;
}

static void el_free(edge_list *e) { free(e->u); free(e->v); e->u = e->v = NULL; e->len = e->cap = 0; }

/* ---------------- CSR build ---------------- */

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Insertion sort for short rows, qsort for long ones. */
static void sort_row(int32_t *a, int64_t len) {
    if (len < 32) {
        for (int64_t i = 1; i < len; i++) {
            int32_t x = a[i];
            int64_t j = i - 1;
            while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; j--; }
            a[j + 1] = x;
        }
    } else {
        qsort(a, (size_t)len, sizeof(int32_t), cmp_i32);
    }
}

/* Builds the symmetric CSR of an undirected edge list (both directions,
 * no self-loops, no duplicates, sorted rows).  Takes ownership of nothing. */
static gen_graph *build_csr(int64_t n, int64_t m, const int32_t *eu, const int32_t *ev) {
    gen_graph *g = (gen_graph *)calloc(1, sizeof(gen_graph));
    if (!g) return NULL;
    g->n = n;
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) { free(g); return NULL; }
    for (int64_t e = 0; e < m; e++) {
        if (eu[e] == ev[e]) continue;
        cnt[eu[e] + 1]++;
        cnt[ev[e] + 1]++;
    }
    for (int64_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
    int64_t raw = cnt[n];
    progress("csr: entries counted", raw);
    int32_t *col = (int32_t *)malloc((size_t)(raw > 0 ? raw : 1) * sizeof(int32_t));
    int64_t *cur = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!col || !cur) { free(cnt); free(col); free(cur); free(g); return NULL; }
    memcpy(cur, cnt, (size_t)n * sizeof(int64_t));
    for (int64_t e = 0; e < m; e++) {
        int32_t a = eu[e], b = ev[e];
        if (a == b) continue;
        col[cur[a]++] = b;
        col[cur[b]++] = a;
    }
    free(cur);
    progress("csr: entries placed", raw);
    /* sort + dedupe each row in place; new lengths in deg[] */
    int64_t *deg = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!deg) { free(cnt); free(col); free(g); return NULL; }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; i++) {
        int32_t *row = col + cnt[i];
        int64_t len = cnt[i + 1] - cnt[i];
        sort_row(row, len);
        int64_t k = 0;
        for (int64_t t = 0; t < len; t++)
            if (k == 0 || row[t] != row[k - 1]) row[k++] = row[t];
        deg[i] = k;
    }
    int64_t *off = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!off) { free(cnt); free(col); free(deg); free(g); return NULL; }
    off[0] = 0;
    for (int64_t i = 0; i < n; i++) off[i + 1] = off[i] + deg[i];
    /* compact rows forward (destination never passes the source) */
    for (int64_t i = 0; i < n; i++)
        if (off[i] != cnt[i]) memmove(col + off[i], col + cnt[i], (size_t)deg[i] * sizeof(int32_t));
    free(cnt);
    free(deg);
    g->nnz = off[n];
    progress("csr: rows sorted, duplicates dropped", g->nnz);
    int32_t *shrunk = (int32_t *)realloc(col, (size_t)(g->nnz > 0 ? g->nnz : 1) * sizeof(int32_t));
    g->col = shrunk ? shrunk : col;
    g->off = off;
    return g;
}

static float edge_weight(int32_t a, int32_t b, uint64_t seed, double lo, double hi) {
    uint64_t x = (uint64_t)(uint32_t)(a < b ? a : b);
    uint64_t y = (uint64_t)(uint32_t)(a < b ? b : a);
    uint64_t h = splitmix64_hash(seed ^ 0x5851f42d4c957f2dULL);
    h = splitmix64_hash(h ^ x);
    h = splitmix64_hash(h ^ (y * 0x9e3779b97f4a7c15ULL));
    double u = (double)(h >> 40) * 0x1.0p-24;
    return (float)(lo + (hi - lo) * u);
}

static int attach_weights(gen_graph *g, uint64_t seed, double lo, double hi) {
    if (g->nnz == 0) { g->w = (float *)malloc(sizeof(float)); return g->w ? 0 : -1; }
    g->w = (float *)malloc((size_t)g->nnz * sizeof(float));
    if (!g->w) return -1;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < g->n; i++)
        for (int64_t e = g->off[i]; e < g->off[i + 1]; e++)
            g->w[e] = edge_weight((int32_t)i, g->col[e], seed, lo, hi);
    return 0;
}

/* random permutation of [0, n) by Fisher-Yates */
static int32_t *random_perm(int64_t n, uint64_t seed) {
    int32_t *p = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!p) return NULL;
    for (int64_t i = 0; i < n; i++) p[i] = (int32_t)i;
    xoshiro r;
    xo_seed(&r, seed ^ 0xa0761d6478bd642fULL);
    for (int64_t i = n - 1; i > 0; i--) {
        int64_t j = (int64_t)(xo_uniform(&r) * (double)(i + 1));
        if (j > i) j = i;
        int32_t t = p[i]; p[i] = p[j]; p[j] = t;
    }
    return p;
}

/* G(n, p) over the vertex range [base, base + s): Batagelj-Brandes skipping.
 * Pairs are (v, w) with w < v, enumerated row by row. */
static int gnp_block(edge_list *el, int64_t base, int64_t s, double p, xoshiro *r) {
    if (p <= 0.0 || s < 2) return 0;
    if (p >= 1.0) {
        for (int64_t v = 1; v < s; v++)
            for (int64_t w = 0; w < v; w++)
                if (el_push(el, (int32_t)(base + v), (int32_t)(base + w))) return -1;
        return 0;
    }
    double lp = log(1.0 - p);
    int64_t v = 1, w = -1;
    while (v < s) {
        double u = xo_uniform(r);
        w += 1 + (int64_t)floor(log(1.0 - u) / lp);
        while (w >= v && v < s) { w -= v; v++; }
        if (v < s)
            if (el_push(el, (int32_t)(base + v), (int32_t)(base + w))) return -1;
    }
    return 0;
}

/* ---------------- public generators ---------------- */

/* Planted-partition SBM: n vertices in `blocks` near-equal consecutive
 * blocks (block b holds [b n / blocks, (b+1) n / blocks) before the
 * relabelling), each intra-block pair an edge with
 * probability p_in, each inter-block pair with probability p_out.  Drawn as
 * the union of G(n, p_out) and, per block, G(s, q) with
 * q = (p_in - p_out) / (1 - p_out), so an intra pair is present with
 * probability 1 - (1 - p_out)(1 - q) = p_in. */
gen_graph *gen_sbm(int64_t n, int64_t blocks, double p_in, double p_out, uint64_t seed, int permute,
                   int weighted, double wlo, double whi) {
    if (n <= 0 || blocks <= 0 || blocks > n) return NULL;
    edge_list el = {0, 0, NULL, NULL};
    xoshiro r;
    xo_seed(&r, seed);
    if (gnp_block(&el, 0, n, p_out, &r)) { el_free(&el); return NULL; }
    double q = p_out < 1.0 ? (p_in - p_out) / (1.0 - p_out) : 0.0;
    for (int64_t b = 0; b < blocks; b++) {
        int64_t lo = b * n / blocks, hi = (b + 1) * n / blocks;
        if (gnp_block(&el, lo, hi - lo, q, &r)) { el_free(&el); return NULL; }
    }
    int32_t *perm = NULL;
    if (permute) {
        perm = random_perm(n, seed);
        if (!perm) { el_free(&el); return NULL; }
        for (int64_t e = 0; e < el.len; e++) { el.u[e] = perm[el.u[e]]; el.v[e] = perm[el.v[e]]; }
    }
    gen_graph *g = build_csr(n, el.len, el.u, el.v);
    el_free(&el);
    if (!g) { free(perm); return NULL; }
    g->block = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (g->block) {
        for (int64_t v = 0; v < n; v++) {
            int64_t b = v * blocks / n;
            while ((b + 1) * n / blocks <= v) b++;
            while (b * n / blocks > v) b--;
            g->block[perm ? perm[v] : v] = b;
        }
    }
    free(perm);
    if (weighted && attach_weights(g, seed, wlo, whi)) return NULL;
    return g;
}

/* R-MAT: `samples` edge draws on 2^scale vertices with quadrant
 * probabilities (a, b, c, 1-a-b-c).  Samples are drawn in blocks of 2^16,
 * each block from its own xoshiro stream seeded by SplitMix64(seed, block),
 * so the result does not depend on the thread count. */
gen_graph *gen_rmat(int scale, int64_t samples, double a, double b, double c, uint64_t seed,
                    int permute, int weighted, double wlo, double whi) {
    if (scale < 1 || scale > 30 || samples < 0) return NULL;
    int64_t n = (int64_t)1 << scale;
    int32_t *eu = (int32_t *)malloc((size_t)(samples > 0 ? samples : 1) * sizeof(int32_t));
    int32_t *ev = (int32_t *)malloc((size_t)(samples > 0 ? samples : 1) * sizeof(int32_t));
    if (!eu || !ev) { free(eu); free(ev); return NULL; }
    const int64_t BLK = (int64_t)1 << 16;
    int64_t nblk = (samples + BLK - 1) / BLK;
    double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < nblk; k++) {
        xoshiro r;
        uint64_t sx = seed * 0x9e3779b97f4a7c15ULL + (uint64_t)k;
        xo_seed(&r, splitmix64_hash(sx));
        int64_t e0 = k * BLK, e1 = e0 + BLK < samples ? e0 + BLK : samples;
        for (int64_t e = e0; e < e1; e++) {
            uint32_t u = 0, v = 0;
            for (int l = 0; l < scale; l++) {
                double x = xo_uniform(&r);
                uint32_t bu, bv;
                if (x < a) { bu = 0; bv = 0; }
                else if (x < ab) { bu = 0; bv = 1; }
                else if (x < abc) { bu = 1; bv = 0; }
                else { bu = 1; bv = 1; }
                u = (u << 1) | bu;
                v = (v << 1) | bv;
            }
            eu[e] = (int32_t)u;
            ev[e] = (int32_t)v;
        }
    }
    progress("rmat: samples drawn", samples);
    if (permute) {
        int32_t *perm = random_perm(n, seed);
        if (!perm) { free(eu); free(ev); return NULL; }
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < samples; e++) { eu[e] = perm[eu[e]]; ev[e] = perm[ev[e]]; }
        free(perm);
        progress("rmat: vertices relabelled", n);
    }
    gen_graph *g = build_csr(n, samples, eu, ev);
    free(eu);
    free(ev);
    if (!g) return NULL;
    if (weighted && attach_weights(g, seed, wlo, whi)) return NULL;
    if (weighted) progress("weights attached", g->nnz);
    return g;
}

/* Discrete power law on [lo, hi] with exponent alpha (P(k) ~ k^-alpha),
 * drawn by inverting the continuous law on [lo, hi + 1) and flooring. */
static int64_t powerlaw_draw(xoshiro *r, double alpha, int64_t lo, int64_t hi) {
    double e = 1.0 - alpha;
    double a = pow((double)lo, e), b = pow((double)(hi + 1), e);
    double x = pow(a + (b - a) * xo_uniform(r), 1.0 / e);
    int64_t k = (int64_t)floor(x);
    return k < lo ? lo : (k > hi ? hi : k);
}

/* Fenwick tree over community capacities (sampling proportional to the
 * remaining capacity of a prefix of communities). */
static void fw_add(int64_t *t, int64_t m, int64_t i, int64_t v) {
    for (i++; i <= m; i += i & -i) t[i] += v;
}
static int64_t fw_prefix(const int64_t *t, int64_t i) {  /* sum of [0, i) */
    int64_t s = 0;
    for (; i > 0; i -= i & -i) s += t[i];
    return s;
}
static int64_t fw_find(const int64_t *t, int64_t m, int64_t x) {  /* smallest i: prefix(i+1) > x */
    int64_t pos = 0, step = 1;
    while (step * 2 <= m) step *= 2;
    for (; step > 0; step >>= 1)
        if (pos + step <= m && t[pos + step] <= x) { pos += step; x -= t[pos]; }
    return pos;
}

/* Index of the first element of cum[0..len) (non-decreasing) exceeding x. */
static int64_t upper_index(const double *cum, int64_t len, double x) {
    int64_t lo = 0, hi = len - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (cum[mid] > x) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* Degree-corrected SBM with power-law degrees and community sizes (LFR-like
 * construction, Chung-Lu edges):
 *   1. target degrees k_i ~ discrete power law (deg_alpha) on [kmin, kmax];
 *   2. community sizes ~ power law (size_alpha) on [smin, smax] until they
 *      cover n (the last one takes the rest; a rest below smin is merged
 *      into the previous community);
 *   3. vertices, highest degree first, join a community drawn with
 *      probability proportional to its free places among the communities
 *      with s - 1 >= (1 - mu) k_i (all communities if none has room);
 *   4. community c receives round(sum_i (1-mu) k_i / 2) edges whose ends
 *      are drawn inside c proportionally to (1-mu) k_i, and the graph
 *      receives round(sum_i mu k_i / 2) edges whose ends are drawn over all
 *      vertices proportionally to mu k_i, redrawn (up to 16 times) while
 *      both ends share a community.
 * Community c's edges come from the stream SplitMix64(seed, c); the mixing
 * edges are drawn in blocks of 2^16, each from its own stream, so the
 * result does not depend on the thread count.  block[v] = community of v. */
gen_graph *gen_dcsbm(int64_t n, double deg_alpha, int64_t kmin, int64_t kmax, double size_alpha, int64_t smin,
                     int64_t smax, double mu, uint64_t seed, int permute, int weighted, double wlo, double whi) {
    if (n <= 1 || kmin < 1 || kmax < kmin || smin < 2 || smax < smin || mu < 0.0 || mu > 1.0) return NULL;
    xoshiro r;
    xo_seed(&r, seed);
    int64_t *k = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *comm = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t ccap = 1024, nc = 0;
    int64_t *size = (int64_t *)malloc((size_t)ccap * sizeof(int64_t));
    if (!k || !comm || !size) { free(k); free(comm); free(size); return NULL; }
    for (int64_t i = 0; i < n; i++) k[i] = powerlaw_draw(&r, deg_alpha, kmin, kmax);
    int64_t covered = 0;
    while (covered < n) {
        int64_t sz = powerlaw_draw(&r, size_alpha, smin, smax);
        if (sz > n - covered) sz = n - covered;
        if (sz < smin && nc > 0) { size[nc - 1] += sz; covered += sz; break; }
        if (nc == ccap) {
            ccap *= 2;
            int64_t *ns = (int64_t *)realloc(size, (size_t)ccap * sizeof(int64_t));
            if (!ns) { free(k); free(comm); free(size); return NULL; }
            size = ns;
        }
        size[nc++] = sz;
        covered += sz;
    }
    /* communities by size, largest first; vertices by degree, largest first */
    int64_t *corder = (int64_t *)malloc((size_t)nc * sizeof(int64_t));
    int64_t *vorder = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *fw = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    int64_t *bucket = (int64_t *)calloc((size_t)(kmax + 2), sizeof(int64_t));
    if (!corder || !vorder || !fw || !bucket) {
        free(k); free(comm); free(size); free(corder); free(vorder); free(fw); free(bucket);
        return NULL;
    }
    for (int64_t c = 0; c < nc; c++) corder[c] = c;
    for (int64_t a = 1; a < nc; a++) {  /* insertion sort on a nearly random list: few thousand items */
        int64_t x = corder[a], b = a - 1;
        while (b >= 0 && size[corder[b]] < size[x]) { corder[b + 1] = corder[b]; b--; }
        corder[b + 1] = x;
    }
    for (int64_t i = 0; i < n; i++) bucket[kmax - k[i] + 1]++;
    for (int64_t d = 0; d <= kmax; d++) bucket[d + 1] += bucket[d];
    for (int64_t i = 0; i < n; i++) vorder[bucket[kmax - k[i]]++] = i;
    free(bucket);
    for (int64_t c = 0; c < nc; c++) fw_add(fw, nc, c, size[corder[c]]);
    int64_t eligible = 0;  /* grows as degrees fall: prefix of corder with room for the vertex */
    for (int64_t t = 0; t < n; t++) {
        int64_t i = vorder[t];
        double need = (1.0 - mu) * (double)k[i];
        while (eligible < nc && (double)(size[corder[eligible]] - 1) >= need) eligible++;
        int64_t pref = eligible > 0 ? eligible : nc;
        int64_t room = fw_prefix(fw, pref);
        if (room == 0) { pref = nc; room = fw_prefix(fw, nc); }
        int64_t x = (int64_t)(xo_uniform(&r) * (double)room);
        if (x >= room) x = room - 1;
        int64_t pos = fw_find(fw, nc, x);
        fw_add(fw, nc, pos, -1);
        comm[i] = corder[pos];
    }
    free(fw);
    free(vorder);
    free(corder);
    /* members of each community */
    int64_t *moff = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    int64_t *mem = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *eoff = (int64_t *)calloc((size_t)nc + 2, sizeof(int64_t));
    double *cum = (double *)malloc((size_t)n * sizeof(double));
    if (!moff || !mem || !eoff || !cum) {
        free(k); free(comm); free(size); free(moff); free(mem); free(eoff); free(cum);
        return NULL;
    }
    for (int64_t i = 0; i < n; i++) moff[comm[i] + 1]++;
    for (int64_t c = 0; c < nc; c++) moff[c + 1] += moff[c];
    {
        int64_t *cur = (int64_t *)malloc((size_t)nc * sizeof(int64_t));
        if (!cur) { free(k); free(comm); free(size); free(moff); free(mem); free(eoff); free(cum); return NULL; }
        memcpy(cur, moff, (size_t)nc * sizeof(int64_t));
        for (int64_t i = 0; i < n; i++) mem[cur[comm[i]]++] = i;
        free(cur);
    }
    double tot_out = 0.0;
    for (int64_t c = 0; c < nc; c++) {
        double s_in = 0.0;
        for (int64_t t = moff[c]; t < moff[c + 1]; t++) {
            s_in += (1.0 - mu) * (double)k[mem[t]];
            cum[t] = s_in;
        }
        eoff[c + 1] = eoff[c] + (moff[c + 1] - moff[c] > 1 ? (int64_t)llround(s_in / 2.0) : 0);
    }
    double *ocum = (double *)malloc((size_t)n * sizeof(double));
    if (!ocum) { free(k); free(comm); free(size); free(moff); free(mem); free(eoff); free(cum); return NULL; }
    for (int64_t i = 0; i < n; i++) {
        tot_out += mu * (double)k[i];
        ocum[i] = tot_out;
    }
    int64_t e_in = eoff[nc], e_out = tot_out > 0.0 ? (int64_t)llround(tot_out / 2.0) : 0;
    int64_t m = e_in + e_out;
    int32_t *eu = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int32_t *ev = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    if (!eu || !ev) {
        free(k); free(comm); free(size); free(moff); free(mem); free(eoff); free(cum); free(ocum); free(eu); free(ev);
        return NULL;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < nc; c++) {
        int64_t len = moff[c + 1] - moff[c];
        if (len < 2) continue;
        xoshiro rc;
        xo_seed(&rc, splitmix64_hash(seed * 0x9e3779b97f4a7c15ULL + 0x632be59bd9b4e019ULL + (uint64_t)c));
        const double *cc = cum + moff[c];
        double tot = cc[len - 1];
        for (int64_t e = eoff[c]; e < eoff[c + 1]; e++) {
            int64_t a = upper_index(cc, len, xo_uniform(&rc) * tot);
            int64_t b = upper_index(cc, len, xo_uniform(&rc) * tot);
            eu[e] = (int32_t)mem[moff[c] + a];
            ev[e] = (int32_t)mem[moff[c] + b];
        }
    }
    const int64_t BLK = (int64_t)1 << 16;
    int64_t nblk = (e_out + BLK - 1) / BLK;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t blk = 0; blk < nblk; blk++) {
        xoshiro rb;
        xo_seed(&rb, splitmix64_hash(seed * 0x9e3779b97f4a7c15ULL + 0x2545f4914f6cdd1dULL + (uint64_t)blk));
        int64_t e0 = blk * BLK, e1 = e0 + BLK < e_out ? e0 + BLK : e_out;
        for (int64_t e = e0; e < e1; e++) {
            int64_t a = 0, b = 0;
            for (int tries = 0; tries < 16; tries++) {
                a = upper_index(ocum, n, xo_uniform(&rb) * tot_out);
                b = upper_index(ocum, n, xo_uniform(&rb) * tot_out);
                if (comm[a] != comm[b]) break;
            }
            eu[e_in + e] = (int32_t)a;
            ev[e_in + e] = (int32_t)b;
        }
    }
    free(cum);
    free(ocum);
    free(mem);
    free(moff);
    free(eoff);
    free(size);
    free(k);
    int32_t *perm = NULL;
    if (permute) {
        perm = random_perm(n, seed);
        if (!perm) { free(eu); free(ev); free(comm); return NULL; }
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < m; e++) { eu[e] = perm[eu[e]]; ev[e] = perm[ev[e]]; }
    }
    gen_graph *g = build_csr(n, m, eu, ev);
    free(eu);
    free(ev);
    if (!g) { free(perm); free(comm); return NULL; }
    g->block = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (g->block)
        for (int64_t v = 0; v < n; v++) g->block[perm ? perm[v] : v] = comm[v];
    free(perm);
    free(comm);
    if (weighted && attach_weights(g, seed, wlo, whi)) return NULL;
    if (weighted) progress("weights attached", g->nnz);
    return g;
}

/* Road-like graph (the low-degree, high-diameter class of road networks
 * and k-mer graphs): a side x side lattice of intersections; each of its
 * 2 side (side - 1) lattice edges is kept with probability `keep` and, when
 * kept, subdivided into a chain with a uniform number of inner vertices in
 * [0, max_inner] (degree-2 vertices, like the road segments between
 * junctions).  Vertex ids: intersections first, then the chains' inner
 * vertices in edge order, then (permute) a random relabelling.  The
 * average degree is 2 E / n, close to 2 when chains are long.  Lattice
 * edges are visited in a fixed order from one xoshiro stream, so the graph
 * depends on the seed only. */
gen_graph *gen_road(int64_t side, double keep, int max_inner, uint64_t seed, int permute) {
    if (side < 2 || max_inner < 0 || !(keep >= 0.0 && keep <= 1.0)) return NULL;
    int64_t ni = side * side;
    xoshiro r;
    xo_seed(&r, seed);
    edge_list el = {0, 0, NULL, NULL};
    int64_t next = ni;
    for (int64_t y = 0; y < side; y++)
        for (int64_t x = 0; x < side; x++)
            for (int dir = 0; dir < 2; dir++) {
                int64_t x2 = x + (dir == 0), y2 = y + (dir == 1);
                if (x2 >= side || y2 >= side) continue;
                double u = xo_uniform(&r);
                int inner = (int)(xo_uniform(&r) * (double)(max_inner + 1));
                if (inner > max_inner) inner = max_inner;
                if (u >= keep) continue;
                if (next + inner > 0x7ffffffe) { el_free(&el); return NULL; }
                int64_t prev = y * side + x;
                for (int k = 0; k < inner; k++) {
                    if (el_push(&el, (int32_t)prev, (int32_t)next)) { el_free(&el); return NULL; }
                    prev = next++;
                }
                if (el_push(&el, (int32_t)prev, (int32_t)(y2 * side + x2))) { el_free(&el); return NULL; }
            }
    int64_t n = next;
    progress("road: chains drawn", el.len);
    if (permute) {
        int32_t *perm = random_perm(n, seed);
        if (!perm) { el_free(&el); return NULL; }
        for (int64_t e = 0; e < el.len; e++) { el.u[e] = perm[el.u[e]]; el.v[e] = perm[el.v[e]]; }
        free(perm);
    }
    gen_graph *g = build_csr(n, el.len, el.u, el.v);
    el_free(&el);
    return g;
}

/* Graph from a caller's undirected edge list (used by hand-built test
 * graphs): symmetrised, deduplicated, self-loops dropped. */
gen_graph *gen_from_edges(int64_t n, int64_t m, const int32_t *eu, const int32_t *ev) {
    if (n <= 0 || m < 0) return NULL;
    for (int64_t e = 0; e < m; e++)
        if (eu[e] < 0 || eu[e] >= n || ev[e] < 0 || ev[e] >= n) return NULL;
    return build_csr(n, m, eu, ev);
}

void gen_free(gen_graph *g) {
    if (!g) return;
    free(g->off);
    free(g->col);
    free(g->w);
    free(g->block);
    free(g);
}

int64_t gen_n(const gen_graph *g) { return g->n; }
int64_t gen_nnz(const gen_graph *g) { return g->nnz; }
int gen_has_weights(const gen_graph *g) { return g->w != NULL; }
int gen_has_blocks(const gen_graph *g) { return g->block != NULL; }

/* Copies the graph into caller buffers (off: n+1, col: nnz, w: nnz or NULL,
 * block: n or NULL). */
void gen_copy(const gen_graph *g, int64_t *off, int32_t *col, float *w, int64_t *block) {
    memcpy(off, g->off, ((size_t)g->n + 1) * sizeof(int64_t));
    if (g->nnz) memcpy(col, g->col, (size_t)g->nnz * sizeof(int32_t));
    if (w && g->w && g->nnz) memcpy(w, g->w, (size_t)g->nnz * sizeof(float));
    if (block && g->block) memcpy(block, g->block, (size_t)g->n * sizeof(int64_t));
}

/* Deterministic uniform draws for callers that need seeded random inputs
 * (e.g. random memberships for parity tests): out[i] in [0, 1). */
void gen_uniform(uint64_t seed, int64_t count, double *out) {
    xoshiro r;
    xo_seed(&r, seed);
    for (int64_t i = 0; i < count; i++) out[i] = xo_uniform(&r);
}
