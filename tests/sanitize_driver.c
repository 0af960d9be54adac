/* Host-side sanitizer driver: the seeded generators and the oracle built
 * with AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitize.py
 * compiles this file with oracle/oracle.c, oracle/prune.c and
 * gsp_inputs/gen.c and runs it).  Every generator family and every oracle
 * entry point runs once on a small graph; a memory error or undefined
 * behaviour ends the program with a non-zero status.  Prints one summary
 * line per graph. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/oracle.h"

typedef struct gen_graph gen_graph;
gen_graph *gen_sbm(int64_t n, int64_t blocks, double p_in, double p_out, uint64_t seed, int permute, int weighted,
                   double wlo, double whi);
gen_graph *gen_rmat(int scale, int64_t samples, double a, double b, double c, uint64_t seed, int permute,
                    int weighted, double wlo, double whi);
gen_graph *gen_dcsbm(int64_t n, double deg_alpha, int64_t kmin, int64_t kmax, double size_alpha, int64_t smin,
                     int64_t smax, double mu, uint64_t seed, int permute, int weighted, double wlo, double whi);
gen_graph *gen_road(int64_t side, double keep, int max_inner, uint64_t seed, int permute);
void gen_free(gen_graph *g);
int64_t gen_n(const gen_graph *g);
int64_t gen_nnz(const gen_graph *g);
int gen_has_weights(const gen_graph *g);
void gen_copy(const gen_graph *g, int64_t *off, int32_t *col, float *w, int64_t *block);
void gen_uniform(uint64_t seed, int64_t count, double *out);

static void *xmalloc(size_t bytes) {
    void *p = malloc(bytes ? bytes : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(3);
    }
    return p;
}

static int fail(const char *what) {
    fprintf(stderr, "check failed: %s\n", what);
    return 1;
}

/* Runs the oracle's steps and whole runs on one graph. */
static int exercise(const char *name, gen_graph *gg, uint64_t seed) {
    if (!gg) return fail("generator returned NULL");
    int64_t n = gen_n(gg), nnz = gen_nnz(gg);
    int64_t *off = xmalloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *col = xmalloc(sizeof(int32_t) * (size_t)nnz);
    float *wf = xmalloc(sizeof(float) * (size_t)nnz);
    double *w = xmalloc(sizeof(double) * (size_t)nnz);
    gen_copy(gg, off, col, gen_has_weights(gg) ? wf : NULL, NULL);
    for (int64_t e = 0; e < nnz; e++) w[e] = gen_has_weights(gg) ? (double)wf[e] : 1.0;
    gen_free(gg);
    int64_t moved = 0;
    if (orc_weight_grid(nnz, w, &moved) < -1000) return fail("weight grid");

    double *K = xmalloc(sizeof(double) * (size_t)n);
    double M2 = orc_vertex_weights(n, off, col, w, K);
    int32_t *memb = xmalloc(sizeof(int32_t) * (size_t)n);
    int32_t *lab = xmalloc(sizeof(int32_t) * (size_t)n);
    int32_t *lab2 = xmalloc(sizeof(int32_t) * (size_t)n);
    int32_t *ren = xmalloc(sizeof(int32_t) * (size_t)n);

    /* one synchronous phase, split both ways, renumber, aggregate */
    for (int64_t i = 0; i < n; i++) memb[i] = (int32_t)i;
    double dq[64];
    int64_t mv[64];
    int32_t li = orc_move_sync(n, off, col, w, M2, K, memb, 1e-2, 20, 8, dq, mv, 0);
    if (orc_split_bfs(n, off, col, memb, lab) < 0) return fail("split bfs");
    if (orc_split_lp(n, off, col, memb, 1, lab2) < 0) return fail("split lpp");
    if (memcmp(lab, lab2, sizeof(int32_t) * (size_t)n) != 0) return fail("split bfs == split lpp");
    int64_t G = orc_renumber(n, lab, ren);
    int64_t *off2 = xmalloc(sizeof(int64_t) * (size_t)(G + 1));
    int32_t *col2 = xmalloc(sizeof(int32_t) * (size_t)nnz);
    double *w2 = xmalloc(sizeof(double) * (size_t)nnz);
    int64_t nnz2 = orc_aggregate(n, off, col, w, ren, G, off2, col2, w2, nnz);
    if (nnz2 < 0) return fail("aggregate capacity");
    double tot = 0.0;
    for (int64_t e = 0; e < nnz2; e++) tot += w2[e];
    if (fabs(tot - M2) > 1e-9 * M2) return fail("aggregation keeps the total weight");
    if (orc_disconnected(n, off, col, ren, NULL) != 0) return fail("split result connected");
    double q1 = orc_modularity(n, off, col, w, ren);

    /* one asynchronous phase from singletons */
    double *sigma = xmalloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; i++) memb[i] = (int32_t)i, sigma[i] = K[i];
    orc_move_async(n, off, col, w, M2, K, memb, sigma, 1e-2, 20, dq);

    /* gated phase with a seeded network and traces */
    float *params = xmalloc(sizeof(float) * ORC_MLP_PARAMS);
    double *u = xmalloc(sizeof(double) * ORC_MLP_PARAMS);
    gen_uniform(seed, ORC_MLP_PARAMS, u);
    for (int k = 0; k < ORC_MLP_PARAMS; k++) params[k] = (float)(u[k] - 0.5);
    orc_trace tr;
    memset(&tr, 0, sizeof tr);
    tr.seed = seed;
    tr.threshold = UINT64_MAX / 2;
    tr.cap = 4096;
    tr.x = xmalloc(sizeof(float) * 8 * (size_t)tr.cap);
    tr.y = xmalloc((size_t)tr.cap);
    tr.vertex = xmalloc(sizeof(int32_t) * (size_t)tr.cap);
    tr.meta = xmalloc(sizeof(int32_t) * (size_t)tr.cap);
    for (int64_t i = 0; i < n; i++) memb[i] = (int32_t)i;
    int64_t cnt[4];
    orc_move_sync_gated(n, off, col, w, M2, K, memb, 1e-2, 20, 8, params, 0.0, 1, &tr, dq, mv, cnt, 0, 1);

    /* training: gradient and a few Adam epochs on the traces */
    int64_t rows = tr.rows < tr.cap ? tr.rows : tr.cap;
    double *grad = xmalloc(sizeof(double) * ORC_MLP_PARAMS);
    double loss = rows ? orc_mlp_loss_grad(params, tr.x, tr.y, rows, 2.0, grad) : 0.0;
    double el[3];
    if (rows) orc_mlp_train_adam(params, tr.x, tr.y, rows, 64, 3, 1e-3, 2.0, el);
    double *logits = xmalloc(sizeof(double) * (size_t)(rows ? rows : 1));
    if (rows) orc_mlp_logits(params, tr.x, rows, 1, logits);

    /* whole runs: SP, SL, none; synchronous and asynchronous; learned */
    orc_options opt;
    memset(&opt, 0, sizeof opt);
    opt.tolerance = 1e-2;
    opt.max_passes = 10;
    opt.max_iterations = 20;
    opt.tolerance_drop = 10.0;
    opt.aggregation_tolerance = 0.8;
    opt.sync_moves = 1;
    opt.sync_rounds = 8;
    orc_stats st;
    double qs[6];
    int k = 0;
    for (int mode = 0; mode < 3; mode++) {
        opt.split_mode = mode;
        orc_louvain(n, off, col, w, &opt, memb, &st);
        qs[k++] = st.modularity;
        if (mode != 2 && orc_disconnected(n, off, col, memb, NULL) != 0) return fail("louvain result connected");
    }
    opt.split_mode = 0;
    opt.sync_moves = 0;
    orc_louvain(n, off, col, w, &opt, memb, &st);
    qs[k++] = st.modularity;
    opt.sync_moves = 1;
    opt.prune_params = params;
    opt.prune_theta_logit = 0.0;
    orc_louvain(n, off, col, w, &opt, memb, &st);
    qs[k++] = st.modularity;
    opt.confirm_final = 1;
    orc_louvain(n, off, col, w, &opt, memb, &st);
    qs[k++] = st.modularity;
    printf("%s: n=%lld nnz=%lld grid moved %lld, l=%d, first-pass Q %.6f, loss %.4f, Q", name, (long long)n,
           (long long)nnz, (long long)moved, li, q1, loss);
    for (int j = 0; j < k; j++) printf(" %.6f", qs[j]);
    printf("\n");

    free(off), free(col), free(wf), free(w), free(K), free(memb), free(lab), free(lab2), free(ren);
    free(off2), free(col2), free(w2), free(params), free(u), free(tr.x), free(tr.y), free(tr.vertex), free(tr.meta);
    free(grad), free(logits), free(sigma);
    return 0;
}

int main(void) {
    int bad = 0;
    bad |= exercise("sbm", gen_sbm(3000, 30, 0.02, 0.0008, 1, 1, 1, 1.0, 4.0), 11);
    bad |= exercise("rmat", gen_rmat(12, 16 << 12, 0.57, 0.19, 0.19, 12, 1, 1, 1.0, 10.0), 12);
    bad |= exercise("dcsbm", gen_dcsbm(6000, 2.5, 5, 300, 1.5, 20, 1000, 0.3, 13, 1, 1, 1.0, 4.0), 13);
    bad |= exercise("road", gen_road(50, 0.7, 8, 14, 1), 14);
    return bad;
}
