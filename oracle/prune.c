/*
 * prune.c - TEST INFRASTRUCTURE ONLY.
 *
 * Oracle of the learned vertex-pruning gate that runs beside GSP-Louvain's
 * local-moving phase: per-vertex features, the 8 -> 64 -> 64 -> 1 network
 * (ReLU hidden layers, sigmoid output), its pos-weighted binary
 * cross-entropy, gradients and Adam, and the synchronous local-moving phase
 * with the gate in front of the scan and a confirming plain sweep before a
 * pass may end.  The gate is not part of the paper; it prunes the vertices
 * that Algorithm "louvainMove" would scan (the unprocessed vertices of an
 * iteration, Section 4.1's pruning), and the plain sweep keeps the paper's
 * convergence test (per-iteration delta-modularity against tau) as the final word.
 *
 * Plain loops, fp64 unless stated.  Only the tests, the smoke check and the
 * bench's CPU leg use it; it shares no code with the GPU library.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* ------------------------------------------------------------------ */
/* Number formats                                                       */
/* ------------------------------------------------------------------ */

/* bfloat16 of an fp32 value (the upper 16 bits of the fp32 pattern after
 * rounding to nearest, ties to even), returned as the fp32 value it
 * represents.  NaN stays NaN. */
float orc_bf16(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
        u |= 0x00400000u;
        u &= 0xffff0000u;
    } else {
        uint32_t lsb = (u >> 16) & 1u;
        u += 0x7fffu + lsb;
        u &= 0xffff0000u;
    }
    float y;
    memcpy(&y, &u, 4);
    return y;
}

/* Piecewise-linear base-2 logarithm for x >= 1: e + (x / 2^e - 1) with
 * 2^e <= x < 2^(e+1).  Exact at powers of two, linear between them, and
 * computed with exact operations only (a scaling by a power of two). */
double orc_plog2(double x) {
    if (!(x >= 1.0)) return 0.0;
    int e = 0;
    double p = 1.0;
    while (p * 2.0 <= x) { p *= 2.0; e++; }
    return (double)e + (x / p - 1.0);
}

/* ------------------------------------------------------------------ */
/* Gate features                                                        */
/* ------------------------------------------------------------------ */

static float feat(double v) { return orc_bf16((float)v); }

/* The 8 features of an unprocessed vertex i, from state the GPU holds per
 * vertex (no scan of i's row):
 *   x0 = plog2(1 + deg_i) / 16       row length at this level
 *   x1 = hfrac_i                     K_{i->d} / K_i at i's last scan this pass
 *   x2 = hgain_i                     normalised best gain at that scan
 *   x3 = min(pass, 8) / 8            pass index
 *   x4 = min(l, 20) / 20             counted iterations so far in the pass
 *   x5 = K_i / Sigma_d               i's share of its community's weight
 *   x6 = 0 never scanned in this pass, 1/2 stayed at its last scan, 1 moved
 *   x7 = min(D_i / K_i, 1)           D_i = weight of the entries (i, j) whose
 *                                    j moved since i's last scan (or since
 *                                    the pass began; pruning keeps it)
 * Each value is computed in fp64, then rounded to fp32 and to bf16. */
void orc_gate_features(int64_t deg, double ki, double sig_d, float hfrac, float hgain, uint8_t hbits, double dmoved,
                       int32_t pass, int32_t iter, float *x) {
    x[0] = feat(orc_plog2(1.0 + (double)deg) / 16.0);
    x[1] = feat((double)hfrac);
    x[2] = feat((double)hgain);
    x[3] = feat((double)(pass < 8 ? pass : 8) / 8.0);
    x[4] = feat((double)(iter < 20 ? iter : 20) / 20.0);
    x[5] = feat(ki > 0.0 && sig_d > 0.0 ? ki / sig_d : 0.0);
    x[6] = feat((hbits & 1u) ? ((hbits & 2u) ? 1.0 : 0.5) : 0.0);
    double r = ki > 0.0 ? dmoved / ki : 0.0;
    x[7] = feat(r < 1.0 ? r : 1.0);
}

/* History written at a scan: K_{i->d} / K_i and the normalised gain
 * (G(best) - G(stay)) / (M2 K_i) clipped to [-1, 1] (-1 with no candidate
 * community, 0 for K_i = 0), each rounded to fp32. */
static void gate_history(double ki, double kid, double M2, int has_best, double g_best, double g_stay, float *hfrac,
                         float *hgain) {
    if (ki > 0.0) {
        *hfrac = (float)(kid / ki);
        double r = has_best ? (g_best - g_stay) / (M2 * ki) : -1.0;
        if (r > 1.0) r = 1.0;
        if (r < -1.0) r = -1.0;
        *hgain = (float)r;
    } else {
        *hfrac = 0.0f;
        *hgain = 0.0f;
    }
}

/* ------------------------------------------------------------------ */
/* The network                                                          */
/* ------------------------------------------------------------------ */

#define NF 8
#define NH 64
#define P_W1 0
#define P_B1 (P_W1 + NH * NF)
#define P_W2 (P_B1 + NH)
#define P_B2 (P_W2 + NH * NH)
#define P_W3 (P_B2 + NH)
#define P_B3 (P_W3 + NH)

/* Forward pass of one row.  Parameters (ORC_MLP_PARAMS fp32 values): W1
 * [64][8] row-major, b1[64], W2 [64][64] (row = output unit), b2[64],
 * w3[64], b3.  z = w3 . relu(W2 relu(W1 x + b1) + b2) + b3.  With bf16 = 1
 * the weight matrices and the first hidden layer's outputs are rounded to
 * bf16 first (the inference kernel's formats); biases stay fp32.  Sums in
 * fp64.  a1, a2 (pre-activations) may be NULL. */
static double mlp_row(const double *p, const float *x, int bf16, double *a1, double *a2) {
    double h1[NH], h2[NH], t1[NH], t2[NH];
    double *A1 = a1 ? a1 : t1, *A2 = a2 ? a2 : t2;
    for (int h = 0; h < NH; h++) {
        double s = 0.0;
        for (int f = 0; f < NF; f++) {
            double wv = bf16 ? orc_bf16((float)p[P_W1 + h * NF + f]) : p[P_W1 + h * NF + f];
            s += wv * (double)x[f];
        }
        A1[h] = s + p[P_B1 + h];
        double r = A1[h] > 0.0 ? A1[h] : 0.0;
        h1[h] = bf16 ? (double)orc_bf16((float)r) : r;
    }
    for (int o = 0; o < NH; o++) {
        double s = 0.0;
        for (int h = 0; h < NH; h++) {
            double wv = bf16 ? orc_bf16((float)p[P_W2 + o * NH + h]) : p[P_W2 + o * NH + h];
            s += wv * h1[h];
        }
        A2[o] = s + p[P_B2 + o];
        h2[o] = A2[o] > 0.0 ? A2[o] : 0.0;
    }
    double z = 0.0;
    for (int o = 0; o < NH; o++) {
        double wv = bf16 ? orc_bf16((float)p[P_W3 + o]) : p[P_W3 + o];
        z += wv * h2[o];
    }
    return z + p[P_B3];
}

static void widen(const float *pf, double *pd) {
    for (int k = 0; k < ORC_MLP_PARAMS; k++) pd[k] = (double)pf[k];
}

void orc_mlp_logits(const float *params, const float *x, int64_t rows, int32_t bf16, double *out) {
    double pd[ORC_MLP_PARAMS];
    widen(params, pd);
    for (int64_t r = 0; r < rows; r++) out[r] = mlp_row(pd, x + r * NF, bf16, NULL, NULL);
}

/* log(1 + e^t) without overflow */
static double softplus(double t) { return (t > 0.0 ? t : 0.0) + log1p(exp(-fabs(t))); }
static double sigmoid(double t) { return t >= 0.0 ? 1.0 / (1.0 + exp(-t)) : exp(t) / (1.0 + exp(t)); }

/* Mean pos-weighted binary cross-entropy of the rows and its gradient with
 * respect to every parameter (fp64 forward, fp32 parameters read as given):
 *   L = (1/B) sum_r [ pw y_r softplus(-z_r) + (1 - y_r) softplus(z_r) ],
 * dL/dz_r = (sigmoid(z_r) (pw y_r + 1 - y_r) - pw y_r) / B, then the chain
 * rule through the layers (ReLU derivative [a > 0]).  grad may be NULL. */
double orc_mlp_loss_grad_f64(const double *params, const float *x, const uint8_t *y, int64_t rows,
                             double pos_weight, double *grad) {
    if (rows <= 0) return 0.0;
    if (grad) memset(grad, 0, ORC_MLP_PARAMS * sizeof(double));
    double loss = 0.0;
    for (int64_t r = 0; r < rows; r++) {
        const float *xr = x + r * NF;
        double a1[NH], a2[NH], h1[NH], h2[NH];
        double z = mlp_row(params, xr, 0, a1, a2);
        for (int h = 0; h < NH; h++) h1[h] = a1[h] > 0.0 ? a1[h] : 0.0;
        for (int h = 0; h < NH; h++) h2[h] = a2[h] > 0.0 ? a2[h] : 0.0;
        double yr = y[r] ? 1.0 : 0.0;
        loss += pos_weight * yr * softplus(-z) + (1.0 - yr) * softplus(z);
        if (!grad) continue;
        double dz = (sigmoid(z) * (pos_weight * yr + 1.0 - yr) - pos_weight * yr) / (double)rows;
        double dh2[NH], dh1[NH];
        grad[P_B3] += dz;
        for (int o = 0; o < NH; o++) {
            grad[P_W3 + o] += dz * h2[o];
            dh2[o] = a2[o] > 0.0 ? dz * params[P_W3 + o] : 0.0;
        }
        for (int o = 0; o < NH; o++) {
            grad[P_B2 + o] += dh2[o];
            for (int h = 0; h < NH; h++) grad[P_W2 + o * NH + h] += dh2[o] * h1[h];
        }
        for (int h = 0; h < NH; h++) {
            double s = 0.0;
            for (int o = 0; o < NH; o++) s += params[P_W2 + o * NH + h] * dh2[o];
            dh1[h] = a1[h] > 0.0 ? s : 0.0;
        }
        for (int h = 0; h < NH; h++) {
            grad[P_B1 + h] += dh1[h];
            for (int f = 0; f < NF; f++) grad[P_W1 + h * NF + f] += dh1[h] * (double)xr[f];
        }
    }
    return loss / (double)rows;
}

double orc_mlp_loss_grad(const float *params, const float *x, const uint8_t *y, int64_t rows, double pos_weight,
                         double *grad) {
    double pd[ORC_MLP_PARAMS];
    widen(params, pd);
    return orc_mlp_loss_grad_f64(pd, x, y, rows, pos_weight, grad);
}

/* Same in fp32 arithmetic throughout (loops in the same order). */
float orc_mlp_loss_grad_f32(const float *p, const float *x, const uint8_t *y, int64_t rows, float pos_weight,
                            float *grad) {
    if (rows <= 0) return 0.0f;
    if (grad) memset(grad, 0, ORC_MLP_PARAMS * sizeof(float));
    float loss = 0.0f;
    for (int64_t r = 0; r < rows; r++) {
        const float *xr = x + r * NF;
        float a1[NH], a2[NH], h1[NH], h2[NH], dh1[NH], dh2[NH];
        for (int h = 0; h < NH; h++) {
            float s = 0.0f;
            for (int f = 0; f < NF; f++) s += p[P_W1 + h * NF + f] * xr[f];
            a1[h] = s + p[P_B1 + h];
            h1[h] = a1[h] > 0.0f ? a1[h] : 0.0f;
        }
        for (int o = 0; o < NH; o++) {
            float s = 0.0f;
            for (int h = 0; h < NH; h++) s += p[P_W2 + o * NH + h] * h1[h];
            a2[o] = s + p[P_B2 + o];
            h2[o] = a2[o] > 0.0f ? a2[o] : 0.0f;
        }
        float z = 0.0f;
        for (int o = 0; o < NH; o++) z += p[P_W3 + o] * h2[o];
        z += p[P_B3];
        float yr = y[r] ? 1.0f : 0.0f;
        float spn = (z < 0.0f ? -z : 0.0f) + log1pf(expf(-fabsf(z)));   /* softplus(-z) */
        float spp = (z > 0.0f ? z : 0.0f) + log1pf(expf(-fabsf(z)));    /* softplus(z) */
        loss += pos_weight * yr * spn + (1.0f - yr) * spp;
        if (!grad) continue;
        float sg = z >= 0.0f ? 1.0f / (1.0f + expf(-z)) : expf(z) / (1.0f + expf(z));
        float dz = (sg * (pos_weight * yr + 1.0f - yr) - pos_weight * yr) / (float)rows;
        grad[P_B3] += dz;
        for (int o = 0; o < NH; o++) {
            grad[P_W3 + o] += dz * h2[o];
            dh2[o] = a2[o] > 0.0f ? dz * p[P_W3 + o] : 0.0f;
        }
        for (int o = 0; o < NH; o++) {
            grad[P_B2 + o] += dh2[o];
            for (int h = 0; h < NH; h++) grad[P_W2 + o * NH + h] += dh2[o] * h1[h];
        }
        for (int h = 0; h < NH; h++) {
            float s = 0.0f;
            for (int o = 0; o < NH; o++) s += p[P_W2 + o * NH + h] * dh2[o];
            dh1[h] = a1[h] > 0.0f ? s : 0.0f;
        }
        for (int h = 0; h < NH; h++) {
            grad[P_B1 + h] += dh1[h];
            for (int f = 0; f < NF; f++) grad[P_W1 + h * NF + f] += dh1[h] * xr[f];
        }
    }
    return loss / (float)rows;
}

/* Adam (Kingma and Ba, ICLR 2015) on mini-batches [b*batch, (b+1)*batch)
 * of the rows in the order given, `epochs` passes; beta1 = 0.9, beta2 =
 * 0.999, eps = 1e-8, bias-corrected moments, step t counted over all
 * batches.  Parameters, moments and arithmetic in fp64; params is updated
 * in place (rounded to fp32 at the end).  epoch_loss[e] (may be NULL)
 * receives the mean of the batch losses of epoch e, each taken before its
 * update.  Returns the number of steps. */
int64_t orc_mlp_train_adam(float *params, const float *x, const uint8_t *y, int64_t rows, int64_t batch,
                           int32_t epochs, double lr, double pos_weight, double *epoch_loss) {
    if (rows <= 0 || batch <= 0 || epochs < 0) return -1;
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    double *p = (double *)malloc(ORC_MLP_PARAMS * sizeof(double));
    double *m = (double *)calloc(ORC_MLP_PARAMS, sizeof(double));
    double *v = (double *)calloc(ORC_MLP_PARAMS, sizeof(double));
    double *g = (double *)malloc(ORC_MLP_PARAMS * sizeof(double));
    float *pf = (float *)malloc(ORC_MLP_PARAMS * sizeof(float));
    if (!p || !m || !v || !g || !pf) { free(p); free(m); free(v); free(g); free(pf); return -1; }
    for (int k = 0; k < ORC_MLP_PARAMS; k++) p[k] = params[k];
    int64_t t = 0;
    for (int32_t e = 0; e < epochs; e++) {
        double lsum = 0.0;
        int64_t nb = 0;
        for (int64_t r0 = 0; r0 < rows; r0 += batch) {
            int64_t len = r0 + batch <= rows ? batch : rows - r0;
            /* gradient at the parameters rounded to fp32, the network's storage format */
            for (int k = 0; k < ORC_MLP_PARAMS; k++) pf[k] = (float)p[k];
            double lb = orc_mlp_loss_grad(pf, x + r0 * NF, y + r0, len, pos_weight, g);
            t++;
            double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
            for (int k = 0; k < ORC_MLP_PARAMS; k++) {
                m[k] = b1 * m[k] + (1.0 - b1) * g[k];
                v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
                double mh = m[k] / c1, vh = v[k] / c2;
                p[k] -= lr * mh / (sqrt(vh) + eps);
            }
            lsum += lb;
            nb++;
        }
        if (epoch_loss) epoch_loss[e] = nb ? lsum / (double)nb : 0.0;
    }
    for (int k = 0; k < ORC_MLP_PARAMS; k++) params[k] = (float)p[k];
    free(p); free(m); free(v); free(g); free(pf);
    return t;
}

/* ------------------------------------------------------------------ */
/* Trace sampling                                                       */
/* ------------------------------------------------------------------ */

/* SplitMix64's output function (Steele, Lea and Flood, 2014) applied to
 * one 64-bit word. */
static uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* A scan of vertex i in sweep `sweep` of pass `pass` is recorded iff
 * mix64(seed ^ (pass << 56) ^ (sweep << 48) ^ i) < threshold. */
int32_t orc_trace_keep(uint64_t seed, int32_t pass, int32_t sweep, int64_t i, uint64_t threshold) {
    uint64_t key = seed ^ ((uint64_t)(uint32_t)pass << 56) ^ ((uint64_t)(uint32_t)sweep << 48) ^ (uint64_t)i;
    return mix64(key) < threshold;
}

/* ------------------------------------------------------------------ */
/* Gated synchronous local-moving phase                                 */
/* ------------------------------------------------------------------ */

static int32_t sub_round(int64_t i, int32_t rounds) {
    if (rounds <= 1) return 0;
    int sh = 0;
    while ((1 << sh) < rounds) sh++;
    return (int32_t)(((uint64_t)i * 0x9E3779B97F4A7C15ULL) >> (64 - sh));
}

static void trace_put(orc_trace *t, const float *x, uint8_t label, int64_t i, int32_t pass, int32_t sweep) {
    if (t->rows < t->cap) {
        memcpy(t->x + t->rows * NF, x, NF * sizeof(float));
        t->y[t->rows] = label;
        t->vertex[t->rows] = (int32_t)i;
        t->meta[t->rows] = pass * 256 + sweep;
        t->rows++;
    }
    t->seen++;
}

/* The synchronous phase of orc_move_sync with two additions.
 *
 * Gate (params != NULL).  The phase starts in "gated" mode: in each
 * sub-round every unprocessed vertex of the group is marked processed as
 * usual, its features (orc_gate_features, from the history of this pass
 * and the sub-round's snapshot) go through the network in the inference
 * formats (bf16 weights and first-layer outputs), and it is scanned only if
 * logit >= theta_logit; pruned vertices keep their community.  When a gated
 * iteration's delta-modularity is <= tau, one "confirming" sweep follows:
 * every vertex unprocessed, no gate.  If its delta-modularity is <= tau the
 * phase ends, otherwise it continues with plain iterations (no gate) until
 * the usual test stops it.  Every iteration counts towards l_i and
 * max_iter except a confirming sweep that moves no vertex.  The last
 * iteration the phase may count (l_i = max_iter - 1) is always a
 * confirming sweep, so a phase that reaches max_iter in gated mode still
 * ends with one sweep of the plain method over every vertex.  An
 * iteration's gain total is the exact sum of the movers' gains in fixed
 * point (orc_gain_fixed).
 *
 * A vertex with an empty row is never gated, scanned or traced (it cannot
 * move).
 *
 * History (both modes, used by the features): at a vertex's scan, bit 0 of
 * hbits (scanned), bit 1 (moved), hfrac and hgain (gate_history) are set
 * and D_i is cleared (D_i is read into the features when i is taken from
 * the unprocessed set, before the gate); when a sub-round's moves are
 * applied every entry (i, j), j != i, of a mover i adds w_ij to D_j.  All
 * start at 0 in the phase.
 *
 * Return moves (returns != 0, as in orc_move_sync, by sweep index): a move
 * of i back into the community it left at its move in the preceding sweep
 * is made, but its gain is not added to the sweep's total.
 *
 * Traces (trace != NULL): every scan kept by orc_trace_keep(seed, pass,
 * sweep, i) appends (features before the scan, moved) to the trace; sweep
 * is the 0-based sweep index of the phase (confirming sweeps included).
 *
 * Counters (may be NULL): out[0] scanned vertices, out[1] scanned entries,
 * out[2] pruned vertices, out[3] confirming sweeps.
 *
 * confirm = 0 drops the confirming sweeps: the gated sweeps run until the
 * usual test stops them (the whole run is then confirmed once, at its end:
 * orc_louvain's final phase). */
int32_t orc_move_sync_gated(int64_t n, const int64_t *off, const int32_t *col, const double *w, double M2,
                            const double *K, int32_t *memb, double tau, int32_t max_iter, int32_t rounds,
                            const float *params, double theta_logit, int32_t pass, orc_trace *trace,
                            double *dq_iter, int64_t *moved_iter, int64_t *counters, int32_t returns,
                            int32_t confirm) {
    if (n < 0 || max_iter < 0 || rounds < 1 || rounds > 64 || (rounds & (rounds - 1))) return -1;
    for (int64_t i = 0; i < n; i++)
        if (memb[i] < 0 || memb[i] >= n) return -1;
    int64_t cnt[4] = {0, 0, 0, 0};
    if (n == 0 || max_iter == 0) {
        if (counters) memcpy(counters, cnt, sizeof(cnt));
        return 0;
    }
    size_t N = (size_t)n;
    double *sigma = (double *)malloc(N * sizeof(double));
    int32_t *csize = (int32_t *)malloc(N * sizeof(int32_t));
    uint8_t *unproc = (uint8_t *)malloc(N);
    uint8_t *scan = (uint8_t *)malloc(N);
    int32_t *dec = (int32_t *)malloc(N * sizeof(int32_t));
    double *gain = (double *)malloc(N * sizeof(double));
    float *hfrac = (float *)calloc(N, sizeof(float));
    float *hgain = (float *)calloc(N, sizeof(float));
    uint8_t *hbits = (uint8_t *)calloc(N, 1);
    double *dmv = (double *)calloc(N, sizeof(double));
    float *xf = (float *)malloc(N * NF * sizeof(float));
    double *acc = (double *)calloc(N, sizeof(double));   /* K_{i->c} accumulator, dense */
    uint8_t *seen = (uint8_t *)calloc(N, 1);
    int32_t *keys = (int32_t *)malloc(N * sizeof(int32_t));
    int32_t *left = (int32_t *)malloc(N * sizeof(int32_t));      /* community left at the last move */
    int32_t *left_sw = (int32_t *)malloc(N * sizeof(int32_t));   /* and that move's sweep */
    if (!sigma || !csize || !unproc || !scan || !dec || !gain || !hfrac || !hgain || !hbits || !dmv || !xf || !acc ||
        !seen || !keys || !left || !left_sw) {
        free(sigma); free(csize); free(unproc); free(scan); free(dec); free(gain); free(hfrac); free(hgain);
        free(hbits); free(dmv); free(xf); free(acc); free(seen); free(keys); free(left); free(left_sw);
        return -1;
    }
    for (size_t i = 0; i < N; i++) { left[i] = -1; left_sw[i] = -2; }
    memset(unproc, 1, N);
    double pd[ORC_MLP_PARAMS];
    if (params) widen(params, pd);
    enum { GATED, CONFIRM, PLAIN } mode = params ? GATED : PLAIN;
    int32_t li = 0;
    for (int32_t sweep = 0; li < max_iter; sweep++) {
        /* the last iteration the phase may count is a confirming sweep: a
         * phase never ends on gated sweeps alone, so every vertex the gate
         * kept from its scans is judged by the plain method once more */
        if (confirm && mode == GATED && li + 1 >= max_iter) mode = CONFIRM;
        if (mode == CONFIRM) {
            memset(unproc, 1, N);
            cnt[3]++;
        }
        int64_t gsum = 0;   /* units of 2^-61 of delta-modularity (orc_gain_fixed) */
        int64_t moved = 0;
        for (int32_t p = 0; p < rounds; p++) {
            for (int64_t c = 0; c < n; c++) { sigma[c] = 0.0; csize[c] = 0; }
            for (int64_t i = 0; i < n; i++) { sigma[memb[i]] += K[i]; csize[memb[i]]++; }
            /* the group's unprocessed vertices; the gate decides which are scanned */
            for (int64_t i = 0; i < n; i++) {
                dec[i] = memb[i];
                gain[i] = 0.0;
                scan[i] = 0;
                if (!unproc[i] || sub_round(i, rounds) != p) continue;
                unproc[i] = 0;
                if (off[i + 1] == off[i]) continue;   /* an empty row: nothing to scan, never moves */
                orc_gate_features(off[i + 1] - off[i], K[i], sigma[memb[i]], hfrac[i], hgain[i], hbits[i], dmv[i],
                                  pass, li, xf + i * NF);
                if (mode == GATED && mlp_row(pd, xf + i * NF, 1, NULL, NULL) < theta_logit) {
                    cnt[2]++;
                    continue;
                }
                scan[i] = 1;
            }
            /* decisions from the snapshot (orc_move_sync_step's rule) */
            for (int64_t i = 0; i < n; i++) {
                if (!scan[i]) continue;
                int32_t d = memb[i];
                int64_t nk = 0;
                for (int64_t e = off[i]; e < off[i + 1]; e++) {
                    int32_t j = col[e];
                    if (j == i) continue;
                    int32_t c = memb[j];
                    if (!seen[c]) { seen[c] = 1; acc[c] = 0.0; keys[nk++] = c; }
                    acc[c] += w ? w[e] : 1.0;
                }
                cnt[0]++;
                cnt[1] += off[i + 1] - off[i];
                double ki = K[i];
                double kid = seen[d] ? acc[d] : 0.0;
                double g_stay = M2 * kid - ki * (sigma[d] - ki);
                int32_t best = -1;
                double g_best = 0.0;
                for (int64_t k = 0; k < nk; k++) {
                    int32_t c = keys[k];
                    if (c == d) continue;
                    double g = M2 * acc[c] - ki * sigma[c];
                    if (best < 0 || g > g_best || (g == g_best && c < best)) { best = c; g_best = g; }
                }
                for (int64_t k = 0; k < nk; k++) seen[keys[k]] = 0;
                int mv = best >= 0 && g_best > g_stay && !(csize[d] == 1 && csize[best] == 1 && best > d);
                if (trace && orc_trace_keep(trace->seed, pass, sweep, i, trace->threshold))
                    trace_put(trace, xf + i * NF, (uint8_t)mv, i, pass, sweep);
                gate_history(ki, kid, M2, best >= 0, g_best, g_stay, &hfrac[i], &hgain[i]);
                hbits[i] = (uint8_t)(1u | (mv ? 2u : 0u));
                dmv[i] = 0.0;   /* scanned: D_i starts again */
                if (mv) {
                    dec[i] = best;
                    gain[i] = g_best - g_stay;
                    moved++;
                }
            }
            for (int64_t i = 0; i < n; i++) {
                if (dec[i] == memb[i]) continue;
                if (!(returns && dec[i] == left[i] && left_sw[i] == sweep - 1)) gsum += orc_gain_fixed(gain[i], M2);   /* not a return move */
                left[i] = memb[i];
                left_sw[i] = sweep;
                for (int64_t e = off[i]; e < off[i + 1]; e++)
                    if (col[e] != i) {
                        unproc[col[e]] = 1;
                        dmv[col[e]] += w ? w[e] : 1.0;
                    }
            }
            for (int64_t i = 0; i < n; i++) memb[i] = dec[i];
        }
        double dq = ldexp((double)gsum, -61);
        int counted = mode != CONFIRM || moved > 0;
        if (counted) {
            if (dq_iter) dq_iter[li] = dq;
            if (moved_iter) moved_iter[li] = moved;
            li++;
        }
        if (dq <= tau) {
            if (mode == GATED && confirm) { mode = CONFIRM; continue; }
            break;
        }
        if (mode == CONFIRM) mode = PLAIN;
    }
    if (counters) memcpy(counters, cnt, sizeof(cnt));
    free(sigma); free(csize); free(unproc); free(scan); free(dec); free(gain); free(hfrac); free(hgain);
    free(hbits); free(dmv); free(xf); free(acc); free(seen); free(keys); free(left); free(left_sw);
    return li;
}
