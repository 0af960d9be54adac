/*
 * oracle.c - TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * A plain, sequential, obviously-correct CPU rendering of GSP-Louvain
 * (arXiv 2402.11454) in fp64.  Every function follows one passage of the
 * paper, cited in its comment.  Nothing here is blocked, fused or reordered
 * beyond what the paper states.  The per-thread "collision-free hashtable"
 * H_t of the local-moving and aggregation phases is a dense array indexed
 * by community id plus a list of the keys touched, which is what a
 * collision-free table keyed by community id is.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared (no fast-math;
 * no FMA contraction, so every product and sum is one IEEE operation).
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* Progress lines on stderr (per iteration and per pass) for long runs. */
static int orc_verbose = 0;
void orc_set_verbose(int32_t on) { orc_verbose = on; }

/* ------------------------------------------------------------------ */
/* helpers                                                              */
/* ------------------------------------------------------------------ */

/* Neumaier's compensated summation (Neumaier 1974). */
typedef struct { double s, c; } nsum;

static void nsum_add(nsum *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double nsum_get(const nsum *a) { return a->s + a->c; }

/* Dense-key table H: val[key] accumulates, keys[] lists touched keys. */
typedef struct {
    double *val;
    uint8_t *used;
    int32_t *keys;
    int64_t nkeys;
} table;

static int table_init(table *h, int64_t size) {
    h->val = (double *)calloc((size_t)(size > 0 ? size : 1), sizeof(double));
    h->used = (uint8_t *)calloc((size_t)(size > 0 ? size : 1), 1);
    h->keys = (int32_t *)malloc((size_t)(size > 0 ? size : 1) * sizeof(int32_t));
    h->nkeys = 0;
    return (h->val && h->used && h->keys) ? 0 : -1;
}

static void table_free(table *h) { free(h->val); free(h->used); free(h->keys); }

static void table_add(table *h, int32_t key, double w) {
    if (!h->used[key]) {
        h->used[key] = 1;
        h->keys[h->nkeys++] = key;
    }
    h->val[key] += w;
}

static void table_clear(table *h) {
    for (int64_t k = 0; k < h->nkeys; k++) {
        h->val[h->keys[k]] = 0.0;
        h->used[h->keys[k]] = 0;
    }
    h->nkeys = 0;
}

/* scanCommunities (Algorithm "louvainMove", second function): adds w_ij to
 * H[C[j]] for every entry of row i, skipping the self-loop unless self. */
static void scan_communities(table *h, const int64_t *off, const int32_t *col, const double *w,
                             const int32_t *memb, int64_t i, int self) {
    for (int64_t e = off[i]; e < off[i + 1]; e++) {
        int32_t j = col[e];
        if (!self && j == i) continue;
        table_add(h, memb[j], w[e]);
    }
}

static int valid_memb(int64_t n, const int32_t *memb) {
    for (int64_t i = 0; i < n; i++)
        if (memb[i] < 0 || memb[i] >= n) return 0;
    return 1;
}

/* ------------------------------------------------------------------ */
/* Exact sums: the weight grid                                          */
/* ------------------------------------------------------------------ */

/* Number of bits of x (0 for x = 0). */
static int bit_length(uint64_t x) {
    int b = 0;
    while (x) { b++; x >>= 1; }
    return b;
}

/* Section 5.1.2 stores edge weights in fp32 and computes in fp64.  A sum of
 * fp32 weights is exact in fp64 only while it stays below 2^53 units of its
 * finest weight, which the largest graphs pass, and a parallel sum beyond
 * that depends on its order.  Reading taken: every weight is replaced by the
 * nearest multiple of 2^-S (ties to even), S the largest integer (kept in
 * [-1000, 1022]) with U 2^S < 2^52, where U >= 2m is an upper bound of the
 * weight total computed exactly:
 *   e with wmax < 2^e (wmax the largest weight), b with nnz < 2^b,
 *   T = 62 - b - e, U_int = sum of max(1, ceil(w 2^T)) over the positive
 *   weights (an exact integer below 2^63), U = U_int 2^-T <= 2^(len - T)
 *   with len the bit length of U_int, so S = 52 - len + T.
 * Then every weight, and every sum or difference of weights the method
 * takes (K_i, 2m, Sigma_c and its updates, K_{i->c}, super-vertex weights)
 * is a multiple of 2^-S of magnitude below 2^52 2^-S: exact in fp64, in any
 * order.  For integer weights, and for fp32 weights of a few units on
 * graphs below about 2^28 entries, nothing changes.  Returns S (0 for a
 * graph without a positive weight); *changed (may be NULL) receives the
 * number of weights that moved. */
int32_t orc_weight_grid(int64_t nnz, double *w, int64_t *changed) {
    if (changed) *changed = 0;
    if (nnz < 0) return -2000;
    double wmax = 0.0;
    for (int64_t e = 0; e < nnz; e++)
        if (w[e] > wmax) wmax = w[e];
    if (!(wmax > 0.0)) return 0;
    int ew;
    frexp(wmax, &ew);                       /* wmax = m 2^ew, 1/2 <= m < 1 */
    int b = bit_length((uint64_t)nnz);
    int T = 62 - b - ew;
    uint64_t U = 0;
    for (int64_t e = 0; e < nnz; e++) {
        if (!(w[e] > 0.0)) continue;
        double t = ceil(ldexp(w[e], T));
        U += t < 1.0 ? 1u : (uint64_t)t;
    }
    int S = 52 - bit_length(U) + T;
    if (S > 1022) S = 1022;
    if (S < -1000) S = -1000;
    int64_t moved = 0;
    for (int64_t e = 0; e < nnz; e++) {
        double q = ldexp(nearbyint(ldexp(w[e], S)), -S);
        if (q != w[e]) moved++;
        w[e] = q;
    }
    if (changed) *changed = moved;
    return S;
}

/* ------------------------------------------------------------------ */
/* Section 3: weights and modularity                                    */
/* ------------------------------------------------------------------ */

/* Section 3 notation: K_i = sum_{j in J_i} w_ij over the stored row (the
 * self-loop entry counted once, as stored); vertexWeights of Algorithm
 * "louvain" (reset step).  Returns M2 = 2m = sum of all entries. */
double orc_vertex_weights(int64_t n, const int64_t *off, const int32_t *col, const double *w, double *K) {
    (void)col;
    double M2 = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double k = 0.0;
        for (int64_t e = off[i]; e < off[i + 1]; e++) k += w[e];
        if (K) K[i] = k;
        M2 += k;
    }
    return M2;
}

/* Eq. 1, right-hand (community) form: Q = sum_c [sigma_c/2m - (Sigma_c/2m)^2]
 * with sigma_c the sum of stored entries whose both ends lie in c and
 * Sigma_c the sum of K_i over i in c. */
double orc_modularity(int64_t n, const int64_t *off, const int32_t *col, const double *w, const int32_t *memb) {
    if (n < 0 || !valid_memb(n, memb)) return NAN;
    nsum *sig_in = (nsum *)calloc((size_t)(n > 0 ? n : 1), sizeof(nsum));
    nsum *sig_tot = (nsum *)calloc((size_t)(n > 0 ? n : 1), sizeof(nsum));
    nsum m2 = {0, 0};
    for (int64_t i = 0; i < n; i++) {
        int32_t c = memb[i];
        for (int64_t e = off[i]; e < off[i + 1]; e++) {
            nsum_add(&m2, w[e]);
            nsum_add(&sig_tot[c], w[e]);
            if (memb[col[e]] == c) nsum_add(&sig_in[c], w[e]);
        }
    }
    double M2 = nsum_get(&m2);
    double q = 0.0;
    if (M2 > 0.0) {
        nsum acc = {0, 0};
        for (int64_t c = 0; c < n; c++) {
            double a = nsum_get(&sig_in[c]) / M2;
            double b = nsum_get(&sig_tot[c]) / M2;
            nsum_add(&acc, a);
            nsum_add(&acc, -(b * b));
        }
        q = nsum_get(&acc);
    }
    free(sig_in);
    free(sig_tot);
    return q;
}

/* Eq. 2: dQ_{i: d->c} = (K_{i->c} - K_{i->d})/m - K_i (K_i + Sigma_c - Sigma_d) / (2 m^2),
 * with K_{i->x} from scanCommunities(self = false) and Sigma_d including K_i. */
double orc_delta_modularity(int64_t n, const int64_t *off, const int32_t *col, const double *w,
                            const int32_t *memb, int64_t i, int32_t c) {
    if (i < 0 || i >= n || c < 0 || c >= n || !valid_memb(n, memb)) return NAN;
    double *K = (double *)malloc((size_t)n * sizeof(double));
    double M2 = orc_vertex_weights(n, off, col, w, K);
    double m = M2 / 2.0;
    int32_t d = memb[i];
    double sig_c = 0.0, sig_d = 0.0, kic = 0.0, kid = 0.0;
    for (int64_t v = 0; v < n; v++) {
        if (memb[v] == c) sig_c += K[v];
        if (memb[v] == d) sig_d += K[v];
    }
    for (int64_t e = off[i]; e < off[i + 1]; e++) {
        if (col[e] == i) continue;
        if (memb[col[e]] == c) kic += w[e];
        if (memb[col[e]] == d) kid += w[e];
    }
    double ki = K[i];
    free(K);
    if (m == 0.0) return 0.0;
    if (c == d) return 0.0;
    return (kic - kid) / m - ki * (ki + sig_c - sig_d) / (2.0 * m * m);
}

/* ------------------------------------------------------------------ */
/* Local-moving phase (Algorithm "louvainMove")                          */
/* ------------------------------------------------------------------ */

/* One thread runs the parallel loop of Algorithm "louvainMove" in vertex
 * order.  For each unprocessed i: mark it processed (pruning), scan its
 * neighbour communities without the self-loop, pick the community c != d
 * with the largest Eq. 2 gain (ties to the lowest id), move only if that
 * gain is positive (staying has gain 0), update Sigma in place, add the gain
 * to the iteration total and mark every neighbour j != i unprocessed.  Stop
 * after an iteration whose total is <= tau, or after max_iter iterations;
 * the count returned includes the last iteration. */
int32_t orc_move_async(int64_t n, const int64_t *off, const int32_t *col, const double *w, double M2,
                       const double *K, int32_t *memb, double *sigma, double tau, int32_t max_iter,
                       double *dq_iter) {
    if (n < 0 || max_iter < 0 || !valid_memb(n, memb)) return -1;
    if (n == 0 || max_iter == 0) return 0;
    uint8_t *unprocessed = (uint8_t *)malloc((size_t)n);
    table h;
    if (!unprocessed || table_init(&h, n)) { free(unprocessed); return -1; }
    memset(unprocessed, 1, (size_t)n);
    double m = M2 / 2.0;
    int32_t li = 0;
    for (int32_t it = 0; it < max_iter; it++) {
        double dq = 0.0;
        for (int64_t i = 0; i < n; i++) {
            if (!unprocessed[i]) continue;
            unprocessed[i] = 0;
            scan_communities(&h, off, col, w, memb, i, 0);
            int32_t d = memb[i];
            double kid = h.used[d] ? h.val[d] : 0.0;
            double ki = K[i];
            int32_t best = -1;
            double best_dq = 0.0;
            for (int64_t k = 0; k < h.nkeys; k++) {
                int32_t c = h.keys[k];
                if (c == d) continue;
                double g = (h.val[c] - kid) / m - ki * (ki + sigma[c] - sigma[d]) / (2.0 * m * m);
                if (best < 0 || g > best_dq || (g == best_dq && c < best)) {
                    best = c;
                    best_dq = g;
                }
            }
            table_clear(&h);
            if (best < 0 || !(best_dq > 0.0)) continue;
            sigma[d] -= ki;
            sigma[best] += ki;
            memb[i] = best;
            dq += best_dq;
            for (int64_t e = off[i]; e < off[i + 1]; e++)
                if (col[e] != i) unprocessed[col[e]] = 1;
        }
        if (dq_iter) dq_iter[it] = dq;
        li = it + 1;
        if (orc_verbose) fprintf(stderr, "[oracle] async iteration %d: dQ %.6g\n", (int)li, dq);
        if (dq <= tau) break;
    }
    table_free(&h);
    free(unprocessed);
    return li;
}

/* Synchronous step.  Scores use Eq. 2 multiplied through by 2m^2 = M2^2/2:
 * for a candidate c != d, G(c) = M2 K_{i->c} - K_i Sigma_c, and for staying
 * G(stay) = M2 K_{i->d} - K_i (Sigma_d - K_i), so that
 * dQ_{i: d->c} = (G(c) - G(stay)) / (M2^2 / 2).  All quantities come from
 * the snapshot.  The best candidate has the largest G (ties to the lowest
 * id); i moves iff G(best) > G(stay), except that a vertex alone in its
 * community does not move to another one-vertex community with a larger id
 * (so two singletons never swap). */
int64_t orc_move_sync_step(int64_t n, const int64_t *off, const int32_t *col, const double *w, double M2,
                           const double *K, const int32_t *memb, const double *sigma, const int32_t *csize,
                           const uint8_t *active, int32_t *dec, double *gain) {
    if (n < 0 || !valid_memb(n, memb)) return -1;
    table h;
    if (table_init(&h, n)) return -1;
    int64_t moved = 0;
    for (int64_t i = 0; i < n; i++) {
        int32_t d = memb[i];
        dec[i] = d;
        if (gain) gain[i] = 0.0;
        if (active && !active[i]) continue;
        scan_communities(&h, off, col, w, memb, i, 0);
        double ki = K[i];
        double kid = h.used[d] ? h.val[d] : 0.0;
        double g_stay = M2 * kid - ki * (sigma[d] - ki);
        int32_t best = -1;
        double g_best = 0.0;
        for (int64_t k = 0; k < h.nkeys; k++) {
            int32_t c = h.keys[k];
            if (c == d) continue;
            double g = M2 * h.val[c] - ki * sigma[c];
            if (best < 0 || g > g_best || (g == g_best && c < best)) {
                best = c;
                g_best = g;
            }
        }
        table_clear(&h);
        if (best < 0 || !(g_best > g_stay)) continue;
        if (csize[d] == 1 && csize[best] == 1 && best > d) continue;
        dec[i] = best;
        if (gain) gain[i] = g_best - g_stay;
        moved++;
    }
    table_free(&h);
    return moved;
}

/* The synchronous decision of one vertex from its row alone (the rule of
 * orc_move_sync_step): cols/w are the row of vertex i (deg entries, w NULL
 * for unit weights), memb/sigma/csize the snapshot.  Writes G(best) -
 * G(stay) to *gain (0 if it stays) and, for margin checks, the two best
 * candidate scores and G(stay) to scores[0..2] (-inf where absent).
 * Returns the chosen community. */
int32_t orc_decide_row(int64_t i, int64_t deg, const int32_t *cols, const double *w, const int32_t *memb,
                       const double *sigma, const int32_t *csize, double ki, double M2, double *gain,
                       double *scores) {
    int32_t d = memb[i];
    /* K_{i->c} over the row's distinct communities (a short list: rows are scanned once) */
    int32_t *keys = (int32_t *)malloc((size_t)(deg > 0 ? deg : 1) * sizeof(int32_t));
    double *vals = (double *)malloc((size_t)(deg > 0 ? deg : 1) * sizeof(double));
    int64_t nk = 0;
    for (int64_t e = 0; e < deg; e++) {
        if (cols[e] == i) continue;
        int32_t c = memb[cols[e]];
        int64_t k = 0;
        while (k < nk && keys[k] != c) k++;
        if (k == nk) { keys[nk] = c; vals[nk] = 0.0; nk++; }
        vals[k] += w ? w[e] : 1.0;
    }
    double kid = 0.0;
    for (int64_t k = 0; k < nk; k++)
        if (keys[k] == d) kid = vals[k];
    double g_stay = M2 * kid - ki * (sigma[d] - ki);
    int32_t best = -1;
    double g_best = -INFINITY, g_second = -INFINITY;
    for (int64_t k = 0; k < nk; k++) {
        int32_t c = keys[k];
        if (c == d) continue;
        double g = M2 * vals[k] - ki * sigma[c];
        if (best < 0 || g > g_best || (g == g_best && c < best)) {
            if (best >= 0) g_second = g_best > g_second ? g_best : g_second;
            best = c;
            g_best = g;
        } else if (g > g_second) {
            g_second = g;
        }
    }
    free(keys);
    free(vals);
    if (scores) { scores[0] = g_best; scores[1] = g_second; scores[2] = g_stay; }
    *gain = 0.0;
    if (best < 0 || !(g_best > g_stay)) return d;
    if (csize[d] == 1 && csize[best] == 1 && best > d) return d;
    *gain = g_best - g_stay;
    return best;
}

/* A mover's gain in the iteration's total (reading of the tolerance test
 * of Algorithm "louvainMove" for simultaneous moves): its delta-modularity
 * 2 (G(c*) - G(stay)) / M2^2 in fixed point, rounded to the nearest
 * multiple of 2^-61 (ties to even).  The total is the exact integer sum of
 * these, so it does not depend on the order in which movers are added; a
 * mover's delta-modularity is at most 2 K_i / M2, so the total of one
 * iteration stays below 2^62 units. */
int64_t orc_gain_fixed(double gain, double M2) {
    if (!(M2 > 0.0)) return 0;
    return (int64_t)llrint(ldexp((2.0 * gain) / (M2 * M2), 61));
}

/* Group of a vertex for the ordered sub-rounds of the synchronous phase:
 * the top log2(rounds) bits of the 64-bit product i * 0x9E3779B97F4A7C15
 * (Fibonacci hashing); rounds is a power of two. */
static int32_t sub_round_of(int64_t i, int32_t rounds) {
    if (rounds <= 1) return 0;
    int sh = 0;
    while ((1 << sh) < rounds) sh++;
    uint64_t x = (uint64_t)i * 0x9E3779B97F4A7C15ULL;
    return (int32_t)(x >> (64 - sh));
}

/* Synchronous local-moving phase, in ordered sub-rounds.  It keeps the
 * structure of Algorithm "louvainMove" (unprocessed flags, pruning, re-marking
 * of neighbours, the per-iteration gain total and its tolerance test), but
 * the parallel vertex loop is split into `rounds` groups taken in order.
 * Within a group every decision comes from one snapshot (orc_move_sync_step);
 * its moves are then applied together, Sigma and the sizes recomputed, and
 * every neighbour j != i of a mover marked unprocessed, so a later group sees
 * them in the same iteration and earlier groups in the next one.
 *
 * Return moves (returns != 0, an option; by default every mover's gain
 * counts, the tolerance test as written).  Moves decided from one snapshot
 * can undo each other (two adjacent vertices of one group each joining the
 * other's community); the next iteration then swaps them back, and so on,
 * each time with positive predicted gains while the modularity does not
 * change.  With the option, a move of i back into the community it left at
 * its move in the immediately preceding iteration is made, but its gain is
 * not added to the iteration's total, so the tolerance test sees the gain
 * that such a cycle does not deliver.  (The paper's loop moves vertices one
 * at a time, where every reported gain is real.) */
int32_t orc_move_sync(int64_t n, const int64_t *off, const int32_t *col, const double *w, double M2,
                      const double *K, int32_t *memb, double tau, int32_t max_iter, int32_t rounds,
                      double *dq_iter, int64_t *moved_iter, int32_t returns) {
    if (n < 0 || max_iter < 0 || rounds < 1 || rounds > 64 || (rounds & (rounds - 1)) || !valid_memb(n, memb))
        return -1;
    if (n == 0 || max_iter == 0) return 0;
    double *sigma = (double *)malloc((size_t)n * sizeof(double));
    int32_t *csize = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    uint8_t *unprocessed = (uint8_t *)malloc((size_t)n);
    uint8_t *active = (uint8_t *)malloc((size_t)n);
    int32_t *dec = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    double *gain = (double *)malloc((size_t)n * sizeof(double));
    if (!sigma || !csize || !unprocessed || !active || !dec || !gain) {
        free(sigma); free(csize); free(unprocessed); free(active); free(dec); free(gain);
        return -1;
    }
    /* per vertex: the community it left at its last move, and that move's iteration */
    int32_t *left = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *left_it = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!left || !left_it) {
        free(sigma); free(csize); free(unprocessed); free(active); free(dec); free(gain); free(left); free(left_it);
        return -1;
    }
    for (int64_t i = 0; i < n; i++) { left[i] = -1; left_it[i] = -2; }
    memset(unprocessed, 1, (size_t)n);
    int32_t li = 0;
    for (int32_t it = 0; it < max_iter; it++) {
        int64_t gsum = 0;   /* units of 2^-61 of delta-modularity (orc_gain_fixed) */
        int64_t moved = 0;
        for (int32_t p = 0; p < rounds; p++) {
            /* snapshot: Sigma_c = sum of K_i over c, and the size of c */
            for (int64_t c = 0; c < n; c++) { sigma[c] = 0.0; csize[c] = 0; }
            for (int64_t i = 0; i < n; i++) { sigma[memb[i]] += K[i]; csize[memb[i]]++; }
            for (int64_t i = 0; i < n; i++) {
                active[i] = unprocessed[i] && sub_round_of(i, rounds) == p;
                if (active[i]) unprocessed[i] = 0;
            }
            moved += orc_move_sync_step(n, off, col, w, M2, K, memb, sigma, csize, active, dec, gain);
            for (int64_t i = 0; i < n; i++) {
                if (dec[i] == memb[i]) continue;
                int back = returns && dec[i] == left[i] && left_it[i] == it - 1;   /* a return move */
                if (!back) gsum += orc_gain_fixed(gain[i], M2);
                left[i] = memb[i];
                left_it[i] = it;
                for (int64_t e = off[i]; e < off[i + 1]; e++)
                    if (col[e] != i) unprocessed[col[e]] = 1;
            }
            for (int64_t i = 0; i < n; i++) memb[i] = dec[i];
        }
        double dq = ldexp((double)gsum, -61);
        if (dq_iter) dq_iter[it] = dq;
        if (moved_iter) moved_iter[it] = moved;
        li = it + 1;
        if (dq <= tau) break;
    }
    free(sigma); free(csize); free(unprocessed); free(active); free(dec); free(gain); free(left); free(left_it);
    return li;
}

/* ------------------------------------------------------------------ */
/* Refinement phase (GSP-Leiden)                                        */
/* ------------------------------------------------------------------ */

/* The refinement phase of the Leiden algorithm (Section 3.5), in the
 * reading this oracle takes for GSP-Leiden (the paper gives prose only):
 * the communities of the local-moving phase are the bounds, and within them
 * vertices build sub-communities.  A vertex may leave its sub-community only
 * while it is alone in it, and may join only the sub-community of a
 * neighbour in its own bound; among those it takes the one of largest
 * delta-modularity (Eq. 2 with the whole graph's K and 2m), ties to the
 * lowest id, and only for a positive gain: the greedy limit of the
 * randomised choice.  The moves run in the ordered synchronous sub-rounds of
 * orc_move_sync, with its gain total, tolerance test and singleton rule; a
 * mover marks its neighbours in the same bound unprocessed.  memb holds the
 * starting sub-communities (normally every vertex alone), each inside one
 * bound, and is updated in place.  Returns the iterations run. */
int32_t orc_refine_sync(int64_t n, const int64_t *off, const int32_t *col, const double *w, double M2,
                        const double *K, const int32_t *bound, int32_t *memb, double tau, int32_t max_iter,
                        int32_t rounds, double *dq_iter, int64_t *moved_iter) {
    if (n < 0 || max_iter < 0 || rounds < 1 || rounds > 64 || (rounds & (rounds - 1)) || !valid_memb(n, memb) ||
        !valid_memb(n, bound))
        return -1;
    if (n == 0 || max_iter == 0) return 0;
    int32_t *home = (int32_t *)malloc((size_t)n * sizeof(int32_t));   /* bound of each sub-community */
    double *sigma = (double *)malloc((size_t)n * sizeof(double));
    int32_t *csize = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    uint8_t *unprocessed = (uint8_t *)malloc((size_t)n);
    int32_t *dec = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    double *gain = (double *)malloc((size_t)n * sizeof(double));
    table h = {0};
    int bad = !home || !sigma || !csize || !unprocessed || !dec || !gain || table_init(&h, n);
    for (int64_t c = 0; !bad && c < n; c++) home[c] = -1;
    for (int64_t i = 0; !bad && i < n; i++) {
        int32_t c = memb[i];
        if (home[c] < 0) home[c] = bound[i];
        else if (home[c] != bound[i]) bad = 1;   /* a sub-community across two bounds */
    }
    if (bad) {
        free(home); free(sigma); free(csize); free(unprocessed); free(dec); free(gain);
        if (h.val) table_free(&h);
        return -1;
    }
    memset(unprocessed, 1, (size_t)n);
    int32_t li = 0;
    for (int32_t it = 0; it < max_iter; it++) {
        int64_t gsum = 0, moved = 0;
        for (int32_t p = 0; p < rounds; p++) {
            for (int64_t c = 0; c < n; c++) { sigma[c] = 0.0; csize[c] = 0; }
            for (int64_t i = 0; i < n; i++) { sigma[memb[i]] += K[i]; csize[memb[i]]++; }
            for (int64_t i = 0; i < n; i++) {
                int32_t d = memb[i];
                dec[i] = d;
                gain[i] = 0.0;
                if (!unprocessed[i] || sub_round_of(i, rounds) != p) continue;
                unprocessed[i] = 0;
                if (csize[d] != 1) continue;   /* merged already: stays */
                for (int64_t e = off[i]; e < off[i + 1]; e++) {
                    int32_t j = col[e];
                    if (j != i && bound[j] == bound[i]) table_add(&h, memb[j], w[e]);
                }
                double ki = K[i];
                double kid = h.used[d] ? h.val[d] : 0.0;
                double g_stay = M2 * kid - ki * (sigma[d] - ki);
                int32_t best = -1;
                double g_best = 0.0;
                for (int64_t k = 0; k < h.nkeys; k++) {
                    int32_t c = h.keys[k];
                    if (c == d) continue;
                    double g = M2 * h.val[c] - ki * sigma[c];
                    if (best < 0 || g > g_best || (g == g_best && c < best)) {
                        best = c;
                        g_best = g;
                    }
                }
                table_clear(&h);
                if (best < 0 || !(g_best > g_stay)) continue;
                if (csize[best] == 1 && best > d) continue;   /* singleton rule */
                dec[i] = best;
                gain[i] = g_best - g_stay;
            }
            for (int64_t i = 0; i < n; i++) {
                if (dec[i] == memb[i]) continue;
                gsum += orc_gain_fixed(gain[i], M2);
                moved++;
                for (int64_t e = off[i]; e < off[i + 1]; e++)
                    if (col[e] != i && bound[col[e]] == bound[i]) unprocessed[col[e]] = 1;
            }
            for (int64_t i = 0; i < n; i++) memb[i] = dec[i];
        }
        double dq = ldexp((double)gsum, -61);
        if (dq_iter) dq_iter[it] = dq;
        if (moved_iter) moved_iter[it] = moved;
        li = it + 1;
        if (dq <= tau) break;
    }
    free(home); free(sigma); free(csize); free(unprocessed); free(dec); free(gain);
    table_free(&h);
    return li;
}

/* ------------------------------------------------------------------ */
/* Split phase                                                          */
/* ------------------------------------------------------------------ */

/* Algorithm "splitDisconnectedBfs" with one thread.  The source of each BFS
 * is the lowest unvisited vertex (the paper picks any unvisited vertex; the
 * partition is the same), the BFS follows entries (x, j) with C[j] equal to
 * the source's community, and every reached vertex gets the source's label.
 * With the lowest source, the label is the component's smallest vertex. */
int32_t orc_split_bfs(int64_t n, const int64_t *off, const int32_t *col, const int32_t *memb, int32_t *labels) {
    if (n < 0 || !valid_memb(n, memb)) return -1;
    uint8_t *vis = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    int32_t *queue = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!vis || !queue) { free(vis); free(queue); return -1; }
    for (int64_t i = 0; i < n; i++) labels[i] = (int32_t)i;
    for (int64_t i = 0; i < n; i++) {
        if (vis[i]) continue;
        int32_t c = memb[i];
        int32_t lab = labels[i];
        int64_t head = 0, tail = 0;
        vis[i] = 1;
        queue[tail++] = (int32_t)i;
        while (head < tail) {
            int32_t x = queue[head++];
            labels[x] = lab;
            for (int64_t e = off[x]; e < off[x + 1]; e++) {
                int32_t j = col[e];
                if (vis[j] || memb[j] != c) continue;
                vis[j] = 1;
                queue[tail++] = j;
            }
        }
    }
    free(vis);
    free(queue);
    return 0;
}

/* Algorithm "splitDisconnectedLp" with one thread (in-place updates). */
int32_t orc_split_lp(int64_t n, const int64_t *off, const int32_t *col, const int32_t *memb, int32_t pruned,
                     int32_t *labels) {
    if (n < 0 || !valid_memb(n, memb)) return -1;
    uint8_t *unprocessed = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    if (!unprocessed) return -1;
    for (int64_t i = 0; i < n; i++) { labels[i] = (int32_t)i; unprocessed[i] = 1; }
    int32_t sweeps = 0;
    for (;;) {
        int64_t changed = 0;
        sweeps++;
        for (int64_t i = 0; i < n; i++) {
            if (!unprocessed[i]) continue;
            if (pruned) unprocessed[i] = 0;
            int32_t cmin = labels[i];
            for (int64_t e = off[i]; e < off[i + 1]; e++)
                if (memb[col[e]] == memb[i] && labels[col[e]] < cmin) cmin = labels[col[e]];
            if (cmin == labels[i]) continue;
            labels[i] = cmin;
            changed++;
            if (pruned)
                for (int64_t e = off[i]; e < off[i + 1]; e++)
                    if (memb[col[e]] == memb[i]) unprocessed[col[e]] = 1;
        }
        if (changed == 0) break;
    }
    free(unprocessed);
    return sweeps;
}

/* ------------------------------------------------------------------ */
/* Renumber, aggregation, disconnected communities                      */
/* ------------------------------------------------------------------ */

/* Renumbering of Algorithm "louvain": distinct labels, ascending, become
 * 0 .. G-1. */
int64_t orc_renumber(int64_t n, const int32_t *labels, int32_t *out) {
    if (n < 0 || !valid_memb(n, labels)) return -1;
    int32_t *map = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!map) return -1;
    for (int64_t i = 0; i < n; i++) map[i] = -1;
    for (int64_t i = 0; i < n; i++) map[labels[i]] = 0;
    int64_t g = 0;
    for (int64_t l = 0; l < n; l++)
        if (map[l] == 0) map[l] = (int32_t)g++;
    for (int64_t i = 0; i < n; i++) out[i] = map[labels[i]];
    free(map);
    return g;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Algorithm "louvainAggregate": the community-vertices CSR from counts and
 * an exclusive scan, then for each community c a table accumulating
 * scanCommunities(self = true) over its members, emitted as row c of the
 * super-vertex graph.  The emitted row is sorted by column (the paper's row
 * order is whatever its atomics give; sorting fixes one canonical order). */
int64_t orc_aggregate(int64_t n, const int64_t *off, const int32_t *col, const double *w, const int32_t *memb,
                      int64_t ncomm, int64_t *off2, int32_t *col2, double *w2, int64_t cap) {
    if (n < 0 || ncomm < 0) return -1;
    for (int64_t i = 0; i < n; i++)
        if (memb[i] < 0 || memb[i] >= ncomm) return -1;
    int64_t *coff = (int64_t *)calloc((size_t)ncomm + 1, sizeof(int64_t));
    int32_t *cver = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t *cur = (int64_t *)malloc((size_t)(ncomm > 0 ? ncomm : 1) * sizeof(int64_t));
    table h;
    if (!coff || !cver || !cur || table_init(&h, ncomm)) { free(coff); free(cver); free(cur); return -1; }
    for (int64_t i = 0; i < n; i++) coff[memb[i] + 1]++;             /* countCommunityVertices */
    for (int64_t c = 0; c < ncomm; c++) coff[c + 1] += coff[c];       /* exclusiveScan */
    for (int64_t c = 0; c < ncomm; c++) cur[c] = coff[c];
    for (int64_t i = 0; i < n; i++) cver[cur[memb[i]]++] = (int32_t)i; /* fill G'_{C'} */
    int64_t nnz = 0;
    off2[0] = 0;
    for (int64_t c = 0; c < ncomm; c++) {
        for (int64_t k = coff[c]; k < coff[c + 1]; k++)
            scan_communities(&h, off, col, w, memb, cver[k], 1);
        qsort(h.keys, (size_t)h.nkeys, sizeof(int32_t), cmp_i32);
        if (nnz + h.nkeys > cap) { nnz = -1; break; }
        for (int64_t k = 0; k < h.nkeys; k++) {
            col2[nnz] = h.keys[k];
            w2[nnz] = h.val[h.keys[k]];
            nnz++;
        }
        table_clear(&h);
        off2[c + 1] = nnz;
    }
    table_free(&h);
    free(coff);
    free(cver);
    free(cur);
    return nnz;
}

/* Algorithm "disconnectedCommunities" with one thread: community sizes,
 * then for each vertex whose community is not yet checked, a BFS within the
 * community counting the vertices reached; fewer than the size means the
 * community is disconnected. */
int64_t orc_disconnected(int64_t n, const int64_t *off, const int32_t *col, const int32_t *memb, uint8_t *flags) {
    if (n < 0 || !valid_memb(n, memb)) return -1;
    int64_t *S = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    uint8_t *vis = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    int32_t *queue = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!S || !vis || !queue) { free(S); free(vis); free(queue); return -1; }
    if (flags) memset(flags, 0, (size_t)n);
    for (int64_t i = 0; i < n; i++) S[memb[i]]++;
    int64_t count = 0;
    for (int64_t i = 0; i < n; i++) {
        int32_t c = memb[i];
        if (S[c] == 0) continue;
        int64_t reached = 0, head = 0, tail = 0;
        vis[i] = 1;
        queue[tail++] = (int32_t)i;
        while (head < tail) {
            int32_t x = queue[head++];
            reached++;
            for (int64_t e = off[x]; e < off[x + 1]; e++) {
                int32_t j = col[e];
                if (vis[j] || memb[j] != c) continue;
                vis[j] = 1;
                queue[tail++] = j;
            }
        }
        if (reached < S[c]) {
            if (flags) flags[c] = 1;
            count++;
        }
        S[c] = 0;
    }
    free(S);
    free(vis);
    free(queue);
    return count;
}

/* ------------------------------------------------------------------ */
/* Algorithm "louvain": the pass loop                                   */
/* ------------------------------------------------------------------ */

/* Numbers communities by ascending smallest vertex id. */
static void canonical_labels(int64_t n, int32_t *memb) {
    int32_t *map = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < n; i++) map[i] = -1;
    int32_t next = 0;
    for (int64_t v = 0; v < n; v++) {
        if (map[memb[v]] < 0) map[memb[v]] = next++;
        memb[v] = map[memb[v]];
    }
    free(map);
}

int32_t orc_louvain(int64_t n, const int64_t *off, const int32_t *col, const double *w, const orc_options *opt,
                    int32_t *memb_out, orc_stats *stats) {
    if (n < 0 || !opt || opt->max_passes < 0) return -1;
    if (opt->leiden && (!opt->sync_moves || opt->prune_params || opt->trace)) return -1;
    if (stats) memset(stats, 0, sizeof(*stats));
    int64_t nnz = off[n];
    /* G' starts as G itself (read only); the super-vertex graphs G'' go to
     * two buffers of G's size in turn (pages only touched as they fill) */
    int64_t *goff = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int32_t *gcol = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    double *gw = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    int64_t *noff = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int32_t *ncol = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    double *nw = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    const int64_t *loff = off;
    const int32_t *lcol = col;
    const double *lw = w;
    double *K = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *sigma = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    int32_t *cm = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *lab = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    /* GSP-Leiden: the refined sub-communities, and each super-vertex's
     * starting community at the next level */
    int32_t *ref = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *init = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!goff || !gcol || !gw || !noff || !ncol || !nw || !K || !sigma || !cm || !lab || !ref || !init) {
        free(goff); free(gcol); free(gw); free(noff); free(ncol); free(nw);
        free(K); free(sigma); free(cm); free(lab); free(ref); free(init);
        return -1;
    }
    int64_t gn = n;
    for (int64_t v = 0; v < n; v++) memb_out[v] = (int32_t)v;       /* C <- [0 .. |V|) */
    double M2 = orc_vertex_weights(n, off, col, w, NULL);            /* 2m of G */
    double tau = opt->tolerance;
    int32_t passes = 0;
    for (int32_t lp = 0; lp < opt->max_passes; lp++) {
        passes = lp + 1;
        /* Sigma' <- K' <- vertexWeights(G'); C' <- [0 .. |V'|); all unprocessed */
        orc_vertex_weights(gn, loff, lcol, lw, K);
        for (int64_t i = 0; i < gn; i++) { sigma[i] = K[i]; cm[i] = (int32_t)i; }
        if (opt->leiden && lp > 0) memcpy(cm, init, (size_t)gn * sizeof(int32_t));   /* C' <- the bounds' communities */
        int32_t li;
        if (opt->sync_moves && (opt->prune_params || opt->trace)) {
            int64_t c4[4];
            li = orc_move_sync_gated(gn, loff, lcol, lw, M2, K, cm, tau, opt->max_iterations, opt->sync_rounds,
                                     opt->prune_params, opt->prune_theta_logit, lp, opt->trace, NULL, NULL, c4,
                                     opt->return_moves, !(opt->prune_params && opt->confirm_final));
            if (stats)
                for (int q = 0; q < 4; q++) stats->counters[q] += c4[q];
        } else if (opt->sync_moves)
            li = orc_move_sync(gn, loff, lcol, lw, M2, K, cm, tau, opt->max_iterations, opt->sync_rounds, NULL, NULL,
                               opt->return_moves);
        else
            li = orc_move_async(gn, loff, lcol, lw, M2, K, cm, sigma, tau, opt->max_iterations, NULL);
        if (opt->split_mode == 0) {                                   /* C' <- split(G', C') */
            orc_split_bfs(gn, loff, lcol, cm, lab);
            memcpy(cm, lab, (size_t)gn * sizeof(int32_t));
        }
        int64_t ng = orc_renumber(gn, cm, lab);                       /* |Gamma| */
        if (stats && lp < 64) {
            stats->tau[lp] = tau;
            stats->iterations[lp] = li;
            stats->communities[lp] = ng;
            stats->vertices[lp] = gn;
        }
        memcpy(cm, lab, (size_t)gn * sizeof(int32_t));
        if (opt->leiden) {
            /* GSP-Leiden: the result is the local-moving communities; the
             * next level's super-vertices are their refined sub-communities,
             * each starting in the community that holds it */
            int stop = li <= 1 || (double)ng / (double)gn > opt->aggregation_tolerance || lp == opt->max_passes - 1;
            int64_t nr = 0;
            if (!stop) {
                for (int64_t i = 0; i < gn; i++) ref[i] = (int32_t)i;
                int32_t ri = orc_refine_sync(gn, loff, lcol, lw, M2, K, cm, ref, tau, opt->max_iterations,
                                             opt->sync_rounds, NULL, NULL);
                if (opt->split_mode == 0) {
                    /* simultaneous moves can leave a sub-community in pieces
                     * (its founder left as others joined it): split it too,
                     * so that every super-vertex is connected */
                    orc_split_bfs(gn, loff, lcol, ref, lab);
                    memcpy(ref, lab, (size_t)gn * sizeof(int32_t));
                }
                nr = orc_renumber(gn, ref, lab);
                if (stats && lp < 64) {
                    stats->refine_iterations[lp] = ri;
                    stats->refined[lp] = nr;
                }
                stop = (double)nr / (double)gn > opt->aggregation_tolerance;
            }
            if (orc_verbose)
                fprintf(stderr, "[oracle] pass %d: %lld vertices, %d iterations, %lld communities, %lld refined\n",
                        (int)lp, (long long)gn, (int)li, (long long)ng, (long long)nr);
            if (stop) {
                for (int64_t v = 0; v < n; v++) memb_out[v] = cm[memb_out[v]];
                break;
            }
            for (int64_t v = 0; v < n; v++) memb_out[v] = lab[memb_out[v]];
            for (int64_t i = 0; i < gn; i++) init[lab[i]] = cm[i];
            int64_t nn = orc_aggregate(gn, loff, lcol, lw, lab, nr, noff, ncol, nw, nnz);
            if (nn < 0) { passes = -1; break; }
            loff = noff; lcol = ncol; lw = nw;
            int64_t *to = goff; goff = noff; noff = to;
            int32_t *tc = gcol; gcol = ncol; ncol = tc;
            double *tw = gw; gw = nw; nw = tw;
            gn = nr;
            tau = tau / opt->tolerance_drop;
            continue;
        }
        /* renumber, then dendrogram lookup C <- C'[C] */
        for (int64_t v = 0; v < n; v++) memb_out[v] = cm[memb_out[v]];
        if (orc_verbose)
            fprintf(stderr, "[oracle] pass %d: %lld vertices, %d iterations, %lld communities\n", (int)lp,
                    (long long)gn, (int)li, (long long)ng);
        if (li <= 1) break;                                           /* globally converged */
        if ((double)ng / (double)gn > opt->aggregation_tolerance) break; /* low shrink */
        if (lp == opt->max_passes - 1) break;                          /* G'' would be unused */
        int64_t nn = orc_aggregate(gn, loff, lcol, lw, cm, ng, noff, ncol, nw, nnz);
        if (nn < 0) { passes = -1; break; }
        loff = noff; lcol = ncol; lw = nw;                              /* G' <- G'' */
        int64_t *to = goff; goff = noff; noff = to;                    /* the next G'' goes to the other buffer */
        int32_t *tc = gcol; gcol = ncol; ncol = tc;
        double *tw = gw; gw = nw; nw = tw;
        gn = ng;
        tau = tau / opt->tolerance_drop;                               /* threshold scaling */
    }
    if (passes > 0 && opt->sync_moves && opt->prune_params && opt->confirm_final) {
        /* the learned gate's confirmation, once per run: one plain
         * local-moving phase (no gate, every vertex unprocessed) over G from
         * the passes' result, with the last pass's tolerance; its first
         * sweep is the final full plain sweep, and further plain sweeps
         * follow while they gain more than tau.  Moves of single vertices
         * can disconnect a community, so the split (split_mode 0) follows,
         * then the renumbering. */
        int64_t c4[4];
        double *K0 = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
        orc_vertex_weights(n, off, col, w, K0);
        double tau_last = opt->tolerance;
        for (int32_t k = 1; k < passes; k++) tau_last = tau_last / opt->tolerance_drop;
        int32_t fi = orc_move_sync_gated(n, off, col, w, M2, K0, memb_out, tau_last, opt->max_iterations,
                                         opt->sync_rounds, NULL, 0.0, passes, opt->trace, NULL, NULL, c4,
                                         opt->return_moves, 1);
        if (stats) {
            stats->final_iterations = fi;
            for (int q = 0; q < 4; q++) stats->counters[q] += c4[q];
        }
        if (opt->split_mode == 0) {
            orc_split_bfs(n, off, col, memb_out, lab);
            memcpy(memb_out, lab, (size_t)n * sizeof(int32_t));
        }
        free(K0);
    }
    if (passes >= 0 && opt->split_mode == 1) {                         /* split last */
        orc_split_bfs(n, off, col, memb_out, lab);
        memcpy(memb_out, lab, (size_t)n * sizeof(int32_t));
    }
    if (passes >= 0) canonical_labels(n, memb_out);
    if (stats && passes >= 0) {
        stats->passes = passes;
        stats->modularity = orc_modularity(n, off, col, w, memb_out);
    }
    free(goff); free(gcol); free(gw); free(noff); free(ncol); free(nw);
    free(K); free(sigma); free(cm); free(lab); free(ref); free(init);
    return passes;
}
