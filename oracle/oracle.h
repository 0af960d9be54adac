/*
 * oracle.h - TEST INFRASTRUCTURE ONLY.
 *
 * Plain, sequential, fp64 CPU oracle of GSP-Louvain (Sahu, "GSP-Louvain:
 * Fast Louvain Algorithm ... for splitting disconnected communities", arXiv
 * 2402.11454).  Only the tests, the smoke check and the bench's CPU-baseline
 * leg may load it; the GPU library never includes, links or calls it, and it
 * shares no code with the GPU library.
 *
 * Graph convention (Section 3, notation): an undirected graph is given as a
 * CSR holding both directions of every edge; row i lists (j, w_ij).  A
 * self-loop is stored once, in its own row.  K_i is the full row sum, and
 * 2m (called M2 below) is the sum of all stored entries.
 *
 * Memberships and labels are int32 values in [0, n).  Weights are fp64.
 * Every function returns a negative value on invalid arguments.
 */
#ifndef GSP_ORACLE_H
#define GSP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Progress lines on stderr (iterations of the asynchronous phase, passes). */
void orc_set_verbose(int32_t on);

/* K_i = sum of row i (self-loop included), returns M2 = sum_i K_i. */
double orc_vertex_weights(int64_t n, const int64_t *off, const int32_t *col, const double *w, double *K);

/* Modularity of a membership, Eq. 1 (community form). 0 when M2 = 0. */
double orc_modularity(int64_t n, const int64_t *off, const int32_t *col, const double *w, const int32_t *memb);

/* Delta-modularity of moving i from its community to c, Eq. 2.  K_{i->x}
 * excludes i's self-loop; Sigma_d includes K_i. */
double orc_delta_modularity(int64_t n, const int64_t *off, const int32_t *col, const double *w,
                            const int32_t *memb, int64_t i, int32_t c);

/* Asynchronous sequential local-moving phase (Algorithm "louvainMove", one
 * thread).  memb/sigma are updated in place; returns l_i (iterations run)
 * and writes the per-iteration delta-modularity sums to dq_iter (length
 * max_iter, may be NULL). */
int32_t orc_move_async(int64_t n, const int64_t *off, const int32_t *col, const double *w, double M2,
                       const double *K, int32_t *memb, double *sigma, double tau, int32_t max_iter,
                       double *dq_iter);

/* One synchronous move step from a snapshot (memb, sigma, csize); vertices
 * with active[i] = 0 keep their community (active NULL = all).  Writes the
 * chosen community (or the current one) to dec and the integer-style gain
 * numerator G(c*) - G(stay) to gain (0 for non-movers).  Returns the number
 * of movers. */
int64_t orc_move_sync_step(int64_t n, const int64_t *off, const int32_t *col, const double *w, double M2,
                           const double *K, const int32_t *memb, const double *sigma, const int32_t *csize,
                           const uint8_t *active, int32_t *dec, double *gain);

/* The synchronous decision of vertex i from its row alone (rule of
 * orc_move_sync_step); scores[3] (may be NULL) receives the best and second
 * candidate scores and G(stay).  Returns the chosen community. */
int32_t orc_decide_row(int64_t i, int64_t deg, const int32_t *cols, const double *w, const int32_t *memb,
                       const double *sigma, const int32_t *csize, double ki, double M2, double *gain,
                       double *scores);

/* Weight grid (exact sums): every weight becomes the nearest multiple of
 * 2^-S, S the largest integer with (an exact upper bound of 2m) * 2^S <
 * 2^52; returns S, *changed = weights that moved (may be NULL). */
int32_t orc_weight_grid(int64_t nnz, double *w, int64_t *changed);

/* A mover's gain numerator as its share of the iteration's gain total:
 * round(2^61 * 2 gain / M2^2) (the total is the exact sum of these). */
int64_t orc_gain_fixed(double gain, double M2);

/* Synchronous local-moving phase in `rounds` ordered sub-rounds (a power of
 * two, 1..64): vertex i belongs to sub-round (i * 0x9E3779B97F4A7C15) >> (64 -
 * log2 rounds).  Each sub-round is one snapshot step over the unprocessed
 * vertices of its group; movers mark their neighbours unprocessed.  memb is
 * updated in place; returns l_i; dq_iter and moved_iter (length max_iter,
 * may be NULL) receive the per-iteration delta-modularity sums and mover
 * counts. */
int32_t orc_move_sync(int64_t n, const int64_t *off, const int32_t *col, const double *w, double M2,
                      const double *K, int32_t *memb, double tau, int32_t max_iter, int32_t rounds,
                      double *dq_iter, int64_t *moved_iter,
                      int32_t returns);

/* Refinement phase of GSP-Leiden (Section 3.5, greedy reading): within
 * each bound community, vertices alone in their sub-community join the
 * sub-community of a same-bound neighbour of largest delta-modularity, in
 * the ordered synchronous sub-rounds of orc_move_sync.  bound[n] holds the
 * local-moving communities; memb (starting sub-communities, each inside one
 * bound; normally memb[i] = i) is updated in place.  Returns the iterations
 * run; dq_iter / moved_iter as for orc_move_sync. */
int32_t orc_refine_sync(int64_t n, const int64_t *off, const int32_t *col, const double *w, double M2,
                        const double *K, const int32_t *bound, int32_t *memb, double tau, int32_t max_iter,
                        int32_t rounds, double *dq_iter, int64_t *moved_iter);

/* Split of internally-disconnected communities by BFS (Algorithm
 * "splitDisconnectedBfs", one thread, lowest unvisited source):
 * labels[i] = smallest vertex id of i's component in the same-community
 * subgraph. */
int32_t orc_split_bfs(int64_t n, const int64_t *off, const int32_t *col, const int32_t *memb, int32_t *labels);

/* Same split by minimum-label propagation (Algorithm "splitDisconnectedLp"),
 * pruned = 1 for LPP.  Returns the number of sweeps. */
int32_t orc_split_lp(int64_t n, const int64_t *off, const int32_t *col, const int32_t *memb, int32_t pruned,
                     int32_t *labels);

/* Renumbers labels (values in [0, n)) to [0, G) in ascending label order;
 * returns G. */
int64_t orc_renumber(int64_t n, const int32_t *labels, int32_t *out);

/* Aggregation (Algorithm "louvainAggregate"): memb holds values in
 * [0, ncomm).  Writes the super-vertex CSR: off2[ncomm+1], col2/w2 with
 * room for cap entries, rows sorted by column.  Returns its entry count, or
 * -1 if cap is too small. */
int64_t orc_aggregate(int64_t n, const int64_t *off, const int32_t *col, const double *w, const int32_t *memb,
                      int64_t ncomm, int64_t *off2, int32_t *col2, double *w2, int64_t cap);

/* Disconnected communities (Algorithm "disconnectedCommunities", one
 * thread): flags[c] = 1 if community c is internally disconnected (flags
 * has length n, may be NULL).  Returns the number of such communities. */
int64_t orc_disconnected(int64_t n, const int64_t *off, const int32_t *col, const int32_t *memb, uint8_t *flags);

/* ---- learned pruning gate (prune.c) ---- */

#define ORC_MLP_PARAMS 4801  /* (8*64 + 64) + (64*64 + 64) + (64 + 1) */

/* bf16 (round to nearest even) of an fp32 value, as fp32. */
float orc_bf16(float x);

/* Piecewise-linear log2 for x >= 1 (0 below): e + x / 2^e - 1. */
double orc_plog2(double x);

/* The gate's 8 features of a vertex (see prune.c), bf16 values as fp32. */
void orc_gate_features(int64_t deg, double ki, double sig_d, float hfrac, float hgain, uint8_t hbits, double dmoved,
                       int32_t pass, int32_t iter, float *x);

/* Logits of rows x[rows][8]; bf16 = 1 emulates the inference formats. */
void orc_mlp_logits(const float *params, const float *x, int64_t rows, int32_t bf16, double *out);

/* Mean pos-weighted BCE and its gradient (grad[ORC_MLP_PARAMS], may be
 * NULL), fp64; _f64 takes fp64 parameters, _f32 computes in fp32. */
double orc_mlp_loss_grad(const float *params, const float *x, const uint8_t *y, int64_t rows, double pos_weight,
                         double *grad);
double orc_mlp_loss_grad_f64(const double *params, const float *x, const uint8_t *y, int64_t rows,
                             double pos_weight, double *grad);
float orc_mlp_loss_grad_f32(const float *params, const float *x, const uint8_t *y, int64_t rows, float pos_weight,
                            float *grad);

/* Adam over contiguous mini-batches, `epochs` passes (fp64). */
int64_t orc_mlp_train_adam(float *params, const float *x, const uint8_t *y, int64_t rows, int64_t batch,
                           int32_t epochs, double lr, double pos_weight, double *epoch_loss);

/* Trace sampling predicate: mix64(seed ^ pass<<56 ^ sweep<<48 ^ i) < threshold. */
int32_t orc_trace_keep(uint64_t seed, int32_t pass, int32_t sweep, int64_t i, uint64_t threshold);

typedef struct orc_trace {
    uint64_t seed, threshold;  /* sampling (orc_trace_keep) */
    int64_t cap;               /* rows the buffers hold */
    float *x;                  /* [cap][8] features before the scan */
    uint8_t *y;                /* [cap] 1 if the vertex moved */
    int32_t *vertex;           /* [cap] vertex id at its level */
    int32_t *meta;             /* [cap] pass * 256 + sweep */
    int64_t rows;              /* rows written (<= cap) */
    int64_t seen;              /* rows kept by the sampling (may exceed cap) */
} orc_trace;

/* Synchronous phase with the learned gate and confirming sweep (prune.c);
 * params = NULL runs it plain.  counters (4, may be NULL): scanned
 * vertices, scanned entries, pruned vertices, confirming sweeps. */
int32_t orc_move_sync_gated(int64_t n, const int64_t *off, const int32_t *col, const double *w, double M2,
                            const double *K, int32_t *memb, double tau, int32_t max_iter, int32_t rounds,
                            const float *params, double theta_logit, int32_t pass, orc_trace *trace,
                            double *dq_iter, int64_t *moved_iter, int64_t *counters,
                            int32_t returns, int32_t confirm);

typedef struct orc_options {
    double tolerance;              /* tau for the first pass */
    int32_t max_passes;
    int32_t max_iterations;
    double tolerance_drop;
    double aggregation_tolerance;  /* tau_agg */
    int32_t sync_moves;            /* 0: asynchronous sequential, 1: synchronous sub-rounds */
    int32_t sync_rounds;           /* sub-rounds per iteration when sync_moves = 1 */
    int32_t split_mode;            /* 0: every pass (SP), 1: after the last pass (SL), 2: none */
    const float *prune_params;     /* learned gate (sync_moves = 1 only), NULL = plain */
    double prune_theta_logit;      /* scan iff logit >= this */
    orc_trace *trace;              /* move traces (sync_moves = 1 only), may be NULL */
    int32_t return_moves;          /* sync_moves = 1: return moves add nothing to the gain total (option) */
    int32_t confirm_final;         /* with prune_params: no confirming sweep per pass; after the passes one
                                      plain local-moving phase over G from the result, then the split */
    int32_t leiden;                /* 1: GSP-Leiden (sync_moves = 1, no gate, no trace): each pass refines the
                                      split communities (orc_refine_sync), splits the refined ones too
                                      (split_mode 0) and aggregates them; they start the next pass in
                                      their community */
} orc_options;

typedef struct orc_stats {
    int32_t passes;
    int32_t iterations[64];        /* l_i per pass */
    int64_t communities[64];       /* |Gamma| after each pass's split */
    int64_t vertices[64];          /* N' of each pass */
    double modularity;
    int64_t counters[4];           /* gated phase: scanned vertices, scanned entries, pruned, confirming sweeps */
    double tau[64];                /* the iteration tolerance each pass ran with (threshold scaling) */
    int32_t final_iterations;      /* confirm_final: iterations of the final plain phase over G */
    int32_t refine_iterations[64]; /* leiden: iterations of each pass's refinement (0 if none ran) */
    int64_t refined[64];           /* leiden: refined sub-communities of each pass (0 if none ran) */
} orc_stats;

/* The whole method (Algorithm "louvain"; with opt->leiden, GSP-Leiden).
 * memb_out[n] gets the top-level membership, numbered by ascending smallest
 * vertex id.  Returns the number of passes run. */
int32_t orc_louvain(int64_t n, const int64_t *off, const int32_t *col, const double *w, const orc_options *opt,
                    int32_t *memb_out, orc_stats *stats);

#ifdef __cplusplus
}
#endif
#endif
