/*
 * gsp.h - C ABI of the GSP-Louvain library for AMD Instinct MI355X (gfx950).
 *
 * GSP-Louvain (Sahu, arXiv 2402.11454) finds disjoint communities of an
 * undirected weighted graph by modularity maximisation (Eq. 1).  Each pass of
 * Algorithm "louvain" runs the local-moving phase (Algorithm "louvainMove",
 * gains by Eq. 2), splits every internally-disconnected community into its
 * connected parts (Section 4.1, split in every pass), renumbers the
 * communities, updates the top-level membership (dendrogram lookup) and
 * aggregates the communities into super-vertices (Algorithm
 * "louvainAggregate").  This library runs every step on one GPU.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 * - Graphs are CSR with both directions of every undirected edge stored
 *   (Section 3: w_ij = w_ji).  A self-loop is stored once, in its own row.
 *   Offsets are int64 (n+1 entries, offsets[0] = 0, non-decreasing,
 *   offsets[n] = nnz); columns are int32 in [0, n); weights are finite and
 *   >= 0, fp32 or fp64, or NULL for unit weights.  Rows may be unsorted.
 *   K_i is the row sum; 2m (M2) is the sum of all entries.
 * - `where` says where a pointer lives: GSP_HOST (pageable or pinned host
 *   memory) or GSP_DEVICE (device memory on the context's GPU).
 * - Memberships and labels are int32 values in [0, n).
 * - Inputs are copied or only read during the call; the caller keeps
 *   ownership of every buffer it passes.  Outputs go to caller buffers.
 * - Every function returns a gsp_status.  On failure the context keeps a
 *   message readable with gsp_last_error(); no exception or abort crosses
 *   the ABI.  GSP_EHIP carries the HIP runtime's error string.
 * - All GPU work is ordered on the context's stream; every entry point
 *   returns after its work has completed (host outputs are valid, device
 *   outputs are written).
 * - A context is not thread-safe: calls on one context must not overlap.
 */
#ifndef GSP_H
#define GSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsp_ctx gsp_ctx;

typedef enum gsp_status {
    GSP_OK = 0,
    GSP_EINVAL = -1,  /* bad argument (NULL pointer, negative size, label out of range) */
    GSP_ENOMEM = -2,  /* device allocation failed or exceeds mem_limit_bytes */
    GSP_EHIP = -3,    /* HIP runtime error */
    GSP_ESTATE = -4,  /* call out of order (no graph loaded, no result yet) */
    GSP_EGRAPH = -5   /* malformed CSR (offsets, columns, weights) */
} gsp_status;

enum { GSP_HOST = 0, GSP_DEVICE = 1 };

/* When the split of internally-disconnected communities runs (Section 4.1). */
enum { GSP_SPLIT_PASS = 0, GSP_SPLIT_LAST = 1, GSP_SPLIT_NONE = 2 };

#define GSP_MAX_PASSES_STATS 64

typedef struct gsp_options {
    int32_t max_iterations;        /* MAX_ITERATIONS of the local-moving phase (default 20) */
    int32_t sub_rounds;            /* ordered sub-rounds per iteration, power of two 1..64 (default 8) */
    double tolerance_drop;         /* TOLERANCE_DROP of threshold scaling (default 10) */
    double aggregation_tolerance;  /* tau_agg: stop when |Gamma|/N' exceeds it (default 0.8) */
    int32_t split_mode;            /* GSP_SPLIT_PASS (default), GSP_SPLIT_LAST or GSP_SPLIT_NONE */
    int32_t timing;                /* 0: none; 1: per-phase HIP-event times; 2: also per-kernel times
                                      (then a sweep's independent scans run one after another instead of
                                      side by side on four streams, so each event pair times one kernel);
                                      3: per-kernel times with the scans side by side (each event pair on
                                      its kernel's stream: the kernel's time as it runs beside the others) */
    uint64_t mem_limit_bytes;      /* refuse device allocations beyond this total (0 = no limit) */
    int32_t prune_mode;            /* GSP_PRUNE_PLAIN (default) or GSP_PRUNE_LEARNED (network set by gsp_pruner_set) */
    float prune_threshold;         /* learned gate: scan a vertex iff p = sigmoid(z) >= this (default 0.5) */
    int32_t use_graphs;            /* 1 (default): replay each pass's plain sweeps from a captured HIP graph */
    uint32_t timing_mask;          /* timing = 2: bit k times kernel class k only (0 = every class) */
    int32_t hub_global;            /* 1: score every hub through global hash tables (default 0: LDS hash
                                      partitions, global tables only for hubs that do not fit them) */
    int32_t hub_max_parts;         /* hubs with more chunks of 2048 entries than this go through their
                                      global table (0 = the limit, 4096; values in [0, 4096]) */
    int32_t return_moves;          /* 0 (default): every mover's gain counts towards the iteration's total,
                                      the tolerance test of Algorithm louvainMove as written; 1: a move back
                                      into the community the vertex left at its move of the preceding sweep
                                      is made but adds nothing, so swap cycles of synchronous moves do not
                                      hold a pass at max_iterations */
    int32_t split_algo;            /* how the split (Section 4.1) finds the components: GSP_SPLIT_UF
                                      (default: concurrent union-find) or GSP_SPLIT_LPP (minimum-label
                                      propagation with pruning, Algorithm splitDisconnectedLp, plus pointer
                                      jumping); both give the same labels */
    int32_t grid_cap;              /* launch schedule: the local-moving scans and apply take at most this many
                                      workgroups each (0, the default: each kernel's own cap, 2048-8192);
                                      results do not depend on it */
    int32_t vertex_order;          /* storage order of the input graph inside gsp_run: GSP_ORDER_AUTO
                                      (default: degree order for graphs of at least 2^25 entries whose
                                      copy fits mem_limit_bytes),
                                      GSP_ORDER_LOADED or GSP_ORDER_DEGREE (vertices renumbered by degree,
                                      largest first, so that the high-degree vertices' words share cache
                                      lines).  The copy in degree order is built by the first run that asks
                                      for it and kept until the next load (device memory: about as much
                                      as the loaded graph).  Results do not depend on it: every rule that
                                      orders vertex or community ids compares the caller's ids.  Batches
                                      and the step entry points use the loaded order. */
    int32_t leiden;                /* 1: GSP-Leiden (the Leiden algorithm's refinement, Section 3.5, taken
                                      greedily, with the split of Section 4.1): after each pass's local
                                      moving and split, a refinement phase runs inside every community
                                      (a vertex alone in its sub-community joins the sub-community of a
                                      same-community neighbour of largest delta-modularity, Eq. 2, in the
                                      same ordered synchronous sub-rounds and tolerance test); with
                                      GSP_SPLIT_PASS the refined sub-communities are split too; they become
                                      the next level's super-vertices, each starting in the community that
                                      holds it.  The result is the local-moving communities.  Single graphs
                                      only, plain pruning, no trace capture (else GSP_EINVAL).
                                      0 (default): GSP-Louvain. */
} gsp_options;

/* split_algo values. */
enum { GSP_SPLIT_UF = 0, GSP_SPLIT_LPP = 1 };

/* vertex_order values. */
enum { GSP_ORDER_AUTO = 0, GSP_ORDER_LOADED = 1, GSP_ORDER_DEGREE = 2 };

/* Vertex pruning of the local-moving phase (prune_mode). */
enum { GSP_PRUNE_PLAIN = 0, GSP_PRUNE_LEARNED = 1 };

/* Per-kernel counters (timing = 2), one class per kernel of the hot path. */
enum {
    GSP_K_MOVE_SMALL = 0,  /* local-move scan+decide, degree <= 64 (lane groups) */
    GSP_K_MOVE_WAVE,       /* local-move scan+decide, 64 < degree <= 512 (a wavefront per vertex) */
    GSP_K_MOVE_BLOCK,      /* local-move scan+decide, 512 < degree <= 2048 (a workgroup per vertex) */
    GSP_K_MOVE_HUB,        /* local-move scan of hubs (degree > 2048): each chunk reduced in LDS and its
                              pairs staged by hash partition (or inserted into global tables) */
    GSP_K_MOVE_HUB_FINISH, /* hub decisions: partial results combined (and the global-table path) */
    GSP_K_MOVE_APPLY,      /* apply moves, community totals */
    GSP_K_FRONTIER,        /* sub-round queue compaction */
    GSP_K_SPLIT,           /* split: union-find hooking and compression */
    GSP_K_AGGREGATE,       /* aggregation kernels */
    GSP_K_GATE,            /* learned gate: features and the network (bf16 matrix cores) */
    GSP_K_MOVE_HUB_GATHER, /* hub partitions: each partition's pairs merged in LDS and scored */
    GSP_K_COUNT
};

typedef struct gsp_kernel_stat {
    int64_t launches;
    double ms;             /* summed HIP-event time of the launches */
    double bytes;          /* algorithmic bytes of those launches (see the library's notes) */
    int64_t items;         /* work items: scanned entries for the move kernels */
} gsp_kernel_stat;

typedef struct gsp_stats {
    int32_t passes;
    int32_t iterations[GSP_MAX_PASSES_STATS];  /* l_i of each pass */
    int64_t vertices[GSP_MAX_PASSES_STATS];    /* N' of each pass */
    int64_t communities[GSP_MAX_PASSES_STATS]; /* |Gamma| after each pass's split */
    int64_t moves;                             /* vertices moved, all passes */
    int64_t scanned_entries;                   /* CSR entries scanned by the local-moving phase */
    double ms_move, ms_split, ms_aggregate, ms_other, ms_total;  /* timing >= 1 */
    gsp_kernel_stat kernels[GSP_K_COUNT];       /* timing = 2 */
    int64_t scanned_vertices;                  /* vertices scanned by the local-moving phase, all passes */
    int64_t pruned;                            /* unprocessed vertices the learned gate kept from the scan */
    int32_t confirm_sweeps;                    /* confirming plain sweeps run after gated convergence */
    int32_t sweeps;                            /* local-moving sweeps run, all passes (counted or not) */
    int32_t split_rounds;                      /* split_algo = GSP_SPLIT_LPP: propagation rounds, all splits */
    int32_t refine_iterations[GSP_MAX_PASSES_STATS]; /* leiden: iterations of each pass's refinement (0: none) */
    int64_t refined[GSP_MAX_PASSES_STATS];     /* leiden: sub-communities of each pass's refinement, after
                                                  their split (0: none ran) */
    double ms_refine;                          /* leiden, timing >= 1: refinement phases (the same-community
                                                  subgraph included; their splits count as split time) */
} gsp_stats;

/* Fills *out with the defaults above. */
gsp_status gsp_default_options(gsp_options *out);

/* Creates a context on HIP device `device`.  hip_stream is a hipStream_t to
 * run on (the caller keeps it alive for the context's life), or NULL for a
 * stream the context creates (default priority) and destroys. */
gsp_status gsp_create(int device, void *hip_stream, gsp_ctx **out);

/* Frees every device buffer of the context and the context itself. */
gsp_status gsp_destroy(gsp_ctx *ctx);

/* Last error message of the context ("" if none).  Valid until the next call
 * on the context.  Accepts NULL (returns a static message). */
const char *gsp_last_error(const gsp_ctx *ctx);

/* Loads the graph G (Section 3) and validates it on the device: offsets
 * start at 0, never decrease and end at nnz; columns lie in [0, n); weights
 * are finite and >= 0.  A malformed graph gives GSP_EGRAPH and leaves no
 * graph loaded.  n must lie in [1, 2^31 - 2] and nnz be >= 0 (an empty
 * graph has no community to find): otherwise GSP_EINVAL, and the graph
 * loaded before, if any, stays.  Symmetry is the caller's promise and is not checked.
 * Replaces any graph loaded before and frees the previous result.
 * weights = NULL means unit weights. */
gsp_status gsp_load_csr(gsp_ctx *ctx, int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols,
                        const float *weights, int where);

/* Exact sums.  Section 5.1.2 keeps edge weights in fp32 and computes in
 * fp64; a sum of fp32 weights is exact in fp64 only while it stays below
 * 2^53 units of its finest weight, and beyond that a parallel sum depends on
 * its order.  Every load therefore takes the weights onto a grid: each
 * weight becomes the nearest multiple of 2^-S (ties to even), with S the
 * largest integer (in [-1000, 1022]) such that an exact upper bound U of the
 * weight total has U 2^S < 2^52 (U = 2^-T sum of max(1, ceil(w 2^T)) over
 * the positive weights, T = 62 - bits(nnz) - e, max weight < 2^e).  Every
 * sum or difference of weights the method forms (K_i, 2m, Sigma_c and its
 * updates, K_{i->c}, super-vertex weights) is then exact, so results do not
 * depend on the order of the GPU's atomics.  Unit weights, and fp32
 * weights of a few units on graphs below about 2^28 entries, do not move;
 * weights in [1, 10) on 2^31 entries move by at most 2^-19.  A batch takes
 * one grid per graph (its own total). */

/* Same with int32 offsets (graphs below 2^31 entries). */
gsp_status gsp_load_csr32(gsp_ctx *ctx, int32_t n, int32_t nnz, const int32_t *offsets, const int32_t *cols,
                          const float *weights, int where);

/* Same with fp64 weights (e.g. super-vertex graphs with self-loops). */
gsp_status gsp_load_csr_f64(gsp_ctx *ctx, int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols,
                            const double *weights, int where);

/* Runs GSP-Louvain (Algorithm "louvain") on the loaded graph with iteration
 * tolerance `tolerance` (tau of the first pass) and at most max_passes
 * passes (max_passes = 0 leaves every vertex alone).  opt = NULL uses
 * gsp_default_options.  The local-moving phase is synchronous in ordered
 * sub-rounds: vertex i belongs to sub-round (i * 0x9E3779B97F4A7C15) >> (64 -
 * log2 sub_rounds); within a sub-round every decision comes from one
 * snapshot of memberships and community totals; ties go to the lowest
 * community id; a vertex moves only for a positive gain, and a vertex alone
 * in its community does not join another one-vertex community with a larger
 * id.  Communities of the result are numbered by ascending smallest vertex
 * id.  The result stays in the context until the next load or run. */
gsp_status gsp_run(gsp_ctx *ctx, double tolerance, int32_t max_passes, const gsp_options *opt);

/* Copies the last run's membership (n values) to out. */
gsp_status gsp_get_membership(gsp_ctx *ctx, int32_t *out, int where);

/* Modularity (Eq. 1) of the last run's membership. */
gsp_status gsp_get_modularity(gsp_ctx *ctx, double *out);

/* The loaded graph's weight grid: weights are multiples of 2^-*scale_exp
 * (the smallest exponent over a batch's graphs; 0 for unit weights), and
 * *moved weights were rounded onto it. */
gsp_status gsp_get_weight_grid(gsp_ctx *ctx, int32_t *scale_exp, int64_t *moved);

/* Statistics of the last run. */
gsp_status gsp_get_stats(gsp_ctx *ctx, gsp_stats *out);

/* Modularity (Eq. 1, community form) of `membership` on the loaded graph,
 * in fp64.  Labels outside [0, n) give GSP_EINVAL. */
gsp_status gsp_modularity(gsp_ctx *ctx, const int32_t *membership, int where, double *out);

/* Number of communities of `membership` that are internally disconnected
 * (Algorithm "disconnectedCommunities"). */
gsp_status gsp_count_disconnected(gsp_ctx *ctx, const int32_t *membership, int where, int64_t *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the count
 * of gsp_count_disconnected for a CSR and a membership given in device
 * memory, with no context and no allocation.  offsets (int64, n + 1),
 * cols (int32, nnz), membership (int32, n) and count_out (one int64) are
 * device pointers on the current device; the work is enqueued on
 * hip_stream (NULL: the null stream) and *count_out is written when the
 * stream reaches it (the call does not wait).  The inputs are not
 * validated on the host: an offset, column or label out of range gives
 * *count_out = -1 (every access is checked on the device).
 * Scratch is a fixed 64 MiB array in device memory (8 bytes per vertex),
 * held by each GPU the library runs on until the process ends and shared
 * by every call on that GPU: calls that overlap on one GPU race (order them
 * on one stream).  n above gsp_noalloc_max_vertices() (8,388,576) gives
 * GSP_EINVAL, as do negative sizes and NULL pointers; a launch failure
 * gives GSP_EHIP.  No context, so there is no gsp_last_error message. */
gsp_status gsp_count_disconnected_noalloc(int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols,
                                          const int32_t *membership, int64_t *count_out, void *hip_stream);

/* The largest n gsp_count_disconnected_noalloc accepts. */
int64_t gsp_noalloc_max_vertices(void);

/* ---- stepwise hooks on the loaded graph (used to check each step) ---- */

/* One synchronous local-moving step (Algorithm "louvainMove", gains by
 * Eq. 2) from the snapshot given by `membership`: community totals and
 * sizes are computed from it.  Vertices with active[i] = 0 stay (active =
 * NULL: all).  dec_out[i] receives the chosen community (or the current
 * one), gain_out[i] the gain numerator G(c*) - G(stay) with
 * G(c) = M2 K_{i->c} - K_i Sigma_c and G(stay) = M2 K_{i->d} - K_i (Sigma_d - K_i)
 * (0 for vertices that stay; gain_out may be NULL), *moved the number of
 * movers.  All pointers share `where`. */
gsp_status gsp_step_move(gsp_ctx *ctx, const int32_t *membership, const uint8_t *active, int where,
                         int32_t *dec_out, double *gain_out, int64_t *moved);

/* The whole local-moving phase (iterations of ordered sub-rounds, as in
 * gsp_run) on the loaded graph, starting from `membership_inout` (updated
 * in place).  Returns l_i in *iterations; dq_iter / moved_iter (length
 * max_iterations, may be NULL) receive each iteration's gain total
 * (delta-modularity) and mover count.  Host pointers for the per-iteration
 * arrays; `where` applies to membership_inout. */
gsp_status gsp_move_phase(gsp_ctx *ctx, int32_t *membership_inout, int where, double tolerance,
                          int32_t max_iterations, int32_t sub_rounds, int32_t *iterations, double *dq_iter,
                          int64_t *moved_iter);

/* Split of internally-disconnected communities (Section 4.1): labels_out[i]
 * = smallest vertex id of i's connected component in the subgraph of edges
 * whose ends share a community. */
gsp_status gsp_step_split(gsp_ctx *ctx, const int32_t *membership, int where, int32_t *labels_out);

/* The same split by minimum-label propagation with pruning (Algorithm
 * "splitDisconnectedLp" with its pruning, plus pointer jumping: see
 * split_algo); *rounds (may be NULL) receives the propagation rounds. */
gsp_status gsp_step_split_lp(gsp_ctx *ctx, const int32_t *membership, int where, int32_t *labels_out,
                             int32_t *rounds);

/* Aggregation (Algorithm "louvainAggregate") of the loaded graph by
 * `membership` after renumbering its labels in ascending order: super-vertex
 * c of G'' is the c-th smallest label.  Row c holds (d, w) with w the sum of
 * w_ij over entries with i in c and j in d (self-loops kept), fp64, in no
 * particular order.  With offsets = NULL only *n_out and *nnz_out are set;
 * otherwise offsets (n_out + 1), cols and weights (nnz_out) are filled. */
gsp_status gsp_step_aggregate(gsp_ctx *ctx, const int32_t *membership, int where, int64_t *n_out,
                              int64_t *nnz_out, int64_t *offsets, int32_t *cols, double *weights);

/* The local-moving phase alone with the run's options (learned gate
 * included): as gsp_move_phase, with opt = NULL for the defaults and
 * pass_index (0..255) the pass the phase stands for (a gate feature and the
 * pass recorded in trace rows).  dq_iter / moved_iter have room for
 * opt->max_iterations values and receive the counted iterations; counters
 * (4 values, may be NULL): vertices scanned, CSR entries scanned, vertices
 * pruned by the gate, confirming sweeps run. */
gsp_status gsp_move_phase_ex(gsp_ctx *ctx, int32_t *membership_inout, int where, double tolerance, int32_t pass_index,
                             const gsp_options *opt, int32_t *iterations, double *dq_iter, int64_t *moved_iter,
                             int64_t *counters);

/* GSP-Leiden's refinement phase on the loaded graph (the Leiden algorithm's
 * refinement, Section 3.5, taken greedily; gsp_options.leiden).  bound
 * (n labels in [0, n)) holds the communities of a local-moving phase;
 * membership_inout holds the starting sub-communities, each inside one bound
 * community (normally membership[i] = i), and receives the refined ones as
 * labels (founding vertex ids, not renumbered).  In every iteration's
 * ordered sub-rounds a vertex alone in its sub-community takes the
 * sub-community of a neighbour in its bound community with the largest
 * delta-modularity (Eq. 2 with the whole graph's K and 2m; ties to the
 * lowest id; a positive gain; the singleton rule of gsp_move_phase); movers
 * mark their same-community neighbours; the iterations stop as
 * gsp_move_phase's do.  Uses opt's max_iterations, sub_rounds, use_graphs,
 * grid_cap and hub options (opt = NULL: the defaults); prune_mode must be
 * GSP_PRUNE_PLAIN.  iterations, dq_iter and moved_iter as for
 * gsp_move_phase.  Both arrays live where `where` says.  GSP_EINVAL for a
 * label outside [0, n), a sub-community across two bound communities, or
 * trace capture on (gsp_capture_traces). */
gsp_status gsp_refine_phase(gsp_ctx *ctx, const int32_t *bound, int32_t *membership_inout, int where,
                            double tolerance, const gsp_options *opt, int32_t *iterations, double *dq_iter,
                            int64_t *moved_iter);

/* ---- batches of independent graphs ----
 *
 * Many graphs (e.g. hundreds of uneven sizes) are run together: every
 * kernel of the method processes all of them in one launch, as one
 * block-diagonal level, while each graph keeps its own 2m (Eq. 1 and 2 use
 * it), its own per-iteration gain total and tolerance test, its own l_i and
 * its own pass-level tests (Algorithm "louvain"); a graph that has finished
 * stays still while the others go on.  Sub-rounds are taken by the vertex's
 * id within its graph, so every graph's result is the one gsp_run gives for
 * it alone, with or without learned pruning (each graph runs its own gated,
 * confirming and plain sweeps). */

/* Loads `graphs` host CSRs (graph k: n[k] >= 1 vertices, nnz[k] entries,
 * offsets[k] int64 [n[k]+1], cols[k] int32 in [0, n[k]), weights[k] fp32 or
 * NULL; weights itself may be NULL for all-unit weights).  The sum of n
 * must stay below 2^31 - 1.  Replaces any graph loaded before. */
gsp_status gsp_load_batch(gsp_ctx *ctx, int32_t graphs, const int64_t *n, const int64_t *nnz,
                          const int64_t *const *offsets, const int32_t *const *cols, const float *const *weights);

/* Runs the method on every graph of the loaded batch (arguments as gsp_run). */
gsp_status gsp_run_batch(gsp_ctx *ctx, double tolerance, int32_t max_passes, const gsp_options *opt);

/* Membership of graph `graph` (n[graph] values, communities numbered by
 * ascending smallest vertex id within the graph). */
gsp_status gsp_get_batch_membership(gsp_ctx *ctx, int32_t graph, int32_t *out, int where);

/* Modularity (Eq. 1, the graph's own 2m) of every graph's result: q_out
 * has one value per graph (host).  Computed on the device at the first call
 * after a run (an evaluation, not part of gsp_run_batch). */
gsp_status gsp_get_batch_modularity(gsp_ctx *ctx, double *q_out);

/* Passes each graph took part in (host, one value per graph). */
gsp_status gsp_get_batch_passes(gsp_ctx *ctx, int32_t *passes_out);

/* ---- learned vertex pruning ----
 *
 * Not part of the paper.  In a run with prune_mode = GSP_PRUNE_LEARNED every
 * unprocessed vertex of a sweep (the vertices Algorithm "louvainMove" would
 * scan after Section 4.1's pruning) first goes through a small network
 * z = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 (8 -> 64 -> 64 -> 1) on 8
 * features that need no scan of its row:
 *   x0 = plog2(1 + row length) / 16, with plog2(v) = e + v / 2^e - 1 for
 *        2^e <= v < 2^(e+1);
 *   x1 = K_{i->d} / K_i at the vertex's last scan in this pass (0 before);
 *   x2 = (G(best) - G(stay)) / (M2 K_i) at that scan, clipped to [-1, 1]
 *        (-1 with no candidate community, 0 for K_i = 0);
 *   x3 = min(pass, 8) / 8;  x4 = min(l, 20) / 20 with l the iterations
 *        counted so far in the pass;
 *   x5 = K_i / Sigma_{C_i} (0 if either is 0);
 *   x6 = 0 if not scanned yet in this pass, 1/2 if it stayed at its last
 *        scan, 1 if it moved;
 *   x7 = min(D_i / K_i, 1) with D_i the weight of the entries (i, j) whose
 *        j moved since the vertex's last scan (or since the pass began; a
 *        pruned vertex keeps it);
 * each computed in fp64 and rounded to fp32, then to bf16 (round to nearest
 * even).  The vertex is scanned iff z >= log(theta / (1 - theta)), theta =
 * prune_threshold; otherwise it keeps its community.  Inference uses bf16
 * weights (W1, W2, w3) and bf16 first-layer outputs with fp32 accumulation.
 * When a gated sweep's gain total is <= tau, a confirming sweep scans every
 * vertex with no gate: if its total is <= tau as well the phase ends,
 * otherwise plain sweeps continue until the usual test stops them.  A
 * confirming sweep that moves no vertex does not count towards l_i or
 * max_iterations.  Vertices with empty rows are never gated or scanned. */

/* Parameters: 4801 fp32 values, W1 [64][8] row-major, b1[64], W2 [64][64]
 * (row = output unit), b2[64], w3[64], b3.  The context keeps the network
 * (in its inference formats) across loads until the next call.  Non-finite
 * values give GSP_EINVAL. */
gsp_status gsp_pruner_set(gsp_ctx *ctx, const float *params, int64_t count, int where);

/* Logits of feature rows x[rows][8] (rounded to bf16 on the device) by the
 * inference kernel, into logits[rows] (fp32).  Needs gsp_pruner_set. */
gsp_status gsp_gate_logits(gsp_ctx *ctx, const float *x, int64_t rows, float *logits, int where);

/* Mean pos-weighted binary cross-entropy of rows (x[rows][8], y[rows] in
 * {0, 1}) at `params` and its gradient grad_out[4801], by the fp32 training
 * kernels:  L = (1/B) sum_r [pw y_r log(1 + e^{-z_r}) + (1 - y_r) log(1 + e^{z_r})].
 * All array pointers share `where`; *loss_out may be NULL. */
gsp_status gsp_pruner_grad(gsp_ctx *ctx, const float *params, const float *x, const uint8_t *y, int64_t rows,
                           float pos_weight, float *grad_out, double *loss_out, int where);

/* Trains the network on the GPU: Adam (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias-corrected) over mini-batches [k*batch, (k+1)*batch) of the rows in
 * the order given, `epochs` passes, learning rate lr, fp32 throughout.
 * params_inout (host, 4801 values) holds the starting point and receives the
 * result; epoch_loss (host, `epochs` values, may be NULL) the mean batch loss
 * of each epoch, each batch's loss taken before its update.  x and y live
 * where `where` says. */
gsp_status gsp_pruner_train(gsp_ctx *ctx, const float *x, const uint8_t *y, int64_t rows, int64_t batch,
                            int32_t epochs, float lr, float pos_weight, float *params_inout, double *epoch_loss,
                            int where);

/* Move traces, the network's training data.  capacity > 0 starts recording
 * (dropping earlier rows) in later gsp_run / gsp_move_phase_ex calls;
 * capacity <= 0 stops and frees.  A scan of vertex i in sweep s of pass p is
 * recorded with probability `rate`: iff SplitMix64's output step applied to
 * seed ^ (p << 56) ^ (s << 48) ^ i is below rate * 2^64.  A row is the
 * vertex's 8 features before the scan, 1 if it moved, its id at its level
 * and p * 256 + s.  Rows land in 16 regions of capacity/16 rows (rounded up);
 * a full region drops its further rows. */
gsp_status gsp_capture_traces(gsp_ctx *ctx, int64_t capacity, double rate, uint64_t seed);

/* Copies up to max_rows recorded rows (in no particular order) into x
 * [rows][8], y, vertex, meta (any may be NULL; all NULL: only counts), all
 * at `where`.  *rows receives the rows copied (or held, when all are
 * NULL), *seen the scans the sampling kept, dropped ones included. */
gsp_status gsp_get_traces(gsp_ctx *ctx, float *x, uint8_t *y, int32_t *vertex, int32_t *meta, int64_t max_rows,
                          int64_t *rows, int64_t *seen, int where);

#ifdef __cplusplus
}
#endif
#endif /* GSP_H */
