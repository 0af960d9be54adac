// gsp_internal.h - host-side declarations shared by the library's sources:
// launch wrappers of every kernel and the per-level work lists.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "gate_common.h"

namespace gsp {

constexpr int kMaxRounds = 64;
constexpr int kNumBuckets = kNumBins * kMaxRounds;  // bucket (bin b, sub-round p) = b * P + p

// A graph level G' in device memory: CSR with int64 offsets, int32 columns
// and weights of type wt (none, fp32 or fp64); deg[i] = off[i+1] - off[i].
struct Level {
    int64_t n = 0, nnz = 0;
    const int64_t *off = nullptr;
    const int32_t *col = nullptr;
    const void *w = nullptr;
    int wt = W_UNIT;
    const int32_t *deg = nullptr;
    // a batch of independent graphs side by side (gid == nullptr: one graph)
    int64_t graphs = 0;
    const int32_t *gid = nullptr;     // graph of each vertex
    const int64_t *vbase = nullptr;   // first vertex of each graph (graphs + 1 entries)
    const double *M2g = nullptr;      // 2m of each graph
    // a graph stored in degree order: orig[v] = the caller's id of vertex v
    // (nullptr: stored as loaded).  Wherever the method orders vertex or
    // community ids (ties, the singleton rule, sub-rounds, traces) it uses
    // orig, so results do not depend on the storage order.
    const int32_t *orig = nullptr;
    // in degree order, rows [0, nlong) are the rows of at least kLongRow
    // entries (0 otherwise)
    int64_t nlong = 0;
};

constexpr int kLongLog = 8;
constexpr int kLongRow = 1 << kLongLog;   // rows this long are cut into entry chunks
constexpr int kScratchU64 = 2 * kNumBuckets + 16;   // counters in Scratch::u64

// The input graph stored in degree order (k_order.hip): vertex p is the
// caller's vertex orig[p], rank is the inverse, and row p is row orig[p]
// with its columns renumbered by rank.
struct DegreeOrder {
    int32_t *orig = nullptr, *rank = nullptr, *deg = nullptr;
    int64_t *off = nullptr;
    int32_t *col = nullptr;
    void *w = nullptr;
    int64_t nlong = 0;
    unsigned long long *hist = nullptr;   // 2 kOrderBucketsMax counters (bucket sizes, cursors)
    int rounds = 0;                       // the sub-rounds the short rows are grouped by
};
constexpr int kOrderBucketsMax = 128 * (kMaxRounds + 1);

// Vertex work lists of a level: every vertex with deg > 0 sits in bucket
// (bin of its degree, its sub-round); bl holds the buckets back to back, in
// bucket order, boff[k]..boff[k+1] is bucket k (host copy).
// Hub vertices (bin BIN_HUB) are cut into chunks of kHubChunk entries:
// chunk k covers entries [ch_beg[k], min(ch_beg[k] + kHubChunk, row end)) of
// vertex ch_vert[k]; chunks of sub-round p are ch_poff[p]..ch_poff[p+1].
// hub_off[i] is the offset of hub i's global table (hub_table_size(deg)).
struct WorkLists {
    int rounds = 1, shift = 0;
    int32_t *bl = nullptr;
    int64_t boff[kNumBuckets + 1] = {0};
    int64_t bucket_entries[kNumBuckets] = {0};
    int32_t *ch_vert = nullptr;
    int64_t *ch_beg = nullptr;
    int64_t nchunks = 0;
    int64_t ch_poff[kMaxRounds + 1] = {0};
    int64_t *hub_off = nullptr;
    int32_t *hub_ch0 = nullptr;
    uint64_t hub_table_total = 0;
    // hash partitions of hub i: as many as its chunks (P_i); chunk s of the
    // hub leaves P_i packed (start, count) pairs at hub_b0[i] + s * P_i
    int64_t *hub_b0 = nullptr;
    uint64_t bucket_total = 0;

    int64_t bucket_begin(int b, int p) const { return boff[b * rounds + p]; }
    int64_t bucket_size(int b, int p) const { return boff[b * rounds + p + 1] - boff[b * rounds + p]; }
    int64_t bin_begin(int b) const { return boff[b * rounds]; }
    int64_t bin_size(int b) const { return boff[(b + 1) * rounds] - boff[b * rounds]; }
};

// Totals of the scan+decide kernels, per kernel class (0 small, 1 wave,
// 2 block, 3 hub scan, 4 hub finish), striped over kStripes cache lines (a
// block adds to stripe blockIdx % kStripes) so thousands of blocks do not
// serialise on one address; the host sums the stripes.
constexpr int kStripes = 16;
// counter classes: 0-2 small / wave / block scan+decide, 3 hub chunk scan,
// 4 hub decisions (and the global-table slices), 5 hub partition gather
constexpr int kMoveClasses = 6;
struct alignas(128) CounterStripe {
    unsigned long long gain;                   // gain total in units of 2^-61 of delta-modularity (gain_units)
    unsigned long long moved;                  // movers
    unsigned long long verts[kMoveClasses];    // vertices decided
    unsigned long long scanned[kMoveClasses];  // CSR entries scanned
    unsigned long long keys[kMoveClasses];     // distinct neighbour communities scored
    unsigned long long ginserts[kMoveClasses]; // hub pairs: staged or inserted (3), read back (5)
    unsigned long long aux[kMoveClasses];      // partition words written (3) / read (5); chunk partials (4)
    unsigned long long pruned;                 // vertices the learned gate kept from the scan
};

// Counters written by the kernels of one local-moving iteration.
struct IterCounters {
    int qcnt[kMaxRounds][kNumBins];   // queued vertices per sub-round and bin
    int ccnt[kMaxRounds][kNumBins];   // gated sweeps: candidates before the gate
    int pad[32];
    CounterStripe st[kStripes];
};

// Trace capture: rows (features before the scan, moved, vertex, pass * 256 +
// sweep) of the sampled scans, in kStripes regions of scap rows; a block
// appends to region blockIdx % kStripes (cnt[r] counts the region's rows,
// also those beyond scap, which are dropped).
struct TraceArgs {
    float *x = nullptr;                 // [kStripes * scap][8]
    uint8_t *y = nullptr;
    int32_t *v = nullptr;
    int32_t *meta = nullptr;
    unsigned long long *cnt = nullptr;  // [kStripes]
    int64_t scap = 0;
    uint64_t seed = 0, thr = 0;
};

// Arguments of the local-moving kernels for one sub-round.
constexpr int kMaxParts = 4096;   // hash partitions (chunks) per hub at most
constexpr int kPartCap = 3072;    // distinct communities per partition at most

struct MoveArgs {
    Level g;
    const double *K;
    const double *sig;
    const int32_t *csize;
    const int32_t *cm;
    double M2;
    uint8_t *flag;           // unprocessed flags (read by compaction, set for neighbours of movers)
    int32_t *dec;            // decision of every queued vertex (its community if it stays)
    double *gain_out;        // per-vertex gain numerator (hooks), or nullptr
    int32_t *queue;          // queued vertices, bin b of this sub-round at qbase[b]
    int64_t qbase[kNumBins];
    int64_t qcap[kNumBins];  // bucket sizes (capacity of each queue)
    IterCounters *ctr;       // this iteration's counters
    int round;               // sub-round index p
    // hubs
    const int32_t *ch_vert;
    const int64_t *ch_beg;
    int64_t ch_first, ch_count;   // static chunk range of this sub-round's hubs
    const int64_t *hub_off;
    uint8_t *hub_act;
    int *hkeys;
    double *hvals;
    const int32_t *hub_ch0;  // per hub vertex: its first chunk id
    double *part_g, *part_kid;  // per chunk: best score and K_{i->d} share
    int *part_c;             // per chunk: best community
    // hubs by hash partitions (hub_parts): staging of each chunk's distinct
    // (community, weight) pairs at the chunk's own entry positions, and the
    // per (chunk, partition) packed start/count words; hub_act[i] = 3 marks
    // a hub sent to its global table instead (by the decision kernel)
    bool hub_parts = false;
    int max_parts = kMaxParts;   // hubs with more chunks: hub_act = 3
    int32_t *skey = nullptr;
    double *sval = nullptr;
    uint32_t *hbuck = nullptr;
    const int64_t *hub_b0 = nullptr;
    // learned gate and traces (hbits == nullptr: neither)
    float *hfrac = nullptr, *hgain = nullptr;   // history of the last scan in this pass
    uint8_t *hbits = nullptr;
    double *dmoved = nullptr;                   // D_i: weight of i's entries to movers since i left the frontier
    double *dsnap = nullptr;                    // D_i as compaction took it (the features' value)
    int32_t *cand = nullptr;                    // gated sweep: candidates (the gate fills `queue`)
    int pass = 0, sweep = 0, iter = 0;          // feature and trace context
    const int64_t *iter_dev = nullptr;          // iter from device memory (sweeps replayed from a graph)
    // return-move option: per vertex, the community it left at its last
    // move (high 32 bits) and that move's sweep (low 32 bits); the sweep
    // index comes from device memory.  mhist == nullptr: every gain counts.
    int64_t *mhist = nullptr;
    const int64_t *sweep_dev = nullptr;
    // batches: per graph, whether the gate applies in this sweep (a graph in
    // its confirming or plain sweeps keeps every candidate) and its l_i
    const uint8_t *ggated = nullptr;
    const int32_t *giter = nullptr;
    TraceArgs tr;                               // tr.x == nullptr: no capture
    // launch schedule: the scans' and apply's grids are at most grid_cap
    // workgroups (0: each kernel's own cap); their loops stride over the
    // grid, so any cap gives the same results
    int grid_cap = 0;
    // GSP-Leiden's refinement: a vertex is queued only while its community
    // (sub-community) holds it alone; the others leave the frontier
    bool single_only = false;
    // batch of graphs (g.gid != nullptr): per-graph totals of the sweep and
    // the graphs still iterating
    unsigned long long *ggain = nullptr;        // per graph, units of gain_units
    unsigned long long *gmoved = nullptr;
    const uint8_t *gactive = nullptr;
};

// ---- k_util.hip ----
void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s);
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);
void launch_fill_f32(float *p, float v, int64_t n, hipStream_t s);
void launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s);
void launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);
void launch_iota_i32(int32_t *p, int64_t n, hipStream_t s);
void launch_copy_i32(int32_t *dst, const int32_t *src, int64_t n, hipStream_t s);
// Exclusive scan of n values into out[0..n]; out[n] is the total.
// tmp must hold scan_tmp_bytes(n) bytes.
size_t scan_tmp_bytes(int64_t n);
void scan_exclusive_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, void *tmp, hipStream_t s);
void scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, void *tmp, hipStream_t s);
void scan_exclusive_i32(const int32_t *in, int32_t *out, int64_t n, void *tmp, hipStream_t s);
// Input checks; err bits: 1 offsets, 2 columns, 4 weights.
void launch_validate(const int64_t *off, const int32_t *col, const void *w, int wt, int64_t n, int64_t nnz,
                     int *err, hipStream_t s);
void launch_offsets_from_i32(const int32_t *in, int64_t *out, int64_t n1, hipStream_t s);
void launch_degrees(const int64_t *off, int32_t *deg, int64_t n, hipStream_t s);
void launch_weights_to_f64(const float *in, double *out, int64_t nnz, hipStream_t s);
// K_i = row sums (one wavefront per row) and *M2 += sum K_i.
void launch_vertex_weights(const Level &g, double *K, double *M2, hipStream_t s);

// ---- k_order.hip ----
struct Scratch;
// K of the long rows of a level in degree order (rows [0, g.nlong)), and
// their part of *M2; the rows after them are launch_vertex_weights' part.
void launch_vertex_weights_long(const Level &g, double *K, double *M2, hipStream_t s);
// Fills o (arrays allocated by the caller: orig, rank, deg n; off n + 1;
// col, w nnz; hist 2 kOrderBucketsMax) with g in degree order, its shorter
// rows grouped by their sub-round out of `rounds`, and sets o.nlong and
// o.rounds.  Synchronizes s.
hipError_t order_by_degree(const Level &g, Scratch &sc, DegreeOrder &o, int rounds, hipStream_t s);
// lab[v] <- the smallest orig[u] over the u with lab[u] = lab[v] (tmp: n ints).
void launch_labels_min_orig(int32_t *lab, const int32_t *orig, int64_t n, int32_t *tmp, hipStream_t s);
// out[v] <- orig[lab[v]].
void launch_labels_orig(const int32_t *lab, const int32_t *orig, int64_t n, int32_t *out, hipStream_t s);
// out[orig[v]] <- in[v].
void launch_scatter_by_orig(const int32_t *in, const int32_t *orig, int64_t n, int32_t *out, hipStream_t s);
// Modularity parts: *sigma_in += sum of entries inside communities,
// sig[c] += K_i; then q = sigma_in/M2 - sum_c (sig[c]/M2)^2, the second sum
// in units of 2^-62 (*out of launch_sum_squares), exact in any order.
void launch_modularity_parts(const Level &g, const int32_t *memb, const double *K, double *sig, double *sigma_in,
                             hipStream_t s);
void launch_sum_squares(const double *sig, int64_t n, double M2, unsigned long long *out, hipStream_t s);
void launch_check_labels(const int32_t *memb, int64_t n, int *err, hipStream_t s);
// Weight grid (exact sums): every weight becomes the nearest multiple of
// 2^-S with S the largest integer (in [-1000, 1022]) such that an exact
// upper bound U of the weight total has U 2^S < 2^52; then every sum or
// difference of weights the method forms is exact in fp64, in any order.
// The host takes S from the largest weight (*out, as fp64 bits) and the
// integer bound *U = sum of max(1, ceil(w 2^T)), T = 62 - bits(nnz) - e with
// wmax < 2^e.
void launch_weight_max(const void *w, int wt, int64_t nnz, unsigned long long *out, hipStream_t s);
void launch_weight_bound(const void *w, int wt, int64_t nnz, int T, unsigned long long *U, hipStream_t s);
void launch_weight_grid(void *w, int wt, int64_t nnz, int S, unsigned long long *moved, hipStream_t s);
// A mover's share of an iteration's gain total: its delta-modularity
// 2 (G(c*) - G(stay)) / M2^2 rounded to the nearest multiple of 2^-61; the
// total is the exact (order-free) integer sum of these.
__device__ __forceinline__ unsigned long long gain_units(double gain, double m2) {
    if (!(m2 > 0.0)) return 0ull;
    return (unsigned long long)(long long)rint(ldexp((2.0 * gain) / (m2 * m2), 61));
}

// ---- k_bins.hip ----
// Builds the work lists of a level (all buckets of all sub-rounds).
// Needs a host sync inside (bucket and chunk offsets are copied back).
struct Scratch;
hipError_t build_work_lists(const Level &g, int rounds, WorkLists &wl, Scratch &sc, hipStream_t s);
// Only the buckets (no hub chunks or tables): items with deg[i] > 0 into
// wl.bl by (bin of deg[i], sub-round of i).
hipError_t bin_vertices(const int32_t *deg, int64_t n, int rounds, WorkLists &wl, Scratch &sc, hipStream_t s,
                        const int32_t *gid = nullptr, const int64_t *vbase = nullptr,
                        const int32_t *orig = nullptr);

// ---- k_move.hip ----
void launch_community_totals(const double *K, const int32_t *cm, int64_t n, double *sig, int32_t *csize,
                             hipStream_t s);
void launch_move_compact(const MoveArgs &a, const WorkLists &wl, hipStream_t s);
void launch_move_small(const MoveArgs &a, const WorkLists &wl, hipStream_t s);
void launch_move_wave(const MoveArgs &a, hipStream_t s);
void launch_move_block(const MoveArgs &a, hipStream_t s);
void launch_move_hub_scan(const MoveArgs &a, hipStream_t s);
void launch_move_hub_finish(const MoveArgs &a, hipStream_t s);
// Hubs by hash partitions: chunk -> LDS reduction -> pairs sorted by
// partition (staging); partition -> LDS table over all chunks -> the
// partition's best candidate and K_{i->d} share (part_* of the chunk with
// the partition's index); a workgroup per hub combines them and decides.
// Hubs with more than max_parts (<= kMaxParts) chunks, or a partition with
// more than kPartCap distinct communities, get hub_act = 3: the decision
// workgroup then takes the hub through its global table.
void launch_move_hub_parts(const MoveArgs &a, hipStream_t s);    // phase 1: chunk reduce, staged pairs
void launch_move_hub_gather(const MoveArgs &a, hipStream_t s);   // phase 2: partitions merged and scored
void launch_move_hub_decide(const MoveArgs &a, hipStream_t s);   // phase 3: a workgroup per hub decides
void launch_move_apply(const MoveArgs &a, int64_t cap, hipStream_t s);

// ---- k_leiden.hip ----
// The same-bound subgraph of a level for GSP-Leiden's refinement: row i
// keeps the entries (i, j) with bound[j] == bound[i], in order.  Writes its
// degrees (deg, n), offsets (off, n + 1) and entries (col; w as fp64 unless
// g has unit weights); wl holds g's work lists (their hub chunks split the
// long rows), ch_cnt one value per hub chunk, kept one byte per entry of g
// (scratch, indexed like g's entries).
hipError_t bound_subgraph(const Level &g, const WorkLists &wl, const int32_t *bound, int32_t *deg, int64_t *off,
                          int32_t *col, double *w, int64_t *ch_cnt, uint8_t *kept, void *scan_tmp,
                          hipStream_t s);
// *err |= 1 if a sub-community has members in two bound communities (home:
// n ints of scratch; *err is not cleared here).
void launch_bound_check(const int32_t *sub, const int32_t *bound, int64_t n, int32_t *home, int *err,
                        hipStream_t s);
// start[sub[i]] <- bound[i]: each sub-community (super-vertex of the next
// level) starts in the community that holds it.
void launch_bound_start(const int32_t *sub, const int32_t *bound, int64_t n, int32_t *start, hipStream_t s);

// ---- k_gate.hip ----
// Gated sweep: the candidates of every bin (cand, ctr->ccnt[round]) go
// through the network; those with logit >= theta_logit are queued (queue,
// ctr->qcnt[round]), the others counted as pruned (a pruned hub's hub_act
// is cleared).
void launch_gate(const MoveArgs &a, const GateNet &net, float theta_logit, int64_t cap, hipStream_t s);
// Logits of feature rows x[rows][8] (fp32, rounded to bf16 here) by the
// inference kernel.
void launch_gate_eval(const GateNet &net, const float *x, int64_t rows, float *logit, hipStream_t s);
// Training (fp32): per-block partial gradients of the mean pos-weighted BCE
// over rows [0, rows) of (x, y) with the batch size `inv_batch` = 1/B, then
// their sum in block order; with `adam` the sum is applied as one Adam step
// (c1 = 1 - beta1^t, c2 = 1 - beta2^t), else written to grad.  The batch
// loss (sum of the rows' losses * inv_batch) is added to *loss.
constexpr int kMlpRowsPerBlock = 64;
void launch_mlp_grad(const float *params, const float *x, const uint8_t *y, int64_t rows, float pos_weight,
                     float inv_batch, float *part, double *part_loss, hipStream_t s);
void launch_mlp_reduce(const float *part, const double *part_loss, int nblocks, float *params, float *m, float *v,
                       bool adam, float lr, float c1, float c2, float *grad, double *loss, hipStream_t s);

// ---- k_batch.hip ----
// gid[v] = graph of vertex v for a level with graph bases vbase[0..G].
void launch_batch_gid(const int64_t *vbase, int64_t G, int64_t n, int32_t *gid, hipStream_t s);
// 2m of each graph (sum of K over its vertices, reproducible order).
void launch_batch_m2(const double *K, const int64_t *vbase, int64_t G, double *M2g, hipStream_t s);
// cfirst[g] = rank[vbase[g]] (g < G), cfirst[G] = *count: first community
// id of each graph after a renumbering with rank = exclusive scan of flags.
void launch_batch_cfirst(const int32_t *rank, const int64_t *vbase, int64_t G, const int64_t *count,
                         int64_t *cfirst, hipStream_t s);
// q[g] = modularity of graph g (level g holds the batch; memb values are
// community ids, graph g's in [cfirst[g], cfirst[g+1]); sig = Sigma_c).
void launch_batch_modularity(const Level &g, const int32_t *memb, const double *sig, const int64_t *cfirst,
                             double *qin, double *q, hipStream_t s);
void launch_add_i32(int32_t *p, int64_t n, int32_t delta, hipStream_t s);
// flag[v] = 1 for every vertex of a graph with gconfirm set (its confirming sweep)
void launch_batch_flag_confirm(const int32_t *gid, const uint8_t *gconfirm, int64_t n, uint8_t *flag, hipStream_t s);

// ---- k_split.hip ----
// labels[i] = smallest vertex of i's component among same-community edges.
// dom, vote_cnt, vote_best: scratch of n entries each (the picked root per
// community and its vote)
void launch_split(const Level &g, const WorkLists &wl, const int32_t *cm, int32_t *labels, int32_t *dom,
                  uint32_t *vote_cnt, unsigned long long *vote_best, hipStream_t s);
// The same labels by minimum-label propagation with pruning (Algorithm
// splitDisconnectedLp with its pruning) and pointer jumping: next (n flags,
// zero on return), q_small / q_large (n each) the rounds' queues, counts (4
// ints, device) and counts_h (2 ints, pinned host) their sizes.  Returns the
// number of rounds (one host read per round), -1 on a HIP error.
int launch_split_lp(const Level &g, const int32_t *cm, int32_t *labels, uint8_t *next, int32_t *q_small,
                    int32_t *q_large, int *counts, int *counts_h, hipStream_t s);
// Renumber labels (values in [0, n)) by ascending label: flag[l] = label l
// in use, rank = exclusive scan of flag, out[i] = rank[labels[i]], *count =
// number of labels in use.  flag/rank are n+1-sized temps.
void launch_renumber(const int32_t *labels, int64_t n, int32_t *out, int32_t *flag, int32_t *rank, int64_t *count,
                     void *tmp, hipStream_t s);
void launch_lookup(int32_t *top, int64_t n, const int32_t *cm, hipStream_t s);
// Counts communities (of memb) with more than one component (labels).
void launch_count_disconnected(const int32_t *labels, const int32_t *memb, int64_t n, int32_t *roots_per_comm,
                               unsigned long long *out, hipStream_t s);
// The disconnected count of a caller's CSR (device pointers, unvalidated)
// with caller-provided scratch: parent and roots of n entries, flags of 2.
// Union-find over every same-community entry (no work lists), then
// communities with more than one root; *out (device) = that count, or -1 if
// an offset, column or label lies out of range (every access is checked).
void launch_count_disconnected_csr(const int64_t *off, const int32_t *col, int64_t n, int64_t nnz,
                                   const int32_t *memb, int32_t *parent, int32_t *roots, unsigned long long *flags,
                                   int64_t *out, hipStream_t s);
// lab[v] = smallest vertex of v's community (then renumber gives the
// numbering by ascending smallest vertex).  first is an n-sized temp.
void launch_canonical_labels(const int32_t *memb, int64_t n, int32_t *first, int32_t *lab, hipStream_t s);

// ---- k_aggregate.hip ----
struct AggOut {
    int64_t *off;     // n2 + 1
    int32_t *col;
    double *w;
    double *K;        // K'' (row sums of G'')
    int32_t *deg;     // deg''
};
// Aggregates g by cm (values in [0, n2)) into `out`, a gapped CSR: row c
// is [out.off[c], out.off[c] + out.deg[c]) (out.off has n2 + 1 entries: the
// row capacities' prefix sums, at most g's entries in all).  *nnz_out = the
// entries written.  stage_* (capacity nnz, not out's arrays) take the giant
// communities' partition pairs when hub_parts; without it every giant
// community goes through a global table.
hipError_t aggregate(const Level &g, const WorkLists &wl, const int32_t *cm, int64_t n2, AggOut out,
                     int32_t *stage_col, double *stage_w, Scratch &sc, int64_t *nnz_out, hipStream_t s,
                     bool hub_parts = true);
// Packs a gapped CSR (eoff, deg) into a plain one (off_out: n2 + 1 entries).
hipError_t compact_rows(const int64_t *eoff, const int32_t *deg, int64_t n2, const int32_t *col, const double *w,
                        int64_t *off_out, int32_t *col_out, double *w_out, Scratch &sc, hipStream_t s);

// Device scratch owned by the context (sized at load).
struct Scratch {
    int64_t n_cap = 0, nnz_cap = 0;
    void *scan_tmp = nullptr;
    size_t scan_tmp_bytes = 0;
    int64_t *i64a = nullptr, *i64b = nullptr, *i64c = nullptr, *i64d = nullptr, *i64e = nullptr, *i64f = nullptr;
    int64_t *i64g = nullptr;   // n_cap + 1
    uint8_t *u8a = nullptr;    // n_cap + 1
    int32_t *i32a = nullptr, *i32b = nullptr, *i32c = nullptr, *i32d = nullptr, *i32e = nullptr;  // n_cap + 1
    int32_t *bl2 = nullptr;  // n_cap: community work lists
    int *err = nullptr;
    unsigned long long *u64 = nullptr;  // 16 counters
    double *f64 = nullptr;              // 16 scalars
    // hub tables (grown on demand): keys and values
    int *hkeys = nullptr;
    double *hvals = nullptr;
    uint64_t hcap = 0;
    // hub partition words (grown on demand)
    uint32_t *hbuck = nullptr;
    uint64_t hbcap = 0;
    // chunk lists (sized for the input graph): vertex hubs of a level, hub
    // communities of an aggregation (entry chunks and table segments), and
    // per-chunk partial results of the hub decisions
    int32_t *ch_vert = nullptr;
    int64_t *ch_beg = nullptr;
    int32_t *cch_comm = nullptr, *cseg_comm = nullptr;
    int64_t *cch_beg = nullptr, *cseg_beg = nullptr;
    int64_t *cch_k0 = nullptr;   // first member position of each chunk
    double *part_g = nullptr, *part_kid = nullptr;   // per chunk
    int *part_c = nullptr;
    int64_t ch_cap = 0;
    uint64_t *mem_used = nullptr;  // not owned
};

// Grows the hub-table pool of sc to at least `slots` (keys empty, values 0).
hipError_t ensure_hub_tables(Scratch &sc, uint64_t slots, hipStream_t s);
// Grows the hub partition words of sc to at least `words`.
hipError_t ensure_hub_buckets(Scratch &sc, uint64_t words, hipStream_t s);

}  // namespace gsp
