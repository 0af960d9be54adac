// capi.hip - the C ABI (include/gsp.h) and the pass driver of Algorithm
// "louvain": per pass, reset -> local moving (synchronous sub-rounds) ->
// split -> renumber + dendrogram lookup -> convergence tests -> aggregation
// -> threshold scaling.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <type_traits>
#include <cmath>
#include <vector>

#include "../../include/gsp.h"
#include "gsp_internal.h"

using namespace gsp;

namespace {

struct EventPair {
    int cls;
    hipEvent_t a, b;
    hipStream_t st;
};

// Records HIP events around phases / kernel classes and sums them later.
struct Timer {
    hipStream_t s = nullptr;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<EventPair> open;
    hipEvent_t get() {
        if (used == pool.size()) {
            hipEvent_t e;
            // timing only (read after a stream synchronisation): no system
            // fence, which would write back and invalidate the caches
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    void reset() {
        used = 0;
        open.clear();
    }
    uint32_t kmask = 0;   // kernel classes (100 + k) to time; 0 = all
    // st: the stream the timed work goes to (default: the context's)
    int begin(int cls, hipStream_t st = nullptr) {
        if (cls >= 100 && kmask && !((kmask >> (cls - 100)) & 1u)) return -1;
        hipEvent_t a = get(), b = get();
        if (!a || !b) return -1;
        if (!st) st = s;
        (void)hipEventRecord(a, st);
        open.push_back({cls, a, b, st});
        return (int)open.size() - 1;
    }
    void end(int k) {
        if (k >= 0) (void)hipEventRecord(open[k].b, open[k].st);
    }
    // Adds elapsed ms per class into out[cls].
    void collect(double *out, int ncls) {
        for (auto &p : open) {
            float ms = 0.f;
            if (p.cls >= 0 && p.cls < ncls && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) out[p.cls] += ms;
        }
        reset();
    }
    ~Timer() {
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

enum { PH_MOVE = 0, PH_SPLIT, PH_AGG, PH_OTHER, PH_REFINE, PH_COUNT };

}  // namespace

struct gsp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;   // where sweeps are captured into graphs
    // the independent scans of a sub-round (wave bin, workgroup bin, hubs)
    // run on side streams beside the small-bin scan; fork / join events per
    // sub-round and side stream
    hipStream_t side[3] = {nullptr, nullptr, nullptr};
    std::vector<hipEvent_t> fork_ev, join_ev;
    bool hub_parts = true;              // hubs by hash partitions (else global tables only); per run
    int hub_max_parts = kMaxParts;      // hubs with more chunks take their global table; per run
    // instantiated sweep graphs, reused while the level and its work lists
    // (everything a sweep's launches take as arguments) are the same
    struct SweepGraph {
        std::vector<int64_t> key;
        hipGraphExec_t exec;
    };
    std::vector<SweepGraph> sweep_graphs;
    void drop_sweep_graphs() {
        for (auto &x : sweep_graphs) (void)hipGraphExecDestroy(x.exec);
        sweep_graphs.clear();
    }
    std::string err;
    std::vector<void *> allocs;
    uint64_t mem_used = 0;
    uint64_t mem_limit = 0;

    // input graph (level 0)
    bool loaded = false;
    int64_t n = 0, nnz = 0;
    int wt0 = W_UNIT;
    int64_t *off0 = nullptr;
    int32_t *col0 = nullptr;
    void *w0 = nullptr;
    int32_t *deg0 = nullptr;
    double *K0 = nullptr;
    double M2 = 0.0;
    // weight grid of the loaded graph (exact sums): weights are multiples of
    // 2^-grid_S; grid_moved weights were rounded onto it at load
    int32_t grid_S = 0;
    int64_t grid_moved = 0;
    int *lp_counts = nullptr;   // queue sizes of the label-propagation split (4 ints)
    // the input graph in degree order (built by the first run asking for it)
    DegreeOrder ord;
    // GSP-Leiden: the level's bound communities and the next level's
    // starting communities (graph-sized, allocated on first use)
    int32_t *bnd = nullptr, *bstart = nullptr;
    double *Kord = nullptr;
    bool ordered = false;

    // super-vertex levels (ping-pong) and the gapped aggregation rows
    int64_t *offL[2] = {nullptr, nullptr};
    int32_t *colL[2] = {nullptr, nullptr};
    double *wL[2] = {nullptr, nullptr};
    int32_t *degL[2] = {nullptr, nullptr};
    double *KL[2] = {nullptr, nullptr};
    int32_t *gap_col = nullptr;
    double *gap_w = nullptr;

    // per-vertex work arrays
    double *sig = nullptr;
    int32_t *cm = nullptr, *csize = nullptr, *dec = nullptr, *queue = nullptr;
    int32_t *lab = nullptr, *top = nullptr, *bl = nullptr, *tmp32 = nullptr;
    uint8_t *flag = nullptr, *hub_act = nullptr;
    int32_t *hub_ch0 = nullptr;
    int64_t *hub_off = nullptr, *hub_b0 = nullptr;
    double *gain_tmp = nullptr;
    Scratch sc;
    IterCounters *ctr = nullptr;      // device, 2 slots
    IterCounters *ctr_h = nullptr;    // pinned host mirror
    int64_t *i64_h = nullptr;         // pinned host scalars
    double *f64_h = nullptr;

    // learned gate: per-vertex history of the current pass and the gated
    // sweeps' candidate lists (graph-sized, allocated on first use)
    float *hfrac = nullptr, *hgain = nullptr;
    uint8_t *hbits = nullptr;
    double *dmoved = nullptr, *dsnap = nullptr;
    int64_t *iter_dev = nullptr;   // [0] l_i, [1] sweep index of the current sweep (kernels read them)
    int64_t *mhist = nullptr;      // per vertex: community left at its last move, and that move's sweep
    int32_t *cand = nullptr;
    // the network in its inference formats (kept across loads)
    bool have_net = false;
    uint16_t *net_w1 = nullptr, *net_w2 = nullptr;
    float *net_f = nullptr;          // b1[64] b2[64] w3[64]
    float net_b3 = 0.0f;
    std::vector<float> net_params;   // fp32 parameters as given
    // a batch of graphs side by side (batch_graphs > 0 after gsp_load_batch)
    int64_t batch_graphs = 0;
    std::vector<int64_t> vbase0_h;        // first vertex of each graph (+ total)
    std::vector<double> M2g_h;            // 2m of each graph
    int64_t *vbase0 = nullptr, *vbaseL[2] = {nullptr, nullptr}, *cfirst = nullptr;
    int32_t *gid0 = nullptr, *gidL[2] = {nullptr, nullptr};
    double *M2g = nullptr, *bq = nullptr, *bqin = nullptr;
    unsigned long long *ggain = nullptr;   // per graph: the sweep's gain total (units of 2^-61)
    unsigned long long *gmoved = nullptr;
    uint8_t *gactive = nullptr;
    uint8_t *ggated = nullptr, *gconfirm = nullptr;   // learned batches: per graph, this sweep's mode
    int32_t *giter = nullptr;                         // learned batches: per graph l_i
    bool have_batch_result = false;
    std::vector<double> bq_h;             // modularity of each graph
    bool bq_pending = false;              // bq_h not computed yet for the last batch run
    int64_t batch_ncomm = 0;              // communities of the last batch run (all graphs)
    std::vector<int32_t> bpasses_h;       // passes each graph took part in
    // trace capture (kept across loads and runs until stopped)
    bool tracing = false;
    TraceArgs trace;
    std::vector<void *> persist;     // device buffers that survive loads

    // last result
    bool have_result = false;
    bool have_q = false;
    double q = 0.0;
    gsp_stats stats;
    Timer timer;
    int64_t kernel_launches[GSP_K_COUNT] = {0};

    gsp_status fail(gsp_status st, const std::string &msg) {
        err = msg;
        return st;
    }
    gsp_status fail_hip(hipError_t e, const char *what) {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? GSP_ENOMEM : GSP_EHIP;
    }
    template <class T>
    T *palloc(size_t count, hipError_t *e) {   // survives loads, freed by gsp_destroy
        void *p = nullptr;
        *e = hipMalloc(&p, (count ? count : 1) * sizeof(T));
        if (*e != hipSuccess) return nullptr;
        persist.push_back(p);
        return (T *)p;
    }
    void pfree(void *p) {
        if (!p) return;
        for (size_t k = 0; k < persist.size(); k++)
            if (persist[k] == p) {
                (void)hipFree(p);
                persist.erase(persist.begin() + (long)k);
                return;
            }
    }
    template <class T>
    T *dalloc(size_t count, hipError_t *e) {
        void *p = nullptr;
        size_t bytes = (count ? count : 1) * sizeof(T);
        *e = hipMalloc(&p, bytes);
        if (*e != hipSuccess) return nullptr;
        allocs.push_back(p);
        mem_used += bytes;
        return (T *)p;
    }
    void free_graph() {
        if (stream) (void)hipStreamSynchronize(stream);
        drop_sweep_graphs();
        for (void *p : allocs) (void)hipFree(p);
        allocs.clear();
        mem_used = 0;
        if (sc.hkeys) (void)hipFree(sc.hkeys);
        if (sc.hvals) (void)hipFree(sc.hvals);
        if (sc.hbuck) (void)hipFree(sc.hbuck);
        sc = Scratch();
        for (int k = 0; k < 2; k++) {
            offL[k] = nullptr;
            colL[k] = nullptr;
            wL[k] = nullptr;
            degL[k] = nullptr;
            KL[k] = nullptr;
        }
        gap_col = nullptr;
        gap_w = nullptr;
        lp_counts = nullptr;
        ord = DegreeOrder();
        bnd = bstart = nullptr;
        Kord = nullptr;
        ordered = false;
        mhist = iter_dev = nullptr;
        ctr = nullptr;
        hfrac = hgain = nullptr;
        hbits = nullptr;
        batch_graphs = 0;
        vbase0_h.clear();
        M2g_h.clear();
        vbase0 = cfirst = nullptr;
        vbaseL[0] = vbaseL[1] = nullptr;
        gid0 = nullptr;
        gidL[0] = gidL[1] = nullptr;
        M2g = bq = bqin = nullptr;
        ggain = nullptr;
        gmoved = nullptr;
        gactive = nullptr;
        ggated = nullptr;
        gconfirm = nullptr;
        giter = nullptr;
        have_batch_result = false;
        dmoved = dsnap = nullptr;
        cand = nullptr;
        loaded = false;
        have_result = false;
        have_q = false;
        n = nnz = 0;
    }
};

namespace gsp {

hipError_t ensure_hub_tables(Scratch &sc, uint64_t slots, hipStream_t s) {
    if (slots <= sc.hcap) return hipSuccess;
    uint64_t cap = std::max<uint64_t>(slots, sc.hcap + sc.hcap / 2);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (sc.hkeys) (void)hipFree(sc.hkeys);
    if (sc.hvals) (void)hipFree(sc.hvals);
    sc.hkeys = nullptr;
    sc.hvals = nullptr;
    sc.hcap = 0;
    e = hipMalloc(&sc.hkeys, cap * sizeof(int));
    if (e != hipSuccess) return e;
    e = hipMalloc(&sc.hvals, cap * sizeof(double));
    if (e != hipSuccess) return e;
    sc.hcap = cap;
    launch_fill_i32(sc.hkeys, kEmpty, (int64_t)cap, s);
    launch_fill_f64(sc.hvals, 0.0, (int64_t)cap, s);
    return hipGetLastError();
}

hipError_t ensure_hub_buckets(Scratch &sc, uint64_t words, hipStream_t s) {
    if (words <= sc.hbcap) return hipSuccess;
    uint64_t cap = std::max<uint64_t>(words, sc.hbcap + sc.hbcap / 2);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (sc.hbuck) (void)hipFree(sc.hbuck);
    sc.hbuck = nullptr;
    sc.hbcap = 0;
    e = hipMalloc(&sc.hbuck, cap * sizeof(uint32_t));
    if (e != hipSuccess) return e;
    sc.hbcap = cap;
    return hipSuccess;
}

}  // namespace gsp

#define HIP_TRY(expr)                                         \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return ctx->fail_hip(_e, #expr); \
    } while (0)

namespace {

Level level0(const gsp_ctx *ctx) {
    Level g;
    g.n = ctx->n;
    g.nnz = ctx->nnz;
    g.off = ctx->off0;
    g.col = ctx->col0;
    g.w = ctx->w0;
    g.wt = ctx->wt0;
    g.deg = ctx->deg0;
    return g;
}

// The input graph in degree order (ensure_order has built it).
Level level_ordered(const gsp_ctx *ctx) {
    Level g = level0(ctx);
    g.off = ctx->ord.off;
    g.col = ctx->ord.col;
    g.w = ctx->wt0 == W_UNIT ? nullptr : ctx->ord.w;
    g.deg = ctx->ord.deg;
    g.orig = ctx->ord.orig;
    g.nlong = ctx->ord.nlong;
    return g;
}

WorkLists make_lists(gsp_ctx *ctx) {
    WorkLists wl;
    wl.bl = ctx->bl;
    wl.hub_off = ctx->hub_off;
    wl.hub_ch0 = ctx->hub_ch0;
    wl.hub_b0 = ctx->hub_b0;
    return wl;
}

bool valid_rounds(int r) { return r >= 1 && r <= kMaxRounds && (r & (r - 1)) == 0; }

gsp_status copy_in_i32(gsp_ctx *ctx, int32_t *dst, const int32_t *src, int64_t count, int where) {
    if (count == 0) return GSP_OK;
    HIP_TRY(hipMemcpyAsync(dst, src, count * sizeof(int32_t),
                           where == GSP_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, ctx->stream));
    return GSP_OK;
}

template <class T>
gsp_status copy_out(gsp_ctx *ctx, T *dst, const T *src, int64_t count, int where) {
    if (count == 0) return GSP_OK;
    HIP_TRY(hipMemcpyAsync(dst, src, count * sizeof(T),
                           where == GSP_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx->stream));
    return GSP_OK;
}

// Copies a caller membership into ctx->cm and checks every label is in [0, n).
gsp_status take_membership(gsp_ctx *ctx, const int32_t *memb, int where) {
    if (!ctx->loaded) return ctx->fail(GSP_ESTATE, "no graph loaded");
    if (!memb && ctx->n > 0) return ctx->fail(GSP_EINVAL, "membership is NULL");
    if (where != GSP_HOST && where != GSP_DEVICE) return ctx->fail(GSP_EINVAL, "bad `where`");
    gsp_status st = copy_in_i32(ctx, ctx->cm, memb, ctx->n, where);
    if (st != GSP_OK) return st;
    HIP_TRY(hipMemsetAsync(ctx->sc.err, 0, sizeof(int), ctx->stream));
    launch_check_labels(ctx->cm, ctx->n, ctx->sc.err, ctx->stream);
    int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, ctx->sc.err, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (bad) return ctx->fail(GSP_EINVAL, "membership label outside [0, n)");
    return GSP_OK;
}

// Renumbers labels (values in [0, n)) by ascending label into out; the
// number of labels in use goes to *count (host).
gsp_status renumber(gsp_ctx *ctx, const int32_t *labels, int64_t n, int32_t *out, int64_t *count) {
    launch_renumber(labels, n, out, ctx->sc.i32a, ctx->sc.i32b, ctx->sc.i64e, ctx->sc.scan_tmp, ctx->stream);
    HIP_TRY(hipMemcpyAsync(ctx->i64_h, ctx->sc.i64e, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    *count = ctx->i64_h[0];
    return GSP_OK;
}

// Algorithmic bytes of the local-moving kernels, per counter class.
//  scan+decide (small, wave, block): per vertex decided 36 B (offset, degree,
//    membership, K, Sigma and size of its community, decision); per entry
//    4 B column + 4 B neighbour membership + the weight (0 / 4 / 8 B); per
//    distinct neighbour community 8 B (its Sigma);
//  hub chunk scan: per entry as above; per staged (chunk, community) pair or
//    global-table insert 12 B (key, value); per partition word 4 B;
//  hub gather: per staged pair read 12 B, per partition word 4 B, per
//    distinct community scored 8 B (its Sigma), per chunk 20 B partial out;
//  hub decisions: per global-table slot scored 20 B (key, value, Sigma);
//    per chunk partial read 20 B; per hub 36 B.
double move_bytes(int cls, const CounterStripe &h, int wt) {
    int ws = wt == W_UNIT ? 0 : (wt == W_F32 ? 4 : 8);
    double v = (double)h.verts[cls], e = (double)h.scanned[cls], k = (double)h.keys[cls];
    double gi = (double)h.ginserts[cls], ax = (double)h.aux[cls];
    switch (cls) {
        case 3: return (8.0 + ws) * e + 12.0 * gi + 4.0 * ax;
        case 4: return 20.0 * k + 20.0 * ax + 36.0 * v;
        case 5: return 12.0 * gi + 4.0 * ax + 8.0 * k + 20.0 * v;
        default: return 36.0 * v + (8.0 + ws) * e + 8.0 * k;
    }
}

// the kernel class each counter class is timed under
constexpr int kClassKernel[kMoveClasses] = {GSP_K_MOVE_SMALL, GSP_K_MOVE_WAVE, GSP_K_MOVE_BLOCK,
                                            GSP_K_MOVE_HUB, GSP_K_MOVE_HUB_FINISH, GSP_K_MOVE_HUB_GATHER};

// What one local-moving phase runs and what it reports.
struct PhaseCfg {
    double tau = 0.0;
    int max_iter = 20;
    bool timing_k = false;
    bool timing_side = false;   // timed scans stay side by side (timing = 3)
    bool return_moves = false;  // return moves add nothing to the gain totals
    bool gated = false;            // learned gate in front of the scan
    bool use_graphs = false;       // replay plain sweeps from a captured graph
    int grid_cap = 0;              // launch schedule (MoveArgs::grid_cap)
    float theta_logit = 0.0f;      // scan iff logit >= theta_logit
    int pass = 0;                  // pass index (a feature, and trace rows)
    double *dq_out = nullptr;      // per counted iteration (max_iter entries)
    int64_t *moved_out = nullptr;
    double *kernel_bytes = nullptr;
    // batch (g.gid != nullptr): graphs already finished stay still; out:
    // each graph's counted iterations
    const uint8_t *gdone = nullptr;   // host, per graph
    std::vector<int32_t> li_g;
    bool single_only = false;         // GSP-Leiden's refinement (MoveArgs::single_only)
    // out
    int32_t li = 0;
    int64_t scanned_vertices = 0, scanned_entries = 0, pruned = 0, confirm_sweeps = 0, sweeps = 0;
};

gsp_status ensure_gate_state(gsp_ctx *ctx) {
    if (ctx->hbits) return GSP_OK;
    hipError_t e = hipSuccess;
    ctx->hfrac = ctx->dalloc<float>(ctx->n, &e);
    if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(gate history)");
    ctx->hgain = ctx->dalloc<float>(ctx->n, &e);
    if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(gate history)");
    ctx->hbits = ctx->dalloc<uint8_t>(ctx->n, &e);
    if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(gate history)");
    ctx->dmoved = ctx->dalloc<double>(ctx->n, &e);
    if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(gate history)");
    ctx->dsnap = ctx->dalloc<double>(ctx->n, &e);
    if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(gate history)");
    ctx->cand = ctx->dalloc<int32_t>(ctx->n, &e);
    if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(gate candidates)");
    return GSP_OK;
}

GateNet net_of(const gsp_ctx *ctx) {
    GateNet net;
    net.w1 = ctx->net_w1;
    net.w2 = ctx->net_w2;
    net.b1 = ctx->net_f;
    net.b2 = ctx->net_f + kGateHidden;
    net.w3 = ctx->net_f + 2 * kGateHidden;
    net.b3 = ctx->net_b3;
    return net;
}

// Side streams (default priority) and the fork / join events of P sub-rounds.
gsp_status ensure_side(gsp_ctx *ctx, int P) {
    for (hipStream_t &q : ctx->side)
        if (!q) HIP_TRY(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
    while ((int)ctx->fork_ev.size() < P) {
        hipEvent_t e;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->fork_ev.push_back(e);
    }
    while ((int)ctx->join_ev.size() < 3 * P) {
        hipEvent_t e;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->join_ev.push_back(e);
    }
    return GSP_OK;
}

// The local-moving phase on level g (Algorithm "louvainMove" in ordered
// sub-rounds).  cm/sig/csize hold the starting state.
//
// With the learned gate the phase starts with gated sweeps (compaction ->
// gate -> scan of the kept vertices).  When a gated sweep's gain total is
// <= tau, a confirming sweep follows with every vertex unprocessed and no
// gate; if its total is <= tau too the phase ends, otherwise plain sweeps
// continue until the usual test stops them.  Every sweep counts towards
// l_i and max_iter except a confirming sweep that moves nothing.  With the
// gate or trace capture on, each scan records the vertex's history (reset
// at the start of the phase) for the features.
gsp_status move_phase(gsp_ctx *ctx, const Level &g, const double *K, const WorkLists &wl, PhaseCfg &cfg) {
    hipStream_t s = ctx->stream;
    int P = wl.rounds;
    {
        gsp_status st = ensure_side(ctx, P);
        if (st != GSP_OK) return st;
    }
    const bool hist = cfg.gated || ctx->tracing;
    if (hist) {
        gsp_status st = ensure_gate_state(ctx);
        if (st != GSP_OK) return st;
        launch_fill_f32(ctx->hfrac, 0.0f, g.n, s);
        launch_fill_f32(ctx->hgain, 0.0f, g.n, s);
        launch_fill_u8(ctx->hbits, 0, g.n, s);
        launch_fill_f64(ctx->dmoved, 0.0, g.n, s);
    }
    const GateNet net = cfg.gated ? net_of(ctx) : GateNet();
    enum { GATED, CONFIRM, PLAIN } mode = cfg.gated ? GATED : PLAIN;
    if (!ctx->mhist || !ctx->iter_dev) return ctx->fail(GSP_ESTATE, "level buffers are not allocated");
    launch_fill_u8(ctx->flag, 1, g.n, s);
    // no vertex has moved: community -1, sweep -2
    if (cfg.return_moves)
        launch_fill_u64(reinterpret_cast<unsigned long long *>(ctx->mhist), 0xFFFFFFFFFFFFFFFEull, g.n, s);
    int li = 0;
    const bool batch = g.gid != nullptr;
    const int64_t G = batch ? g.graphs : 0;
    std::vector<uint8_t> act;
    std::vector<unsigned long long> gg, gm;
    // batches: each graph runs the single graph's sweep sequence (gated,
    // confirming, plain) on its own; gmode holds its current mode
    std::vector<uint8_t> gmode, ggated_h, gconfirm_h;
    std::vector<int32_t> giter_h;
    if (batch) {
        gmode.assign(G, cfg.gated ? (uint8_t)GATED : (uint8_t)PLAIN);
        ggated_h.assign(G, 0);
        gconfirm_h.assign(G, 0);
        giter_h.assign(G, 0);
        act.assign(G, 1);
        for (int64_t k = 0; k < G; k++) act[k] = cfg.gdone && cfg.gdone[k] ? 0 : 1;
        cfg.li_g.assign(G, 0);
        gg.resize(G);
        gm.resize(G);
    }
    // One sweep: clear its counters (a fill kernel, so that the sweep can be
    // captured), then every sub-round's kernels, on stream cs.
    // Sweeps repeat the same launches with the same arguments within a pass
    // (per mode: plain, gated, confirming): each is captured once as a graph
    // and replayed; l_i, the one argument that changes, is read from device
    // memory in replays.  Trace capture and per-kernel timing run launch by
    // launch.
    const bool capture = cfg.use_graphs && !ctx->tracing && !cfg.timing_k;
    auto enqueue_sweep = [&](int sweep, IterCounters *ctr, hipStream_t cs) {
        int64_t *launches = ctx->kernel_launches;
        launch_fill_u64(reinterpret_cast<unsigned long long *>(ctr), 0, sizeof(IterCounters) / 8, cs);
        if (batch) {
            launch_fill_u64(ctx->ggain, 0, G, cs);
            launch_fill_u64(ctx->gmoved, 0, G, cs);
        }
        for (int p = 0; p < P; p++) {
            MoveArgs a;
            a.g = g;
            a.K = K;
            a.sig = ctx->sig;
            a.csize = ctx->csize;
            a.cm = ctx->cm;
            a.M2 = ctx->M2;
            a.flag = ctx->flag;
            a.dec = ctx->dec;
            a.gain_out = nullptr;
            a.queue = ctx->queue;
            int64_t cap = 0;
            for (int b = 0; b < kNumBins; b++) {
                a.qbase[b] = wl.bucket_begin(b, p);
                a.qcap[b] = wl.bucket_size(b, p);
                cap += a.qcap[b];
            }
            a.ctr = ctr;
            a.round = p;
            a.ch_vert = wl.ch_vert;
            a.ch_beg = wl.ch_beg;
            a.ch_first = wl.ch_poff[p];
            a.ch_count = wl.ch_poff[p + 1] - wl.ch_poff[p];
            a.hub_off = wl.hub_off;
            a.hub_act = ctx->hub_act;
            a.hkeys = ctx->sc.hkeys;
            a.hvals = ctx->sc.hvals;
            a.hub_ch0 = ctx->hub_ch0;
            a.part_g = ctx->sc.part_g;
            a.part_kid = ctx->sc.part_kid;
            a.part_c = ctx->sc.part_c;
            a.hub_parts = ctx->hub_parts && ctx->gap_col;
            a.max_parts = ctx->hub_max_parts;
            a.skey = ctx->gap_col;
            a.sval = ctx->gap_w;
            a.hbuck = ctx->sc.hbuck;
            a.hub_b0 = wl.hub_b0;
            a.grid_cap = cfg.grid_cap;
            a.single_only = cfg.single_only;
            // the history feeds the gate's features: once a pass has left its
            // gated sweeps it never returns to them, so later sweeps skip it
            // (the history's per-entry adds to D_j cost most of it); trace
            // capture keeps it in every sweep
            if (hist && (ctx->tracing || mode == GATED)) {
                a.hfrac = ctx->hfrac;
                a.hgain = ctx->hgain;
                a.hbits = ctx->hbits;
                a.dmoved = ctx->dmoved;
                a.dsnap = ctx->dsnap;
                a.pass = cfg.pass;
                a.sweep = sweep;
                a.iter = li;
                a.iter_dev = capture ? ctx->iter_dev : nullptr;   // replays read l_i from memory
                if (ctx->tracing) a.tr = ctx->trace;
            }
            if (mode == GATED) a.cand = ctx->cand;
            if (cfg.return_moves) {
                a.mhist = ctx->mhist;
                a.sweep_dev = ctx->iter_dev + 1;
            }
            if (batch) {
                a.ggain = ctx->ggain;
                a.gmoved = ctx->gmoved;
                a.gactive = ctx->gactive;
                if (mode == GATED) {
                    a.ggated = ctx->ggated;
                    a.giter = ctx->giter;
                }
            }
            if (cap == 0) continue;
            const bool tk = cfg.timing_k && cs == s;
            int t;
            t = tk ? ctx->timer.begin(100 + GSP_K_FRONTIER, cs) : -1;
            launch_move_compact(a, wl, cs);
            ctx->timer.end(t);
            if (mode == GATED) {
                t = tk ? ctx->timer.begin(100 + GSP_K_GATE, cs) : -1;
                launch_gate(a, net, cfg.theta_logit, cap, cs);
                ctx->timer.end(t);
            }
            // the four scans read the same state and write disjoint
            // decisions: the wave-bin, workgroup-bin and hub scans fork onto
            // side streams and join before the moves are applied.  Timed
            // sweeps stay on one stream (timing = 2), so that an event pair
            // around a kernel holds that kernel alone, or keep the side
            // streams (timing = 3): each pair is then on its kernel's own
            // stream and times it as it runs beside the others.
            const bool fork = !cfg.timing_k || cfg.timing_side;
            hipStream_t sw = fork ? ctx->side[0] : cs, sb = fork ? ctx->side[1] : cs, sh = fork ? ctx->side[2] : cs;
            if (fork) {
                hipEvent_t fe = ctx->fork_ev[p];
                (void)hipEventRecord(fe, cs);
                for (hipStream_t q : ctx->side) (void)hipStreamWaitEvent(q, fe, 0);
            }
            // hubs first: their chain of three kernels is the longest path of
            // the sub-round, and enqueued first it gets the compute units
            // first (measured: R-MAT 20 8.5 -> 7.9 ms per run).  On the
            // partition path the chunk scan, the partitions' gather and the
            // decisions; on the global-table path the chunk scan, then the
            // table slices and the decisions
            t = tk && a.qcap[BIN_HUB] ? ctx->timer.begin(100 + GSP_K_MOVE_HUB, sh) : -1;
            if (a.hub_parts) launch_move_hub_parts(a, sh); else launch_move_hub_scan(a, sh);
            ctx->timer.end(t);
            if (a.hub_parts) {
                t = tk && a.qcap[BIN_HUB] ? ctx->timer.begin(100 + GSP_K_MOVE_HUB_GATHER, sh) : -1;
                launch_move_hub_gather(a, sh);
                ctx->timer.end(t);
            }
            t = tk && a.qcap[BIN_HUB] ? ctx->timer.begin(100 + GSP_K_MOVE_HUB_FINISH, sh) : -1;
            if (a.hub_parts) launch_move_hub_decide(a, sh); else launch_move_hub_finish(a, sh);
            ctx->timer.end(t);
            t = tk ? ctx->timer.begin(100 + GSP_K_MOVE_SMALL, cs) : -1;
            launch_move_small(a, wl, cs);
            ctx->timer.end(t);
            t = tk && a.qcap[BIN_WAVE] ? ctx->timer.begin(100 + GSP_K_MOVE_WAVE, sw) : -1;
            launch_move_wave(a, sw);
            ctx->timer.end(t);
            t = tk && a.qcap[BIN_BLOCK] ? ctx->timer.begin(100 + GSP_K_MOVE_BLOCK, sb) : -1;
            launch_move_block(a, sb);
            ctx->timer.end(t);
            for (int q = 0; fork && q < 3; q++) {
                hipEvent_t je = ctx->join_ev[3 * p + q];
                (void)hipEventRecord(je, ctx->side[q]);
                (void)hipStreamWaitEvent(cs, je, 0);
            }
            t = tk ? ctx->timer.begin(100 + GSP_K_MOVE_APPLY, cs) : -1;
            launch_move_apply(a, cap, cs);
            ctx->timer.end(t);
            if (tk) {
                launches[GSP_K_FRONTIER]++;
                launches[GSP_K_GATE] += mode == GATED;
                launches[GSP_K_MOVE_SMALL] += cap - a.qcap[BIN_WAVE] - a.qcap[BIN_BLOCK] -
                                                          a.qcap[BIN_HUB] > 0;
                launches[GSP_K_MOVE_WAVE] += a.qcap[BIN_WAVE] > 0;
                launches[GSP_K_MOVE_BLOCK] += a.qcap[BIN_BLOCK] > 0;
                launches[GSP_K_MOVE_HUB] += a.qcap[BIN_HUB] > 0;
                launches[GSP_K_MOVE_HUB_GATHER] += a.hub_parts && a.qcap[BIN_HUB] > 0;
                launches[GSP_K_MOVE_HUB_FINISH] += (a.hub_parts ? 1 : 2) * (a.qcap[BIN_HUB] > 0);
                launches[GSP_K_MOVE_APPLY]++;
            }
        }
    };
    std::vector<int64_t> key;
    if (capture) {
        if (!ctx->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        auto ptr = [](const void *q) { return (int64_t)(intptr_t)q; };
        key = {g.n, g.nnz, g.wt, g.graphs, ptr(g.off), ptr(g.col), ptr(g.w), ptr(g.deg), ptr(g.gid), ptr(g.vbase),
               ptr(K), P, (int64_t)cfg.grid_cap, ptr(wl.bl), ptr(wl.ch_vert), ptr(wl.ch_beg), ptr(wl.hub_off), ptr(ctx->sc.hkeys),
               ptr(ctx->sc.hvals), ptr(ctx->sc.part_g), ptr(ctx->sc.hbuck), (int64_t)(batch ? 1 : 0),
               ptr(ctx->ggated), ptr(ctx->giter), ptr(g.orig), g.nlong};
        for (int k = 0; k <= kNumBins * P; k++) key.push_back(wl.boff[k]);
        for (int p = 0; p <= P; p++) key.push_back(wl.ch_poff[p]);
        int64_t m2bits;
        memcpy(&m2bits, &ctx->M2, sizeof(m2bits));
        key.push_back(m2bits);
        // the gate's inputs: its network (b3 is a kernel argument), the pass
        // (a feature) and theta; the hub paths the sweep launches
        int32_t thbits, b3bits;
        memcpy(&thbits, &cfg.theta_logit, sizeof(thbits));
        memcpy(&b3bits, &net.b3, sizeof(b3bits));
        key.push_back((int64_t)cfg.return_moves);   // the kernels' move records (or none)
        key.push_back((int64_t)cfg.single_only);
        key.insert(key.end(), {(int64_t)hist, (int64_t)cfg.pass, (int64_t)thbits, (int64_t)b3bits, ptr(net.w1),
                               ptr(net.w2), ptr(net.b1), ptr(ctx->hbits), (int64_t)ctx->hub_parts,
                               (int64_t)ctx->hub_max_parts});
    }
    for (int sweep = 0;; sweep++) {
        if (batch) {
            bool any = false, any_gated = false, any_confirm = false;
            for (int64_t k = 0; k < G; k++) {
                // a graph's last countable iteration is a confirming sweep
                if (act[k] && gmode[k] == GATED && cfg.li_g[k] + 1 >= cfg.max_iter) gmode[k] = CONFIRM;
                any = any || act[k] != 0;
                ggated_h[k] = act[k] && gmode[k] == GATED;
                gconfirm_h[k] = act[k] && gmode[k] == CONFIRM;
                giter_h[k] = cfg.li_g[k];
                any_gated = any_gated || ggated_h[k];
                any_confirm = any_confirm || gconfirm_h[k];
            }
            if (!any) break;
            HIP_TRY(hipMemcpyAsync(ctx->gactive, act.data(), G, hipMemcpyHostToDevice, s));
            if (cfg.gated) {
                HIP_TRY(hipMemcpyAsync(ctx->ggated, ggated_h.data(), G, hipMemcpyHostToDevice, s));
                HIP_TRY(hipMemcpyAsync(ctx->giter, giter_h.data(), G * sizeof(int32_t), hipMemcpyHostToDevice, s));
            }
            if (any_confirm) {
                HIP_TRY(hipMemcpyAsync(ctx->gconfirm, gconfirm_h.data(), G, hipMemcpyHostToDevice, s));
                launch_batch_flag_confirm(g.gid, ctx->gconfirm, g.n, ctx->flag, s);
                cfg.confirm_sweeps++;
            }
            // the sweep runs the gate if any graph is in its gated sweeps
            mode = any_gated ? GATED : PLAIN;
        } else if (li >= cfg.max_iter) {
            break;
        } else if (mode == GATED && li + 1 >= cfg.max_iter) {
            // the last iteration the phase may count is a confirming sweep:
            // a phase never ends on gated sweeps alone
            mode = CONFIRM;
        }
        cfg.sweeps++;
        if (!batch && mode == CONFIRM) {
            launch_fill_u8(ctx->flag, 1, g.n, s);
            cfg.confirm_sweeps++;
        }
        IterCounters *ctr = capture ? ctx->ctr : ctx->ctr + (sweep & 1);
        // l_i (the gate's feature) and the sweep index, read by the kernels
        ctx->i64_h[6] = li;
        ctx->i64_h[7] = sweep;
        HIP_TRY(hipMemcpyAsync(ctx->iter_dev, &ctx->i64_h[6], 2 * sizeof(int64_t), hipMemcpyHostToDevice, s));
        if (capture) {
            std::vector<int64_t> km = key;
            km.push_back((int64_t)mode);
            hipGraphExec_t exec = nullptr;
            for (auto &x : ctx->sweep_graphs)
                if (x.key == km) exec = x.exec;
            if (!exec) {
                HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
                enqueue_sweep(sweep, ctr, ctx->cap_stream);
                hipGraph_t graph = nullptr;
                hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
                if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                if (graph) (void)hipGraphDestroy(graph);
                if (e != hipSuccess) return ctx->fail_hip(e, "sweep graph capture");
                if (ctx->sweep_graphs.size() >= 64) ctx->drop_sweep_graphs();
                ctx->sweep_graphs.push_back({km, exec});
            }
            HIP_TRY(hipGraphLaunch(exec, s));
        } else {
            enqueue_sweep(sweep, ctr, s);
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(ctx->ctr_h, ctr, sizeof(IterCounters), hipMemcpyDeviceToHost, s));
        if (batch) {
            HIP_TRY(hipMemcpyAsync(gg.data(), ctx->ggain, G * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(gm.data(), ctx->gmoved, G * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        }
        HIP_TRY(hipStreamSynchronize(s));
        CounterStripe h;
        memset(&h, 0, sizeof(h));
        for (int q = 0; q < kStripes; q++) {
            const CounterStripe &x = ctx->ctr_h->st[q];
            h.gain += x.gain;   // integer units: exact, in any order
            h.moved += x.moved;
            h.pruned += x.pruned;
            for (int c = 0; c < kMoveClasses; c++) {
                h.verts[c] += x.verts[c];
                h.scanned[c] += x.scanned[c];
                h.keys[c] += x.keys[c];
                h.ginserts[c] += x.ginserts[c];
                h.aux[c] += x.aux[c];
            }
        }
        const double dq = ldexp((double)h.gain, -61);   // the movers' delta-modularity (gain_units)
        ctx->stats.moves += (int64_t)h.moved;
        cfg.pruned += (int64_t)h.pruned;
        for (int c = 0; c < kMoveClasses; c++) {
            cfg.scanned_entries += (int64_t)h.scanned[c];
            // hubs are counted once, by the decision kernel (class 5 counts chunks)
            if (c != 5) cfg.scanned_vertices += (int64_t)h.verts[c];
            ctx->stats.kernels[kClassKernel[c]].items += (int64_t)(c == 5 ? h.ginserts[c] : h.scanned[c]);
            if (cfg.kernel_bytes) cfg.kernel_bytes[kClassKernel[c]] += move_bytes(c, h, g.wt);
        }
        if (mode == GATED && cfg.kernel_bytes) {
            // per candidate: vertex id, degree, K, membership, Sigma, history
            // (9 B) in; queue slot out
            int64_t nc = 0;
            for (int p = 0; p < P; p++)
                for (int b = 0; b < kNumBins; b++) nc += ctx->ctr_h->ccnt[p][b];
            cfg.kernel_bytes[GSP_K_GATE] += 41.0 * (double)nc;
            ctx->stats.kernels[GSP_K_GATE].items += nc;
        }
        if (batch) {
            // each graph's own convergence test (its movers' delta-modularity)
            for (int64_t k = 0; k < G; k++) {
                if (!act[k]) continue;
                const double dqk = ldexp((double)gg[k], -61);
                if (gmode[k] != CONFIRM || gm[k] > 0) cfg.li_g[k]++;   // as counted for one graph
                if (dqk <= cfg.tau) {
                    if (gmode[k] == GATED)
                        gmode[k] = CONFIRM;
                    else
                        act[k] = 0;
                } else if (gmode[k] == CONFIRM) {
                    gmode[k] = PLAIN;
                }
                if (cfg.li_g[k] >= cfg.max_iter) act[k] = 0;
            }
            li++;
            continue;
        }
        const bool counted = mode != CONFIRM || h.moved > 0;
        if (counted) {
            if (cfg.dq_out) cfg.dq_out[li] = dq;
            if (cfg.moved_out) cfg.moved_out[li] = (int64_t)h.moved;
            li++;
        }
        if (dq <= cfg.tau) {
            if (mode == GATED) {
                mode = CONFIRM;
                continue;
            }
            break;
        }
        if (mode == CONFIRM) mode = PLAIN;
    }
    cfg.li = li;
    return GSP_OK;
}

gsp_status ensure_levels(gsp_ctx *ctx) {
    if (ctx->offL[0]) return GSP_OK;
    if (ctx->mem_limit) {
        uint64_t need = 2 * ((ctx->n + 1) * 8 + ctx->nnz * 12 + ctx->n * 12) + ctx->nnz * 12 + ctx->n * 8 + 16;
        if (ctx->mem_used + need > ctx->mem_limit)
            return ctx->fail(GSP_ENOMEM, "device memory limit (mem_limit_bytes) reached");
    }
    hipError_t e = hipSuccess;
    for (int k = 0; k < 2; k++) {
        ctx->offL[k] = ctx->dalloc<int64_t>(ctx->n + 1, &e);
        if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(level offsets)");
        ctx->colL[k] = ctx->dalloc<int32_t>(ctx->nnz, &e);
        if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(level columns)");
        ctx->wL[k] = ctx->dalloc<double>(ctx->nnz, &e);
        if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(level weights)");
        ctx->degL[k] = ctx->dalloc<int32_t>(ctx->n, &e);
        if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(level degrees)");
        ctx->KL[k] = ctx->dalloc<double>(ctx->n, &e);
        if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(level weights K)");
    }
    ctx->gap_col = ctx->dalloc<int32_t>(ctx->nnz, &e);
    if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(gap columns)");
    ctx->gap_w = ctx->dalloc<double>(ctx->nnz, &e);
    if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(gap weights)");
    ctx->mhist = ctx->dalloc<int64_t>(ctx->n, &e);
    if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(move records)");
    ctx->iter_dev = ctx->dalloc<int64_t>(2, &e);
    if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(sweep index)");
    return GSP_OK;
}

gsp_status ensure_leiden(gsp_ctx *ctx) {
    if (ctx->bnd) return GSP_OK;
    if (ctx->mem_limit && ctx->mem_used + 8 * (uint64_t)ctx->n + 16 > ctx->mem_limit)
        return ctx->fail(GSP_ENOMEM, "device memory limit (mem_limit_bytes) reached (refinement)");
    hipError_t e = hipSuccess;
    ctx->bnd = ctx->dalloc<int32_t>(ctx->n, &e);
    if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(bound communities)");
    ctx->bstart = ctx->dalloc<int32_t>(ctx->n, &e);
    if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(starting communities)");
    return GSP_OK;
}

// GSP-Leiden's refinement of level g (Section 3.5, read greedily) within the
// communities ctx->bnd, from the sub-communities in ctx->cm / sig / csize:
// the local-moving phase over the same-bound subgraph (built in the level
// buffers of `slot`, which the caller's next aggregation overwrites) with
// g's K and 2m, only vertices alone in their sub-community moving.  wl holds
// g's work lists; its buffers then hold the subgraph's, so the caller builds
// g's again before it uses them.
gsp_status refine_level(gsp_ctx *ctx, const Level &g, const double *K, const WorkLists &wl, int slot,
                        PhaseCfg &pc, int rounds) {
    hipStream_t s = ctx->stream;
    Level r = g;
    r.nlong = 0;
    r.off = ctx->offL[slot];
    r.col = ctx->colL[slot];
    r.deg = ctx->degL[slot];
    r.wt = g.wt == W_UNIT ? W_UNIT : W_F64;
    r.w = r.wt == W_UNIT ? nullptr : ctx->wL[slot];
    // the gap buffer (hub staging of the local-moving phases, the
    // aggregation's rows) is idle here: a byte per entry of g
    HIP_TRY(bound_subgraph(g, wl, ctx->bnd, ctx->degL[slot], ctx->offL[slot], ctx->colL[slot], ctx->wL[slot],
                           ctx->sc.cch_k0, reinterpret_cast<uint8_t *>(ctx->gap_col), ctx->sc.scan_tmp, s));
    HIP_TRY(hipMemcpyAsync(ctx->i64_h, ctx->offL[slot] + g.n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    r.nnz = ctx->i64_h[0];
    WorkLists wr = make_lists(ctx);
    HIP_TRY(build_work_lists(r, rounds, wr, ctx->sc, s));
    pc.single_only = true;
    pc.return_moves = false;
    pc.gated = false;
    return move_phase(ctx, r, K, wr, pc);
}

// Whether gsp_run stores the input graph in degree order (vertex_order;
// batches never).
constexpr int64_t kAutoOrderEntries = int64_t(1) << 25;
// Device bytes of the copy in degree order.
uint64_t order_bytes(const gsp_ctx *ctx) {
    const int wb = ctx->wt0 == W_UNIT ? 0 : (ctx->wt0 == W_F32 ? 4 : 8);
    return (uint64_t)ctx->n * 20 + (uint64_t)(ctx->n + 1) * 8 + (uint64_t)ctx->nnz * (4 + wb) +
           16 * (uint64_t)kOrderBucketsMax + 64;
}

// AUTO keeps the loaded order where the copy would pass mem_limit_bytes.
bool wants_order(const gsp_ctx *ctx, const gsp_options &opt, bool batch, int32_t max_passes) {
    if (batch || max_passes == 0 || ctx->n == 0 || ctx->nnz == 0) return false;
    if (opt.vertex_order == GSP_ORDER_DEGREE) return true;
    if (opt.vertex_order != GSP_ORDER_AUTO || ctx->nnz < kAutoOrderEntries) return false;
    return ctx->ordered || !ctx->mem_limit || ctx->mem_used + order_bytes(ctx) <= ctx->mem_limit;
}

// Builds the input graph's copy in degree order once per load (again when
// a run asks for another number of sub-rounds: the layout groups the
// shorter rows by sub-round).
gsp_status ensure_order(gsp_ctx *ctx, int rounds) {
    if (ctx->ordered && ctx->ord.rounds == rounds) return GSP_OK;
    if (ctx->ordered) {
        ctx->drop_sweep_graphs();   // captured sweeps hold the old layout's work lists
        HIP_TRY(order_by_degree(level0(ctx), ctx->sc, ctx->ord, rounds, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        return GSP_OK;
    }
    const int64_t n = ctx->n, nnz = ctx->nnz;
    const int wb = ctx->wt0 == W_UNIT ? 0 : (ctx->wt0 == W_F32 ? 4 : 8);
    if (ctx->mem_limit) {
        if (ctx->mem_used + order_bytes(ctx) > ctx->mem_limit)
            return ctx->fail(GSP_ENOMEM, "device memory limit (mem_limit_bytes) reached (degree order)");
    }
    hipError_t e = hipSuccess;
    DegreeOrder o;
    auto fail = [&](const char *what) { return ctx->fail_hip(e, what); };
    if (!(o.orig = ctx->dalloc<int32_t>(n, &e))) return fail("hipMalloc(order)");
    if (!(o.rank = ctx->dalloc<int32_t>(n, &e))) return fail("hipMalloc(order rank)");
    if (!(o.deg = ctx->dalloc<int32_t>(n, &e))) return fail("hipMalloc(order degrees)");
    if (!(o.off = ctx->dalloc<int64_t>(n + 1, &e))) return fail("hipMalloc(order offsets)");
    if (!(o.col = ctx->dalloc<int32_t>(nnz, &e))) return fail("hipMalloc(order columns)");
    if (wb == 4 && !(o.w = ctx->dalloc<float>(nnz, &e))) return fail("hipMalloc(order weights)");
    if (wb == 8 && !(o.w = ctx->dalloc<double>(nnz, &e))) return fail("hipMalloc(order weights)");
    if (!(o.hist = ctx->dalloc<unsigned long long>(2 * kOrderBucketsMax, &e))) return fail("hipMalloc(order counters)");
    double *K = ctx->dalloc<double>(n, &e);
    if (!K) return fail("hipMalloc(order K)");
    HIP_TRY(order_by_degree(level0(ctx), ctx->sc, o, rounds, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->ord = o;
    ctx->Kord = K;
    ctx->ordered = true;
    return GSP_OK;
}

int bit_length(uint64_t x) {
    int b = 0;
    while (x) {
        b++;
        x >>= 1;
    }
    return b;
}

// The grid of exact sums for weights w[0..nnz) (host copy, fp32): returns S
// with every weight rounded to the nearest multiple of 2^-S (ties to even)
// in place, *moved = weights that changed.  Same rule as the device kernels
// (launch_weight_grid): S = 52 - bits(U) + T, U = sum of max(1, ceil(w 2^T))
// over the positive weights, T = 62 - bits(nnz) - e with max(w) < 2^e.
int32_t host_weight_grid(float *w, int64_t nnz, int64_t *moved) {
    *moved = 0;
    double wmax = 0.0;
    for (int64_t e = 0; e < nnz; e++) wmax = std::max(wmax, (double)w[e]);
    if (!(wmax > 0.0)) return 0;
    int ew = 0;
    (void)std::frexp(wmax, &ew);
    const int T = 62 - bit_length((uint64_t)nnz) - ew;
    uint64_t U = 0;
    for (int64_t e = 0; e < nnz; e++) {
        if (!(w[e] > 0.0f)) continue;
        const double t = std::ceil(std::ldexp((double)w[e], T));
        U += t < 1.0 ? 1u : (uint64_t)t;
    }
    const int S = std::min(1022, std::max(-1000, 52 - bit_length(U) + T));
    for (int64_t e = 0; e < nnz; e++) {
        const double q = std::ldexp(std::nearbyint(std::ldexp((double)w[e], S)), -S);
        if (q != (double)w[e]) {
            w[e] = (float)q;
            (*moved)++;
        }
    }
    return S;
}

// Loads a CSR given as int64 offsets (off64) or int32 offsets (off32).
// grid = false when the caller has taken the weights onto their grids
// already (a batch: one grid per graph).
gsp_status load_impl(gsp_ctx *ctx, int64_t n, int64_t nnz, const int64_t *off64, const int32_t *off32,
                     const int32_t *cols, const void *weights, int wt, int where, bool grid = true) {
    if (n < 1 || nnz < 0) return ctx->fail(GSP_EINVAL, "n must be >= 1 and nnz >= 0");
    if (n > 0x7fffffffLL - 1) return ctx->fail(GSP_EINVAL, "n must be below 2^31 - 1 (int32 vertex ids)");
    if (where != GSP_HOST && where != GSP_DEVICE) return ctx->fail(GSP_EINVAL, "bad `where`");
    if (!off64 && !off32) return ctx->fail(GSP_EINVAL, "offsets is NULL");
    if (nnz > 0 && !cols) return ctx->fail(GSP_EINVAL, "cols is NULL");
    ctx->free_graph();
    hipError_t e = hipSuccess;
    hipStream_t s = ctx->stream;
    auto A = [&](auto *&ptr, size_t count, const char *what) -> gsp_status {
        using T = std::remove_reference_t<decltype(*ptr)>;
        ptr = ctx->dalloc<T>(count, &e);
        if (e != hipSuccess) {
            gsp_status st = ctx->fail_hip(e, what);
            ctx->free_graph();
            return st;
        }
        return GSP_OK;
    };
    gsp_status st;
    int64_t n1 = n + 1;
    if ((st = A(ctx->off0, n1, "hipMalloc(offsets)")) != GSP_OK) return st;
    if ((st = A(ctx->col0, nnz, "hipMalloc(cols)")) != GSP_OK) return st;
    if (wt == W_F32) {
        float *w = nullptr;
        if ((st = A(w, nnz, "hipMalloc(weights)")) != GSP_OK) return st;
        ctx->w0 = w;
    } else if (wt == W_F64) {
        double *w = nullptr;
        if ((st = A(w, nnz, "hipMalloc(weights)")) != GSP_OK) return st;
        ctx->w0 = w;
    }
    if ((st = A(ctx->deg0, n, "hipMalloc(deg)")) != GSP_OK) return st;
    if ((st = A(ctx->K0, n, "hipMalloc(K)")) != GSP_OK) return st;
    if ((st = A(ctx->sig, n, "hipMalloc(sigma)")) != GSP_OK) return st;
    if ((st = A(ctx->cm, n, "hipMalloc(membership)")) != GSP_OK) return st;
    if ((st = A(ctx->csize, n, "hipMalloc(sizes)")) != GSP_OK) return st;
    if ((st = A(ctx->dec, n, "hipMalloc(decisions)")) != GSP_OK) return st;
    if ((st = A(ctx->queue, n, "hipMalloc(queue)")) != GSP_OK) return st;
    if ((st = A(ctx->lab, n, "hipMalloc(labels)")) != GSP_OK) return st;
    if ((st = A(ctx->top, n, "hipMalloc(top membership)")) != GSP_OK) return st;
    if ((st = A(ctx->bl, n, "hipMalloc(work lists)")) != GSP_OK) return st;
    if ((st = A(ctx->tmp32, n + 1, "hipMalloc(tmp)")) != GSP_OK) return st;
    if ((st = A(ctx->flag, n, "hipMalloc(flags)")) != GSP_OK) return st;
    if ((st = A(ctx->hub_act, n, "hipMalloc(hub flags)")) != GSP_OK) return st;
    if ((st = A(ctx->hub_off, n, "hipMalloc(hub offsets)")) != GSP_OK) return st;
    if ((st = A(ctx->hub_ch0, n, "hipMalloc(hub chunk ids)")) != GSP_OK) return st;
    if ((st = A(ctx->hub_b0, n, "hipMalloc(hub partition offsets)")) != GSP_OK) return st;
    if ((st = A(ctx->gain_tmp, n, "hipMalloc(gains)")) != GSP_OK) return st;
    Scratch &sc = ctx->sc;
    sc.n_cap = n;
    sc.nnz_cap = nnz;
    sc.scan_tmp_bytes = scan_tmp_bytes(n1 > nnz ? n1 : nnz);
    char *stmp = nullptr;
    if ((st = A(stmp, sc.scan_tmp_bytes, "hipMalloc(scan)")) != GSP_OK) return st;
    sc.scan_tmp = stmp;
    for (int64_t **p : {&sc.i64a, &sc.i64b, &sc.i64c, &sc.i64d, &sc.i64e, &sc.i64f, &sc.i64g})
        if ((st = A(*p, n1, "hipMalloc(scratch)")) != GSP_OK) return st;
    if ((st = A(sc.u8a, n1, "hipMalloc(scratch)")) != GSP_OK) return st;
    for (int32_t **p : {&sc.i32a, &sc.i32b, &sc.i32c, &sc.i32d, &sc.i32e, &sc.bl2})
        if ((st = A(*p, n1, "hipMalloc(scratch)")) != GSP_OK) return st;
    if ((st = A(sc.err, 4, "hipMalloc(err)")) != GSP_OK) return st;
    if ((st = A(sc.u64, kScratchU64, "hipMalloc(counters)")) != GSP_OK) return st;
    if ((st = A(sc.f64, 16, "hipMalloc(scalars)")) != GSP_OK) return st;
    // chunks: vertex hubs need <= nnz/2048 + #hubs, hub communities <=
    // nnz/1024 + #hubs, with #hubs <= nnz/2049
    sc.ch_cap = nnz / 512 + 16;
    if ((st = A(sc.ch_vert, sc.ch_cap, "hipMalloc(chunks)")) != GSP_OK) return st;
    if ((st = A(sc.ch_beg, sc.ch_cap, "hipMalloc(chunks)")) != GSP_OK) return st;
    if ((st = A(sc.cch_comm, sc.ch_cap, "hipMalloc(chunks)")) != GSP_OK) return st;
    if ((st = A(sc.cch_beg, sc.ch_cap, "hipMalloc(chunks)")) != GSP_OK) return st;
    if ((st = A(sc.cch_k0, sc.ch_cap, "hipMalloc(chunks)")) != GSP_OK) return st;
    if ((st = A(sc.cseg_comm, sc.ch_cap, "hipMalloc(segments)")) != GSP_OK) return st;
    if ((st = A(sc.cseg_beg, sc.ch_cap, "hipMalloc(segments)")) != GSP_OK) return st;
    if ((st = A(sc.part_g, sc.ch_cap, "hipMalloc(hub partials)")) != GSP_OK) return st;
    if ((st = A(sc.part_kid, sc.ch_cap, "hipMalloc(hub partials)")) != GSP_OK) return st;
    if ((st = A(sc.part_c, sc.ch_cap, "hipMalloc(hub partials)")) != GSP_OK) return st;
    if ((st = A(ctx->ctr, 2, "hipMalloc(iteration counters)")) != GSP_OK) return st;
    if ((st = A(ctx->lp_counts, 4, "hipMalloc(split counters)")) != GSP_OK) return st;

    // copy in
    hipMemcpyKind kind = where == GSP_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (off64) {
        HIP_TRY(hipMemcpyAsync(ctx->off0, off64, n1 * sizeof(int64_t), kind, s));
    } else {
        HIP_TRY(hipMemcpyAsync(ctx->tmp32, off32, n1 * sizeof(int32_t), kind, s));
        launch_offsets_from_i32(ctx->tmp32, ctx->off0, n1, s);
    }
    if (nnz) HIP_TRY(hipMemcpyAsync(ctx->col0, cols, nnz * sizeof(int32_t), kind, s));
    if (wt == W_F32 && nnz) HIP_TRY(hipMemcpyAsync(ctx->w0, weights, nnz * sizeof(float), kind, s));
    if (wt == W_F64 && nnz) HIP_TRY(hipMemcpyAsync(ctx->w0, weights, nnz * sizeof(double), kind, s));
    HIP_TRY(hipMemsetAsync(sc.err, 0, sizeof(int), s));
    launch_validate(ctx->off0, ctx->col0, ctx->w0, wt, n, nnz, sc.err, s);
    int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, sc.err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (bad) {
        ctx->free_graph();
        std::string m = "malformed CSR:";
        if (bad & 1) m += " offsets (must start at 0, not decrease, end at nnz, rows below 2^31 entries)";
        if (bad & 2) m += " column outside [0, n)";
        if (bad & 4) m += " weight negative, NaN or infinite";
        return ctx->fail(GSP_EGRAPH, m);
    }
    ctx->n = n;
    ctx->nnz = nnz;
    ctx->wt0 = wt;
    launch_degrees(ctx->off0, ctx->deg0, n, s);
    // the weight grid (exact sums): the largest weight, the exact bound of
    // the total, then the rounding (a no-op unless the total needs it)
    ctx->grid_S = 0;
    ctx->grid_moved = 0;
    if (grid && wt != W_UNIT && nnz > 0) {
        unsigned long long *u = sc.u64;
        launch_fill_u64(u, 0, 3, s);
        launch_weight_max(ctx->w0, wt, nnz, u, s);
        HIP_TRY(hipMemcpyAsync(ctx->i64_h, u, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        double wmax = 0.0;
        memcpy(&wmax, ctx->i64_h, sizeof(double));
        if (wmax > 0.0) {
            int ew = 0;
            (void)std::frexp(wmax, &ew);
            const int T = 62 - bit_length((uint64_t)nnz) - ew;
            launch_weight_bound(ctx->w0, wt, nnz, T, u + 1, s);
            HIP_TRY(hipMemcpyAsync(ctx->i64_h, u + 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            const int S = std::min(1022, std::max(-1000, 52 - bit_length((uint64_t)ctx->i64_h[0]) + T));
            launch_weight_grid(ctx->w0, wt, nnz, S, u + 2, s);
            HIP_TRY(hipMemcpyAsync(ctx->i64_h, u + 2, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            ctx->grid_S = S;
            ctx->grid_moved = ctx->i64_h[0];
        }
    }
    HIP_TRY(hipMemsetAsync(sc.f64, 0, sizeof(double), s));
    Level g = level0(ctx);
    launch_vertex_weights(g, ctx->K0, sc.f64, s);
    HIP_TRY(hipMemcpyAsync(ctx->f64_h, sc.f64, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    ctx->M2 = ctx->f64_h[0];
    ctx->loaded = true;
    return GSP_OK;
}

gsp_status check_where(gsp_ctx *ctx, int where) {
    if (where != GSP_HOST && where != GSP_DEVICE) return ctx->fail(GSP_EINVAL, "bad `where`");
    return GSP_OK;
}

// Q = sigma_in / M2 - sum_c (Sigma_c / M2)^2 of membership m (device, valid).
gsp_status modularity_of(gsp_ctx *ctx, const int32_t *m, double *out) {
    hipStream_t s = ctx->stream;
    if (ctx->M2 <= 0.0) {
        *out = 0.0;
        return GSP_OK;
    }
    launch_fill_f64(ctx->sig, 0.0, ctx->n, s);
    launch_fill_f64(ctx->sc.f64, 0.0, 1, s);
    launch_fill_u64(ctx->sc.u64, 0, 1, s);
    launch_community_totals(ctx->K0, m, ctx->n, ctx->sig, nullptr, s);
    launch_modularity_parts(level0(ctx), m, ctx->K0, ctx->sig, ctx->sc.f64, s);
    launch_sum_squares(ctx->sig, ctx->n, ctx->M2, ctx->sc.u64, s);
    HIP_TRY(hipMemcpyAsync(ctx->f64_h, ctx->sc.f64, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(ctx->i64_h, ctx->sc.u64, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    *out = ctx->f64_h[0] / ctx->M2 - ldexp((double)(uint64_t)ctx->i64_h[0], -62);
    return GSP_OK;
}

}  // namespace

// =====================================================================
// C ABI
// =====================================================================

gsp_status check_options(gsp_ctx *ctx, const gsp_options &opt) {
    if (opt.max_iterations < 0 || opt.max_iterations > 100 || !valid_rounds(opt.sub_rounds) ||
        !(opt.tolerance_drop > 0.0) || opt.split_mode < 0 || opt.split_mode > 2)
        return ctx->fail(GSP_EINVAL,
                         "bad options (max_iterations in [0, 100]; sub_rounds a power of two in [1, 64])");
    if (opt.prune_mode != GSP_PRUNE_PLAIN && opt.prune_mode != GSP_PRUNE_LEARNED)
        return ctx->fail(GSP_EINVAL, "bad prune_mode");
    if (opt.timing < 0 || opt.timing > 3) return ctx->fail(GSP_EINVAL, "timing must lie in [0, 3]");
    if (opt.return_moves != 0 && opt.return_moves != 1) return ctx->fail(GSP_EINVAL, "return_moves must be 0 or 1");
    if (opt.grid_cap < 0) return ctx->fail(GSP_EINVAL, "grid_cap must be >= 0");
    if (opt.vertex_order < GSP_ORDER_AUTO || opt.vertex_order > GSP_ORDER_DEGREE)
        return ctx->fail(GSP_EINVAL, "vertex_order must be GSP_ORDER_AUTO, GSP_ORDER_LOADED or GSP_ORDER_DEGREE");
    if (opt.split_algo != GSP_SPLIT_UF && opt.split_algo != GSP_SPLIT_LPP)
        return ctx->fail(GSP_EINVAL, "split_algo must be GSP_SPLIT_UF or GSP_SPLIT_LPP");
    if (opt.hub_max_parts < 0 || opt.hub_max_parts > kMaxParts)
        return ctx->fail(GSP_EINVAL, "hub_max_parts must lie in [0, 4096]");
    if (opt.leiden != 0 && opt.leiden != 1) return ctx->fail(GSP_EINVAL, "leiden must be 0 or 1");
    if (opt.leiden && opt.prune_mode != GSP_PRUNE_PLAIN)
        return ctx->fail(GSP_EINVAL, "GSP-Leiden (leiden = 1) runs with prune_mode GSP_PRUNE_PLAIN");
    if (opt.prune_mode == GSP_PRUNE_LEARNED) {
        if (!(opt.prune_threshold > 0.0f && opt.prune_threshold < 1.0f))
            return ctx->fail(GSP_EINVAL, "prune_threshold must lie in (0, 1)");
        if (!ctx->have_net) return ctx->fail(GSP_ESTATE, "learned pruning needs a network (gsp_pruner_set)");
    }
    return GSP_OK;
}

// The gate compares the logit z with logit(theta) (p >= theta <=> z >= logit(theta)).
float theta_logit(float theta) {
    double t = (double)theta;
    return (float)std::log(t / (1.0 - t));
}

extern "C" {

gsp_status gsp_default_options(gsp_options *out) {
    if (!out) return GSP_EINVAL;
    memset(out, 0, sizeof(*out));
    out->max_iterations = 20;
    out->sub_rounds = 8;
    out->tolerance_drop = 10.0;
    out->aggregation_tolerance = 0.8;
    out->split_mode = GSP_SPLIT_PASS;
    out->timing = 0;
    out->mem_limit_bytes = 0;
    out->prune_mode = GSP_PRUNE_PLAIN;
    out->prune_threshold = 0.5f;
    out->use_graphs = 1;
    out->timing_mask = 0;
    out->hub_global = 0;
    out->hub_max_parts = 0;
    out->return_moves = 0;
    out->split_algo = GSP_SPLIT_UF;
    out->vertex_order = GSP_ORDER_AUTO;
    out->leiden = 0;
    return GSP_OK;
}

gsp_status gsp_create(int device, void *hip_stream, gsp_ctx **out) {
    if (!out) return GSP_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return GSP_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return GSP_EHIP;
    gsp_ctx *ctx = new (std::nothrow) gsp_ctx();
    if (!ctx) return GSP_ENOMEM;
    ctx->device = device;
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return GSP_EHIP;
        }
        ctx->own_stream = true;
    }
    if (hipHostMalloc((void **)&ctx->ctr_h, sizeof(IterCounters), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&ctx->i64_h, 16 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&ctx->f64_h, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        gsp_destroy(ctx);
        return GSP_ENOMEM;
    }
    ctx->timer.s = ctx->stream;
    memset(&ctx->stats, 0, sizeof(ctx->stats));
    *out = ctx;
    return GSP_OK;
}

gsp_status gsp_destroy(gsp_ctx *ctx) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    ctx->free_graph();
    for (void *p : ctx->persist) (void)hipFree(p);
    ctx->persist.clear();
    if (ctx->ctr_h) (void)hipHostFree(ctx->ctr_h);
    if (ctx->i64_h) (void)hipHostFree(ctx->i64_h);
    if (ctx->f64_h) (void)hipHostFree(ctx->f64_h);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    ctx->drop_sweep_graphs();
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    for (hipStream_t q : ctx->side)
        if (q) (void)hipStreamDestroy(q);
    for (hipEvent_t e : ctx->fork_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->join_ev) (void)hipEventDestroy(e);
    delete ctx;
    return GSP_OK;
}

const char *gsp_last_error(const gsp_ctx *ctx) {
    if (!ctx) return "no context";
    return ctx->err.c_str();
}

gsp_status gsp_load_csr(gsp_ctx *ctx, int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols,
                        const float *weights, int where) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    return load_impl(ctx, n, nnz, offsets, nullptr, cols, weights, weights ? W_F32 : W_UNIT, where);
}

gsp_status gsp_load_csr32(gsp_ctx *ctx, int32_t n, int32_t nnz, const int32_t *offsets, const int32_t *cols,
                          const float *weights, int where) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (!offsets) return ctx->fail(GSP_EINVAL, "offsets is NULL");
    return load_impl(ctx, n, nnz, nullptr, offsets, cols, weights, weights ? W_F32 : W_UNIT, where);
}

gsp_status gsp_load_csr_f64(gsp_ctx *ctx, int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols,
                            const double *weights, int where) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    return load_impl(ctx, n, nnz, offsets, nullptr, cols, weights, weights ? W_F64 : W_UNIT, where);
}

}  // extern "C"

namespace {

// The split of level g by membership cm into labels: union-find, or
// minimum-label propagation (split_algo).  *rounds += the propagation rounds.
gsp_status run_split(gsp_ctx *ctx, const Level &g, const WorkLists &wl, const int32_t *cm, int32_t *labels,
                     int algo, int32_t *rounds) {
    hipStream_t s = ctx->stream;
    if (algo == GSP_SPLIT_LPP) {
        int r = launch_split_lp(g, cm, labels, ctx->sc.u8a, ctx->sc.i32d, ctx->sc.i32e, ctx->lp_counts,
                                reinterpret_cast<int *>(ctx->i64_h + 12), s);
        if (r < 0) return ctx->fail_hip(hipGetLastError(), "split by label propagation");
        if (rounds) *rounds += r;
        return GSP_OK;
    }
    launch_split(g, wl, cm, labels, ctx->sc.i32c, reinterpret_cast<uint32_t *>(ctx->sc.i32a),
                 reinterpret_cast<unsigned long long *>(ctx->sc.i64a), s);
    return GSP_OK;
}

// Algorithm "louvain" on the loaded graph, or on the loaded batch of graphs
// (batch = true): then every graph keeps its own 2m, convergence tests,
// iteration counts and passes, and a graph that has finished stays still
// while the others go on; its levels are still aggregated with the rest.
gsp_status run_passes(gsp_ctx *ctx, double tolerance, int32_t max_passes, const gsp_options *optp, bool batch) {
    if (!ctx->loaded) return ctx->fail(GSP_ESTATE, "no graph loaded");
    if (batch && ctx->batch_graphs == 0) return ctx->fail(GSP_ESTATE, "no batch loaded (gsp_load_batch)");
    gsp_options opt;
    if (optp)
        opt = *optp;
    else
        gsp_default_options(&opt);
    if (!(tolerance >= 0.0) || max_passes < 0) return ctx->fail(GSP_EINVAL, "tolerance < 0 or max_passes < 0");
    gsp_status st0 = check_options(ctx, opt);
    if (st0 != GSP_OK) return st0;
    const bool leiden = opt.leiden != 0;
    if (leiden && (batch || ctx->tracing))
        return ctx->fail(GSP_EINVAL, "GSP-Leiden (leiden = 1) runs single graphs without trace capture");
    ctx->mem_limit = opt.mem_limit_bytes;
    if (ctx->mem_limit && ctx->mem_used > ctx->mem_limit)
        return ctx->fail(GSP_ENOMEM, "device memory limit (mem_limit_bytes) reached");
    gsp_status st = ensure_levels(ctx);
    if (st != GSP_OK) return st;
    if (leiden && (st = ensure_leiden(ctx)) != GSP_OK) return st;
    const bool ordered = wants_order(ctx, opt, batch, max_passes);
    if (ordered && (st = ensure_order(ctx, opt.sub_rounds)) != GSP_OK) return st;
    hipStream_t s = ctx->stream;
    ctx->have_result = false;
    ctx->have_batch_result = false;
    ctx->have_q = false;
    memset(&ctx->stats, 0, sizeof(ctx->stats));
    ctx->timer.reset();
    ctx->timer.kmask = opt.timing_mask;
    ctx->hub_parts = opt.hub_global == 0;
    ctx->hub_max_parts = opt.hub_max_parts ? opt.hub_max_parts : kMaxParts;
    bool tphase = opt.timing >= 1, tk = opt.timing >= 2;
    double kbytes[GSP_K_COUNT] = {0};
    for (int k = 0; k < GSP_K_COUNT; k++) ctx->kernel_launches[k] = 0;
    int t_all = tphase ? ctx->timer.begin(PH_COUNT) : -1;

    const int64_t G = batch ? ctx->batch_graphs : 0;
    std::vector<uint8_t> gdone(G, 0);
    std::vector<int64_t> cfirst_h(G + 1, 0);
    if (batch) ctx->bpasses_h.assign(G, 0);

    launch_iota_i32(ctx->top, ctx->n, s);   // level-0 ids (in degree order if ordered)
    Level g = ordered ? level_ordered(ctx) : level0(ctx);
    double *K0 = ordered ? ctx->Kord : ctx->K0;
    if (batch) {
        g.graphs = G;
        g.gid = ctx->gid0;
        g.vbase = ctx->vbase0;
        g.M2g = ctx->M2g;
    }
    {
        // the reset step's vertexWeights of the first pass (Algorithm
        // louvain) and 2m, inside the run (later passes take K'' from the
        // aggregation); exact sums, so equal to the load's values
        int t = tphase ? ctx->timer.begin(PH_OTHER) : -1;
        launch_fill_f64(ctx->sc.f64, 0.0, 1, s);
        launch_vertex_weights(g, K0, ctx->sc.f64, s);
        if (batch) launch_batch_m2(K0, ctx->vbase0, G, ctx->M2g, s);
        HIP_TRY(hipMemcpyAsync(ctx->f64_h, ctx->sc.f64, sizeof(double), hipMemcpyDeviceToHost, s));
        if (batch) HIP_TRY(hipMemcpyAsync(ctx->M2g_h.data(), ctx->M2g, G * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        ctx->M2 = ctx->f64_h[0];
        ctx->timer.end(t);
    }
    const double *K = K0;
    double tau = tolerance;
    int next = 0;
    int passes = 0;
    for (int lp = 0; lp < max_passes; lp++) {
        passes = lp + 1;
        int t = tphase ? ctx->timer.begin(PH_OTHER) : -1;
        WorkLists wl = make_lists(ctx);
        HIP_TRY(build_work_lists(g, opt.sub_rounds, wl, ctx->sc, s));
        if (leiden && lp > 0) {
            // GSP-Leiden: each super-vertex starts in the community that
            // holds its sub-community
            launch_copy_i32(ctx->cm, ctx->bstart, g.n, s);
            launch_fill_f64(ctx->sig, 0.0, g.n, s);
            launch_fill_i32(ctx->csize, 0, g.n, s);
            launch_community_totals(K, ctx->cm, g.n, ctx->sig, ctx->csize, s);
        } else {
            // Sigma' <- K'; C' <- [0 .. |V'|); sizes 1
            launch_iota_i32(ctx->cm, g.n, s);
            HIP_TRY(hipMemcpyAsync(ctx->sig, K, g.n * sizeof(double), hipMemcpyDeviceToDevice, s));
            launch_fill_i32(ctx->csize, 1, g.n, s);
        }
        ctx->timer.end(t);
        t = tphase ? ctx->timer.begin(PH_MOVE) : -1;
        PhaseCfg pc;
        pc.tau = tau;
        pc.max_iter = opt.max_iterations;
        pc.timing_k = tk;
        pc.timing_side = opt.timing == 3;
        pc.return_moves = opt.return_moves != 0;
        pc.gated = opt.prune_mode == GSP_PRUNE_LEARNED;
        pc.theta_logit = theta_logit(opt.prune_threshold);
        pc.pass = lp;
        pc.use_graphs = opt.use_graphs != 0;
        pc.grid_cap = opt.grid_cap;
        pc.kernel_bytes = kbytes;
        if (batch) pc.gdone = gdone.data();
        st = move_phase(ctx, g, K, wl, pc);
        if (st != GSP_OK) return st;
        int32_t li = pc.li;
        if (batch) {
            li = 0;
            for (int64_t k = 0; k < G; k++) li = std::max(li, pc.li_g[k]);
        }
        ctx->stats.scanned_entries += pc.scanned_entries;
        ctx->stats.scanned_vertices += pc.scanned_vertices;
        ctx->stats.pruned += pc.pruned;
        ctx->stats.confirm_sweeps += (int32_t)pc.confirm_sweeps;
        ctx->stats.sweeps += (int32_t)pc.sweeps;
        ctx->timer.end(t);
        const int32_t *labels = ctx->cm;
        if (opt.split_mode == GSP_SPLIT_PASS) {
            t = tphase ? ctx->timer.begin(PH_SPLIT) : -1;
            int tk1 = tk ? ctx->timer.begin(100 + GSP_K_SPLIT) : -1;
            st = run_split(ctx, g, wl, ctx->cm, ctx->lab, opt.split_algo, &ctx->stats.split_rounds);
            if (st != GSP_OK) return st;
            ctx->timer.end(tk1);
            if (tk) ctx->kernel_launches[GSP_K_SPLIT] += 6;
            // one pass over the level: column + membership of both ends per
            // entry; offset, degree, membership, label write per vertex
            kbytes[GSP_K_SPLIT] += 8.0 * (double)g.nnz + 24.0 * (double)g.n;
            ctx->timer.end(t);
            labels = ctx->lab;
        }
        t = tphase ? ctx->timer.begin(PH_OTHER) : -1;
        // level 0 in degree order: number the communities as in the caller's
        // order, split components by their smallest vertex and communities
        // by their founding vertex, both as caller's ids
        auto caller_labels = [&](const int32_t *l) -> const int32_t * {
            if (!g.orig) return l;
            if (l == ctx->lab)
                launch_labels_min_orig(ctx->lab, g.orig, g.n, ctx->sc.i32c, s);
            else
                launch_labels_orig(l, g.orig, g.n, ctx->lab, s);
            return ctx->lab;
        };
        labels = caller_labels(labels);
        int64_t ncomm = 0;
        st = renumber(ctx, labels, g.n, ctx->cm, &ncomm);
        if (st != GSP_OK) return st;
        bool stop = false;
        int64_t nnext = ncomm;   // vertices of the next level
        if (leiden) {
            // GSP-Leiden: the result stays the local-moving communities
            // (ctx->cm, then ctx->bnd); the next level's super-vertices are
            // their refined sub-communities
            stop = li <= 1 || (double)ncomm / (double)g.n > opt.aggregation_tolerance || lp == max_passes - 1;
            const int32_t *result = ctx->cm;
            if (!stop) {
                launch_copy_i32(ctx->bnd, ctx->cm, g.n, s);
                result = ctx->bnd;
                launch_iota_i32(ctx->cm, g.n, s);
                HIP_TRY(hipMemcpyAsync(ctx->sig, K, g.n * sizeof(double), hipMemcpyDeviceToDevice, s));
                launch_fill_i32(ctx->csize, 1, g.n, s);
                ctx->timer.end(t);
                t = tphase ? ctx->timer.begin(PH_REFINE) : -1;
                PhaseCfg rc;
                rc.tau = tau;
                rc.max_iter = opt.max_iterations;
                rc.timing_k = tk;
                rc.timing_side = opt.timing == 3;
                rc.pass = lp;
                rc.use_graphs = opt.use_graphs != 0;
                rc.grid_cap = opt.grid_cap;
                rc.kernel_bytes = kbytes;
                st = refine_level(ctx, g, K, wl, next, rc, opt.sub_rounds);
                if (st != GSP_OK) return st;
                ctx->stats.scanned_entries += rc.scanned_entries;
                ctx->stats.scanned_vertices += rc.scanned_vertices;
                ctx->stats.sweeps += (int32_t)rc.sweeps;
                ctx->timer.end(t);
                t = tphase ? ctx->timer.begin(PH_OTHER) : -1;
                HIP_TRY(build_work_lists(g, opt.sub_rounds, wl, ctx->sc, s));   // g's lists again
                ctx->timer.end(t);
                const int32_t *rl = ctx->cm;
                if (opt.split_mode == GSP_SPLIT_PASS) {
                    // synchronous moves can leave a sub-community in pieces
                    // (its founder left as others joined it): split it too
                    t = tphase ? ctx->timer.begin(PH_SPLIT) : -1;
                    st = run_split(ctx, g, wl, ctx->cm, ctx->lab, opt.split_algo, &ctx->stats.split_rounds);
                    if (st != GSP_OK) return st;
                    kbytes[GSP_K_SPLIT] += 8.0 * (double)g.nnz + 24.0 * (double)g.n;
                    ctx->timer.end(t);
                    rl = ctx->lab;
                }
                t = tphase ? ctx->timer.begin(PH_OTHER) : -1;
                rl = caller_labels(rl);
                st = renumber(ctx, rl, g.n, ctx->cm, &nnext);
                if (st != GSP_OK) return st;
                if (lp < GSP_MAX_PASSES_STATS) {
                    ctx->stats.refine_iterations[lp] = rc.li;
                    ctx->stats.refined[lp] = nnext;
                }
                stop = (double)nnext / (double)g.n > opt.aggregation_tolerance;
            }
            launch_lookup(ctx->top, ctx->n, stop ? result : ctx->cm, s);
        } else if (batch) {
            launch_lookup(ctx->top, ctx->n, ctx->cm, s);
            // each graph's communities: [cfirst[k], cfirst[k+1])
            launch_batch_cfirst(ctx->sc.i32b, g.vbase, G, ctx->sc.i64e, ctx->cfirst, s);
            HIP_TRY(hipMemcpyAsync(cfirst_h.data(), ctx->cfirst, (G + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
            std::vector<int64_t> vb(G + 1);
            HIP_TRY(hipMemcpyAsync(vb.data(), g.vbase, (G + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            bool all = true;
            for (int64_t k = 0; k < G; k++) {
                if (gdone[k]) continue;
                ctx->bpasses_h[k] = lp + 1;
                int64_t nk = vb[k + 1] - vb[k], ck = cfirst_h[k + 1] - cfirst_h[k];
                if (pc.li_g[k] <= 1 || (double)ck / (double)nk > opt.aggregation_tolerance) gdone[k] = 1;
                all = all && gdone[k];
            }
            stop = all;
        } else {
            launch_lookup(ctx->top, ctx->n, ctx->cm, s);
            stop = li <= 1 ||                                                // globally converged
                   (double)ncomm / (double)g.n > opt.aggregation_tolerance;    // low shrink
        }
        ctx->timer.end(t);
        if (lp < GSP_MAX_PASSES_STATS) {
            ctx->stats.iterations[lp] = li;
            ctx->stats.vertices[lp] = g.n;
            ctx->stats.communities[lp] = ncomm;
        }
        if (stop) break;
        if (lp == max_passes - 1) break;                                   // G'' would be unused
        t = tphase ? ctx->timer.begin(PH_AGG) : -1;
        int tk2 = tk ? ctx->timer.begin(100 + GSP_K_AGGREGATE) : -1;
        AggOut out{ctx->offL[next], ctx->colL[next], ctx->wL[next], ctx->KL[next], ctx->degL[next]};
        int64_t nnz2 = 0;
        HIP_TRY(aggregate(g, wl, ctx->cm, nnext, out, ctx->gap_col, ctx->gap_w, ctx->sc, &nnz2, s, ctx->hub_parts));
        ctx->timer.end(tk2);
        if (leiden) launch_bound_start(ctx->cm, ctx->bnd, g.n, ctx->bstart, s);
        {
            // read every entry (column, weight, neighbour membership), write
            // the gapped rows of G'' (12 B per entry); per vertex membership,
            // degree, offset and the member list
            int ws = g.wt == W_UNIT ? 0 : (g.wt == W_F32 ? 4 : 8);
            kbytes[GSP_K_AGGREGATE] += (8.0 + ws) * (double)g.nnz + 12.0 * (double)nnz2 + 28.0 * (double)g.n +
                                       40.0 * (double)nnext;
            if (tk) ctx->kernel_launches[GSP_K_AGGREGATE] += 1;
        }
        ctx->timer.end(t);
        Level g2;
        g2.n = nnext;
        g2.nnz = nnz2;
        g2.off = out.off;
        g2.col = out.col;
        g2.w = out.w;
        g2.wt = W_F64;
        g2.deg = out.deg;
        if (batch) {
            // super-vertex c of graph k: ids [cfirst[k], cfirst[k+1])
            HIP_TRY(hipMemcpyAsync(ctx->vbaseL[next], ctx->cfirst, (G + 1) * sizeof(int64_t),
                                   hipMemcpyDeviceToDevice, s));
            launch_batch_gid(ctx->vbaseL[next], G, ncomm, ctx->gidL[next], s);
            g2.graphs = G;
            g2.gid = ctx->gidL[next];
            g2.vbase = ctx->vbaseL[next];
            g2.M2g = ctx->M2g;
        }
        g = g2;
        K = out.K;
        next ^= 1;
        tau = tau / opt.tolerance_drop;                                    // threshold scaling
    }
    if (ordered) {
        // the top-level membership back in the caller's vertex order
        launch_scatter_by_orig(ctx->top, ctx->ord.orig, ctx->n, ctx->lab, s);
        HIP_TRY(hipMemcpyAsync(ctx->top, ctx->lab, ctx->n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    if (opt.split_mode == GSP_SPLIT_LAST && ctx->n > 0) {
        Level g0 = level0(ctx);
        WorkLists wl = make_lists(ctx);
        HIP_TRY(build_work_lists(g0, 1, wl, ctx->sc, s));
        st = run_split(ctx, g0, wl, ctx->top, ctx->lab, opt.split_algo, &ctx->stats.split_rounds);
        if (st != GSP_OK) return st;
        HIP_TRY(hipMemcpyAsync(ctx->top, ctx->lab, ctx->n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    if (opt.split_mode != GSP_SPLIT_PASS && ctx->n > 0) {
        // number communities by ascending smallest vertex id
        launch_canonical_labels(ctx->top, ctx->n, ctx->sc.i32c, ctx->lab, s);
        int64_t ncan = 0;
        st = renumber(ctx, ctx->lab, ctx->n, ctx->top, &ncan);
        if (st != GSP_OK) return st;
    }
    if (batch) {
        // the last renumbering left the community count in sc.i64e (none ran
        // when max_passes = 0: then every vertex is its own community); the
        // graphs' modularities are computed when first asked for
        if (passes == 0) launch_fill_i64(ctx->sc.i64e, ctx->n, 1, s);
        HIP_TRY(hipMemcpyAsync(&ctx->i64_h[8], ctx->sc.i64e, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    }
    ctx->timer.end(t_all);
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    if (batch) {
        ctx->batch_ncomm = ctx->i64_h[8];
        ctx->bq_pending = true;
    }
    ctx->stats.passes = passes;
    if (tphase) {
        double acc[100 + GSP_K_COUNT] = {0};
        ctx->timer.collect(acc, 100 + GSP_K_COUNT);
        ctx->stats.ms_move = acc[PH_MOVE];
        ctx->stats.ms_split = acc[PH_SPLIT];
        ctx->stats.ms_aggregate = acc[PH_AGG];
        ctx->stats.ms_other = acc[PH_OTHER];
        ctx->stats.ms_refine = acc[PH_REFINE];
        ctx->stats.ms_total = acc[PH_COUNT];
        for (int k = 0; k < GSP_K_COUNT; k++) {
            ctx->stats.kernels[k].ms = acc[100 + k];
            ctx->stats.kernels[k].launches = ctx->kernel_launches[k];
            ctx->stats.kernels[k].bytes = kbytes[k];
        }
    }
    ctx->have_result = true;
    ctx->have_batch_result = batch;
    return GSP_OK;
}

}  // namespace

extern "C" {

gsp_status gsp_run(gsp_ctx *ctx, double tolerance, int32_t max_passes, const gsp_options *optp) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    return run_passes(ctx, tolerance, max_passes, optp, false);
}

// ---- batches of graphs ----

gsp_status gsp_load_batch(gsp_ctx *ctx, int32_t graphs, const int64_t *n, const int64_t *nnz,
                          const int64_t *const *offsets, const int32_t *const *cols, const float *const *weights) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (graphs <= 0 || !n || !nnz || !offsets || !cols) return ctx->fail(GSP_EINVAL, "bad batch arguments");
    int64_t N = 0, E = 0;
    bool any_w = false;
    for (int32_t k = 0; k < graphs; k++) {
        if (n[k] <= 0 || nnz[k] < 0 || !offsets[k] || (nnz[k] > 0 && !cols[k]))
            return ctx->fail(GSP_EINVAL, "every graph of a batch needs n >= 1, nnz >= 0, offsets and columns");
        if (offsets[k][0] != 0 || offsets[k][n[k]] != nnz[k])
            return ctx->fail(GSP_EGRAPH, "a graph's offsets must start at 0 and end at its nnz");
        N += n[k];
        E += nnz[k];
        any_w = any_w || (weights && weights[k]);
        if (N > 0x7fffffffLL - 1) return ctx->fail(GSP_EINVAL, "a batch must hold fewer than 2^31 - 1 vertices");
    }
    // one block-diagonal CSR: graph k's vertex v is vertex vbase[k] + v
    std::vector<int64_t> off(N + 1);
    std::vector<int32_t> col(E);
    std::vector<float> w(any_w ? E : 0);
    std::vector<int64_t> vbase(graphs + 1);
    int64_t vb = 0, eb = 0;
    int32_t grid_S = 1022;
    int64_t grid_moved = 0;
    for (int32_t k = 0; k < graphs; k++) {
        vbase[k] = vb;
        for (int64_t v = 0; v < n[k]; v++) off[vb + v] = eb + offsets[k][v];
        for (int64_t e = 0; e < nnz[k]; e++) {
            int32_t c = cols[k][e];
            if (c < 0 || c >= n[k]) return ctx->fail(GSP_EGRAPH, "a column lies outside its graph");
            col[eb + e] = (int32_t)(vb + c);
        }
        if (any_w) {
            for (int64_t e = 0; e < nnz[k]; e++) w[eb + e] = weights[k] ? weights[k][e] : 1.0f;
            // each graph on the grid of its own total: every sum of one graph's
            // weights is then exact (no sum mixes graphs)
            int64_t mv = 0;
            grid_S = std::min(grid_S, host_weight_grid(w.data() + eb, nnz[k], &mv));
            grid_moved += mv;
        }
        vb += n[k];
        eb += nnz[k];
    }
    off[N] = E;
    vbase[graphs] = N;
    gsp_status st = load_impl(ctx, N, E, off.data(), nullptr, col.data(), any_w ? (const void *)w.data() : nullptr,
                              any_w ? W_F32 : W_UNIT, GSP_HOST, false);
    if (st != GSP_OK) return st;
    ctx->grid_S = any_w ? grid_S : 0;
    ctx->grid_moved = grid_moved;
    hipError_t e = hipSuccess;
    const int64_t G = graphs;
    ctx->vbase0 = ctx->dalloc<int64_t>(G + 1, &e);
    for (int k = 0; k < 2 && e == hipSuccess; k++) {
        ctx->vbaseL[k] = ctx->dalloc<int64_t>(G + 1, &e);
        if (e == hipSuccess) ctx->gidL[k] = ctx->dalloc<int32_t>(N, &e);
    }
    if (e == hipSuccess) ctx->cfirst = ctx->dalloc<int64_t>(G + 1, &e);
    if (e == hipSuccess) ctx->gid0 = ctx->dalloc<int32_t>(N, &e);
    if (e == hipSuccess) ctx->M2g = ctx->dalloc<double>(G, &e);
    if (e == hipSuccess) ctx->ggain = ctx->dalloc<unsigned long long>(G, &e);
    if (e == hipSuccess) ctx->bq = ctx->dalloc<double>(G, &e);
    if (e == hipSuccess) ctx->bqin = ctx->dalloc<double>(G, &e);
    if (e == hipSuccess) ctx->gmoved = ctx->dalloc<unsigned long long>(G, &e);
    if (e == hipSuccess) ctx->gactive = ctx->dalloc<uint8_t>(G, &e);
    if (e == hipSuccess) ctx->ggated = ctx->dalloc<uint8_t>(G, &e);
    if (e == hipSuccess) ctx->gconfirm = ctx->dalloc<uint8_t>(G, &e);
    if (e == hipSuccess) ctx->giter = ctx->dalloc<int32_t>(G, &e);
    if (e != hipSuccess) {
        ctx->free_graph();
        return ctx->fail_hip(e, "hipMalloc(batch state)");
    }
    hipStream_t s = ctx->stream;
    HIP_TRY(hipMemcpyAsync(ctx->vbase0, vbase.data(), (G + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    launch_batch_gid(ctx->vbase0, G, N, ctx->gid0, s);
    launch_batch_m2(ctx->K0, ctx->vbase0, G, ctx->M2g, s);
    ctx->M2g_h.assign(G, 0.0);
    HIP_TRY(hipMemcpyAsync(ctx->M2g_h.data(), ctx->M2g, G * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    ctx->vbase0_h = vbase;
    ctx->batch_graphs = G;
    return GSP_OK;
}

gsp_status gsp_run_batch(gsp_ctx *ctx, double tolerance, int32_t max_passes, const gsp_options *opt) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    return run_passes(ctx, tolerance, max_passes, opt, true);
}

gsp_status gsp_get_batch_membership(gsp_ctx *ctx, int32_t graph, int32_t *out, int where) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (!ctx->have_batch_result) return ctx->fail(GSP_ESTATE, "no batch result (call gsp_run_batch)");
    if (graph < 0 || graph >= ctx->batch_graphs || !out) return ctx->fail(GSP_EINVAL, "bad graph index or NULL out");
    if (check_where(ctx, where) != GSP_OK) return GSP_EINVAL;
    hipStream_t s = ctx->stream;
    int64_t b = ctx->vbase0_h[graph], len = ctx->vbase0_h[graph + 1] - b;
    int32_t first = 0;
    HIP_TRY(hipMemcpyAsync(&first, ctx->top + b, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (where == GSP_DEVICE) {
        HIP_TRY(hipMemcpyAsync(out, ctx->top + b, len * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        launch_add_i32(out, len, -first, s);
    } else {
        HIP_TRY(hipMemcpyAsync(out, ctx->top + b, len * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    if (where == GSP_HOST)
        for (int64_t v = 0; v < len; v++) out[v] -= first;
    return GSP_OK;
}

gsp_status gsp_get_batch_modularity(gsp_ctx *ctx, double *q_out) {
    if (!ctx || !q_out) return GSP_EINVAL;
    if (!ctx->have_batch_result) return ctx->fail(GSP_ESTATE, "no batch result (call gsp_run_batch)");
    (void)hipSetDevice(ctx->device);
    if (ctx->bq_pending) {
        // each graph's modularity (Eq. 1) with its own 2m; communities of
        // graph k are [top[vbase0[k]], top[vbase0[k + 1]]) in the final
        // numbering
        hipStream_t s = ctx->stream;
        const int64_t G = ctx->batch_graphs;
        Level g0 = level0(ctx);
        g0.graphs = G;
        g0.gid = ctx->gid0;
        g0.vbase = ctx->vbase0;
        g0.M2g = ctx->M2g;
        launch_fill_f64(ctx->sig, 0.0, ctx->n, s);
        launch_fill_i32(ctx->csize, 0, ctx->n, s);
        launch_community_totals(ctx->K0, ctx->top, ctx->n, ctx->sig, ctx->csize, s);
        ctx->i64_h[8] = ctx->batch_ncomm;
        HIP_TRY(hipMemcpyAsync(ctx->sc.i64e, &ctx->i64_h[8], sizeof(int64_t), hipMemcpyHostToDevice, s));
        launch_batch_cfirst(ctx->top, ctx->vbase0, G, ctx->sc.i64e, ctx->cfirst, s);
        launch_batch_modularity(g0, ctx->top, ctx->sig, ctx->cfirst, ctx->bqin, ctx->bq, s);
        ctx->bq_h.assign(G, 0.0);
        HIP_TRY(hipMemcpyAsync(ctx->bq_h.data(), ctx->bq, G * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipGetLastError());
        ctx->bq_pending = false;
    }
    for (int64_t k = 0; k < ctx->batch_graphs; k++) q_out[k] = ctx->bq_h[k];
    return GSP_OK;
}

gsp_status gsp_get_batch_passes(gsp_ctx *ctx, int32_t *passes_out) {
    if (!ctx || !passes_out) return GSP_EINVAL;
    if (!ctx->have_batch_result) return ctx->fail(GSP_ESTATE, "no batch result (call gsp_run_batch)");
    for (int64_t k = 0; k < ctx->batch_graphs; k++) passes_out[k] = ctx->bpasses_h[k];
    return GSP_OK;
}

gsp_status gsp_get_membership(gsp_ctx *ctx, int32_t *out, int where) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (!ctx->have_result) return ctx->fail(GSP_ESTATE, "no result (call gsp_run)");
    if (check_where(ctx, where) != GSP_OK) return GSP_EINVAL;
    if (!out && ctx->n) return ctx->fail(GSP_EINVAL, "out is NULL");
    gsp_status st = copy_out(ctx, out, ctx->top, ctx->n, where);
    if (st != GSP_OK) return st;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return GSP_OK;
}

gsp_status gsp_get_modularity(gsp_ctx *ctx, double *out) {
    if (!ctx || !out) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (!ctx->have_result) return ctx->fail(GSP_ESTATE, "no result (call gsp_run)");
    if (!ctx->have_q) {
        gsp_status st = modularity_of(ctx, ctx->top, &ctx->q);
        if (st != GSP_OK) return st;
        ctx->have_q = true;
    }
    *out = ctx->q;
    return GSP_OK;
}

gsp_status gsp_get_weight_grid(gsp_ctx *ctx, int32_t *scale_exp, int64_t *moved) {
    if (!ctx || !scale_exp || !moved) return GSP_EINVAL;
    if (!ctx->loaded) return ctx->fail(GSP_ESTATE, "no graph loaded");
    *scale_exp = ctx->grid_S;
    *moved = ctx->grid_moved;
    return GSP_OK;
}

gsp_status gsp_get_stats(gsp_ctx *ctx, gsp_stats *out) {
    if (!ctx || !out) return GSP_EINVAL;
    if (!ctx->have_result) return ctx->fail(GSP_ESTATE, "no result (call gsp_run)");
    *out = ctx->stats;
    return GSP_OK;
}

gsp_status gsp_modularity(gsp_ctx *ctx, const int32_t *membership, int where, double *out) {
    if (!ctx || !out) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    gsp_status st = take_membership(ctx, membership, where);
    if (st != GSP_OK) return st;
    return modularity_of(ctx, ctx->cm, out);
}

gsp_status gsp_count_disconnected(gsp_ctx *ctx, const int32_t *membership, int where, int64_t *out) {
    if (!ctx || !out) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    gsp_status st = take_membership(ctx, membership, where);
    if (st != GSP_OK) return st;
    hipStream_t s = ctx->stream;
    Level g = level0(ctx);
    WorkLists wl = make_lists(ctx);
    HIP_TRY(build_work_lists(g, 1, wl, ctx->sc, s));
    launch_split(g, wl, ctx->cm, ctx->lab, ctx->sc.i32c, reinterpret_cast<uint32_t *>(ctx->sc.i32a),
                 reinterpret_cast<unsigned long long *>(ctx->sc.i64a), s);
    HIP_TRY(hipMemsetAsync(ctx->sc.u64, 0, sizeof(unsigned long long), s));
    launch_count_disconnected(ctx->lab, ctx->cm, ctx->n, ctx->sc.i32a, ctx->sc.u64, s);
    HIP_TRY(hipMemcpyAsync(ctx->i64_h, ctx->sc.u64, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    *out = ctx->i64_h[0];
    return GSP_OK;
}

gsp_status gsp_step_move(gsp_ctx *ctx, const int32_t *membership, const uint8_t *active, int where,
                         int32_t *dec_out, double *gain_out, int64_t *moved) {
    if (!ctx || !moved) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (!dec_out && ctx->n) return ctx->fail(GSP_EINVAL, "dec_out is NULL");
    gsp_status st0 = ensure_levels(ctx);   // the hub staging lives in the aggregation buffers
    if (st0 != GSP_OK) return st0;
    gsp_status st = take_membership(ctx, membership, where);
    if (st != GSP_OK) return st;
    hipStream_t s = ctx->stream;
    Level g = level0(ctx);
    launch_fill_f64(ctx->sig, 0.0, g.n, s);
    launch_fill_i32(ctx->csize, 0, g.n, s);
    launch_community_totals(ctx->K0, ctx->cm, g.n, ctx->sig, ctx->csize, s);
    if (active) {
        if (g.n)
            HIP_TRY(hipMemcpyAsync(ctx->flag, active, g.n, where == GSP_DEVICE ? hipMemcpyDeviceToDevice
                                                                                : hipMemcpyHostToDevice, s));
    } else {
        launch_fill_u8(ctx->flag, 1, g.n, s);
    }
    WorkLists wl = make_lists(ctx);
    HIP_TRY(build_work_lists(g, 1, wl, ctx->sc, s));
    launch_copy_i32(ctx->dec, ctx->cm, g.n, s);
    launch_fill_f64(ctx->gain_tmp, 0.0, g.n, s);
    IterCounters *ctr = ctx->ctr;
    HIP_TRY(hipMemsetAsync(ctr, 0, sizeof(IterCounters), s));
    MoveArgs a;
    a.g = g;
    a.K = ctx->K0;
    a.sig = ctx->sig;
    a.csize = ctx->csize;
    a.cm = ctx->cm;
    a.M2 = ctx->M2;
    a.flag = ctx->flag;
    a.dec = ctx->dec;
    a.gain_out = ctx->gain_tmp;
    a.queue = ctx->queue;
    for (int b = 0; b < kNumBins; b++) {
        a.qbase[b] = wl.bucket_begin(b, 0);
        a.qcap[b] = wl.bucket_size(b, 0);
    }
    a.ctr = ctr;
    a.round = 0;
    a.ch_vert = wl.ch_vert;
    a.ch_beg = wl.ch_beg;
    a.ch_first = wl.ch_poff[0];
    a.ch_count = wl.ch_poff[1] - wl.ch_poff[0];
    a.hub_off = wl.hub_off;
    a.hub_act = ctx->hub_act;
    a.hkeys = ctx->sc.hkeys;
    a.hvals = ctx->sc.hvals;
    a.hub_ch0 = ctx->hub_ch0;
    a.part_g = ctx->sc.part_g;
    a.part_kid = ctx->sc.part_kid;
    a.part_c = ctx->sc.part_c;
    a.hub_parts = ctx->hub_parts && ctx->gap_col;
    a.max_parts = ctx->hub_max_parts;
    a.skey = ctx->gap_col;
    a.sval = ctx->gap_w;
    a.hbuck = ctx->sc.hbuck;
    a.hub_b0 = wl.hub_b0;
    launch_move_compact(a, wl, s);
    launch_move_small(a, wl, s);
    launch_move_wave(a, s);
    launch_move_block(a, s);
    if (a.hub_parts) {
        launch_move_hub_parts(a, s);
        launch_move_hub_gather(a, s);
        launch_move_hub_decide(a, s);
    } else {
        launch_move_hub_scan(a, s);
        launch_move_hub_finish(a, s);
    }
    HIP_TRY(hipGetLastError());
    st = copy_out(ctx, dec_out, ctx->dec, g.n, where);
    if (st != GSP_OK) return st;
    if (gain_out) {
        st = copy_out(ctx, gain_out, ctx->gain_tmp, g.n, where);
        if (st != GSP_OK) return st;
    }
    HIP_TRY(hipMemcpyAsync(ctx->ctr_h, ctr, sizeof(IterCounters), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int64_t mv = 0;
    for (int q = 0; q < kStripes; q++) mv += (int64_t)ctx->ctr_h->st[q].moved;
    *moved = mv;
    return GSP_OK;
}

gsp_status gsp_move_phase_ex(gsp_ctx *ctx, int32_t *membership_inout, int where, double tolerance, int32_t pass_index,
                             const gsp_options *optp, int32_t *iterations, double *dq_iter, int64_t *moved_iter,
                             int64_t *counters) {
    if (!ctx || !iterations) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    gsp_options opt;
    if (optp)
        opt = *optp;
    else
        gsp_default_options(&opt);
    gsp_status st = check_options(ctx, opt);
    if (st != GSP_OK) return st;
    if (!(tolerance >= 0.0) || pass_index < 0 || pass_index > 255)
        return ctx->fail(GSP_EINVAL, "bad tolerance or pass_index");
    st = ensure_levels(ctx);   // the hub staging lives in the aggregation buffers
    if (st != GSP_OK) return st;
    ctx->hub_parts = opt.hub_global == 0;
    ctx->hub_max_parts = opt.hub_max_parts ? opt.hub_max_parts : kMaxParts;
    st = take_membership(ctx, membership_inout, where);
    if (st != GSP_OK) return st;
    hipStream_t s = ctx->stream;
    Level g = level0(ctx);
    launch_fill_f64(ctx->sig, 0.0, g.n, s);
    launch_fill_i32(ctx->csize, 0, g.n, s);
    launch_community_totals(ctx->K0, ctx->cm, g.n, ctx->sig, ctx->csize, s);
    WorkLists wl = make_lists(ctx);
    HIP_TRY(build_work_lists(g, opt.sub_rounds, wl, ctx->sc, s));
    int mi = opt.max_iterations;
    std::vector<double> dq(mi > 0 ? mi : 1);
    std::vector<int64_t> mv(mi > 0 ? mi : 1);
    PhaseCfg pc;
    pc.tau = tolerance;
    pc.return_moves = opt.return_moves != 0;
    pc.max_iter = mi;
    pc.gated = opt.prune_mode == GSP_PRUNE_LEARNED;
    pc.theta_logit = theta_logit(opt.prune_threshold);
    pc.pass = pass_index;
    pc.use_graphs = opt.use_graphs != 0;
    pc.grid_cap = opt.grid_cap;
    pc.dq_out = dq.data();
    pc.moved_out = mv.data();
    st = move_phase(ctx, g, ctx->K0, wl, pc);
    if (st != GSP_OK) return st;
    st = copy_out(ctx, membership_inout, ctx->cm, g.n, where);
    if (st != GSP_OK) return st;
    HIP_TRY(hipStreamSynchronize(s));
    *iterations = pc.li;
    for (int k = 0; k < pc.li; k++) {
        if (dq_iter) dq_iter[k] = dq[k];
        if (moved_iter) moved_iter[k] = mv[k];
    }
    if (counters) {
        counters[0] = pc.scanned_vertices;
        counters[1] = pc.scanned_entries;
        counters[2] = pc.pruned;
        counters[3] = pc.confirm_sweeps;
    }
    return GSP_OK;
}

gsp_status gsp_refine_phase(gsp_ctx *ctx, const int32_t *bound, int32_t *membership_inout, int where,
                            double tolerance, const gsp_options *optp, int32_t *iterations, double *dq_iter,
                            int64_t *moved_iter) {
    if (!ctx || !iterations) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    gsp_options opt;
    if (optp)
        opt = *optp;
    else
        gsp_default_options(&opt);
    opt.leiden = 1;
    gsp_status st = check_options(ctx, opt);
    if (st != GSP_OK) return st;
    if (!(tolerance >= 0.0)) return ctx->fail(GSP_EINVAL, "bad tolerance");
    if (!ctx->loaded) return ctx->fail(GSP_ESTATE, "no graph loaded");
    if (!bound && ctx->n > 0) return ctx->fail(GSP_EINVAL, "bound is NULL");
    if (ctx->tracing) return ctx->fail(GSP_EINVAL, "the refinement runs without trace capture");
    if ((st = ensure_levels(ctx)) != GSP_OK) return st;   // the subgraph and the hub staging
    if ((st = ensure_leiden(ctx)) != GSP_OK) return st;
    ctx->hub_parts = opt.hub_global == 0;
    ctx->hub_max_parts = opt.hub_max_parts ? opt.hub_max_parts : kMaxParts;
    // the bound communities (checked as a membership), then the start
    if ((st = take_membership(ctx, bound, where)) != GSP_OK) return st;
    hipStream_t s = ctx->stream;
    launch_copy_i32(ctx->bnd, ctx->cm, ctx->n, s);
    if ((st = take_membership(ctx, membership_inout, where)) != GSP_OK) return st;
    HIP_TRY(hipMemsetAsync(ctx->sc.err, 0, sizeof(int), s));
    launch_bound_check(ctx->cm, ctx->bnd, ctx->n, ctx->sc.i32c, ctx->sc.err, s);
    int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, ctx->sc.err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (bad) return ctx->fail(GSP_EINVAL, "a starting sub-community lies in two bound communities");
    Level g = level0(ctx);
    launch_fill_f64(ctx->sig, 0.0, g.n, s);
    launch_fill_i32(ctx->csize, 0, g.n, s);
    launch_community_totals(ctx->K0, ctx->cm, g.n, ctx->sig, ctx->csize, s);
    WorkLists wl = make_lists(ctx);
    HIP_TRY(build_work_lists(g, opt.sub_rounds, wl, ctx->sc, s));
    int mi = opt.max_iterations;
    std::vector<double> dq(mi > 0 ? mi : 1);
    std::vector<int64_t> mv(mi > 0 ? mi : 1);
    PhaseCfg pc;
    pc.tau = tolerance;
    pc.max_iter = mi;
    pc.use_graphs = opt.use_graphs != 0;
    pc.grid_cap = opt.grid_cap;
    pc.dq_out = dq.data();
    pc.moved_out = mv.data();
    st = refine_level(ctx, g, ctx->K0, wl, 0, pc, opt.sub_rounds);
    if (st != GSP_OK) return st;
    st = copy_out(ctx, membership_inout, ctx->cm, g.n, where);
    if (st != GSP_OK) return st;
    HIP_TRY(hipStreamSynchronize(s));
    *iterations = pc.li;
    for (int k = 0; k < pc.li; k++) {
        if (dq_iter) dq_iter[k] = dq[k];
        if (moved_iter) moved_iter[k] = mv[k];
    }
    return GSP_OK;
}

gsp_status gsp_move_phase(gsp_ctx *ctx, int32_t *membership_inout, int where, double tolerance,
                          int32_t max_iterations, int32_t sub_rounds, int32_t *iterations, double *dq_iter,
                          int64_t *moved_iter) {
    if (!ctx) return GSP_EINVAL;
    gsp_options opt;
    gsp_default_options(&opt);
    opt.max_iterations = max_iterations;
    opt.sub_rounds = sub_rounds;
    return gsp_move_phase_ex(ctx, membership_inout, where, tolerance, 0, &opt, iterations, dq_iter, moved_iter,
                             nullptr);
}

// ---- the disconnected count without allocation ----

}  // extern "C"

namespace {

// Scratch of gsp_count_disconnected_noalloc: a fixed array in device memory
// (each GPU holds its own copy for the life of the process).  Layout: two
// 64-bit counters in the first 256 bytes, then parent[n] and roots[n]
// (int32).  Host code never passes `scratch` itself to a kernel (in host
// code it is a stand-in, not a device address): it takes the device
// address of this GPU's copy from hipGetSymbolAddress once per device.
constexpr size_t kNoallocBytes = (size_t)64 << 20;
constexpr int64_t kNoallocMaxN = (int64_t)((kNoallocBytes - 256) / 8);
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {nullptr};

// This device's address of `scratch` (looked up on the first call per
// device, with that device current).
hipError_t noalloc_scratch(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

gsp_status gsp_count_disconnected_noalloc(int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols,
                                          const int32_t *membership, int64_t *count_out, void *hip_stream) {
    if (n < 0 || nnz < 0 || n > kNoallocMaxN || !offsets || !count_out || (n > 0 && !membership) ||
        (nnz > 0 && !cols))
        return GSP_EINVAL;
    void *base = nullptr;
    if (noalloc_scratch(&base) != hipSuccess) return GSP_EHIP;
    unsigned char *b = static_cast<unsigned char *>(base);
    unsigned long long *flags = reinterpret_cast<unsigned long long *>(b);
    int32_t *parent = reinterpret_cast<int32_t *>(b + 256);
    int32_t *roots = parent + n;
    hipStream_t s = (hipStream_t)hip_stream;
    launch_count_disconnected_csr(offsets, cols, n, nnz, membership, parent, roots, flags, count_out, s);
    return hipGetLastError() == hipSuccess ? GSP_OK : GSP_EHIP;
}

int64_t gsp_noalloc_max_vertices(void) { return kNoallocMaxN; }

// ---- learned pruning gate ----

gsp_status gsp_pruner_set(gsp_ctx *ctx, const float *params, int64_t count, int where) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (!params || count != kGateParams) return ctx->fail(GSP_EINVAL, "params must hold 4801 values");
    if (where != GSP_HOST && where != GSP_DEVICE) return ctx->fail(GSP_EINVAL, "bad `where`");
    std::vector<float> p(kGateParams);
    if (where == GSP_DEVICE) {
        HIP_TRY(hipMemcpyAsync(p.data(), params, kGateParams * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    } else {
        memcpy(p.data(), params, kGateParams * sizeof(float));
    }
    for (float v : p)
        if (!std::isfinite(v)) return ctx->fail(GSP_EINVAL, "params must be finite");
    hipError_t e = hipSuccess;
    if (!ctx->net_w1) {
        ctx->net_w1 = ctx->palloc<uint16_t>(kGateHidden * kGateFeatures, &e);
        if (e == hipSuccess) ctx->net_w2 = ctx->palloc<uint16_t>(kGateHidden * kGateHidden, &e);
        if (e == hipSuccess) ctx->net_f = ctx->palloc<float>(3 * kGateHidden, &e);
        if (e != hipSuccess) return ctx->fail_hip(e, "hipMalloc(network)");
    }
    std::vector<uint16_t> w1(kGateHidden * kGateFeatures), w2(kGateHidden * kGateHidden);
    std::vector<float> f(3 * kGateHidden);
    for (int k = 0; k < kGateHidden * kGateFeatures; k++) w1[k] = bf16_bits(p[kPW1 + k]);
    for (int k = 0; k < kGateHidden * kGateHidden; k++) w2[k] = bf16_bits(p[kPW2 + k]);
    for (int k = 0; k < kGateHidden; k++) {
        f[k] = p[kPB1 + k];
        f[kGateHidden + k] = p[kPB2 + k];
        f[2 * kGateHidden + k] = bf16_round(p[kPW3 + k]);
    }
    HIP_TRY(hipMemcpyAsync(ctx->net_w1, w1.data(), w1.size() * 2, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(ctx->net_w2, w2.data(), w2.size() * 2, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(ctx->net_f, f.data(), f.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->net_b3 = p[kPB3];
    ctx->net_params = p;
    ctx->have_net = true;
    ctx->drop_sweep_graphs();   // captured gated sweeps hold the old network's arguments
    return GSP_OK;
}

gsp_status gsp_gate_logits(gsp_ctx *ctx, const float *x, int64_t rows, float *logits, int where) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (!ctx->have_net) return ctx->fail(GSP_ESTATE, "no network (gsp_pruner_set)");
    if (rows < 0 || (rows > 0 && (!x || !logits))) return ctx->fail(GSP_EINVAL, "bad rows or NULL buffer");
    if (where != GSP_HOST && where != GSP_DEVICE) return ctx->fail(GSP_EINVAL, "bad `where`");
    if (rows == 0) return GSP_OK;
    hipStream_t s = ctx->stream;
    const float *dx = x;
    float *dz = logits;
    float *tx = nullptr, *tz = nullptr;
    if (where == GSP_HOST) {
        HIP_TRY(hipMalloc(&tx, rows * kGateFeatures * sizeof(float)));
        hipError_t e = hipMalloc(&tz, rows * sizeof(float));
        if (e != hipSuccess) {
            (void)hipFree(tx);
            return ctx->fail_hip(e, "hipMalloc(logits)");
        }
        (void)hipMemcpyAsync(tx, x, rows * kGateFeatures * sizeof(float), hipMemcpyHostToDevice, s);
        dx = tx;
        dz = tz;
    }
    launch_gate_eval(net_of(ctx), dx, rows, dz, s);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && where == GSP_HOST)
        e = hipMemcpyAsync(logits, dz, rows * sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (tx) (void)hipFree(tx);
    if (tz) (void)hipFree(tz);
    if (e != hipSuccess) return ctx->fail_hip(e, "gate logits");
    return GSP_OK;
}

namespace {

// Device copies of training rows (or the caller's device pointers).
struct TrainRows {
    const float *x = nullptr;
    const uint8_t *y = nullptr;
    float *tx = nullptr;
    uint8_t *ty = nullptr;
    ~TrainRows() {
        if (tx) (void)hipFree(tx);
        if (ty) (void)hipFree(ty);
    }
};

gsp_status take_rows(gsp_ctx *ctx, const float *x, const uint8_t *y, int64_t rows, int where, TrainRows &r) {
    if (rows <= 0 || !x || !y) return ctx->fail(GSP_EINVAL, "rows must be > 0 with x and y given");
    if (where != GSP_HOST && where != GSP_DEVICE) return ctx->fail(GSP_EINVAL, "bad `where`");
    if (where == GSP_DEVICE) {
        r.x = x;
        r.y = y;
        return GSP_OK;
    }
    HIP_TRY(hipMalloc(&r.tx, rows * kGateFeatures * sizeof(float)));
    HIP_TRY(hipMalloc(&r.ty, rows));
    HIP_TRY(hipMemcpyAsync(r.tx, x, rows * kGateFeatures * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(r.ty, y, rows, hipMemcpyHostToDevice, ctx->stream));
    r.x = r.tx;
    r.y = r.ty;
    return GSP_OK;
}

// Device scratch of one training call, freed on return.
struct TrainScratch {
    float *params = nullptr, *m = nullptr, *v = nullptr, *part = nullptr, *grad = nullptr;
    double *ploss = nullptr, *loss = nullptr;
    ~TrainScratch() {
        for (void *p : {(void *)params, (void *)m, (void *)v, (void *)part, (void *)grad, (void *)ploss, (void *)loss})
            if (p) (void)hipFree(p);
    }
};

}  // namespace

gsp_status gsp_pruner_grad(gsp_ctx *ctx, const float *params, const float *x, const uint8_t *y, int64_t rows,
                           float pos_weight, float *grad_out, double *loss_out, int where) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (!params || !grad_out) return ctx->fail(GSP_EINVAL, "params and grad_out are required");
    if (!(pos_weight > 0.0f) || !std::isfinite(pos_weight)) return ctx->fail(GSP_EINVAL, "pos_weight must be > 0");
    TrainRows r;
    gsp_status st = take_rows(ctx, x, y, rows, where, r);
    if (st != GSP_OK) return st;
    hipStream_t s = ctx->stream;
    int nb = (int)((rows + kMlpRowsPerBlock - 1) / kMlpRowsPerBlock);
    TrainScratch t;
    HIP_TRY(hipMalloc(&t.params, kGateParams * sizeof(float)));
    HIP_TRY(hipMalloc(&t.grad, kGateParams * sizeof(float)));
    HIP_TRY(hipMalloc(&t.part, (size_t)nb * kGateParams * sizeof(float)));
    HIP_TRY(hipMalloc(&t.ploss, (size_t)nb * sizeof(double)));
    HIP_TRY(hipMalloc(&t.loss, sizeof(double)));
    HIP_TRY(hipMemcpyAsync(t.params, params, kGateParams * sizeof(float),
                           where == GSP_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    launch_fill_f64(t.loss, 0.0, 1, s);
    launch_mlp_grad(t.params, r.x, r.y, rows, pos_weight, 1.0f / (float)rows, t.part, t.ploss, s);
    launch_mlp_reduce(t.part, t.ploss, nb, nullptr, nullptr, nullptr, false, 0.0f, 1.0f, 1.0f, t.grad, t.loss, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(grad_out, t.grad, kGateParams * sizeof(float),
                           where == GSP_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    double L = 0.0;
    HIP_TRY(hipMemcpyAsync(&L, t.loss, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (loss_out) *loss_out = L;
    return GSP_OK;
}

gsp_status gsp_pruner_train(gsp_ctx *ctx, const float *x, const uint8_t *y, int64_t rows, int64_t batch,
                            int32_t epochs, float lr, float pos_weight, float *params_inout, double *epoch_loss,
                            int where) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (!params_inout) return ctx->fail(GSP_EINVAL, "params_inout is NULL");
    if (batch <= 0 || batch > (1 << 20) || epochs < 0 || !(lr > 0.0f) || !(pos_weight > 0.0f))
        return ctx->fail(GSP_EINVAL, "bad batch (1..2^20), epochs, lr or pos_weight");
    TrainRows r;
    gsp_status st = take_rows(ctx, x, y, rows, where, r);
    if (st != GSP_OK) return st;
    hipStream_t s = ctx->stream;
    int64_t bmax = std::min<int64_t>(batch, rows);
    int nbmax = (int)((bmax + kMlpRowsPerBlock - 1) / kMlpRowsPerBlock);
    TrainScratch t;
    HIP_TRY(hipMalloc(&t.params, kGateParams * sizeof(float)));
    HIP_TRY(hipMalloc(&t.m, kGateParams * sizeof(float)));
    HIP_TRY(hipMalloc(&t.v, kGateParams * sizeof(float)));
    HIP_TRY(hipMalloc(&t.part, (size_t)nbmax * kGateParams * sizeof(float)));
    HIP_TRY(hipMalloc(&t.ploss, (size_t)nbmax * sizeof(double)));
    HIP_TRY(hipMalloc(&t.loss, (size_t)(epochs > 0 ? epochs : 1) * sizeof(double)));
    HIP_TRY(hipMemcpyAsync(t.params, params_inout, kGateParams * sizeof(float), hipMemcpyHostToDevice, s));
    launch_fill_f32(t.m, 0.0f, kGateParams, s);
    launch_fill_f32(t.v, 0.0f, kGateParams, s);
    launch_fill_f64(t.loss, 0.0, epochs > 0 ? epochs : 1, s);
    int64_t step = 0, nbatches = (rows + batch - 1) / batch;
    for (int ep = 0; ep < epochs; ep++) {
        for (int64_t r0 = 0; r0 < rows; r0 += batch) {
            int64_t len = std::min<int64_t>(batch, rows - r0);
            int nb = (int)((len + kMlpRowsPerBlock - 1) / kMlpRowsPerBlock);
            step++;
            float c1 = (float)(1.0 - std::pow(0.9, (double)step));
            float c2 = (float)(1.0 - std::pow(0.999, (double)step));
            launch_mlp_grad(t.params, r.x + r0 * kGateFeatures, r.y + r0, len, pos_weight, 1.0f / (float)len, t.part,
                            t.ploss, s);
            launch_mlp_reduce(t.part, t.ploss, nb, t.params, t.m, t.v, true, lr, c1, c2, nullptr, t.loss + ep, s);
        }
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipMemcpyAsync(params_inout, t.params, kGateParams * sizeof(float), hipMemcpyDeviceToHost, s));
    std::vector<double> el(epochs > 0 ? epochs : 1);
    HIP_TRY(hipMemcpyAsync(el.data(), t.loss, el.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (epoch_loss)
        for (int ep = 0; ep < epochs; ep++) epoch_loss[ep] = el[ep] / (double)nbatches;
    return GSP_OK;
}

// ---- move traces ----

gsp_status gsp_capture_traces(gsp_ctx *ctx, int64_t capacity, double rate, uint64_t seed) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (void *p : {(void *)ctx->trace.x, (void *)ctx->trace.y, (void *)ctx->trace.v, (void *)ctx->trace.meta,
                    (void *)ctx->trace.cnt})
        ctx->pfree(p);
    ctx->trace = TraceArgs();
    ctx->tracing = false;
    if (capacity <= 0) return GSP_OK;
    if (!(rate > 0.0) || !(rate <= 1.0)) return ctx->fail(GSP_EINVAL, "rate must lie in (0, 1]");
    int64_t scap = (capacity + kStripes - 1) / kStripes;
    int64_t rows = scap * kStripes;
    hipError_t e = hipSuccess;
    TraceArgs t;
    t.x = ctx->palloc<float>(rows * kGateFeatures, &e);
    if (e == hipSuccess) t.y = ctx->palloc<uint8_t>(rows, &e);
    if (e == hipSuccess) t.v = ctx->palloc<int32_t>(rows, &e);
    if (e == hipSuccess) t.meta = ctx->palloc<int32_t>(rows, &e);
    if (e == hipSuccess) t.cnt = ctx->palloc<unsigned long long>(kStripes, &e);
    ctx->trace = t;   // owned through ctx->persist either way
    if (e != hipSuccess) {
        gsp_capture_traces(ctx, 0, 1.0, 0);
        return ctx->fail_hip(e, "hipMalloc(traces)");
    }
    HIP_TRY(hipMemsetAsync(t.cnt, 0, kStripes * sizeof(unsigned long long), ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->trace.scap = scap;
    ctx->trace.seed = seed;
    ctx->trace.thr = rate >= 1.0 ? ~0ull : (uint64_t)std::ldexp(rate, 64);
    ctx->tracing = true;
    return GSP_OK;
}

gsp_status gsp_get_traces(gsp_ctx *ctx, float *x, uint8_t *y, int32_t *vertex, int32_t *meta, int64_t max_rows,
                          int64_t *rows, int64_t *seen, int where) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (!ctx->tracing) return ctx->fail(GSP_ESTATE, "trace capture is off (gsp_capture_traces)");
    if (where != GSP_HOST && where != GSP_DEVICE) return ctx->fail(GSP_EINVAL, "bad `where`");
    hipStream_t s = ctx->stream;
    unsigned long long cnt[kStripes];
    HIP_TRY(hipMemcpyAsync(cnt, ctx->trace.cnt, sizeof(cnt), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int64_t tot = 0, kept = 0;
    for (int q = 0; q < kStripes; q++) {
        tot += (int64_t)cnt[q];
        kept += std::min<int64_t>((int64_t)cnt[q], ctx->trace.scap);
    }
    if (seen) *seen = tot;
    int64_t out = 0;
    hipMemcpyKind kind = where == GSP_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    for (int q = 0; q < kStripes && out < max_rows; q++) {
        int64_t k = std::min<int64_t>(std::min<int64_t>((int64_t)cnt[q], ctx->trace.scap), max_rows - out);
        if (k <= 0) continue;
        int64_t src = q * ctx->trace.scap;
        if (x)
            HIP_TRY(hipMemcpyAsync(x + out * kGateFeatures, ctx->trace.x + src * kGateFeatures,
                                   k * kGateFeatures * sizeof(float), kind, s));
        if (y) HIP_TRY(hipMemcpyAsync(y + out, ctx->trace.y + src, k, kind, s));
        if (vertex) HIP_TRY(hipMemcpyAsync(vertex + out, ctx->trace.v + src, k * sizeof(int32_t), kind, s));
        if (meta) HIP_TRY(hipMemcpyAsync(meta + out, ctx->trace.meta + src, k * sizeof(int32_t), kind, s));
        out += k;
    }
    HIP_TRY(hipStreamSynchronize(s));
    if (rows) *rows = (x || y || vertex || meta) ? out : kept;
    return GSP_OK;
}

gsp_status gsp_step_split(gsp_ctx *ctx, const int32_t *membership, int where, int32_t *labels_out) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (!labels_out && ctx->n) return ctx->fail(GSP_EINVAL, "labels_out is NULL");
    gsp_status st = take_membership(ctx, membership, where);
    if (st != GSP_OK) return st;
    hipStream_t s = ctx->stream;
    Level g = level0(ctx);
    WorkLists wl = make_lists(ctx);
    HIP_TRY(build_work_lists(g, 1, wl, ctx->sc, s));
    launch_split(g, wl, ctx->cm, ctx->lab, ctx->sc.i32c, reinterpret_cast<uint32_t *>(ctx->sc.i32a),
                 reinterpret_cast<unsigned long long *>(ctx->sc.i64a), s);
    HIP_TRY(hipGetLastError());
    st = copy_out(ctx, labels_out, ctx->lab, g.n, where);
    if (st != GSP_OK) return st;
    HIP_TRY(hipStreamSynchronize(s));
    return GSP_OK;
}

gsp_status gsp_step_split_lp(gsp_ctx *ctx, const int32_t *membership, int where, int32_t *labels_out,
                             int32_t *rounds) {
    if (!ctx) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (!labels_out && ctx->n) return ctx->fail(GSP_EINVAL, "labels_out is NULL");
    gsp_status st = take_membership(ctx, membership, where);
    if (st != GSP_OK) return st;
    Level g = level0(ctx);
    WorkLists wl = make_lists(ctx);
    int32_t r = 0;
    st = run_split(ctx, g, wl, ctx->cm, ctx->lab, GSP_SPLIT_LPP, &r);
    if (st != GSP_OK) return st;
    HIP_TRY(hipGetLastError());
    st = copy_out(ctx, labels_out, ctx->lab, g.n, where);
    if (st != GSP_OK) return st;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (rounds) *rounds = r;
    return GSP_OK;
}

gsp_status gsp_step_aggregate(gsp_ctx *ctx, const int32_t *membership, int where, int64_t *n_out,
                              int64_t *nnz_out, int64_t *offsets, int32_t *cols, double *weights) {
    if (!ctx || !n_out || !nnz_out) return GSP_EINVAL;
    (void)hipSetDevice(ctx->device);
    gsp_status st = take_membership(ctx, membership, where);
    if (st != GSP_OK) return st;
    st = ensure_levels(ctx);
    if (st != GSP_OK) return st;
    hipStream_t s = ctx->stream;
    Level g = level0(ctx);
    int64_t ncomm = 0;
    HIP_TRY(hipMemcpyAsync(ctx->lab, ctx->cm, g.n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    st = renumber(ctx, ctx->lab, g.n, ctx->cm, &ncomm);
    if (st != GSP_OK) return st;
    WorkLists wl = make_lists(ctx);
    HIP_TRY(build_work_lists(g, 1, wl, ctx->sc, s));
    AggOut out{ctx->offL[0], ctx->colL[0], ctx->wL[0], ctx->KL[0], ctx->degL[0]};
    int64_t nnz2 = 0;
    HIP_TRY(aggregate(g, wl, ctx->cm, ncomm, out, ctx->gap_col, ctx->gap_w, ctx->sc, &nnz2, s, ctx->hub_parts));
    *n_out = ncomm;
    *nnz_out = nnz2;
    if (offsets) {
        if ((nnz2 && (!cols || !weights))) return ctx->fail(GSP_EINVAL, "cols/weights NULL");
        // the gapped rows packed into a plain CSR (in the staging arrays)
        int64_t *off_c = ctx->sc.i64f;
        HIP_TRY(compact_rows(out.off, out.deg, ncomm, out.col, out.w, off_c, ctx->gap_col, ctx->gap_w, ctx->sc, s));
        st = copy_out(ctx, offsets, off_c, ncomm + 1, where);
        if (st != GSP_OK) return st;
        st = copy_out(ctx, cols, ctx->gap_col, nnz2, where);
        if (st != GSP_OK) return st;
        st = copy_out(ctx, weights, ctx->gap_w, nnz2, where);
        if (st != GSP_OK) return st;
    }
    HIP_TRY(hipStreamSynchronize(s));
    return GSP_OK;
}

}  // extern "C"
