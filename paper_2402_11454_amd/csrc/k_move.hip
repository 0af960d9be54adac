// k_move.hip - the local-moving phase (Algorithm "louvainMove") as
// synchronous sub-rounds.  Per sub-round:
//   compact : unprocessed vertices of the sub-round -> per-bin queues (and
//             mark them processed: pruning);
//   small   : degree <= 64, a group of 4..64 lanes per vertex;
//   large   : degree <= 2048, a wavefront or a workgroup per vertex;
//   hub     : degree > 2048, chunks of the row into a global table, then a
//             workgroup per hub picks the best community;
//   apply   : moves of the sub-round, community totals Sigma and sizes.
// Each scan+decide kernel builds the table K_{i->c} of scanCommunities
// (self-loop skipped), evaluates Eq. 2 multiplied through by 2m^2:
//   G(c)    = M2 K_{i->c} - K_i Sigma_c            (candidate c != d)
//   G(stay) = M2 K_{i->d} - K_i (Sigma_d - K_i)
// so dQ_{i:d->c} = (G(c) - G(stay)) / (M2^2/2), takes the best candidate
// (ties to the lowest id), moves i only if G(best) > G(stay) unless i and the
// target are both one-vertex communities and the target id is larger, and
// marks every neighbour j != i of a mover unprocessed.  Everything is read
// from the sub-round's snapshot: memberships and totals change only in
// `apply`.  Built with -ffp-contract=off so every product and difference is
// a single IEEE operation.
#include <math.h>

#include "gsp_internal.h"

namespace gsp {

namespace {


struct Acc {          // per-thread counters, reduced per block at the end
    unsigned long long gain = 0;   // units of 2^-61 of delta-modularity (gain_units)
    unsigned long long moved = 0, verts = 0, scanned = 0, keys = 0, ginserts = 0, aux = 0;
};

__device__ void flush_acc(const Acc &acc, IterCounters *ctr, int cls) {
    constexpr int F = 6;
    __shared__ unsigned long long sg[kBlock / kWave];
    __shared__ unsigned long long sv[F][kBlock / kWave];
    const unsigned long long g = (unsigned long long)group_sum_ll<kWave>((long long)acc.gain);
    long long v[F] = {(long long)acc.moved, (long long)acc.verts, (long long)acc.scanned, (long long)acc.keys,
                      (long long)acc.ginserts, (long long)acc.aux};
#pragma unroll
    for (int f = 0; f < F; f++) v[f] = group_sum_ll<kWave>(v[f]);
    int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
        sg[w] = g;
#pragma unroll
        for (int f = 0; f < F; f++) sv[f][w] = (unsigned long long)v[f];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tg = 0;
        unsigned long long t[F] = {0, 0, 0, 0, 0, 0};
        for (int q = 0; q < kBlock / kWave; q++) {
            tg += sg[q];
            for (int f = 0; f < F; f++) t[f] += sv[f][q];
        }
        CounterStripe &st = ctr->st[blockIdx.x % kStripes];
        if (tg) atomicAdd(&st.gain, tg);
        if (t[0]) atomicAdd(&st.moved, t[0]);
        if (t[1]) atomicAdd(&st.verts[cls], t[1]);
        if (t[2]) atomicAdd(&st.scanned[cls], t[2]);
        if (t[3]) atomicAdd(&st.keys[cls], t[3]);
        if (t[4]) atomicAdd(&st.ginserts[cls], t[4]);
        if (t[5]) atomicAdd(&st.aux[cls], t[5]);
    }
}

// Batch: a mover's gain and count into its graph's totals (one lane).
__device__ __forceinline__ void graph_totals(const MoveArgs &a, int i, unsigned long long gain) {
    int gk = a.g.gid[i];
    atomicAdd(&a.ggain[gk], gain);
    atomicAdd(&a.gmoved[gk], 1ull);
}

// The part of a mover's gain (i: d -> bc) that counts towards the sweep's
// total, in fixed point (gain_units): all of it, unless the return-move
// option gives move records (mhist).  Then a move back into the community i
// left at its move of the preceding sweep, which undoes a swap made from one
// snapshot, counts nothing (the move is still made), and this move is
// recorded.  One lane per mover.
__device__ __forceinline__ unsigned long long counted_gain(const MoveArgs &a, int i, int d, int bc, double gain,
                                                           double m2) {
    if (a.mhist) {
        const int32_t sw = (int32_t)*a.sweep_dev;
        const uint64_t h = (uint64_t)a.mhist[i];
        a.mhist[i] = (int64_t)(((uint64_t)(uint32_t)d << 32) | (uint32_t)sw);
        if ((int32_t)(h >> 32) == bc && (int32_t)(uint32_t)h == sw - 1) return 0ull;
    }
    return gain_units(gain, m2);
}

// 2m of vertex i's graph (the level's 2m unless it holds a batch).
__device__ __forceinline__ double m2_of(const MoveArgs &a, int i) { return a.g.M2g ? a.g.M2g[a.g.gid[i]] : a.M2; }

// Decision from the group's best candidate; identical on every lane.
// sig_d = Sigma_d and csz_d = |d| are loaded early by the callers;
// bc_single says whether the best community bc is a singleton (see
// best_single: looked up only when the rule can apply).
__device__ __forceinline__ bool decide(double m2, int d, double ki, double kid, double bg, int bc, double sig_d,
                                       int csz_d, int bc_single, double *gain) {
    if (bc == kIntMax) return false;
    double gstay = m2 * kid - ki * (sig_d - ki);
    if (!(bg > gstay)) return false;
    if (bc_single) return false;
    *gain = bg - gstay;
    return true;
}

// Whether community bc is a singleton, read only where the singleton rule
// can reject the move (d a singleton, bc > d).
__device__ __forceinline__ int best_single(const MoveArgs &a, int d, int csz_d, int bc) {
    if (csz_d != 1 || bc == kIntMax) return 0;
    const int32_t *o = a.g.orig;
    if (!(o ? o[bc] > o[d] : bc > d)) return 0;
    return a.csize[bc] == 1;
}

// History of a scan (for the learned gate's features) and, if sampled, a
// trace row with the features the vertex had before this scan and whether
// it moves.  Called by one lane per decided vertex; no-op unless enabled.
__device__ __forceinline__ void record_scan(const MoveArgs &a, double m2, int i, int d, int di, double ki, double kid,
                                           double bg, int bc, bool mv) {
    uint8_t hb = a.hbits[i];
    float hf = a.hfrac[i], hg = a.hgain[i];
    const int vid = a.g.orig ? a.g.orig[i] : i;   // the caller's id of i
    if (a.tr.x && trace_keep(a.tr.seed, a.pass, a.sweep, vid, a.tr.thr)) {
        uint16_t x[kGateFeatures];
        gate_features(di, ki, a.sig[d], hf, hg, hb, a.dsnap[i], a.pass, a.iter, x);
        int r = blockIdx.x % kStripes;
        unsigned long long slot = atomicAdd(&a.tr.cnt[r], 1ull);
        if ((int64_t)slot < a.tr.scap) {
            int64_t row = r * a.tr.scap + (int64_t)slot;
#pragma unroll
            for (int f = 0; f < kGateFeatures; f++) a.tr.x[row * kGateFeatures + f] = bf16_value(x[f]);
            a.tr.y[row] = mv ? 1 : 0;
            a.tr.v[row] = vid;
            a.tr.meta[row] = a.pass * 256 + a.sweep;
        }
    }
    float nf = 0.0f, ng = 0.0f;
    if (ki > 0.0) {
        nf = (float)(kid / ki);
        double gstay = m2 * kid - ki * (a.sig[d] - ki);
        double r = bc != kIntMax ? (bg - gstay) / (m2 * ki) : -1.0;
        if (r > 1.0) r = 1.0;
        if (r < -1.0) r = -1.0;
        ng = (float)r;
    }
    a.hfrac[i] = nf;
    a.hgain[i] = ng;
    a.hbits[i] = kHistScanned | (mv ? kHistMoved : 0);
    // D_i starts again at a scan.  Movers of this sub-round may be adding to
    // it right now; taking away exactly the value the features saw (which is
    // all D_i held before this sub-round's moves) leaves just their adds, in
    // any order, as the sums are exact.
    if (a.dsnap[i] != 0.0) unsafeAtomicAdd(&a.dmoved[i], -a.dsnap[i]);
}

// A mover's entry (i, j), j != i: j is unprocessed again and, with the
// gate's history on, D_j grows by w_ij.
__device__ __forceinline__ void mark_neighbour(const MoveArgs &a, int j, double w) {
    a.flag[j] = 1;
    if (a.dmoved) unsafeAtomicAdd(&a.dmoved[j], w);
}

// Folds the entry (key, v) of a scan table into (bg, bc, kid).
__device__ __forceinline__ void fold_key(const MoveArgs &a, double m2, int key, double v, int d, double ki, double &bg,
                                         int &bc, double &kid) {
    if (key == d) {
        kid = v;
    } else {
        double g = m2 * v - ki * a.sig[key];
        if (better(g, key, bg, bc, a.g.orig)) {
            bg = g;
            bc = key;
        }
    }
}

// Value type of the wave and workgroup LDS tables: on unit weights every
// K_{i->c} is a count (< 2^31), kept as an int (8-byte slots, a quarter
// more resident waves); otherwise the fp64 sum.
template <int WT> struct TabVal { using T = double; };
template <> struct TabVal<W_UNIT> { using T = int; };

__device__ __forceinline__ void lds_count_add(int *keys, int *vals, uint32_t mask, int key) {
    uint32_t s = key_hash(key) & mask;
    while (true) {
        int prev = atomicCAS(&keys[s], kEmpty, key);
        if (prev == kEmpty || prev == key) {
            atomicAdd(&vals[s], 1);
            return;
        }
        s = (s + 1) & mask;
    }
}
__device__ __forceinline__ void lds_table_put(int *keys, int *vals, uint32_t mask, int key, double) {
    lds_count_add(keys, vals, mask, key);
}
__device__ __forceinline__ void lds_table_put(int *keys, double *vals, uint32_t mask, int key, double w) {
    lds_table_add(keys, vals, mask, key, w);
}

// Reads one table slot, resets it and folds it into (bg, bc, kid).
template <typename V>
__device__ __forceinline__ void take_slot(const MoveArgs &a, double m2, int *keys, V *vals, int64_t s, int d,
                                          double ki, double &bg, int &bc, double &kid, unsigned long long &nkeys) {
    int key = keys[s];
    if (key == kEmpty) return;
    double v = (double)vals[s];
    keys[s] = kEmpty;
    vals[s] = 0;
    nkeys++;
    if (key == d) {
        kid = v;
    } else {
        double g = m2 * v - ki * a.sig[key];
        if (better(g, key, bg, bc, a.g.orig)) {
            bg = g;
            bc = key;
        }
    }
}

// Scores a whole table of T slots with NT threads (t = this thread's
// index), resetting it: each thread reads CH slots, then the Sigma of their
// communities together, then folds them.  The argmax does not depend on the
// order of the slots.
template <int NT, int CH, typename V>
__device__ __forceinline__ void fold_table(const MoveArgs &a, double m2, int *keys, V *vals, int T, int t, int d,
                                           double ki, double &bg, int &bc, double &kid,
                                           unsigned long long &nkeys) {
    for (int s0 = 0; s0 < T; s0 += NT * CH) {
        int key[CH];
        double v[CH], sg[CH];
#pragma unroll
        for (int u = 0; u < CH; u++) {
            const int sl = s0 + u * NT + t;
            key[u] = sl < T ? keys[sl] : kEmpty;
            v[u] = 0.0;
            if (key[u] != kEmpty) {
                v[u] = (double)vals[sl];
                keys[sl] = kEmpty;
                vals[sl] = 0;
            }
        }
#pragma unroll
        for (int u = 0; u < CH; u++) sg[u] = (key[u] != kEmpty && key[u] != d) ? a.sig[key[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < CH; u++) {
            if (key[u] == kEmpty) continue;
            nkeys++;
            if (key[u] == d) {
                kid = v[u];
            } else {
                double g = m2 * v[u] - ki * sg[u];
                if (better(g, key[u], bg, bc, a.g.orig)) {
                    bg = g;
                    bc = key[u];
                }
            }
        }
    }
}

// ---------------------------------------------------------------- compact

constexpr int kCompactSpan = 4096;   // entries of the buckets per compaction workgroup, at most

// Unprocessed vertices of the sub-round's buckets -> per-bin queues (or,
// in a gated sweep, per-bin candidate lists for the gate).  Workgroup k
// takes the contiguous range [k span, (k + 1) span) of the buckets (span <=
// kCompactSpan), stages its active vertices in LDS with their rank in their
// bin, reserves their queue slots with one atomic per bin, then writes them.
// The queue counters are shared by every workgroup, so their atomics, not
// the reads, bound this kernel on large levels: one per bin per workgroup
// (not per 256 entries) keeps them few.
__global__ void __launch_bounds__(kBlock) k_move_compact(MoveArgs a, const int32_t *bl, int64_t span) {
    __shared__ int lcnt[kNumBins];
    __shared__ int lbase[kNumBins];
    __shared__ int32_t sv[kCompactSpan];      // staged vertex
    __shared__ uint32_t sbr[kCompactSpan];    // its bin (top 4 bits) and rank in the bin
    int64_t pre[kNumBins + 1];
    pre[0] = 0;
#pragma unroll
    for (int b = 0; b < kNumBins; b++) pre[b + 1] = pre[b] + a.qcap[b];
    const int64_t total = pre[kNumBins];
    const bool gated = a.cand != nullptr;   // the gate fills the queue from the candidates
    int *qcnt = gated ? a.ctr->ccnt[a.round] : a.ctr->qcnt[a.round];
    int32_t *qout = gated ? a.cand : a.queue;
    const int64_t lo = blockIdx.x * span;
    const int64_t hi = lo + span < total ? lo + span : total;
    if (threadIdx.x < kNumBins) lcnt[threadIdx.x] = 0;
    __shared__ int nst;
    if (threadIdx.x == 0) nst = 0;
    __syncthreads();
    for (int64_t t = lo + threadIdx.x; t < hi; t += kBlock) {
        int b = 0;
        while (t >= pre[b + 1]) b++;
        const int i = bl[a.qbase[b] + (t - pre[b])];
        bool act = a.flag[i] != 0 && (!a.gactive || a.gactive[a.g.gid[i]]);
        if (act && a.single_only && a.csize[a.cm[i]] != 1) {
            a.flag[i] = 0;   // merged into a sub-community: stays
            act = false;
        }
        if (b == BIN_HUB) a.hub_act[i] = act ? 1 : 0;
        if (act) {
            a.flag[i] = 0;
            if (a.dmoved) a.dsnap[i] = a.dmoved[i];   // the features' D_i
            const int rank = atomicAdd(&lcnt[b], 1);
            const int slot = atomicAdd(&nst, 1);
            sv[slot] = i;
            sbr[slot] = ((uint32_t)b << 28) | (uint32_t)rank;
        }
    }
    __syncthreads();
    if (threadIdx.x < kNumBins && lcnt[threadIdx.x] > 0)
        lbase[threadIdx.x] = atomicAdd(&qcnt[threadIdx.x], lcnt[threadIdx.x]);
    __syncthreads();
    for (int k = threadIdx.x; k < nst; k += kBlock) {
        const uint32_t br = sbr[k];
        const int b = (int)(br >> 28);
        qout[a.qbase[b] + lbase[b] + (int64_t)(br & 0x0FFFFFFFu)] = sv[k];
    }
}

// ---------------------------------------------------------------- small

// Orders the LDS operations of one wavefront (its lanes are the only users
// of their table region): no workgroup barrier, so the waves of a block run
// their units independently.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
}

// Argmax / sum over aligned groups of G lanes, G a runtime power of two.
__device__ __forceinline__ void group_argmax_rt(double &g, int &c, int G, const int32_t *orig) {
    for (int off = G >> 1; off > 0; off >>= 1) {
        double og = __shfl_xor(g, off);
        int oc = __shfl_xor(c, off);
        if (better(og, oc, g, c, orig)) {
            g = og;
            c = oc;
        }
    }
}

__device__ __forceinline__ double group_sum_rt(double x, int G) {
    for (int off = G >> 1; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// Small bins (degree <= G = 4, 8, ..., 64): a group of L = max(G /
// kSmallE, 1) lanes per vertex, up to kSmallE entries per lane (loaded
// together), a table of 2G slots per vertex in the wave's LDS; a wavefront
// takes 64 / L vertices.  G is a runtime value, so the five bins share one
// code path.
constexpr int kSmallE = 4;
__host__ __device__ inline int small_lanes(int G) { return G > kSmallE ? G / kSmallE : 1; }

template <int WT>
__device__ void small_unit(const MoveArgs &a, int bin, int G, int64_t unit, int cnt, int *wkeys, double *wvals,
                           Acc &acc) {
    const int kSlots = 2 * G, L = small_lanes(G);
    const int lane = lane_id();
    const int grp = lane / L, gl = lane & (L - 1);
    const int64_t qi = unit * (kWave / L) + grp;
    const bool valid = qi < cnt;
    int *keys = wkeys + grp * kSlots;
    double *vals = wvals + grp * kSlots;
    int i = -1, di = 0, d = -1, csd = 0;
    int j[kSmallE];
    double w[kSmallE];
    double ki = 0.0, m2 = a.M2, sgd = 0.0;
#pragma unroll
    for (int r = 0; r < kSmallE; r++) {
        j[r] = -1;
        w[r] = 0.0;
    }
    if (valid) {
        i = a.queue[a.qbase[bin] + qi];
        m2 = m2_of(a, i);
        di = a.g.deg[i];
        d = a.cm[i];
        ki = a.K[i];
        sgd = a.sig[d];
        csd = a.csize[d];
        const int64_t b0 = a.g.off[i];
#pragma unroll
        for (int r = 0; r < kSmallE; r++) {
            const int e = gl + r * L;
            if (e < di) {
                j[r] = load_col(a.g.col, b0 + e);
                w[r] = edge_weight<WT>(a.g.w, b0 + e);
            }
        }
        int c[kSmallE];
#pragma unroll
        for (int r = 0; r < kSmallE; r++) c[r] = (j[r] >= 0 && j[r] != i) ? a.cm[j[r]] : kEmpty;
#pragma unroll
        for (int r = 0; r < kSmallE; r++)
            if (c[r] != kEmpty) lds_table_add(keys, vals, kSlots - 1, c[r], w[r]);
    }
    wave_lds_sync();
    double bg = -INFINITY, kid = 0.0;
    int bc = kIntMax;
    if (valid) {
#pragma unroll
        for (int q = 0; q < 2 * kSmallE; q++)
            if (gl + q * L < kSlots) take_slot(a, m2, keys, vals, gl + q * L, d, ki, bg, bc, kid, acc.keys);
    }
    group_argmax_rt(bg, bc, L, a.g.orig);
    kid = group_sum_rt(kid, L);
    double gain = 0.0;
    bool mv = valid && decide(m2, d, ki, kid, bg, bc, sgd, csd, best_single(a, d, csd, bc), &gain);
    if (mv)
#pragma unroll
        for (int r = 0; r < kSmallE; r++)
            if (j[r] >= 0 && j[r] != i) mark_neighbour(a, j[r], w[r]);
    bool lead = valid && gl == 0;
    const unsigned long long cg = lead && mv ? counted_gain(a, i, d, bc, gain, m2) : 0ull;
    if (a.ggain) {   // batch: per-graph totals, one atomic per graph met by the wavefront
        int gk = valid ? a.g.gid[i] : 0;
        wave_add_u64_by_key(a.ggain, gk, cg, lead && mv);
        wave_add_u64_by_key(a.gmoved, gk, 1ull, lead && mv);
    }
    if (lead) {
        acc.verts++;
        acc.scanned += (unsigned long long)di;
        if (a.hbits) record_scan(a, m2, i, d, di, ki, kid, bg, bc, mv);
        a.dec[i] = mv ? bc : d;
        if (mv) {
            acc.gain += cg;
            acc.moved++;
        }
        if (a.gain_out) a.gain_out[i] = mv ? gain : 0.0;
    }
    wave_lds_sync();
}

// vertices of small bin b per wavefront
__host__ __device__ inline int small_vpw(int b) { return kWave / small_lanes(4 << b); }

template <int WT>
__global__ void __launch_bounds__(kBlock, WT == W_UNIT ? 5 : 4) k_move_small(MoveArgs a) {
    constexpr int kWaveSlots = 2 * kWave * kSmallE;   // (64 / L) vertices x 2G slots, at most
    __shared__ int tkeys[kWaveSlots * (kBlock / kWave)];
    __shared__ double tvals[kWaveSlots * (kBlock / kWave)];
    const int w = threadIdx.x / kWave;
    int *wkeys = tkeys + w * kWaveSlots;
    double *wvals = tvals + w * kWaveSlots;
    for (int k = lane_id(); k < kWaveSlots; k += kWave) {
        wkeys[k] = kEmpty;
        wvals[k] = 0.0;
    }
    wave_lds_sync();
    int cnt[kNumSmallBins];
    int64_t pre[kNumSmallBins + 1];
    pre[0] = 0;
#pragma unroll
    for (int b = 0; b < kNumSmallBins; b++) {
        cnt[b] = a.ctr->qcnt[a.round][b];
        int vpw = small_vpw(b);
        pre[b + 1] = pre[b] + (cnt[b] + vpw - 1) / vpw;
    }
    Acc acc;
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t u = (int64_t)blockIdx.x * (kBlock / kWave) + w; u < pre[kNumSmallBins]; u += nw) {
        int b = 0;
        while (u >= pre[b + 1]) b++;
        small_unit<WT>(a, b, 4 << b, u - pre[b], cnt[b], wkeys, wvals, acc);
    }
    flush_acc(acc, a.ctr, 0);
}

// ---------------------------------------------------------------- large

// Block-wide argmax / sum through LDS; every thread gets the result.
__device__ void block_argmax_sum(double &bg, int &bc, double &x, const int32_t *orig) {
    __shared__ double sg[kBlock / kWave], sx[kBlock / kWave];
    __shared__ int sc[kBlock / kWave];
    group_argmax<kWave>(bg, bc, orig);
    x = group_sum<kWave>(x);
    int w = threadIdx.x / kWave;
    if (lane_id() == 0) { sg[w] = bg; sc[w] = bc; sx[w] = x; }
    __syncthreads();
    bg = sg[0];
    bc = sc[0];
    x = sx[0];
#pragma unroll
    for (int q = 1; q < kBlock / kWave; q++) {
        if (better(sg[q], sc[q], bg, bc, orig)) { bg = sg[q]; bc = sc[q]; }
        x += sx[q];
    }
    __syncthreads();
}

// The LDS tables of the wave and workgroup bins (and of the hub chunks).
// With fp64 values they have 768 and 3072 slots, at most two thirds full for
// 512 and 2048 entries: 36 KB per workgroup of four wave tables or one
// workgroup table, so four workgroups share a CU's LDS where half-full
// tables let three (R-MAT 26: 3 % less time per run).  A key's first slot is
// then the multiply-shift reduction of its hash onto the T slots in use, and
// probing is linear with wrap-around.  On unit weights (int values) the
// half-full power-of-two tables already fit four workgroups, and the
// fuller ones only lengthened the probes (R-MAT 20: 2.6 % more time), so
// they stay.
template <int WT> struct ScanSlots {
    static constexpr int wave = WT == W_UNIT ? kWaveTable : 3 * kWaveMaxDeg / 2;
    static constexpr int block = WT == W_UNIT ? kBlockTable : 3 * kBlockMaxDeg / 2;
    // slots a vertex of d entries uses in a table of `cap` slots
    __device__ static int of(int d, int cap) {
        return WT == W_UNIT || d <= cap / 3 ? (int)hub_table_size(d) : cap;
    }
};
__device__ __forceinline__ uint32_t block_slot(int key, uint32_t T) {
    return (uint32_t)(((uint64_t)key_hash(key) * T) >> 32);
}
__device__ __forceinline__ void block_put(int *keys, int *vals, uint32_t T, int key, double) {
    uint32_t s = block_slot(key, T);
    while (true) {
        const int prev = atomicCAS(&keys[s], kEmpty, key);
        if (prev == kEmpty || prev == key) {
            atomicAdd(&vals[s], 1);
            return;
        }
        s = s + 1 == T ? 0 : s + 1;
    }
}
__device__ __forceinline__ void block_put(int *keys, double *vals, uint32_t T, int key, double w) {
    uint32_t s = block_slot(key, T);
    while (true) {
        const int prev = atomicCAS(&keys[s], kEmpty, key);
        if (prev == kEmpty || prev == key) {
            atomicAdd(&vals[s], w);
            return;
        }
        s = s + 1 == T ? 0 : s + 1;
    }
}
template <int WT, typename V>
__device__ __forceinline__ void scan_put(int *keys, V *vals, int T, int key, double w) {
    if constexpr (WT == W_UNIT)
        lds_table_put(keys, vals, (uint32_t)T - 1, key, w);   // T a power of two
    else
        block_put(keys, vals, (uint32_t)T, key, w);
}

// One wavefront per vertex of 65..512 entries, table in its LDS.
template <int WT>
__global__ void __launch_bounds__(kBlock, 4) k_move_wave(MoveArgs a) {
    using V = typename TabVal<WT>::T;
    constexpr int S = ScanSlots<WT>::wave;
    __shared__ int tkeys[kBlock / kWave * S];
    __shared__ V tvals[kBlock / kWave * S];
    const int w = threadIdx.x / kWave, lane = lane_id();
    int *keys = tkeys + w * S;
    V *vals = tvals + w * S;
    for (int k = lane; k < S; k += kWave) {
        keys[k] = kEmpty;
        vals[k] = 0;
    }
    wave_lds_sync();
    const int cnt = a.ctr->qcnt[a.round][BIN_WAVE];
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    Acc acc;
    for (int64_t qi = (int64_t)blockIdx.x * (kBlock / kWave) + w; qi < cnt; qi += nw) {
        int i = a.queue[a.qbase[BIN_WAVE] + qi];
        const double m2 = m2_of(a, i);
        int di = a.g.deg[i];
        int64_t beg = a.g.off[i];
        int d = a.cm[i];
        double ki = a.K[i];
        const double sgd = a.sig[d];
        const int csd = a.csize[d];
        const int T = ScanSlots<WT>::of(di, S);
        // the lane's entries (at most R) are loaded together, then their
        // memberships: two round trips to memory instead of 2R
        constexpr int R = kWaveMaxDeg / kWave;
        int jj[R];
        double ww[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int e = lane + r * kWave;
            jj[r] = e < di ? load_col(a.g.col, beg + e) : i;
            ww[r] = e < di ? edge_weight<WT>(a.g.w, beg + e) : 0.0;
        }
        int cj[R];
#pragma unroll
        for (int r = 0; r < R; r++) cj[r] = jj[r] != i ? a.cm[jj[r]] : kEmpty;
#pragma unroll
        for (int r = 0; r < R; r++)
            if (cj[r] != kEmpty) scan_put<WT>(keys, vals, T, cj[r], ww[r]);
        wave_lds_sync();
        double bg = -INFINITY, kid = 0.0;
        int bc = kIntMax;
        fold_table<kWave, 4>(a, m2, keys, vals, T, lane, d, ki, bg, bc, kid, acc.keys);
        group_argmax<kWave>(bg, bc, a.g.orig);
        kid = group_sum<kWave>(kid);
        double gain = 0.0;
        bool mv = decide(m2, d, ki, kid, bg, bc, sgd, csd, best_single(a, d, csd, bc), &gain);
        if (mv)   // the lane's columns are still in registers (weights reloaded)
#pragma unroll
            for (int r = 0; r < R; r++)
                if (jj[r] != i) mark_neighbour(a, jj[r], a.dmoved ? edge_weight<WT>(a.g.w, beg + lane + r * kWave) : 0.0);
        if (lane == 0) {
            acc.verts++;
            acc.scanned += (unsigned long long)di;
            if (a.hbits) record_scan(a, m2, i, d, di, ki, kid, bg, bc, mv);
            a.dec[i] = mv ? bc : d;
            if (mv) {
                const unsigned long long cg = counted_gain(a, i, d, bc, gain, m2);
                acc.gain += cg;
                acc.moved++;
                if (a.ggain) graph_totals(a, i, cg);
            }
            if (a.gain_out) a.gain_out[i] = mv ? gain : 0.0;
        }
        wave_lds_sync();
    }
    flush_acc(acc, a.ctr, 1);
}

// One workgroup per vertex of 513..2048 entries, table in LDS.
template <int WT>
__global__ void __launch_bounds__(kBlock, 4) k_move_block(MoveArgs a) {
    using V = typename TabVal<WT>::T;
    constexpr int S = ScanSlots<WT>::block;
    __shared__ int keys[S];
    __shared__ V vals[S];
    const int tid = threadIdx.x;
    for (int k = tid; k < S; k += kBlock) {
        keys[k] = kEmpty;
        vals[k] = 0;
    }
    __syncthreads();
    const int cnt = a.ctr->qcnt[a.round][BIN_BLOCK];
    Acc acc;
    for (int64_t qi = blockIdx.x; qi < cnt; qi += gridDim.x) {
        int i = a.queue[a.qbase[BIN_BLOCK] + qi];
        const double m2 = m2_of(a, i);
        int di = a.g.deg[i];
        int64_t beg = a.g.off[i];
        int d = a.cm[i];
        double ki = a.K[i];
        const double sgd = a.sig[d];
        const int csd = a.csize[d];
        const int T = ScanSlots<WT>::of(di, S);
        constexpr int R = kBlockMaxDeg / kBlock;   // entries per thread, loaded together
        int jj[R];
        double ww[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int e = tid + r * kBlock;
            jj[r] = e < di ? load_col(a.g.col, beg + e) : i;
            ww[r] = e < di ? edge_weight<WT>(a.g.w, beg + e) : 0.0;
        }
        int cj[R];
#pragma unroll
        for (int r = 0; r < R; r++) cj[r] = jj[r] != i ? a.cm[jj[r]] : kEmpty;
#pragma unroll
        for (int r = 0; r < R; r++)
            if (cj[r] != kEmpty) scan_put<WT>(keys, vals, T, cj[r], ww[r]);
        __syncthreads();
        double bg = -INFINITY, kid = 0.0;
        int bc = kIntMax;
        fold_table<kBlock, 4>(a, m2, keys, vals, T, tid, d, ki, bg, bc, kid, acc.keys);
        block_argmax_sum(bg, bc, kid, a.g.orig);
        double gain = 0.0;
        bool mv = decide(m2, d, ki, kid, bg, bc, sgd, csd, best_single(a, d, csd, bc), &gain);
        if (mv)   // the thread's columns are still in registers (weights reloaded)
#pragma unroll
            for (int r = 0; r < R; r++)
                if (jj[r] != i) mark_neighbour(a, jj[r], a.dmoved ? edge_weight<WT>(a.g.w, beg + tid + r * kBlock) : 0.0);
        if (tid == 0) {
            acc.verts++;
            acc.scanned += (unsigned long long)di;
            if (a.hbits) record_scan(a, m2, i, d, di, ki, kid, bg, bc, mv);
            a.dec[i] = mv ? bc : d;
            if (mv) {
                const unsigned long long cg = counted_gain(a, i, d, bc, gain, m2);
                acc.gain += cg;
                acc.moved++;
                if (a.ggain) graph_totals(a, i, cg);
            }
            if (a.gain_out) a.gain_out[i] = mv ? gain : 0.0;
        }
        __syncthreads();
    }
    flush_acc(acc, a.ctr, 2);
}

// ---------------------------------------------------------------- hubs

// One workgroup per chunk of kHubChunk entries of an active hub: the chunk
// is first reduced in an LDS table (so a community met many times in the
// chunk costs one global atomic), then each distinct (community, partial
// sum) goes into the hub's global table.
template <int WT>
__global__ void __launch_bounds__(kBlock) k_move_hub_insert(MoveArgs a) {
    __shared__ int tkeys[kBlockTable];
    __shared__ double tvals[kBlockTable];
    for (int k = threadIdx.x; k < kBlockTable; k += kBlock) {
        tkeys[k] = kEmpty;
        tvals[k] = 0.0;
    }
    __syncthreads();
    Acc acc;
    for (int64_t k = a.ch_first + blockIdx.x; k < a.ch_first + a.ch_count; k += gridDim.x) {
        int i = a.ch_vert[k];
        if (!a.hub_act[i]) continue;
        int64_t beg = a.ch_beg[k];
        int64_t end = a.g.off[i] + a.g.deg[i];
        if (end > beg + kHubChunk) end = beg + kHubChunk;
        for (int64_t e = beg + threadIdx.x; e < end; e += kBlock) {
            int j = load_col(a.g.col, e);
            double wt = edge_weight<WT>(a.g.w, e);
            if (j != i) lds_table_add(tkeys, tvals, kBlockTable - 1, a.cm[j], wt);
        }
        __syncthreads();
        int64_t tb = a.hub_off[i];
        uint64_t mask = hub_table_size(a.g.deg[i]) - 1;
        int *gk = a.hkeys + tb;
        double *gv = a.hvals + tb;
        // batches of 4 slots: the first compare-and-swaps are issued together
        for (int s0 = threadIdx.x; s0 < kBlockTable; s0 += 4 * kBlock) {
            int key[4], prev[4];
            double v[4];
            uint64_t gs[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                int sl = s0 + u * kBlock;
                key[u] = tkeys[sl];
                v[u] = tvals[sl];
                tkeys[sl] = kEmpty;
                tvals[sl] = 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                prev[u] = kEmpty;
                if (key[u] != kEmpty) {
                    gs[u] = key_hash(key[u]) & mask;
                    prev[u] = atomicCAS(&gk[gs[u]], kEmpty, key[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if (key[u] == kEmpty) continue;
                acc.ginserts++;
                if (prev[u] == kEmpty || prev[u] == key[u])
                    unsafeAtomicAdd(&gv[gs[u]], v[u]);
                else
                    gbl_table_add(gk, gv, mask, key[u], v[u]);
            }
        }
        if (threadIdx.x == 0) acc.scanned += (unsigned long long)(end - beg);
        __syncthreads();
    }
    flush_acc(acc, a.ctr, 3);
}

// ---------------------------------------------------------------- hubs by hash partitions
//
// A hub's distinct neighbour communities are split into P hash partitions
// (P = its number of chunks).  Phase 1, per chunk: reduce the chunk's entries
// in LDS and write the distinct (community, weight) pairs to staging at the
// chunk's own entry positions, grouped by partition, plus one word per
// partition (start << 16 | count).  Phase 2, per partition: gather that
// partition's pairs from every chunk of the hub into one LDS table and score
// it.  Each (chunk, community) pair is written once and read once; nothing
// goes through a global hash table.

template <int WT>
__global__ void __launch_bounds__(kBlock) k_hub_bucket(MoveArgs a) {
    using V = typename TabVal<WT>::T;
    constexpr int S = ScanSlots<WT>::block;   // a chunk's <= 2048 communities
    __shared__ int tkeys[S];
    __shared__ V tvals[S];
    __shared__ int pcnt[kMaxParts + 1];
    const int tid = threadIdx.x;
    for (int k = tid; k < S; k += kBlock) {
        tkeys[k] = kEmpty;
        tvals[k] = 0;
    }
    __syncthreads();
    Acc acc;
    for (int64_t k = a.ch_first + blockIdx.x; k < a.ch_first + a.ch_count; k += gridDim.x) {
        int i = a.ch_vert[k];
        if (a.hub_act[i] != 1) continue;
        int di = a.g.deg[i];
        int P = (di + kHubChunk - 1) / kHubChunk;
        if (P > a.max_parts) {   // too many partitions: the hub's global table
            if (tid == 0) a.hub_act[i] = 3;
            continue;
        }
        int64_t beg = a.ch_beg[k];
        int64_t end = a.g.off[i] + di;
        if (end > beg + kHubChunk) end = beg + kHubChunk;
        int s = (int)((beg - a.g.off[i]) / kHubChunk);
        {
            constexpr int R = kHubChunk / kBlock;   // entries per thread, loaded together
            int jj[R];
            double ww[R];
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int64_t e = beg + tid + r * kBlock;
                jj[r] = e < end ? load_col(a.g.col, e) : i;
                ww[r] = e < end ? edge_weight<WT>(a.g.w, e) : 0.0;
            }
            int cj[R];
#pragma unroll
            for (int r = 0; r < R; r++) cj[r] = jj[r] != i ? a.cm[jj[r]] : kEmpty;
#pragma unroll
            for (int r = 0; r < R; r++)
                if (cj[r] != kEmpty) scan_put<WT>(tkeys, tvals, S, cj[r], ww[r]);
        }
        for (int b = tid; b <= P; b += kBlock) pcnt[b] = 0;
        __syncthreads();
        for (int sl = tid; sl < S; sl += kBlock) {
            int key = tkeys[sl];
            if (key != kEmpty) atomicAdd(&pcnt[part_of(key, P)], 1);
        }
        __syncthreads();
        block_scan_excl(pcnt, P);
        uint32_t *words = a.hbuck + a.hub_b0[i] + (int64_t)s * P;
        for (int b = tid; b < P; b += kBlock) words[b] = ((uint32_t)pcnt[b] << 16) | (uint32_t)(pcnt[b + 1] - pcnt[b]);
        if (tid == 0) acc.aux += (unsigned long long)P;
        __syncthreads();
        for (int sl = tid; sl < S; sl += kBlock) {
            int key = tkeys[sl];
            if (key == kEmpty) continue;
            double v = (double)tvals[sl];
            tkeys[sl] = kEmpty;
            tvals[sl] = 0;
            int pos = atomicAdd(&pcnt[part_of(key, P)], 1);
            a.skey[beg + pos] = key;
            a.sval[beg + pos] = v;
            acc.ginserts++;
        }
        if (tid == 0) acc.scanned += (unsigned long long)(end - beg);
        __syncthreads();
    }
    flush_acc(acc, a.ctr, 3);
}

// A hub's decision from (bg, bc, kid) (block-uniform): records it, counts
// it in acc (class of the hub decisions) and leaves hub_act = 2 (moves: its
// neighbours are marked chunk by chunk in apply) or 0.  Thread 0 writes.
__device__ __forceinline__ void hub_decide(const MoveArgs &a, int i, double bg, int bc, double kid, int nch,
                                           Acc &acc) {
    if (threadIdx.x != 0) return;
    const double m2 = m2_of(a, i);
    const int d = a.cm[i], di = a.g.deg[i];
    const double ki = a.K[i];
    const int csd = a.csize[d];
    double gain = 0.0;
    bool mv = decide(m2, d, ki, kid, bg, bc, a.sig[d], csd, best_single(a, d, csd, bc), &gain);
    acc.verts++;
    acc.aux += (unsigned long long)nch;
    a.hub_act[i] = mv ? 2 : 0;
    if (a.hbits) record_scan(a, m2, i, d, di, ki, kid, bg, bc, mv);
    a.dec[i] = mv ? bc : d;
    if (mv) {
        const unsigned long long cg = counted_gain(a, i, d, bc, gain, m2);
        acc.gain += cg;
        acc.moved++;
        if (a.ggain) graph_totals(a, i, cg);
    }
    if (a.gain_out) a.gain_out[i] = mv ? gain : 0.0;
}

// A hub's decision after its partitions (all results in part_*): combine
// the P partitions' best candidates and decide.  If a partition overflowed
// or the hub has more than max_parts chunks (hub_act = 3), the workgroup
// takes the whole hub through its global table instead: insert every entry,
// then score and reset the table (rare; slow for enormous hubs, but exact).
template <int WT>
__device__ void hub_finish_block(const MoveArgs &a, int i, int P, Acc &acc) {
    const int tid = threadIdx.x;
    const int d = a.cm[i];
    const double ki = a.K[i];
    const double m2 = m2_of(a, i);
    double bg = -INFINITY, kid = 0.0;
    int bc = kIntMax;
    if (a.hub_act[i] == 3) {
        const int di = a.g.deg[i];
        const int64_t beg = a.g.off[i], T = (int64_t)hub_table_size(di), tb = a.hub_off[i];
        int *gk = a.hkeys + tb;
        double *gv = a.hvals + tb;
        for (int64_t e = beg + tid; e < beg + di; e += kBlock) {
            int j = load_col(a.g.col, e);
            if (j != i) gbl_table_add(gk, gv, (uint64_t)(T - 1), a.cm[j], edge_weight<WT>(a.g.w, e));
        }
        __threadfence();   // the table was built with device-scope atomics
        __syncthreads();
        for (int64_t q = tid; q < T; q += kBlock) {
            int key = __hip_atomic_load(gk + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (key == kEmpty) continue;
            double v = __hip_atomic_load(gv + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            gk[q] = kEmpty;
            gv[q] = 0.0;
            acc.keys++;
            fold_key(a, m2, key, v, d, ki, bg, bc, kid);
        }
    } else {
        const int64_t c0 = a.hub_ch0[i];
        for (int q = tid; q < P; q += kBlock) {
            double g = a.part_g[c0 + q];
            int c = a.part_c[c0 + q];
            if (better(g, c, bg, bc, a.g.orig)) {
                bg = g;
                bc = c;
            }
            kid += a.part_kid[c0 + q];
        }
    }
    block_argmax_sum(bg, bc, kid, a.g.orig);
    hub_decide(a, i, bg, bc, kid, P, acc);
    __syncthreads();
}

// One workgroup per active hub of the sub-round (partition path).
template <int WT>
__global__ void __launch_bounds__(kBlock) k_hub_decide(MoveArgs a) {
    const int cnt = a.ctr->qcnt[a.round][BIN_HUB];
    Acc acc;
    for (int64_t qi = blockIdx.x; qi < cnt; qi += gridDim.x) {
        int i = a.queue[a.qbase[BIN_HUB] + qi];
        hub_finish_block<WT>(a, i, (a.g.deg[i] + kHubChunk - 1) / kHubChunk, acc);
    }
    flush_acc(acc, a.ctr, 4);
}

// Per partition of an active hub: merges the partition's pairs from every
// chunk of the hub (source chunks taken kHubWin at a time) in one LDS table
// and scores it.  On unit weights the values are counts (int slots).
constexpr int kHubWin = 512;

// A hub partition's merge table: on unit weights (int values, 32 KB) 4096
// slots and at most kPartCap distinct communities; otherwise 3072 slots and
// at most 2560 (a partition holds about 2048 on average, as a hub has one
// partition per chunk of 2048 entries), so that four workgroups share a
// CU's LDS where the 4096-slot fp64 table let three.  Past the cap the hub
// takes its global table.  Fewer than kBlock inserts overshoot the cap.
template <int WT> struct GatherSlots {
    static constexpr int slots = WT == W_UNIT ? kBlockTable : 3 * kBlockMaxDeg / 2;
    static constexpr int cap = WT == W_UNIT ? kPartCap : 2560;
    static_assert(cap + kBlock < slots, "the merge table never fills");
    __device__ static uint32_t first(int key) {
        if constexpr (WT == W_UNIT)
            return key_hash(key) & (uint32_t)(slots - 1);
        else
            return (uint32_t)(((uint64_t)key_hash(key) * slots) >> 32);
    }
};

template <int WT>
__global__ void __launch_bounds__(kBlock) k_hub_gather(MoveArgs a) {
    using V = typename TabVal<WT>::T;
    constexpr int S = GatherSlots<WT>::slots;
    __shared__ int tkeys[S];
    __shared__ V tvals[S];
    __shared__ int pst[kHubWin + 1];
    __shared__ short srcst[kHubWin];   // this partition's start within each source chunk
    __shared__ int nkeys, ovf;
    const int tid = threadIdx.x;
    for (int k = tid; k < S; k += kBlock) {
        tkeys[k] = kEmpty;
        tvals[k] = 0;
    }
    __syncthreads();
    Acc acc;
    for (int64_t k = a.ch_first + blockIdx.x; k < a.ch_first + a.ch_count; k += gridDim.x) {
        int i = a.ch_vert[k];
        // 0: not in this sub-round's frontier; 3: the hub goes through its
        // global table (set by the chunk kernel, or by a partition that
        // overflowed: the decision kernel takes it)
        if (a.hub_act[i] != 1) continue;
        int di = a.g.deg[i];
        int P = (di + kHubChunk - 1) / kHubChunk;
        {
        int p = (int)((a.ch_beg[k] - a.g.off[i]) / kHubChunk);
        const uint32_t *words = a.hbuck + a.hub_b0[i];
        const int64_t base = a.g.off[i];
        if (tid == 0) {
            nkeys = 0;
            ovf = 0;
            acc.verts++;   // chunks (partitions) gathered
            acc.aux += (unsigned long long)P;
        }
        for (int w0 = 0; w0 < P; w0 += kHubWin) {
            const int nw = P - w0 < kHubWin ? P - w0 : kHubWin;
            for (int s = tid; s < nw; s += kBlock) {
                uint32_t wd = words[(int64_t)(w0 + s) * P + p];
                pst[s] = (int)(wd & 0xFFFFu);
                srcst[s] = (short)(wd >> 16);
            }
            __syncthreads();
            block_scan_excl(pst, nw);
            const int total = pst[nw];
            if (tid == 0) acc.ginserts += (unsigned long long)total;
            for (int t = tid; t < total; t += kBlock) {
                if (*(volatile int *)&ovf) break;
                int s = last_le(pst, nw, t);
                int64_t idx = base + (int64_t)(w0 + s) * kHubChunk + (int64_t)srcst[s] + (t - pst[s]);
                int key = a.skey[idx];
                double v = a.sval[idx];
                // insert, counting distinct keys; past kPartCap the partition
                // stops (at most kBlock inserts overshoot: the table never fills)
                uint32_t sl = GatherSlots<WT>::first(key);
                while (true) {
                    int prev = atomicCAS(&tkeys[sl], kEmpty, key);
                    if (prev == kEmpty) {
                        if (atomicAdd(&nkeys, 1) >= GatherSlots<WT>::cap) ovf = 1;
                        atomicAdd(&tvals[sl], (V)v);
                        break;
                    }
                    if (prev == key) {
                        atomicAdd(&tvals[sl], (V)v);
                        break;
                    }
                    sl = sl + 1 == (uint32_t)S ? 0 : sl + 1;
                }
            }
            __syncthreads();
            if (ovf) break;
        }
        if (ovf) {   // rare: this hub goes through its global table
            for (int q = tid; q < S; q += kBlock) {
                tkeys[q] = kEmpty;
                tvals[q] = 0;
            }
            if (tid == 0) a.hub_act[i] = 3;
        } else {
            int d = a.cm[i];
            double ki = a.K[i];
            const double m2 = m2_of(a, i);
            double bg = -INFINITY, kid = 0.0;
            int bc = kIntMax;
            fold_table<kBlock, 8>(a, m2, tkeys, tvals, S, tid, d, ki, bg, bc, kid, acc.keys);
            block_argmax_sum(bg, bc, kid, a.g.orig);
            if (tid == 0) {
                a.part_g[k] = bg;
                a.part_c[k] = bc;
                a.part_kid[k] = kid;
            }
        }
        }
        __syncthreads();
    }
    flush_acc(acc, a.ctr, 5);
}

// One workgroup per chunk again: chunk s of a hub with nch chunks scores and
// resets the slice [s*seg, (s+1)*seg) of the hub's table (seg = ceil(T /
// nch) <= 8192 slots; the table is complete now) and leaves the slice's best
// candidate and its share of K_{i->d} in part_*[chunk].
__global__ void __launch_bounds__(kBlock) k_move_hub_part(MoveArgs a) {
    Acc acc;
    for (int64_t k = a.ch_first + blockIdx.x; k < a.ch_first + a.ch_count; k += gridDim.x) {
        int i = a.ch_vert[k];
        if (!a.hub_act[i]) continue;
        int di = a.g.deg[i];
        int64_t T = (int64_t)hub_table_size(di);
        int64_t nch = (di + kHubChunk - 1) / kHubChunk;
        int64_t seg = (T + nch - 1) / nch;
        int64_t sidx = (a.ch_beg[k] - a.g.off[i]) / kHubChunk;
        int64_t s0 = sidx * seg, s1 = s0 + seg < T ? s0 + seg : T;
        int d = a.cm[i];
        double ki = a.K[i];
        const double m2 = m2_of(a, i);
        int64_t tb = a.hub_off[i];
        double bg = -INFINITY, kid = 0.0;
        int bc = kIntMax;
        int *gk = a.hkeys + tb;
        double *gv = a.hvals + tb;
        for (int64_t q0 = s0 + threadIdx.x; q0 < s1; q0 += 4 * kBlock) {
            int key[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                int64_t q = q0 + u * kBlock;
                key[u] = q < s1 ? gk[q] : kEmpty;
            }
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                v[u] = 0.0;
                if (key[u] != kEmpty) {
                    int64_t q = q0 + u * kBlock;
                    v[u] = gv[q];
                    gk[q] = kEmpty;
                    gv[q] = 0.0;
                    acc.keys++;
                }
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (key[u] != kEmpty) fold_key(a, m2, key[u], v[u], d, ki, bg, bc, kid);
        }
        block_argmax_sum(bg, bc, kid, a.g.orig);
        if (threadIdx.x == 0) {
            a.part_g[k] = bg;
            a.part_c[k] = bc;
            a.part_kid[k] = kid;
        }
    }
    flush_acc(acc, a.ctr, 4);
}

// One wavefront per active hub: combines its chunks' partial results and
// decides (the neighbours of a moving hub are marked by the apply kernel).
__global__ void __launch_bounds__(kBlock) k_move_hub_final(MoveArgs a) {
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int cnt = a.ctr->qcnt[a.round][BIN_HUB];
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    Acc acc;
    for (int64_t qi = (int64_t)blockIdx.x * (kBlock / kWave) + w; qi < cnt; qi += nw) {
        int i = a.queue[a.qbase[BIN_HUB] + qi];
        const double m2 = m2_of(a, i);
        int di = a.g.deg[i];
        int d = a.cm[i];
        double ki = a.K[i];
        int64_t c0 = a.hub_ch0[i];
        int nch = (di + kHubChunk - 1) / kHubChunk;
        double bg = -INFINITY, kid = 0.0;
        int bc = kIntMax;
        for (int q = lane; q < nch; q += kWave) {
            double g = a.part_g[c0 + q];
            int c = a.part_c[c0 + q];
            if (better(g, c, bg, bc, a.g.orig)) { bg = g; bc = c; }
            kid += a.part_kid[c0 + q];
        }
        group_argmax<kWave>(bg, bc, a.g.orig);
        kid = group_sum<kWave>(kid);
        double gain = 0.0;
        const int csd = a.csize[d];
        bool mv = decide(m2, d, ki, kid, bg, bc, a.sig[d], csd, best_single(a, d, csd, bc), &gain);
        if (lane == 0) {
            acc.verts++;
            acc.aux += (unsigned long long)nch;
            a.hub_act[i] = mv ? 2 : 0;   // 2: its neighbours are marked chunk by chunk in apply
            if (a.hbits) record_scan(a, m2, i, d, di, ki, kid, bg, bc, mv);
            a.dec[i] = mv ? bc : d;
            if (mv) {
                const unsigned long long cg = counted_gain(a, i, d, bc, gain, m2);
                acc.gain += cg;
                acc.moved++;
                if (a.ggain) graph_totals(a, i, cg);
            }
            if (a.gain_out) a.gain_out[i] = mv ? gain : 0.0;
        }
    }
    flush_acc(acc, a.ctr, 4);
}

// ---------------------------------------------------------------- apply

// Moves of the sub-round.  Blocks [0, nq) walk the sub-round's queue: every
// vertex whose decision differs from its community moves (C'[i] <- c*);
// the Sigma and size changes of a tile are summed per community in LDS
// first (movers crowd into a few popular communities).  Blocks [nq, ...)
// take the sub-round's hub chunks and mark the chunk's neighbours of a hub
// that moved.
constexpr int kApplyTable = 4 * kBlock;

__global__ void __launch_bounds__(kBlock) k_move_apply(MoveArgs a, int nq) {
    __shared__ int tk[kApplyTable];
    __shared__ double tv[kApplyTable];
    __shared__ int tc[kApplyTable];
    if ((int)blockIdx.x >= nq) {
        for (int64_t k = a.ch_first + (blockIdx.x - nq); k < a.ch_first + a.ch_count; k += gridDim.x - nq) {
            int i = a.ch_vert[k];
            if (a.hub_act[i] != 2) continue;
            int64_t beg = a.ch_beg[k];
            int64_t end = a.g.off[i] + a.g.deg[i];
            if (end > beg + kHubChunk) end = beg + kHubChunk;
            for (int64_t e = beg + threadIdx.x; e < end; e += kBlock) {
                int j = load_col(a.g.col, e);
                if (j == i) continue;
                double w = 0.0;
                if (a.dmoved)
                    w = a.g.wt == W_UNIT ? 1.0
                                         : (a.g.wt == W_F32 ? edge_weight<W_F32>(a.g.w, e) : edge_weight<W_F64>(a.g.w, e));
                mark_neighbour(a, j, w);
            }
        }
        return;
    }
    for (int s = threadIdx.x; s < kApplyTable; s += kBlock) {
        tk[s] = kEmpty;
        tv[s] = 0.0;
        tc[s] = 0;
    }
    __syncthreads();
    int64_t pre[kNumBins + 1];
    pre[0] = 0;
#pragma unroll
    for (int b = 0; b < kNumBins; b++) pre[b + 1] = pre[b] + a.ctr->qcnt[a.round][b];
    int32_t *cm = const_cast<int32_t *>(a.cm);
    double *sig = const_cast<double *>(a.sig);
    int32_t *csize = const_cast<int32_t *>(a.csize);
    for (int64_t t0 = blockIdx.x * (int64_t)kBlock; t0 < pre[kNumBins]; t0 += (int64_t)nq * kBlock) {
        int64_t t = t0 + threadIdx.x;
        if (t < pre[kNumBins]) {
            int b = 0;
            while (t >= pre[b + 1]) b++;
            int i = a.queue[a.qbase[b] + (t - pre[b])];
            int c = a.dec[i];
            int d = cm[i];
            if (c != d) {
                double ki = a.K[i];
                cm[i] = c;
                int sd = lds_table_slot(tk, kApplyTable - 1, d);
                int sc = lds_table_slot(tk, kApplyTable - 1, c);
                if (ki != 0.0) {
                    atomicAdd(&tv[sd], -ki);
                    atomicAdd(&tv[sc], ki);
                }
                atomicSub(&tc[sd], 1);
                atomicAdd(&tc[sc], 1);
            }
        }
        __syncthreads();
        for (int s = threadIdx.x; s < kApplyTable; s += kBlock) {
            int key = tk[s];
            if (key == kEmpty) continue;
            if (tv[s] != 0.0) unsafeAtomicAdd(&sig[key], tv[s]);
            if (tc[s] != 0) atomicAdd(&csize[key], tc[s]);
            tk[s] = kEmpty;
            tv[s] = 0.0;
            tc[s] = 0;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kBlock) k_community_totals(const double *K, const int32_t *cm, int64_t n,
                                                            double *sig, int32_t *csize) {
    for (int64_t i0 = blockIdx.x * (int64_t)kBlock; i0 < n; i0 += (int64_t)gridDim.x * kBlock) {
        int64_t i = i0 + threadIdx.x;
        bool ok = i < n;
        int c = ok ? cm[i] : 0;
        double k = ok ? K[i] : 0.0;
        wave_add_f64_by_key(sig, c, k, ok && k != 0.0);
        if (csize) wave_add_i32_by_key(csize, c, 1, ok);
    }
}

inline unsigned cap_grid(int64_t units, int64_t cap) {
    if (units < 1) units = 1;
    return (unsigned)(units < cap ? units : cap);
}

// A kernel's cap under the run's launch schedule.
inline int64_t sched_cap(const MoveArgs &a, int64_t cap) { return a.grid_cap > 0 && a.grid_cap < cap ? a.grid_cap : cap; }

}  // namespace

void launch_community_totals(const double *K, const int32_t *cm, int64_t n, double *sig, int32_t *csize,
                             hipStream_t s) {
    if (n > 0) k_community_totals<<<cap_grid((n + kBlock - 1) / kBlock, 8192), kBlock, 0, s>>>(K, cm, n, sig, csize);
}

void launch_move_compact(const MoveArgs &a, const WorkLists &wl, hipStream_t s) {
    int64_t total = 0;
    for (int b = 0; b < kNumBins; b++) total += a.qcap[b];
    if (total == 0) return;
    // one pass of 256 entries per workgroup while that gives at most 1024
    // workgroups, then longer ranges (at most kCompactSpan entries)
    int64_t blocks = (total + kBlock - 1) / kBlock;
    if (blocks > 1024) blocks = 1024;
    if (blocks < (total + kCompactSpan - 1) / kCompactSpan) blocks = (total + kCompactSpan - 1) / kCompactSpan;
    int64_t span = (total + blocks - 1) / blocks;
    span = (span + kBlock - 1) / kBlock * kBlock;
    blocks = (total + span - 1) / span;
    k_move_compact<<<(unsigned)blocks, kBlock, 0, s>>>(a, wl.bl, span);
}

void launch_move_small(const MoveArgs &a, const WorkLists &wl, hipStream_t s) {
    (void)wl;
    int64_t units = 0;   // wave units
    for (int b = 0; b < kNumSmallBins; b++) {
        int vpw = small_vpw(b);
        units += (a.qcap[b] + vpw - 1) / vpw;
    }
    if (units == 0) return;
    unsigned gr = cap_grid((units + 3) / 4, sched_cap(a, 8192));
    if (a.g.wt == W_UNIT)
        k_move_small<W_UNIT><<<gr, kBlock, 0, s>>>(a);
    else if (a.g.wt == W_F32)
        k_move_small<W_F32><<<gr, kBlock, 0, s>>>(a);
    else
        k_move_small<W_F64><<<gr, kBlock, 0, s>>>(a);
}

void launch_move_wave(const MoveArgs &a, hipStream_t s) {
    if (a.qcap[BIN_WAVE] == 0) return;
    unsigned gr = cap_grid((a.qcap[BIN_WAVE] + 3) / 4, sched_cap(a, 4096));
    if (a.g.wt == W_UNIT)
        k_move_wave<W_UNIT><<<gr, kBlock, 0, s>>>(a);
    else if (a.g.wt == W_F32)
        k_move_wave<W_F32><<<gr, kBlock, 0, s>>>(a);
    else
        k_move_wave<W_F64><<<gr, kBlock, 0, s>>>(a);
}

void launch_move_block(const MoveArgs &a, hipStream_t s) {
    if (a.qcap[BIN_BLOCK] == 0) return;
    unsigned gr = cap_grid(a.qcap[BIN_BLOCK], sched_cap(a, 2048));
    if (a.g.wt == W_UNIT)
        k_move_block<W_UNIT><<<gr, kBlock, 0, s>>>(a);
    else if (a.g.wt == W_F32)
        k_move_block<W_F32><<<gr, kBlock, 0, s>>>(a);
    else
        k_move_block<W_F64><<<gr, kBlock, 0, s>>>(a);
}

void launch_move_hub_scan(const MoveArgs &a, hipStream_t s) {
    if (a.qcap[BIN_HUB] == 0) return;
    unsigned gr = cap_grid(a.ch_count, 4096);
    if (a.g.wt == W_UNIT)
        k_move_hub_insert<W_UNIT><<<gr, kBlock, 0, s>>>(a);
    else if (a.g.wt == W_F32)
        k_move_hub_insert<W_F32><<<gr, kBlock, 0, s>>>(a);
    else
        k_move_hub_insert<W_F64><<<gr, kBlock, 0, s>>>(a);
}

void launch_move_hub_parts(const MoveArgs &a, hipStream_t s) {
    if (a.qcap[BIN_HUB] == 0) return;
    unsigned gr = cap_grid(a.ch_count, sched_cap(a, 4096));
    if (a.g.wt == W_UNIT)
        k_hub_bucket<W_UNIT><<<gr, kBlock, 0, s>>>(a);
    else if (a.g.wt == W_F32)
        k_hub_bucket<W_F32><<<gr, kBlock, 0, s>>>(a);
    else
        k_hub_bucket<W_F64><<<gr, kBlock, 0, s>>>(a);
}

void launch_move_hub_gather(const MoveArgs &a, hipStream_t s) {
    if (a.qcap[BIN_HUB] == 0) return;
    unsigned gr = cap_grid(a.ch_count, sched_cap(a, 4096));
    if (a.g.wt == W_UNIT)
        k_hub_gather<W_UNIT><<<gr, kBlock, 0, s>>>(a);
    else
        k_hub_gather<W_F64><<<gr, kBlock, 0, s>>>(a);   // staged values are fp64 sums
}

void launch_move_hub_decide(const MoveArgs &a, hipStream_t s) {
    if (a.qcap[BIN_HUB] == 0) return;
    unsigned gr = cap_grid(a.qcap[BIN_HUB], sched_cap(a, 2048));
    if (a.g.wt == W_UNIT)
        k_hub_decide<W_UNIT><<<gr, kBlock, 0, s>>>(a);
    else if (a.g.wt == W_F32)
        k_hub_decide<W_F32><<<gr, kBlock, 0, s>>>(a);
    else
        k_hub_decide<W_F64><<<gr, kBlock, 0, s>>>(a);
}

void launch_move_hub_finish(const MoveArgs &a, hipStream_t s) {
    if (a.qcap[BIN_HUB] == 0) return;
    k_move_hub_part<<<cap_grid(a.ch_count, 4096), kBlock, 0, s>>>(a);
    k_move_hub_final<<<cap_grid((a.qcap[BIN_HUB] + 3) / 4, 1024), kBlock, 0, s>>>(a);
}

void launch_move_apply(const MoveArgs &a, int64_t cap, hipStream_t s) {
    if (cap == 0) return;
    int nq = (int)cap_grid((cap + kBlock - 1) / kBlock, sched_cap(a, 2048));
    int nh = a.qcap[BIN_HUB] ? (int)cap_grid(a.ch_count, sched_cap(a, 2048)) : 0;
    k_move_apply<<<nq + nh, kBlock, 0, s>>>(a, nq);
}

}  // namespace gsp
