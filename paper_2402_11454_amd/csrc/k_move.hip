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

constexpr int kIntMax = 0x7fffffff;

struct Acc {          // per-thread counters, reduced per block at the end
    double gain = 0.0;
    unsigned long long moved = 0, verts = 0, scanned = 0, keys = 0;
};

__device__ void flush_acc(const Acc &acc, IterCounters *ctr, int cls) {
    __shared__ double sg[kBlock / kWave];
    __shared__ unsigned long long sm[kBlock / kWave], sv[kBlock / kWave], ss[kBlock / kWave], sk[kBlock / kWave];
    double g = group_sum<kWave>(acc.gain);
    long long m = group_sum_ll<kWave>((long long)acc.moved);
    long long v = group_sum_ll<kWave>((long long)acc.verts);
    long long s = group_sum_ll<kWave>((long long)acc.scanned);
    long long k = group_sum_ll<kWave>((long long)acc.keys);
    int w = threadIdx.x / kWave;
    if (lane_id() == 0) { sg[w] = g; sm[w] = m; sv[w] = v; ss[w] = s; sk[w] = k; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tg = 0.0;
        unsigned long long tm = 0, tv = 0, ts = 0, tk = 0;
        for (int q = 0; q < kBlock / kWave; q++) { tg += sg[q]; tm += sm[q]; tv += sv[q]; ts += ss[q]; tk += sk[q]; }
        if (tg != 0.0) unsafeAtomicAdd(&ctr->gain, tg);
        if (tm) atomicAdd(&ctr->moved, tm);
        if (tv) atomicAdd(&ctr->verts[cls], tv);
        if (ts) atomicAdd(&ctr->scanned[cls], ts);
        if (tk) atomicAdd(&ctr->keys[cls], tk);
    }
}

// Decision from the group's best candidate; identical on every lane.
__device__ __forceinline__ bool decide(const MoveArgs &a, int i, int d, double ki, double kid, double bg, int bc,
                                       double *gain) {
    if (bc == kIntMax) return false;
    double gstay = a.M2 * kid - ki * (a.sig[d] - ki);
    if (!(bg > gstay)) return false;
    if (a.csize[d] == 1 && a.csize[bc] == 1 && bc > d) return false;
    *gain = bg - gstay;
    return true;
}

// Reads one table slot, resets it and folds it into (bg, bc, kid).
__device__ __forceinline__ void take_slot(const MoveArgs &a, int *keys, double *vals, int64_t s, int d, double ki,
                                          double &bg, int &bc, double &kid, unsigned long long &nkeys) {
    int key = keys[s];
    if (key == kEmpty) return;
    double v = vals[s];
    keys[s] = kEmpty;
    vals[s] = 0.0;
    nkeys++;
    if (key == d) {
        kid = v;
    } else {
        double g = a.M2 * v - ki * a.sig[key];
        if (better(g, key, bg, bc)) {
            bg = g;
            bc = key;
        }
    }
}

// ---------------------------------------------------------------- compact

__global__ void __launch_bounds__(kBlock) k_move_compact(MoveArgs a, const int32_t *bl) {
    int64_t pre[kNumBins + 1];
    pre[0] = 0;
#pragma unroll
    for (int b = 0; b < kNumBins; b++) pre[b + 1] = pre[b] + a.qcap[b];
    int64_t total = pre[kNumBins];
    int *qcnt = a.ctr->qcnt[a.round];
    for (int64_t t0 = blockIdx.x * (int64_t)kBlock; t0 < total; t0 += (int64_t)gridDim.x * kBlock) {
        int64_t t = t0 + threadIdx.x;
        int b = -1, i = -1;
        bool act = false;
        if (t < total) {
            b = 0;
            while (t >= pre[b + 1]) b++;
            i = bl[a.qbase[b] + (t - pre[b])];
            act = a.flag[i] != 0;
            if (act) {
                a.flag[i] = 0;
                if (b == BIN_HUB) a.hub_act[i] = 1;
            }
        }
        unsigned long long pending = __ballot(act);
        while (pending) {
            int leader = __ffsll((long long)pending) - 1;
            int lb = __shfl(b, leader);
            bool mine = act && b == lb;
            int slot = wave_append(mine, &qcnt[lb]);
            if (mine) a.queue[a.qbase[lb] + slot] = i;
            pending &= ~__ballot(mine);
        }
    }
}

// ---------------------------------------------------------------- small

template <int G, int WT>
__device__ void small_unit(const MoveArgs &a, int bin, int64_t unit, int cnt, int *tkeys, double *tvals, Acc &acc) {
    constexpr int kSlots = 2 * G;
    const int grp = threadIdx.x / G, gl = threadIdx.x % G;
    const int64_t qi = unit * (kBlock / G) + grp;
    const bool valid = qi < cnt;
    int *keys = tkeys + grp * kSlots;
    double *vals = tvals + grp * kSlots;
    int i = -1, di = 0, d = -1, j = -1;
    double ki = 0.0;
    if (valid) {
        i = a.queue[a.qbase[bin] + qi];
        di = a.g.deg[i];
        d = a.cm[i];
        ki = a.K[i];
        if (gl < di) {
            int64_t e = a.g.off[i] + gl;
            j = load_col(a.g.col, e);
            double w = edge_weight<WT>(a.g.w, e);
            if (j != i) lds_table_add(keys, vals, kSlots - 1, a.cm[j], w);
        }
    }
    __syncthreads();
    double bg = -INFINITY, kid = 0.0;
    int bc = kIntMax;
    if (valid) {
        take_slot(a, keys, vals, gl, d, ki, bg, bc, kid, acc.keys);
        take_slot(a, keys, vals, gl + G, d, ki, bg, bc, kid, acc.keys);
    }
    group_argmax<G>(bg, bc);
    kid = group_sum<G>(kid);
    double gain = 0.0;
    bool mv = valid && decide(a, i, d, ki, kid, bg, bc, &gain);
    if (mv && j >= 0 && j != i) a.flag[j] = 1;
    bool lead = valid && gl == 0;
    if (lead) {
        acc.verts++;
        acc.scanned += (unsigned long long)di;
        if (mv) {
            a.dec[i] = bc;
            acc.gain += gain;
            acc.moved++;
        }
        if (a.gain_out) a.gain_out[i] = mv ? gain : 0.0;
    }
    int slot = wave_append(lead && mv, &a.ctr->nmov[a.round]);
    if (slot >= 0) a.movers[slot] = i;
    __syncthreads();
}

template <int WT>
__global__ void __launch_bounds__(kBlock) k_move_small(MoveArgs a) {
    __shared__ int tkeys[2 * kBlock];
    __shared__ double tvals[2 * kBlock];
    for (int k = threadIdx.x; k < 2 * kBlock; k += kBlock) {
        tkeys[k] = kEmpty;
        tvals[k] = 0.0;
    }
    __syncthreads();
    int cnt[kNumSmallBins];
    int64_t pre[kNumSmallBins + 1];
    pre[0] = 0;
#pragma unroll
    for (int b = 0; b < kNumSmallBins; b++) {
        cnt[b] = a.ctr->qcnt[a.round][b];
        int vpb = kBlock / (4 << b);
        pre[b + 1] = pre[b] + (cnt[b] + vpb - 1) / vpb;
    }
    Acc acc;
    for (int64_t u = blockIdx.x; u < pre[kNumSmallBins]; u += gridDim.x) {
        int b = 0;
        while (u >= pre[b + 1]) b++;
        int64_t uu = u - pre[b];
        switch (b) {
            case 0: small_unit<4, WT>(a, 0, uu, cnt[0], tkeys, tvals, acc); break;
            case 1: small_unit<8, WT>(a, 1, uu, cnt[1], tkeys, tvals, acc); break;
            case 2: small_unit<16, WT>(a, 2, uu, cnt[2], tkeys, tvals, acc); break;
            case 3: small_unit<32, WT>(a, 3, uu, cnt[3], tkeys, tvals, acc); break;
            default: small_unit<64, WT>(a, 4, uu, cnt[4], tkeys, tvals, acc); break;
        }
    }
    flush_acc(acc, a.ctr, 0);
}

// ---------------------------------------------------------------- large

// Block-wide argmax / sum through LDS; every thread gets the result.
__device__ void block_argmax_sum(double &bg, int &bc, double &x) {
    __shared__ double sg[kBlock / kWave], sx[kBlock / kWave];
    __shared__ int sc[kBlock / kWave];
    group_argmax<kWave>(bg, bc);
    x = group_sum<kWave>(x);
    int w = threadIdx.x / kWave;
    if (lane_id() == 0) { sg[w] = bg; sc[w] = bc; sx[w] = x; }
    __syncthreads();
    bg = sg[0];
    bc = sc[0];
    x = sx[0];
#pragma unroll
    for (int q = 1; q < kBlock / kWave; q++) {
        if (better(sg[q], sc[q], bg, bc)) { bg = sg[q]; bc = sc[q]; }
        x += sx[q];
    }
    __syncthreads();
}

template <int WT>
__device__ void wave_unit(const MoveArgs &a, int64_t unit, int cnt, int *tkeys, double *tvals, Acc &acc) {
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int64_t qi = unit * (kBlock / kWave) + w;
    const bool valid = qi < cnt;
    int *keys = tkeys + w * kWaveTable;
    double *vals = tvals + w * kWaveTable;
    int i = -1, di = 0, d = -1;
    int64_t beg = 0;
    double ki = 0.0;
    if (valid) {
        i = a.queue[a.qbase[BIN_WAVE] + qi];
        di = a.g.deg[i];
        beg = a.g.off[i];
        d = a.cm[i];
        ki = a.K[i];
        for (int e = lane; e < di; e += kWave) {
            int j = load_col(a.g.col, beg + e);
            double wt = edge_weight<WT>(a.g.w, beg + e);
            if (j != i) lds_table_add(keys, vals, kWaveTable - 1, a.cm[j], wt);
        }
    }
    __syncthreads();
    double bg = -INFINITY, kid = 0.0;
    int bc = kIntMax;
    if (valid)
        for (int s = lane; s < kWaveTable; s += kWave) take_slot(a, keys, vals, s, d, ki, bg, bc, kid, acc.keys);
    group_argmax<kWave>(bg, bc);
    kid = group_sum<kWave>(kid);
    double gain = 0.0;
    bool mv = valid && decide(a, i, d, ki, kid, bg, bc, &gain);
    if (mv)
        for (int e = lane; e < di; e += kWave) {
            int j = load_col(a.g.col, beg + e);
            if (j != i) a.flag[j] = 1;
        }
    bool lead = valid && lane == 0;
    if (lead) {
        acc.verts++;
        acc.scanned += (unsigned long long)di;
        if (mv) {
            a.dec[i] = bc;
            acc.gain += gain;
            acc.moved++;
        }
        if (a.gain_out) a.gain_out[i] = mv ? gain : 0.0;
    }
    int slot = wave_append(lead && mv, &a.ctr->nmov[a.round]);
    if (slot >= 0) a.movers[slot] = i;
    __syncthreads();
}

template <int WT>
__device__ void block_unit(const MoveArgs &a, int64_t qi, int *keys, double *vals, Acc &acc) {
    const int tid = threadIdx.x;
    int i = a.queue[a.qbase[BIN_BLOCK] + qi];
    int di = a.g.deg[i];
    int64_t beg = a.g.off[i];
    int d = a.cm[i];
    double ki = a.K[i];
    for (int e = tid; e < di; e += kBlock) {
        int j = load_col(a.g.col, beg + e);
        double wt = edge_weight<WT>(a.g.w, beg + e);
        if (j != i) lds_table_add(keys, vals, kBlockTable - 1, a.cm[j], wt);
    }
    __syncthreads();
    double bg = -INFINITY, kid = 0.0;
    int bc = kIntMax;
    for (int s = tid; s < kBlockTable; s += kBlock) take_slot(a, keys, vals, s, d, ki, bg, bc, kid, acc.keys);
    block_argmax_sum(bg, bc, kid);
    double gain = 0.0;
    bool mv = decide(a, i, d, ki, kid, bg, bc, &gain);
    if (mv)
        for (int e = tid; e < di; e += kBlock) {
            int j = load_col(a.g.col, beg + e);
            if (j != i) a.flag[j] = 1;
        }
    if (tid == 0) {
        acc.verts++;
        acc.scanned += (unsigned long long)di;
        if (mv) {
            a.dec[i] = bc;
            acc.gain += gain;
            acc.moved++;
            int slot = atomicAdd(&a.ctr->nmov[a.round], 1);
            a.movers[slot] = i;
        }
        if (a.gain_out) a.gain_out[i] = mv ? gain : 0.0;
    }
    __syncthreads();
}

template <int WT>
__global__ void __launch_bounds__(kBlock) k_move_large(MoveArgs a) {
    __shared__ int tkeys[kBlockTable];
    __shared__ double tvals[kBlockTable];
    for (int k = threadIdx.x; k < kBlockTable; k += kBlock) {
        tkeys[k] = kEmpty;
        tvals[k] = 0.0;
    }
    __syncthreads();
    int cw = a.ctr->qcnt[a.round][BIN_WAVE];
    int cb = a.ctr->qcnt[a.round][BIN_BLOCK];
    int64_t uw = (cw + (kBlock / kWave) - 1) / (kBlock / kWave);
    int64_t total = uw + cb;
    Acc acc;
    for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
        if (u < uw)
            wave_unit<WT>(a, u, cw, tkeys, tvals, acc);
        else
            block_unit<WT>(a, u - uw, tkeys, tvals, acc);
    }
    flush_acc(acc, a.ctr, 1);
}

// ---------------------------------------------------------------- hubs

template <int WT>
__global__ void __launch_bounds__(kBlock) k_move_hub_insert(MoveArgs a) {
    Acc acc;
    for (int64_t k = a.ch_first + blockIdx.x; k < a.ch_first + a.ch_count; k += gridDim.x) {
        int i = a.ch_vert[k];
        if (!a.hub_act[i]) continue;
        int64_t beg = a.ch_beg[k];
        int64_t end = a.g.off[i] + a.g.deg[i];
        if (end > beg + kHubChunk) end = beg + kHubChunk;
        int64_t tb = a.hub_off[i];
        uint64_t mask = hub_table_size(a.g.deg[i]) - 1;
        for (int64_t e = beg + threadIdx.x; e < end; e += kBlock) {
            int j = load_col(a.g.col, e);
            double wt = edge_weight<WT>(a.g.w, e);
            if (j != i) gbl_table_add(a.hkeys + tb, a.hvals + tb, mask, a.cm[j], wt);
        }
        if (threadIdx.x == 0) acc.scanned += (unsigned long long)(end - beg);
    }
    flush_acc(acc, a.ctr, 2);
}

__global__ void __launch_bounds__(kBlock) k_move_hub_final(MoveArgs a) {
    int cnt = a.ctr->qcnt[a.round][BIN_HUB];
    Acc acc;
    for (int64_t qi = blockIdx.x; qi < cnt; qi += gridDim.x) {
        int i = a.queue[a.qbase[BIN_HUB] + qi];
        int di = a.g.deg[i];
        int64_t beg = a.g.off[i];
        int d = a.cm[i];
        double ki = a.K[i];
        int64_t tb = a.hub_off[i];
        int64_t T = (int64_t)hub_table_size(di);
        double bg = -INFINITY, kid = 0.0;
        int bc = kIntMax;
        for (int64_t s = threadIdx.x; s < T; s += kBlock)
            take_slot(a, a.hkeys + tb, a.hvals + tb, s, d, ki, bg, bc, kid, acc.keys);
        block_argmax_sum(bg, bc, kid);
        double gain = 0.0;
        bool mv = decide(a, i, d, ki, kid, bg, bc, &gain);
        if (mv)
            for (int64_t e = threadIdx.x; e < di; e += kBlock) {
                int j = load_col(a.g.col, beg + e);
                if (j != i) a.flag[j] = 1;
            }
        if (threadIdx.x == 0) {
            acc.verts++;
            a.hub_act[i] = 0;
            if (mv) {
                a.dec[i] = bc;
                acc.gain += gain;
                acc.moved++;
                int slot = atomicAdd(&a.ctr->nmov[a.round], 1);
                a.movers[slot] = i;
            }
            if (a.gain_out) a.gain_out[i] = mv ? gain : 0.0;
        }
        __syncthreads();
    }
    flush_acc(acc, a.ctr, 2);
}

// ---------------------------------------------------------------- apply

__global__ void __launch_bounds__(kBlock) k_move_apply(MoveArgs a) {
    int n = a.ctr->nmov[a.round];
    int32_t *cm = const_cast<int32_t *>(a.cm);
    double *sig = const_cast<double *>(a.sig);
    int32_t *csize = const_cast<int32_t *>(a.csize);
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock) {
        int i = a.movers[k];
        int c = a.dec[i];
        int d = cm[i];
        double ki = a.K[i];
        cm[i] = c;
        unsafeAtomicAdd(&sig[d], -ki);
        unsafeAtomicAdd(&sig[c], ki);
        atomicSub(&csize[d], 1);
        atomicAdd(&csize[c], 1);
    }
}

__global__ void __launch_bounds__(kBlock) k_community_totals(const double *K, const int32_t *cm, int64_t n,
                                                            double *sig, int32_t *csize) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        int c = cm[i];
        if (K[i] != 0.0) unsafeAtomicAdd(&sig[c], K[i]);
        atomicAdd(&csize[c], 1);
    }
}

inline unsigned cap_grid(int64_t units, int64_t cap) {
    if (units < 1) units = 1;
    return (unsigned)(units < cap ? units : cap);
}

}  // namespace

void launch_community_totals(const double *K, const int32_t *cm, int64_t n, double *sig, int32_t *csize,
                             hipStream_t s) {
    if (n > 0) k_community_totals<<<cap_grid((n + kBlock - 1) / kBlock, 8192), kBlock, 0, s>>>(K, cm, n, sig, csize);
}

void launch_move_compact(const MoveArgs &a, const WorkLists &wl, hipStream_t s) {
    int64_t total = 0;
    for (int b = 0; b < kNumBins; b++) total += a.qcap[b];
    if (total == 0) return;
    k_move_compact<<<cap_grid((total + kBlock - 1) / kBlock, 4096), kBlock, 0, s>>>(a, wl.bl);
}

void launch_move_small(const MoveArgs &a, const WorkLists &wl, hipStream_t s) {
    (void)wl;
    int64_t units = 0;
    for (int b = 0; b < kNumSmallBins; b++) {
        int vpb = kBlock / (4 << b);
        units += (a.qcap[b] + vpb - 1) / vpb;
    }
    if (units == 0) return;
    unsigned gr = cap_grid(units, 4096);
    if (a.g.wt == W_UNIT)
        k_move_small<W_UNIT><<<gr, kBlock, 0, s>>>(a);
    else if (a.g.wt == W_F32)
        k_move_small<W_F32><<<gr, kBlock, 0, s>>>(a);
    else
        k_move_small<W_F64><<<gr, kBlock, 0, s>>>(a);
}

void launch_move_large(const MoveArgs &a, const WorkLists &wl, hipStream_t s) {
    (void)wl;
    int64_t units = (a.qcap[BIN_WAVE] + 3) / 4 + a.qcap[BIN_BLOCK];
    if (units == 0) return;
    unsigned gr = cap_grid(units, 2048);
    if (a.g.wt == W_UNIT)
        k_move_large<W_UNIT><<<gr, kBlock, 0, s>>>(a);
    else if (a.g.wt == W_F32)
        k_move_large<W_F32><<<gr, kBlock, 0, s>>>(a);
    else
        k_move_large<W_F64><<<gr, kBlock, 0, s>>>(a);
}

void launch_move_hub(const MoveArgs &a, const WorkLists &wl, hipStream_t s) {
    (void)wl;
    if (a.qcap[BIN_HUB] == 0) return;
    unsigned gr = cap_grid(a.ch_count, 2048);
    if (a.g.wt == W_UNIT)
        k_move_hub_insert<W_UNIT><<<gr, kBlock, 0, s>>>(a);
    else if (a.g.wt == W_F32)
        k_move_hub_insert<W_F32><<<gr, kBlock, 0, s>>>(a);
    else
        k_move_hub_insert<W_F64><<<gr, kBlock, 0, s>>>(a);
    k_move_hub_final<<<cap_grid(a.qcap[BIN_HUB], 1024), kBlock, 0, s>>>(a);
}

void launch_move_apply(const MoveArgs &a, int64_t cap, hipStream_t s) {
    if (cap == 0) return;
    k_move_apply<<<cap_grid((cap + kBlock - 1) / kBlock, 2048), kBlock, 0, s>>>(a);
}

}  // namespace gsp
