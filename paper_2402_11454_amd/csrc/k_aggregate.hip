// k_aggregate.hip - the aggregation phase (Algorithm "louvainAggregate").
//
// 1. community sizes and total degrees, exclusive scans -> the community
//    vertices CSR (members) and the upper-bound offsets eoff of the
//    super-vertex rows (a gapped CSR, as in the paper);
// 2. communities are binned by total degree; each one accumulates
//    scanCommunities(self = true) over its members into a table keyed by the
//    neighbour community: a lane group (<= 64 entries), a wavefront (<= 512),
//    a workgroup (<= 2048) -- all in LDS -- or, beyond, a table in global
//    memory filled vertex by vertex;
// 3. each table is emitted as row c of G'' (fp64 weights, order of the
//    table), with deg''[c] and K''[c] = row sum.
// G'' stays gapped ("holey"): row c is [eoff[c], eoff[c] + deg''[c]) of the
// output arrays, the paper's layout; no kernel reads past deg''.
// compact_rows packs it for callers that want a plain CSR.
// Sums are fp64; on integer weights (and fp32 weights whose totals stay
// below 2^30 in units of their spacing) they are exact, so G'' does not
// depend on the order of the atomics.
#include <vector>

#include "gsp_internal.h"

namespace gsp {

namespace {

inline unsigned grid1(int64_t n, int64_t cap = 8192) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// Community sizes and total degrees.  A tile of kCountTile vertices is
// first reduced in an LDS table keyed by community, so a giant community
// costs one global atomic per tile instead of one per member.
constexpr int kCountTile = 4 * kBlock;
constexpr int kCountTable = 2 * kCountTile;

__global__ void __launch_bounds__(kBlock) k_agg_count(Level g, const int32_t *cm, int32_t *csz, int64_t *ctot) {
    __shared__ int tk[kCountTable];
    __shared__ int tc[kCountTable];
    __shared__ unsigned long long td[kCountTable];
    for (int s = threadIdx.x; s < kCountTable; s += kBlock) { tk[s] = kEmpty; tc[s] = 0; td[s] = 0; }
    __syncthreads();
    for (int64_t t0 = blockIdx.x * (int64_t)kCountTile; t0 < g.n; t0 += (int64_t)gridDim.x * kCountTile) {
#pragma unroll
        for (int r = 0; r < kCountTile / kBlock; r++) {
            int64_t v = t0 + r * kBlock + threadIdx.x;
            if (v < g.n) {
                int slot = lds_table_slot(tk, kCountTable - 1, cm[v]);
                atomicAdd(&tc[slot], 1);
                int d = g.deg[v];
                if (d) atomicAdd(&td[slot], (unsigned long long)d);
            }
        }
        __syncthreads();
        for (int s = threadIdx.x; s < kCountTable; s += kBlock) {
            int c = tk[s];
            if (c == kEmpty) continue;
            atomicAdd(&csz[c], tc[s]);
            if (td[s]) atomicAdd((unsigned long long *)&ctot[c], td[s]);
            tk[s] = kEmpty;
            tc[s] = 0;
            td[s] = 0;
        }
        __syncthreads();
    }
}

// Community vertices CSR: members with entries fill each community's range
// from the front, members without entries from the back, so the first
// members of a community all have at least one entry.  Each tile reserves
// its slots with one atomic per community and side.
__global__ void __launch_bounds__(kBlock) k_agg_fill(Level g, const int32_t *cm, const int64_t *coff,
                                                    int32_t *front, int32_t *back, int32_t *members) {
    __shared__ int tk[kCountTable];
    __shared__ int nf[kCountTable], nb[kCountTable];
    __shared__ int bf[kCountTable], bb[kCountTable];
    for (int s = threadIdx.x; s < kCountTable; s += kBlock) { tk[s] = kEmpty; nf[s] = 0; nb[s] = 0; }
    __syncthreads();
    constexpr int R = kCountTile / kBlock;
    for (int64_t t0 = blockIdx.x * (int64_t)kCountTile; t0 < g.n; t0 += (int64_t)gridDim.x * kCountTile) {
        int slot[R], rank[R], comm[R];
        bool has[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            int64_t v = t0 + r * kBlock + threadIdx.x;
            slot[r] = -1;
            if (v < g.n) {
                comm[r] = cm[v];
                has[r] = g.deg[v] > 0;
                slot[r] = lds_table_slot(tk, kCountTable - 1, comm[r]);
                rank[r] = atomicAdd(has[r] ? &nf[slot[r]] : &nb[slot[r]], 1);
            }
        }
        __syncthreads();
        for (int s = threadIdx.x; s < kCountTable; s += kBlock) {
            int c = tk[s];
            if (c == kEmpty) continue;
            if (nf[s]) bf[s] = atomicAdd(&front[c], nf[s]);
            if (nb[s]) bb[s] = atomicAdd(&back[c], nb[s]);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; r++) {
            if (slot[r] < 0) continue;
            int64_t v = t0 + r * kBlock + threadIdx.x;
            int c = comm[r];
            if (has[r])
                members[coff[c] + bf[slot[r]] + rank[r]] = (int32_t)v;
            else
                members[coff[c + 1] - 1 - (bb[slot[r]] + rank[r])] = (int32_t)v;
        }
        __syncthreads();
        for (int s = threadIdx.x; s < kCountTable; s += kBlock) { tk[s] = kEmpty; nf[s] = 0; nb[s] = 0; }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kBlock) k_member_degrees(const int32_t *members, int64_t n, const int32_t *deg,
                                                          int32_t *mdeg) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock)
        mdeg[k] = deg[members[k]];
}

__global__ void __launch_bounds__(kBlock) k_agg_cdeg(const int64_t *eoff, int64_t n2, int32_t *cdeg) {
    for (int64_t c = blockIdx.x * (int64_t)kBlock + threadIdx.x; c < n2; c += (int64_t)gridDim.x * kBlock) {
        int64_t t = eoff[c + 1] - eoff[c];
        cdeg[c] = (int32_t)(t < 0x7fffffff ? t : 0x7fffffff);
    }
}

__device__ __forceinline__ uint64_t comm_table_size(int64_t ctot, int64_t n2) {
    return hub_table_size(ctot < n2 ? ctot : n2);
}

__global__ void __launch_bounds__(kBlock) k_agg_hub_sizes(const int32_t *bl, int64_t hb, int64_t H,
                                                         const int64_t *eoff, int64_t n2, int64_t *tsize) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < H; k += (int64_t)gridDim.x * kBlock) {
        int c = bl[hb + k];
        tsize[k] = (int64_t)comm_table_size(eoff[c + 1] - eoff[c], n2);
    }
}

__global__ void __launch_bounds__(kBlock) k_agg_hub_off(const int32_t *bl, int64_t hb, int64_t H,
                                                       const int64_t *toff, int64_t *ctab) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < H; k += (int64_t)gridDim.x * kBlock)
        ctab[bl[hb + k]] = toff[k];
}

constexpr int kAggChunk = 1024;          // entries per workgroup for hub communities
constexpr int kAggChunkTable = 2 * kAggChunk;

__global__ void __launch_bounds__(kBlock) k_agg_hub_nchunks(const int32_t *bl, int64_t hb, int64_t H,
                                                           const int64_t *eoff, int64_t *nch) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < H; k += (int64_t)gridDim.x * kBlock) {
        int c = bl[hb + k];
        nch[k] = (eoff[c + 1] - eoff[c] + kAggChunk - 1) / kAggChunk;
    }
}

// Fills a list of pieces: hub h (h < H, id bl[hb + h]) owns pieces
// [poff[h], poff[h+1]); piece k of it starts at base(h) + (k - poff[h]) *
// step.  One thread per piece (binary search for its hub).
__global__ void __launch_bounds__(kBlock) k_fill_pieces(const int32_t *bl, int64_t hb, int64_t H,
                                                       const int64_t *poff, const int64_t *base_of, int64_t step,
                                                       int32_t *pid, int64_t *pbeg) {
    int64_t total = poff[H];
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < total; k += (int64_t)gridDim.x * kBlock) {
        int64_t lo = 0, hi = H - 1;
        while (lo < hi) {
            int64_t mid = (lo + hi + 1) / 2;
            if (poff[mid] <= k) lo = mid; else hi = mid - 1;
        }
        int c = bl[hb + lo];
        pid[k] = c;
        pbeg[k] = (base_of ? base_of[c] : 0) + (k - poff[lo]) * step;
    }
}

constexpr int kEmitSeg = 4096;          // table slots per workgroup when emitting hub rows

__global__ void __launch_bounds__(kBlock) k_agg_hub_nsegs(const int32_t *bl, int64_t hb, int64_t H,
                                                         const int64_t *eoff, int64_t n2, int64_t *nseg) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < H; k += (int64_t)gridDim.x * kBlock) {
        int c = bl[hb + k];
        int64_t T = (int64_t)comm_table_size(eoff[c + 1] - eoff[c], n2);
        nseg[k] = (T + kEmitSeg - 1) / kEmitSeg;
    }
}

struct AggArgs {
    Level g;
    const int32_t *cm;
    const int64_t *coff;     // community c's members: members[coff[c] .. coff[c+1])
    const int32_t *members;
    const int64_t *eoff;     // gapped row of c: [eoff[c], eoff[c+1])
    int32_t *gap_col;
    double *gap_w;
    int32_t *deg2;
    double *K2;
    const int32_t *cbl;      // community work lists
    int64_t cbeg[kNumBins], cn[kNumBins];
    int64_t n2;
    const int64_t *ctab;     // hub community table offsets (-1: not a hub)
    const int64_t *mpre;     // exclusive scan of member degrees (flattened entry index)
    const int64_t *ck0;      // per hub chunk: the member position holding its first entry
    int *hkeys;
    double *hvals;
    // hub partitions (null stage_col: every hub community through its global table)
    int32_t *stage_col;      // staged pairs at flattened entry positions
    double *stage_w;
    uint32_t *words;         // per chunk and partition: start << 16 | count
    const int64_t *woff;     // community c's words begin at words + woff[c]
    uint8_t *spill;          // community c has a partition in its global table
};

template <int W>
__device__ __forceinline__ int group_incl_scan(int x, int gl) {
#pragma unroll
    for (int off = 1; off < W; off <<= 1) {
        int y = __shfl_up(x, off, W);
        if (gl >= off) x += y;
    }
    return x;
}

// Smallest k with incl[k] > x over the W lanes of a group (incl
// non-decreasing); uniform across the group.
template <int W>
__device__ __forceinline__ int group_search(int incl, int x) {
    int k = 0;
#pragma unroll
    for (int step = W / 2; step > 0; step >>= 1) {
        int v = __shfl(incl, k + step - 1, W);
        if (v <= x) k += step;
    }
    return k;
}

// Inserts the entries of a chunk of at most W members (positions
// [m0, m1) of c's member list) into the table; uniform across the group.
// Adds w to `key` in an LDS table of T slots (any T): first slot by the
// multiply-shift reduction of the hash, linear probing with wrap-around.
__device__ __forceinline__ void lds_table_add_mod(int *keys, double *vals, uint32_t T, int key, double w) {
    uint32_t s = (uint32_t)(((uint64_t)key_hash(key) * T) >> 32);
    while (true) {
        const int prev = atomicCAS(&keys[s], kEmpty, key);
        if (prev == kEmpty || prev == key) {
            atomicAdd(&vals[s], w);
            return;
        }
        s = s + 1 == T ? 0 : s + 1;
    }
}

// GLOBAL: a global table of mask + 1 slots; else an LDS table of mask + 1
// slots, or (MOD) of `mask` slots.
template <int W, int WT, bool GLOBAL, bool MOD = false>
__device__ void insert_member_chunk(const AggArgs &a, int64_t m0, int64_t m1, int gl, int *keys, double *vals,
                                    uint64_t mask) {
    int dm = 0;
    int64_t bm = 0;
    if (m0 + gl < m1) {
        int v = a.members[m0 + gl];
        dm = a.g.deg[v];
        bm = a.g.off[v];
    }
    int incl = group_incl_scan<W>(dm, gl);
    int total = __shfl(incl, W - 1, W);
    // R rounds of W entries at a time: positions first, then their columns,
    // then the memberships, so the loads of a batch are in flight together
    constexpr int R = 4;
    for (int x0 = 0; x0 < total; x0 += W * R) {
        int64_t e[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            int x = x0 + r * W + gl;
            int k = group_search<W>(incl, x);
            int ik = __shfl(incl, k, W), dk = __shfl(dm, k, W);
            int64_t bk = __shfl(bm, k, W);
            e[r] = x < total ? bk + (x - (ik - dk)) : -1;
        }
        int32_t j[R];
        double w[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            j[r] = e[r] >= 0 ? load_col(a.g.col, e[r]) : 0;
            w[r] = e[r] >= 0 ? edge_weight<WT>(a.g.w, e[r]) : 0.0;
        }
        int c[R];
#pragma unroll
        for (int r = 0; r < R; r++) c[r] = e[r] >= 0 ? a.cm[j[r]] : 0;
#pragma unroll
        for (int r = 0; r < R; r++) {
            if (e[r] < 0) continue;
            if constexpr (GLOBAL)
                gbl_table_add(keys, vals, mask, c[r], w[r]);
            else if constexpr (MOD)
                lds_table_add_mod(keys, vals, (uint32_t)mask, c[r], w[r]);
            else
                lds_table_add(keys, vals, (uint32_t)mask, c[r], w[r]);
        }
    }
}

template <int W>
__device__ __forceinline__ int group_excl_scan(int x, int gl, int *total) {
    int inc = group_incl_scan<W>(x, gl);
    *total = __shfl(inc, W - 1, W);
    return inc - x;
}

// ---------------------------------------------------------------- small

template <int G, int WT>
__device__ void agg_small_unit(const AggArgs &a, int bin, int64_t unit, int *tkeys, double *tvals) {
    constexpr int kSlots = 2 * G;
    const int grp = threadIdx.x / G, gl = threadIdx.x % G;
    const int64_t qi = unit * (kBlock / G) + grp;
    const bool valid = qi < a.cn[bin];
    int *keys = tkeys + grp * kSlots;
    double *vals = tvals + grp * kSlots;
    int c = valid ? a.cbl[a.cbeg[bin] + qi] : 0;
    // members of degree 0 contribute nothing, so a community may have more
    // members than entries: take them G at a time
    if (valid)
        for (int64_t m0 = a.coff[c]; m0 < a.coff[c + 1]; m0 += G) {
            int64_t m1 = m0 + G < a.coff[c + 1] ? m0 + G : a.coff[c + 1];
            insert_member_chunk<G, WT, false>(a, m0, m1, gl, keys, vals, kSlots - 1);
        }
    __syncthreads();
    if (valid) {
        int k0 = keys[gl], k1 = keys[gl + G];
        double v0 = vals[gl], v1 = vals[gl + G];
        keys[gl] = kEmpty; keys[gl + G] = kEmpty;
        vals[gl] = 0.0; vals[gl + G] = 0.0;
        int cntl = (k0 != kEmpty) + (k1 != kEmpty);
        int tot;
        int pos = group_excl_scan<G>(cntl, gl, &tot);
        int64_t base = a.eoff[c];
        double s = 0.0;
        if (k0 != kEmpty) { a.gap_col[base + pos] = k0; a.gap_w[base + pos] = v0; pos++; s += v0; }
        if (k1 != kEmpty) { a.gap_col[base + pos] = k1; a.gap_w[base + pos] = v1; s += v1; }
        s = group_sum<G>(s);
        if (gl == 0) { a.deg2[c] = tot; a.K2[c] = s; }
    }
    __syncthreads();
}

template <int WT>
__global__ void __launch_bounds__(kBlock) k_agg_small(AggArgs a) {
    __shared__ int tkeys[2 * kBlock];
    __shared__ double tvals[2 * kBlock];
    for (int k = threadIdx.x; k < 2 * kBlock; k += kBlock) { tkeys[k] = kEmpty; tvals[k] = 0.0; }
    __syncthreads();
    int64_t pre[kNumSmallBins + 1];
    pre[0] = 0;
#pragma unroll
    for (int b = 0; b < kNumSmallBins; b++) {
        int vpb = kBlock / (4 << b);
        pre[b + 1] = pre[b] + (a.cn[b] + vpb - 1) / vpb;
    }
    for (int64_t u = blockIdx.x; u < pre[kNumSmallBins]; u += gridDim.x) {
        int b = 0;
        while (u >= pre[b + 1]) b++;
        int64_t uu = u - pre[b];
        switch (b) {
            case 0: agg_small_unit<4, WT>(a, 0, uu, tkeys, tvals); break;
            case 1: agg_small_unit<8, WT>(a, 1, uu, tkeys, tvals); break;
            case 2: agg_small_unit<16, WT>(a, 2, uu, tkeys, tvals); break;
            case 3: agg_small_unit<32, WT>(a, 3, uu, tkeys, tvals); break;
            default: agg_small_unit<64, WT>(a, 4, uu, tkeys, tvals); break;
        }
    }
}

// ---------------------------------------------------------------- large

// Emits a table of T slots (in LDS, or global when GLOBAL) with `nthreads`
// lanes of a wave (nthreads = 64) or the whole block (256).
template <int NT>
__device__ void emit_table(const AggArgs &a, int c, int *keys, double *vals, int64_t T) {
    __shared__ int s_tot[kBlock / kWave];
    __shared__ double s_sum[kBlock / kWave];
    const int t = (NT == kWave) ? lane_id() : (int)threadIdx.x;
    int64_t base = a.eoff[c];
    int64_t written = 0;
    double sum = 0.0;
    for (int64_t s0 = 0; s0 < T; s0 += NT) {
        int64_t s = s0 + t;
        int key = kEmpty;
        double v = 0.0;
        if (s < T) {
            key = keys[s];
            if (key != kEmpty) {
                v = vals[s];
                keys[s] = kEmpty;
                vals[s] = 0.0;
            }
        }
        int f = key != kEmpty;
        int wt;
        int pos = group_excl_scan<kWave>(f, lane_id(), &wt);
        int64_t wbase = written;
        if constexpr (NT == kBlock) {
            int w = threadIdx.x / kWave;
            if (lane_id() == 0) s_tot[w] = wt;
            __syncthreads();
            int before = 0, all = 0;
            for (int q = 0; q < kBlock / kWave; q++) {
                if (q < w) before += s_tot[q];
                all += s_tot[q];
            }
            __syncthreads();
            wbase += before;
            written += all;
        } else {
            written += wt;
        }
        if (f) {
            a.gap_col[base + wbase + pos] = key;
            a.gap_w[base + wbase + pos] = v;
            sum += v;
        }
    }
    sum = group_sum<kWave>(sum);
    if constexpr (NT == kBlock) {
        if (lane_id() == 0) s_sum[threadIdx.x / kWave] = sum;
        __syncthreads();
        if (threadIdx.x == 0) {
            double tsum = 0.0;
            for (int q = 0; q < kBlock / kWave; q++) tsum += s_sum[q];
            a.deg2[c] = (int32_t)written;
            a.K2[c] = tsum;
        }
        __syncthreads();
    } else {
        if (lane_id() == 0) {
            a.deg2[c] = (int32_t)written;
            a.K2[c] = sum;
        }
    }
}

// Communities of 65..512 entries (four per workgroup, a wavefront and a
// table of up to 768 slots each) and of 513..2048 entries (a workgroup and
// a table of up to 3072 slots): 36 KB, so that four workgroups share a CU's
// LDS (half-full tables of 48 KB let three).  A community of at most a third
// of the capacity in entries keeps a half-full power-of-two table (and the
// emit scans only that); larger ones fill theirs at most two thirds.
constexpr int kAggWaveSlots = 3 * kWaveMaxDeg / 2;
constexpr int kAggBlockSlots = 3 * kBlockMaxDeg / 2;
static_assert(kAggBlockSlots == (kBlock / kWave) * kAggWaveSlots, "the wave tables tile the workgroup table");
__device__ __forceinline__ int agg_slots(int64_t entries, int cap) {
    return entries <= cap / 3 ? (int)hub_table_size(entries) : cap;
}

template <int WT>
__global__ void __launch_bounds__(kBlock, 4) k_agg_large(AggArgs a) {
    __shared__ int tkeys[kAggBlockSlots];
    __shared__ double tvals[kAggBlockSlots];
    for (int k = threadIdx.x; k < kAggBlockSlots; k += kBlock) { tkeys[k] = kEmpty; tvals[k] = 0.0; }
    __syncthreads();
    int64_t uw = (a.cn[BIN_WAVE] + 3) / 4;
    int64_t total = uw + a.cn[BIN_BLOCK];
    const int w = threadIdx.x / kWave, lane = lane_id();
    for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
        if (u < uw) {
            int64_t qi = u * 4 + w;
            bool valid = qi < a.cn[BIN_WAVE];
            int *keys = tkeys + w * kAggWaveSlots;
            double *vals = tvals + w * kAggWaveSlots;
            int c = valid ? a.cbl[a.cbeg[BIN_WAVE] + qi] : 0;
            const int T = valid ? agg_slots(a.eoff[c + 1] - a.eoff[c], kAggWaveSlots) : 0;
            if (valid)
                for (int64_t m0 = a.coff[c]; m0 < a.coff[c + 1]; m0 += kWave) {
                    int64_t m1 = m0 + kWave < a.coff[c + 1] ? m0 + kWave : a.coff[c + 1];
                    insert_member_chunk<kWave, WT, false, true>(a, m0, m1, lane, keys, vals, T);
                }
            __syncthreads();
            if (valid) emit_table<kWave>(a, c, keys, vals, T);
            __syncthreads();
        } else {
            int c = a.cbl[a.cbeg[BIN_BLOCK] + (u - uw)];
            const int T = agg_slots(a.eoff[c + 1] - a.eoff[c], kAggBlockSlots);
            // the four waves take member chunks in turn
            for (int64_t m0 = a.coff[c] + (int64_t)w * kWave; m0 < a.coff[c + 1]; m0 += kBlock) {
                int64_t m1 = m0 + kWave < a.coff[c + 1] ? m0 + kWave : a.coff[c + 1];
                insert_member_chunk<kWave, WT, false, true>(a, m0, m1, lane, tkeys, tvals, T);
            }
            __syncthreads();
            emit_table<kBlock>(a, c, tkeys, tvals, T);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------- hubs

// First member of every hub chunk: the last position k among c's members
// with mpre[k] <= X0 (one thread per chunk).
__global__ void __launch_bounds__(kBlock) k_agg_chunk_k0(const int32_t *cch_comm, const int64_t *cch_beg,
                                                        int64_t nchunks, const int64_t *coff, const int64_t *mpre,
                                                        int64_t *k0) {
    for (int64_t ch = blockIdx.x * (int64_t)kBlock + threadIdx.x; ch < nchunks; ch += (int64_t)gridDim.x * kBlock) {
        int c = cch_comm[ch];
        int64_t X0 = cch_beg[ch];
        int64_t lo = coff[c], hi = coff[c + 1] - 1;
        while (lo < hi) {
            int64_t mid = (lo + hi + 1) / 2;
            if (mpre[mid] <= X0) lo = mid; else hi = mid - 1;
        }
        k0[ch] = lo;
    }
}

// Reduces hub chunk ch (entries [X0, X1) of community c's flattened member
// rows) into the LDS table.  The window holds, for the chunk's candidate
// members k0 .. k0 + nm - 1, the offset of each one's first entry relative to
// X0 (win, at least -2^31 + 1 as a row has fewer than 2^31 entries) and its
// row start (moff); win[nm] = X1 - X0.  Ends with a barrier (the window is
// free again).  The candidates end
// at the member holding the next chunk's first entry (or at c's last
// member); members with entries come first, so there are at most kAggChunk.
// Each thread resolves its four entries first and then issues their loads
// together.
template <int WT>
__device__ __forceinline__ void reduce_hub_chunk(const AggArgs &a, const int32_t *cch_comm, int64_t nchunks,
                                                 int64_t ch, int c, int64_t X0, int64_t X1, int *tkeys,
                                                 double *tvals, int *win, int64_t *moff) {
    const int tid = threadIdx.x;
    const int64_t k0 = a.ck0[ch];
    const int64_t m_end = a.coff[c + 1];
    int64_t k1 = (ch + 1 < nchunks && cch_comm[ch + 1] == c) ? a.ck0[ch + 1] + 1 : m_end;
    if (k1 > k0 + kAggChunk) k1 = k0 + kAggChunk;
    const int nm = (int)(k1 - k0);
    for (int t = tid; t < nm; t += kBlock) {
        win[t] = (int)(a.mpre[k0 + t] - X0);
        moff[t] = a.g.off[a.members[k0 + t]];
    }
    if (tid == 0) win[nm] = (int)(X1 - X0);
    __syncthreads();
    constexpr int R = kAggChunk / kBlock;
    int64_t e[R];
    bool ok[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int x = r * kBlock + tid;
        ok[r] = X0 + x < X1;
        e[r] = 0;
        if (ok[r]) {
            int lo = 0, hi = nm - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (win[mid] <= x) lo = mid; else hi = mid - 1;
            }
            e[r] = moff[lo] + (x - win[lo]);
        }
    }
    int32_t j[R];
    double w[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        j[r] = ok[r] ? load_col(a.g.col, e[r]) : 0;
        w[r] = ok[r] ? edge_weight<WT>(a.g.w, e[r]) : 0.0;
    }
    int cj[R];
#pragma unroll
    for (int r = 0; r < R; r++) cj[r] = ok[r] ? a.cm[j[r]] : 0;
#pragma unroll
    for (int r = 0; r < R; r++)
        if (ok[r]) lds_table_add(tkeys, tvals, kAggChunkTable - 1, cj[r], w[r]);
    __syncthreads();
}

// Hub communities, one workgroup per chunk of kAggChunk entries of the
// community's flattened member rows (entry X of the level's member order is
// entry X - mpre[k] of member k).  The chunk is reduced in LDS, then each
// distinct (neighbour community, partial sum) goes to the community's global
// table.
template <int WT>
__global__ void __launch_bounds__(kBlock) k_agg_hub_chunks(AggArgs a, const int32_t *cch_comm,
                                                          const int64_t *cch_beg, int64_t nchunks) {
    __shared__ int tkeys[kAggChunkTable];
    __shared__ double tvals[kAggChunkTable];
    __shared__ int win[kAggChunk + 1];
    __shared__ int64_t moff[kAggChunk];
    for (int k = threadIdx.x; k < kAggChunkTable; k += kBlock) {
        tkeys[k] = kEmpty;
        tvals[k] = 0.0;
    }
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        int c = cch_comm[ch];
        int64_t X0 = cch_beg[ch];
        int64_t X1 = X0 + kAggChunk < a.eoff[c + 1] ? X0 + kAggChunk : a.eoff[c + 1];
        reduce_hub_chunk<WT>(a, cch_comm, nchunks, ch, c, X0, X1, tkeys, tvals, win, moff);
        int64_t tb = a.ctab[c];
        uint64_t mask = comm_table_size(a.eoff[c + 1] - a.eoff[c], a.n2) - 1;
        for (int s = threadIdx.x; s < kAggChunkTable; s += kBlock) {
            int key = tkeys[s];
            if (key == kEmpty) continue;
            double v = tvals[s];
            tkeys[s] = kEmpty;
            tvals[s] = 0.0;
            gbl_table_add(a.hkeys + tb, a.hvals + tb, mask, key, v);
        }
        __syncthreads();
    }
}

// One workgroup per segment of kEmitSeg slots of a hub community's table:
// the occupied slots become entries of row c of G'' (the block reserves its
// range of the row with one atomic on deg''[c]) and are reset.
__global__ void __launch_bounds__(kBlock) k_agg_hub_emit(AggArgs a, const int32_t *seg_comm, const int64_t *seg_beg,
                                                        int64_t nseg) {
    __shared__ int s_cnt[kBlock / kWave];
    __shared__ double s_sum[kBlock / kWave];
    __shared__ int s_base;
    constexpr int R = kEmitSeg / kBlock;
    for (int64_t q = blockIdx.x; q < nseg; q += gridDim.x) {
        int c = seg_comm[q];
        if (a.stage_col && !a.spill[c]) continue;   // its table is empty
        int64_t tb = a.ctab[c];
        int64_t T = (int64_t)comm_table_size(a.eoff[c + 1] - a.eoff[c], a.n2);
        int64_t s0 = seg_beg[q];
        int key[R];
        double val[R];
        int cnt = 0;
        double sum = 0.0;
#pragma unroll
        for (int r = 0; r < R; r++) {
            int64_t s = s0 + (int64_t)r * kBlock + threadIdx.x;
            key[r] = kEmpty;
            val[r] = 0.0;
            if (s < T) {
                key[r] = a.hkeys[tb + s];
                if (key[r] != kEmpty) {
                    val[r] = a.hvals[tb + s];
                    a.hkeys[tb + s] = kEmpty;
                    a.hvals[tb + s] = 0.0;
                    cnt++;
                    sum += val[r];
                }
            }
        }
        int wt;
        int pos = group_excl_scan<kWave>(cnt, lane_id(), &wt);
        sum = group_sum<kWave>(sum);
        int w = threadIdx.x / kWave;
        if (lane_id() == 0) { s_cnt[w] = wt; s_sum[w] = sum; }
        __syncthreads();
        int before = 0, all = 0;
        double tsum = 0.0;
        for (int x = 0; x < kBlock / kWave; x++) {
            if (x < w) before += s_cnt[x];
            all += s_cnt[x];
            tsum += s_sum[x];
        }
        if (threadIdx.x == 0) {
            s_base = all ? atomicAdd(&a.deg2[c], all) : 0;
            if (tsum != 0.0) unsafeAtomicAdd(&a.K2[c], tsum);
        }
        __syncthreads();
        int64_t dst = a.eoff[c] + s_base + before + pos;
#pragma unroll
        for (int r = 0; r < R; r++)
            if (key[r] != kEmpty) {
                a.gap_col[dst] = key[r];
                a.gap_w[dst] = val[r];
                dst++;
            }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- hub partitions

// Giant communities without global tables.  Community c's distinct
// neighbour communities are split into P_c hash partitions.  Phase 1, per
// chunk of kAggChunk entries: reduce the chunk in LDS and stage its distinct
// (community, weight) pairs, grouped by partition, at the chunk's own
// positions of the staging arrays, with one word per partition (start << 16
// | count).  Phase 2, per partition: merge that partition's pairs from every
// chunk of c in one LDS table and append the table to row c.  Each pair is
// written once and read once.  A partition with more than kAggGatherCap
// distinct communities (its table would not fit) spills its pairs into c's
// global table instead; the emit kernel appends those.

constexpr int kAggPartTarget = 1536;   // distinct communities aimed at per partition
constexpr int kAggMaxParts = 4086;     // partition counts (+1) fit the bucket kernel's 40 KB of LDS
constexpr int kGatherWin = 2048;       // source chunks per window of the gather
// The gather's LDS table: 3072 slots, at most kAggGatherCap distinct
// communities per partition (a third above the target; past it the
// partition spills) plus fewer than kBlock inserts in flight, so at most
// three quarters full: 49 KB of LDS with the window, three workgroups per
// CU where the 4096-slot table allowed two.
constexpr int kAggGatherSlots = 3072;
constexpr int kAggGatherCap = 2048;
static_assert(kAggGatherCap + kBlock < kAggGatherSlots, "the gather's table never fills");

// P_c: one partition per kAggPartTarget possible distinct neighbours (at most
// min(total degree, n2)); at most kAggMaxParts and at most the chunk count.
__device__ __forceinline__ int agg_parts(int64_t tot, int64_t n2) {
    int64_t d = tot < n2 ? tot : n2;
    int64_t p = (d + kAggPartTarget - 1) / kAggPartTarget;
    if (p < 1) p = 1;
    return (int)(p < kAggMaxParts ? p : kAggMaxParts);
}

__global__ void __launch_bounds__(kBlock) k_agg_part_words(const int32_t *bl, int64_t hb, int64_t H,
                                                          const int64_t *eoff, int64_t n2, int64_t *nw) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < H; k += (int64_t)gridDim.x * kBlock) {
        int c = bl[hb + k];
        int64_t tot = eoff[c + 1] - eoff[c];
        nw[k] = (tot + kAggChunk - 1) / kAggChunk * (int64_t)agg_parts(tot, n2);
    }
}

__global__ void __launch_bounds__(kBlock) k_agg_part_scatter(const int32_t *bl, int64_t hb, int64_t H,
                                                            const int64_t *wk, int64_t *woff) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < H; k += (int64_t)gridDim.x * kBlock)
        woff[bl[hb + k]] = wk[k];
}

template <int WT>
__global__ void __launch_bounds__(kBlock) k_agg_part_bucket(AggArgs a, const int32_t *cch_comm,
                                                           const int64_t *cch_beg, int64_t nchunks) {
    __shared__ int tkeys[kAggChunkTable];
    __shared__ double tvals[kAggChunkTable];
    // the window (during the reduce) and the partition counts (after it)
    // share one LDS region: the block stays at 40 KB, four blocks per CU
    __shared__ int64_t wm[kAggMaxParts / 2 + 1];
    static_assert(sizeof(int64_t) * kAggChunk + sizeof(int) * (kAggChunk + 1) <= sizeof(wm), "window");
    int64_t *moff = wm;
    int *win = (int *)(wm + kAggChunk);
    int *pcnt = (int *)wm;
    const int tid = threadIdx.x;
    for (int k = tid; k < kAggChunkTable; k += kBlock) {
        tkeys[k] = kEmpty;
        tvals[k] = 0.0;
    }
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        int c = cch_comm[ch];
        int64_t X0 = cch_beg[ch];
        int64_t X1 = X0 + kAggChunk < a.eoff[c + 1] ? X0 + kAggChunk : a.eoff[c + 1];
        reduce_hub_chunk<WT>(a, cch_comm, nchunks, ch, c, X0, X1, tkeys, tvals, win, moff);
        const int64_t tot = a.eoff[c + 1] - a.eoff[c];
        const int P = agg_parts(tot, a.n2);
        const int64_t s = (X0 - a.eoff[c]) / kAggChunk;
        for (int b = tid; b <= P; b += kBlock) pcnt[b] = 0;
        __syncthreads();
        for (int sl = tid; sl < kAggChunkTable; sl += kBlock) {
            int key = tkeys[sl];
            if (key != kEmpty) atomicAdd(&pcnt[part_of(key, P)], 1);
        }
        __syncthreads();
        block_scan_excl(pcnt, P);
        uint32_t *wd = a.words + a.woff[c] + s * P;
        for (int b = tid; b < P; b += kBlock) wd[b] = ((uint32_t)pcnt[b] << 16) | (uint32_t)(pcnt[b + 1] - pcnt[b]);
        __syncthreads();
        for (int sl = tid; sl < kAggChunkTable; sl += kBlock) {
            int key = tkeys[sl];
            if (key == kEmpty) continue;
            double v = tvals[sl];
            tkeys[sl] = kEmpty;
            tvals[sl] = 0.0;
            int pos = atomicAdd(&pcnt[part_of(key, P)], 1);
            a.stage_col[X0 + pos] = key;
            a.stage_w[X0 + pos] = v;
        }
        __syncthreads();
    }
}

// Loads the words of source chunks [w0, w0 + nw) for partition p into
// (count -> exclusive offsets in pst, starts in srcst); returns the pair total.
__device__ __forceinline__ int load_window(const uint32_t *wd, int P, int p, int64_t w0, int nw, int *pst,
                                           short *srcst) {
    for (int s = threadIdx.x; s < nw; s += kBlock) {
        uint32_t x = wd[(w0 + s) * P + p];
        pst[s] = (int)(x & 0xFFFFu);
        srcst[s] = (short)(x >> 16);
    }
    __syncthreads();
    block_scan_excl(pst, nw);
    return pst[nw];
}

// One workgroup per (hub community, partition): the pieces are the chunk
// list again, chunk s of community c standing for partition s (chunks with
// s >= P_c have nothing to do).
__global__ void __launch_bounds__(kBlock) k_agg_part_gather(AggArgs a, const int32_t *cch_comm,
                                                           const int64_t *cch_beg, int64_t nchunks) {
    __shared__ int tkeys[kAggGatherSlots];
    __shared__ double tvals[kAggGatherSlots];
    __shared__ int pst[kGatherWin + 1];
    __shared__ short srcst[kGatherWin];
    __shared__ int s_cnt[kBlock / kWave];
    __shared__ double s_sum[kBlock / kWave];
    __shared__ int nkeys, ovf, s_base;
    const int tid = threadIdx.x;
    for (int k = tid; k < kAggGatherSlots; k += kBlock) {
        tkeys[k] = kEmpty;
        tvals[k] = 0.0;
    }
    __syncthreads();
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int c = cch_comm[ch];
        const int64_t e0 = a.eoff[c], tot = a.eoff[c + 1] - e0;
        const int P = agg_parts(tot, a.n2);
        const int p = (int)((cch_beg[ch] - e0) / kAggChunk);
        if (p >= P) continue;
        const int64_t nch = (tot + kAggChunk - 1) / kAggChunk;
        const uint32_t *wd = a.words + a.woff[c];
        if (tid == 0) {
            nkeys = 0;
            ovf = 0;
        }
        for (int64_t w0 = 0; w0 < nch; w0 += kGatherWin) {
            int nw = (int)(nch - w0 < kGatherWin ? nch - w0 : kGatherWin);
            int total = load_window(wd, P, p, w0, nw, pst, srcst);
            for (int t = tid; t < total; t += kBlock) {
                if (*(volatile int *)&ovf) break;
                int s = last_le(pst, nw, t);
                int64_t idx = e0 + (w0 + s) * kAggChunk + (int64_t)srcst[s] + (t - pst[s]);
                int key = a.stage_col[idx];
                double v = a.stage_w[idx];
                // at most kAggGatherCap distinct keys (plus fewer than kBlock
                // in flight): the table never fills
                uint32_t sl = (uint32_t)(((uint64_t)key_hash(key) * kAggGatherSlots) >> 32);
                while (true) {
                    int prev = atomicCAS(&tkeys[sl], kEmpty, key);
                    if (prev == kEmpty) {
                        if (atomicAdd(&nkeys, 1) >= kAggGatherCap) ovf = 1;
                        atomicAdd(&tvals[sl], v);
                        break;
                    }
                    if (prev == key) {
                        atomicAdd(&tvals[sl], v);
                        break;
                    }
                    sl = sl + 1 == kAggGatherSlots ? 0 : sl + 1;
                }
            }
            __syncthreads();
            if (ovf) break;
        }
        if (ovf) {
            // spill: the partition's pairs go to c's global table
            for (int q = tid; q < kAggGatherSlots; q += kBlock) {
                tkeys[q] = kEmpty;
                tvals[q] = 0.0;
            }
            if (tid == 0) a.spill[c] = 1;
            const int64_t tb = a.ctab[c];
            const uint64_t mask = comm_table_size(tot, a.n2) - 1;
            for (int64_t w0 = 0; w0 < nch; w0 += kGatherWin) {
                int nw = (int)(nch - w0 < kGatherWin ? nch - w0 : kGatherWin);
                int total = load_window(wd, P, p, w0, nw, pst, srcst);
                for (int t = tid; t < total; t += kBlock) {
                    int s = last_le(pst, nw, t);
                    int64_t idx = e0 + (w0 + s) * kAggChunk + (int64_t)srcst[s] + (t - pst[s]);
                    gbl_table_add(a.hkeys + tb, a.hvals + tb, mask, a.stage_col[idx], a.stage_w[idx]);
                }
                __syncthreads();
            }
            continue;
        }
        // append the table to row c: one reservation on deg''[c] per block
        constexpr int R = kAggGatherSlots / kBlock;
        int key[R];
        double val[R];
        int cnt = 0;
        double sum = 0.0;
#pragma unroll
        for (int r = 0; r < R; r++) {
            int sl = r * kBlock + tid;
            key[r] = tkeys[sl];
            val[r] = 0.0;
            if (key[r] != kEmpty) {
                val[r] = tvals[sl];
                tkeys[sl] = kEmpty;
                tvals[sl] = 0.0;
                cnt++;
                sum += val[r];
            }
        }
        int wt;
        int pos = group_excl_scan<kWave>(cnt, lane_id(), &wt);
        sum = group_sum<kWave>(sum);
        const int w = tid / kWave;
        if (lane_id() == 0) {
            s_cnt[w] = wt;
            s_sum[w] = sum;
        }
        __syncthreads();
        int before = 0, all = 0;
        double tsum = 0.0;
        for (int x = 0; x < kBlock / kWave; x++) {
            if (x < w) before += s_cnt[x];
            all += s_cnt[x];
            tsum += s_sum[x];
        }
        if (tid == 0) {
            s_base = all ? atomicAdd(&a.deg2[c], all) : 0;
            if (tsum != 0.0) unsafeAtomicAdd(&a.K2[c], tsum);
        }
        __syncthreads();
        int64_t dst = e0 + s_base + before + pos;
#pragma unroll
        for (int r = 0; r < R; r++)
            if (key[r] != kEmpty) {
                a.gap_col[dst] = key[r];
                a.gap_w[dst] = val[r];
                dst++;
            }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- compact

__global__ void __launch_bounds__(kBlock) k_agg_copy(const int64_t *eoff, const int64_t *off2, int64_t n2,
                                                    const int32_t *gap_col, const double *gap_w, int32_t *col2,
                                                    double *w2) {
    const int w = threadIdx.x / kWave;
    for (int64_t c = (int64_t)blockIdx.x * 4 + w; c < n2; c += (int64_t)gridDim.x * 4) {
        int64_t src = eoff[c], dst = off2[c], len = off2[c + 1] - off2[c];
        for (int64_t k = lane_id(); k < len; k += kWave) {
            col2[dst + k] = gap_col[src + k];
            w2[dst + k] = gap_w[src + k];
        }
    }
}

}  // namespace

hipError_t aggregate(const Level &g, const WorkLists &wl, const int32_t *cm, int64_t n2, AggOut out,
                     int32_t *stage_col, double *stage_w, Scratch &sc, int64_t *nnz_out, hipStream_t s,
                     bool hub_parts) {
    (void)wl;
    int32_t *csz = sc.i32a, *ccur = sc.i32b, *members = sc.i32c, *cdeg = sc.i32d, *mdeg = sc.i32e;
    int64_t *coff = sc.i64a, *ctot = sc.i64b, *eoff = out.off, *mpre = sc.i64d, *ctab = sc.i64e, *tmp = sc.i64f;
    launch_fill_i32(csz, 0, n2, s);
    launch_fill_i64(ctot, 0, n2, s);
    k_agg_count<<<grid1((g.n + 3) / 4, 4096), kBlock, 0, s>>>(g, cm, csz, ctot);
    scan_exclusive_i32_to_i64(csz, coff, n2, sc.scan_tmp, s);
    scan_exclusive_i64(ctot, eoff, n2, sc.scan_tmp, s);
    launch_fill_i32(ccur, 0, n2, s);
    launch_fill_i32(csz, 0, n2, s);                  // csz becomes the back cursor
    k_agg_fill<<<grid1((g.n + 3) / 4, 4096), kBlock, 0, s>>>(g, cm, coff, ccur, csz, members);
    k_agg_cdeg<<<grid1(n2), kBlock, 0, s>>>(eoff, n2, cdeg);
    WorkLists cwl;
    cwl.bl = sc.bl2;
    hipError_t e = bin_vertices(cdeg, n2, 1, cwl, sc, s);
    if (e != hipSuccess) return e;
    launch_fill_i32(out.deg, 0, n2, s);
    launch_fill_f64(out.K, 0.0, n2, s);

    AggArgs a;
    a.g = g;
    a.cm = cm;
    a.coff = coff;
    a.members = members;
    a.eoff = eoff;
    a.gap_col = out.col;   // rows written in place: the gapped level
    a.gap_w = out.w;
    a.deg2 = out.deg;
    a.K2 = out.K;
    a.cbl = cwl.bl;
    for (int b = 0; b < kNumBins; b++) {
        a.cbeg[b] = cwl.bin_begin(b);
        a.cn[b] = cwl.bin_size(b);
    }
    a.n2 = n2;
    a.ctab = ctab;
    a.mpre = mpre;
    a.ck0 = sc.cch_k0;
    a.stage_col = nullptr;
    a.stage_w = nullptr;
    a.words = nullptr;
    a.woff = nullptr;
    a.spill = nullptr;

    // hub communities: table offsets in the global pool, entry chunks and
    // table segments
    int64_t H = a.cn[BIN_HUB], nchunks = 0, nsegs = 0;
    if (H > 0) {
        unsigned gr = grid1(H, 4096);
        int64_t hb = a.cbeg[BIN_HUB];
        k_agg_hub_sizes<<<gr, kBlock, 0, s>>>(cwl.bl, hb, H, eoff, n2, ctot);    // ctot is free now
        scan_exclusive_i64(ctot, tmp, H, sc.scan_tmp, s);
        k_agg_hub_off<<<gr, kBlock, 0, s>>>(cwl.bl, hb, H, tmp, ctab);
        int64_t host[4] = {0, 0, 0, 0};
        e = hipMemcpyAsync(&host[0], tmp + H, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        k_agg_hub_nchunks<<<gr, kBlock, 0, s>>>(cwl.bl, hb, H, eoff, ctot);
        scan_exclusive_i64(ctot, mpre, H, sc.scan_tmp, s);                        // mpre as temp
        e = hipMemcpyAsync(&host[1], mpre + H, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        k_agg_hub_nsegs<<<gr, kBlock, 0, s>>>(cwl.bl, hb, H, eoff, n2, ctot);
        scan_exclusive_i64(ctot, tmp, H, sc.scan_tmp, s);
        e = hipMemcpyAsync(&host[2], tmp + H, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        if (hub_parts) {   // partition words per hub community (scan by hub index in i64g)
            k_agg_part_words<<<gr, kBlock, 0, s>>>(cwl.bl, hb, H, eoff, n2, ctot);
            scan_exclusive_i64(ctot, sc.i64g, H, sc.scan_tmp, s);
            e = hipMemcpyAsync(&host[3], sc.i64g + H, sizeof(int64_t), hipMemcpyDeviceToHost, s);
            if (e != hipSuccess) return e;
        }
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        nchunks = host[1];
        nsegs = host[2];
        if (nchunks > sc.ch_cap || nsegs > sc.ch_cap) return hipErrorInvalidValue;
        if (nchunks)
            k_fill_pieces<<<grid1(nchunks, 8192), kBlock, 0, s>>>(cwl.bl, hb, H, mpre, eoff, kAggChunk, sc.cch_comm,
                                                                  sc.cch_beg);
        if (nsegs)
            k_fill_pieces<<<grid1(nsegs, 8192), kBlock, 0, s>>>(cwl.bl, hb, H, tmp, nullptr, kEmitSeg, sc.cseg_comm,
                                                                sc.cseg_beg);
        e = ensure_hub_tables(sc, (uint64_t)host[0], s);
        if (e != hipSuccess) return e;
        if (hub_parts) {
            e = ensure_hub_buckets(sc, (uint64_t)host[3], s);
            if (e != hipSuccess) return e;
            k_agg_part_scatter<<<gr, kBlock, 0, s>>>(cwl.bl, hb, H, sc.i64g, ctot);   // ctot: words offset by community
            launch_fill_u8(sc.u8a, 0, n2, s);
            a.stage_col = stage_col;
            a.stage_w = stage_w;
            a.words = sc.hbuck;
            a.woff = ctot;
            a.spill = sc.u8a;
        }
        // flattened entry index of every member
        k_member_degrees<<<grid1(g.n), kBlock, 0, s>>>(members, g.n, g.deg, mdeg);
        scan_exclusive_i32_to_i64(mdeg, mpre, g.n, sc.scan_tmp, s);
        if (nchunks)
            k_agg_chunk_k0<<<grid1(nchunks, 8192), kBlock, 0, s>>>(sc.cch_comm, sc.cch_beg, nchunks, coff, mpre,
                                                                   sc.cch_k0);
    }
    a.hkeys = sc.hkeys;
    a.hvals = sc.hvals;

    int64_t us = 0;
    for (int b = 0; b < kNumSmallBins; b++) {
        int vpb = kBlock / (4 << b);
        us += (a.cn[b] + vpb - 1) / vpb;
    }
    int64_t ul = (a.cn[BIN_WAVE] + 3) / 4 + a.cn[BIN_BLOCK];
    unsigned gs = (unsigned)(us < 8192 ? us : 8192), gl = (unsigned)(ul < 2048 ? ul : 2048);
    unsigned gh = (unsigned)(nchunks < 4096 ? nchunks : 4096);
    const bool parts = a.stage_col != nullptr;
    if (g.wt == W_UNIT) {
        if (us) k_agg_small<W_UNIT><<<gs, kBlock, 0, s>>>(a);
        if (ul) k_agg_large<W_UNIT><<<gl, kBlock, 0, s>>>(a);
        if (nchunks && parts) k_agg_part_bucket<W_UNIT><<<gh, kBlock, 0, s>>>(a, sc.cch_comm, sc.cch_beg, nchunks);
        if (nchunks && !parts) k_agg_hub_chunks<W_UNIT><<<gh, kBlock, 0, s>>>(a, sc.cch_comm, sc.cch_beg, nchunks);
    } else if (g.wt == W_F32) {
        if (us) k_agg_small<W_F32><<<gs, kBlock, 0, s>>>(a);
        if (ul) k_agg_large<W_F32><<<gl, kBlock, 0, s>>>(a);
        if (nchunks && parts) k_agg_part_bucket<W_F32><<<gh, kBlock, 0, s>>>(a, sc.cch_comm, sc.cch_beg, nchunks);
        if (nchunks && !parts) k_agg_hub_chunks<W_F32><<<gh, kBlock, 0, s>>>(a, sc.cch_comm, sc.cch_beg, nchunks);
    } else {
        if (us) k_agg_small<W_F64><<<gs, kBlock, 0, s>>>(a);
        if (ul) k_agg_large<W_F64><<<gl, kBlock, 0, s>>>(a);
        if (nchunks && parts) k_agg_part_bucket<W_F64><<<gh, kBlock, 0, s>>>(a, sc.cch_comm, sc.cch_beg, nchunks);
        if (nchunks && !parts) k_agg_hub_chunks<W_F64><<<gh, kBlock, 0, s>>>(a, sc.cch_comm, sc.cch_beg, nchunks);
    }
    if (nchunks && parts) k_agg_part_gather<<<gh, kBlock, 0, s>>>(a, sc.cch_comm, sc.cch_beg, nchunks);
    if (nsegs) k_agg_hub_emit<<<(unsigned)(nsegs < 8192 ? nsegs : 8192), kBlock, 0, s>>>(a, sc.cseg_comm, sc.cseg_beg, nsegs);
    // entries of G'' (the row lengths' total)
    scan_exclusive_i32_to_i64(out.deg, tmp, n2, sc.scan_tmp, s);
    e = hipMemcpyAsync(nnz_out, tmp + n2, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t compact_rows(const int64_t *eoff, const int32_t *deg, int64_t n2, const int32_t *col, const double *w,
                        int64_t *off_out, int32_t *col_out, double *w_out, Scratch &sc, hipStream_t s) {
    scan_exclusive_i32_to_i64(deg, off_out, n2, sc.scan_tmp, s);
    if (n2 > 0) k_agg_copy<<<grid1(n2 * kWave, 65536), kBlock, 0, s>>>(eoff, off_out, n2, col, w, col_out, w_out);
    return hipGetLastError();
}

}  // namespace gsp
