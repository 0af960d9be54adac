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
//    table), with deg''[c] and K''[c] = row sum;
// 4. deg'' is scanned into compact offsets and the rows are copied.
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
    int *hkeys;
    double *hvals;
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
template <int W, int WT, bool GLOBAL>
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
    for (int x0 = 0; x0 < total; x0 += W) {
        int x = x0 + gl;
        int k = group_search<W>(incl, x);
        int ik = __shfl(incl, k, W), dk = __shfl(dm, k, W);
        int64_t bk = __shfl(bm, k, W);
        if (x < total) {
            int64_t e = bk + (x - (ik - dk));
            int32_t j = load_col(a.g.col, e);
            double w = edge_weight<WT>(a.g.w, e);
            if constexpr (GLOBAL)
                gbl_table_add(keys, vals, mask, a.cm[j], w);
            else
                lds_table_add(keys, vals, (uint32_t)mask, a.cm[j], w);
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

template <int WT>
__global__ void __launch_bounds__(kBlock) k_agg_large(AggArgs a) {
    __shared__ int tkeys[kBlockTable];
    __shared__ double tvals[kBlockTable];
    for (int k = threadIdx.x; k < kBlockTable; k += kBlock) { tkeys[k] = kEmpty; tvals[k] = 0.0; }
    __syncthreads();
    int64_t uw = (a.cn[BIN_WAVE] + 3) / 4;
    int64_t total = uw + a.cn[BIN_BLOCK];
    const int w = threadIdx.x / kWave, lane = lane_id();
    for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
        if (u < uw) {
            int64_t qi = u * 4 + w;
            bool valid = qi < a.cn[BIN_WAVE];
            int *keys = tkeys + w * kWaveTable;
            double *vals = tvals + w * kWaveTable;
            int c = valid ? a.cbl[a.cbeg[BIN_WAVE] + qi] : 0;
            if (valid)
                for (int64_t m0 = a.coff[c]; m0 < a.coff[c + 1]; m0 += kWave) {
                    int64_t m1 = m0 + kWave < a.coff[c + 1] ? m0 + kWave : a.coff[c + 1];
                    insert_member_chunk<kWave, WT, false>(a, m0, m1, lane, keys, vals, kWaveTable - 1);
                }
            __syncthreads();
            if (valid) emit_table<kWave>(a, c, keys, vals, kWaveTable);
            __syncthreads();
        } else {
            int c = a.cbl[a.cbeg[BIN_BLOCK] + (u - uw)];
            // the four waves take member chunks in turn
            for (int64_t m0 = a.coff[c] + (int64_t)w * kWave; m0 < a.coff[c + 1]; m0 += kBlock) {
                int64_t m1 = m0 + kWave < a.coff[c + 1] ? m0 + kWave : a.coff[c + 1];
                insert_member_chunk<kWave, WT, false>(a, m0, m1, lane, tkeys, tvals, kBlockTable - 1);
            }
            __syncthreads();
            emit_table<kBlock>(a, c, tkeys, tvals, kBlockTable);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------- hubs

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
    __shared__ int64_t win[kAggChunk + 1];
    __shared__ int64_t s_k0;
    for (int k = threadIdx.x; k < kAggChunkTable; k += kBlock) {
        tkeys[k] = kEmpty;
        tvals[k] = 0.0;
    }
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        int c = cch_comm[ch];
        int64_t X0 = cch_beg[ch];
        int64_t X1 = X0 + kAggChunk < a.eoff[c + 1] ? X0 + kAggChunk : a.eoff[c + 1];
        int64_t m_end = a.coff[c + 1];
        if (threadIdx.x == 0) {
            // last member position k with mpre[k] <= X0 among c's members
            int64_t lo = a.coff[c], hi = m_end - 1;
            while (lo < hi) {
                int64_t mid = (lo + hi + 1) / 2;
                if (a.mpre[mid] <= X0) lo = mid; else hi = mid - 1;
            }
            s_k0 = lo;
        }
        __syncthreads();
        int64_t k0 = s_k0;
        // members with entries come first, so the chunk's members lie in
        // [k0, k0 + kAggChunk); the window holds their prefix values
        for (int t = threadIdx.x; t <= kAggChunk; t += kBlock)
            win[t] = (k0 + t < m_end) ? a.mpre[k0 + t] : a.eoff[c + 1];
        __syncthreads();
        for (int64_t X = X0 + threadIdx.x; X < X1; X += kBlock) {
            int lo = 0, hi = kAggChunk - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) / 2;
                if (win[mid] <= X) lo = mid; else hi = mid - 1;
            }
            int v = a.members[k0 + lo];
            int64_t e = a.g.off[v] + (X - win[lo]);
            int32_t j = load_col(a.g.col, e);
            lds_table_add(tkeys, tvals, kAggChunkTable - 1, a.cm[j], edge_weight<WT>(a.g.w, e));
        }
        __syncthreads();
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
                     int32_t *gap_col, double *gap_w, Scratch &sc, int64_t *nnz_out, hipStream_t s,
                     bool hub_parts) {
    (void)wl;
    (void)hub_parts;
    int32_t *csz = sc.i32a, *ccur = sc.i32b, *members = sc.i32c, *cdeg = sc.i32d, *mdeg = sc.i32e;
    int64_t *coff = sc.i64a, *ctot = sc.i64b, *eoff = sc.i64c, *mpre = sc.i64d, *ctab = sc.i64e, *tmp = sc.i64f;
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
    a.gap_col = gap_col;
    a.gap_w = gap_w;
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

    // hub communities: table offsets in the global pool, entry chunks and
    // table segments
    int64_t H = a.cn[BIN_HUB], nchunks = 0, nsegs = 0;
    if (H > 0) {
        unsigned gr = grid1(H, 4096);
        int64_t hb = a.cbeg[BIN_HUB];
        k_agg_hub_sizes<<<gr, kBlock, 0, s>>>(cwl.bl, hb, H, eoff, n2, ctot);    // ctot is free now
        scan_exclusive_i64(ctot, tmp, H, sc.scan_tmp, s);
        k_agg_hub_off<<<gr, kBlock, 0, s>>>(cwl.bl, hb, H, tmp, ctab);
        int64_t host[3] = {0, 0, 0};
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
        // flattened entry index of every member
        k_member_degrees<<<grid1(g.n), kBlock, 0, s>>>(members, g.n, g.deg, mdeg);
        scan_exclusive_i32_to_i64(mdeg, mpre, g.n, sc.scan_tmp, s);
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
    if (g.wt == W_UNIT) {
        if (us) k_agg_small<W_UNIT><<<gs, kBlock, 0, s>>>(a);
        if (ul) k_agg_large<W_UNIT><<<gl, kBlock, 0, s>>>(a);
        if (nchunks) k_agg_hub_chunks<W_UNIT><<<gh, kBlock, 0, s>>>(a, sc.cch_comm, sc.cch_beg, nchunks);
    } else if (g.wt == W_F32) {
        if (us) k_agg_small<W_F32><<<gs, kBlock, 0, s>>>(a);
        if (ul) k_agg_large<W_F32><<<gl, kBlock, 0, s>>>(a);
        if (nchunks) k_agg_hub_chunks<W_F32><<<gh, kBlock, 0, s>>>(a, sc.cch_comm, sc.cch_beg, nchunks);
    } else {
        if (us) k_agg_small<W_F64><<<gs, kBlock, 0, s>>>(a);
        if (ul) k_agg_large<W_F64><<<gl, kBlock, 0, s>>>(a);
        if (nchunks) k_agg_hub_chunks<W_F64><<<gh, kBlock, 0, s>>>(a, sc.cch_comm, sc.cch_beg, nchunks);
    }
    if (nsegs) k_agg_hub_emit<<<(unsigned)(nsegs < 8192 ? nsegs : 8192), kBlock, 0, s>>>(a, sc.cseg_comm, sc.cseg_beg, nsegs);
    // compact
    scan_exclusive_i32_to_i64(out.deg, out.off, n2, sc.scan_tmp, s);
    e = hipMemcpyAsync(nnz_out, out.off + n2, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    if (n2 > 0) k_agg_copy<<<grid1(n2 * kWave, 65536), kBlock, 0, s>>>(eoff, out.off, n2, gap_col, gap_w, out.col, out.w);
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace gsp
