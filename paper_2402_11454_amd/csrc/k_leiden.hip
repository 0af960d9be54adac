// k_leiden.hip - the steps GSP-Leiden adds around its refinement phase
// (Section 3.5, the Leiden algorithm's refinement, read greedily):
//
//   * the same-bound subgraph: row i keeps the entries (i, j) whose j lies
//     in i's bound community.  Sub-communities never leave their bound, so
//     these are the only entries that reach a candidate sub-community of i
//     or i's own; the refinement is the local-moving kernels run over this
//     subgraph (with the whole graph's K and 2m, and only vertices alone in
//     their sub-community moving), and a mover marks exactly its same-bound
//     neighbours.  Each row keeps its entries in their order.
//   * the next level's starting communities: super-vertex r (a refined
//     sub-community) starts in the bound community that holds it.
//
// A level's row i is [off[i], off[i] + deg[i]) (aggregated levels leave a
// gap after each row, whose stale contents are never read).
//
// Rows of at most kBlockMaxDeg entries are counted and copied by tiles of
// rows whose entries stream through a workgroup in order; hub rows by their
// work list chunks of kHubChunk entries, one workgroup each, a chunk's place
// in its row being the kept entries of the row's earlier chunks.  The count
// pass leaves a byte per entry (kept or not) for the copy pass, which so
// reads bytes in order instead of gathering bound[j] again.
#include "device_common.h"
#include "gsp_internal.h"

namespace gsp {
namespace {

constexpr int kTileRows = kBlock;

template <int WT>
__device__ __forceinline__ void put_entry(const Level &g, int64_t e, int64_t at, int32_t *colR, double *wR) {
    colR[at] = g.col[e];
    if constexpr (WT != W_UNIT) wR[at] = edge_weight<WT>(g.w, e);
}

// Rows that are not hubs, kTileRows per workgroup: the tile's rows' entries
// are taken as one sequence (row after row, each [off, off + deg); hub rows
// count as empty), kBlock at a time, each entry's row found by binary
// search in the tile's prefix of row lengths, so the loads of consecutive
// threads are consecutive.  FILL = false writes each row's kept-entry count
// (0 for hubs, whose chunks add theirs after); FILL = true writes the kept
// entries in order: an entry's place is the number of kept entries of the
// tile before it, less that number at its row's first entry.
template <int WT, bool FILL>
__global__ void __launch_bounds__(kBlock) k_bound_tile(Level g, const int32_t *bound, uint8_t *kept, int32_t *cnt,
                                                      const int64_t *offR, int32_t *colR, double *wR) {
    __shared__ int32_t pre[kTileRows + 1];   // exclusive prefix of the tile's row lengths
    __shared__ int32_t acc[kTileRows];       // kept entries per row / kept before the row's first entry
    __shared__ int32_t wsum[kBlock / kWave];
    const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
    static_assert(kTileRows == kBlock, "one row length per thread");
    for (int64_t r0 = (int64_t)blockIdx.x * kTileRows; r0 < g.n; r0 += (int64_t)gridDim.x * kTileRows) {
        const int nr = g.n - r0 < kTileRows ? (int)(g.n - r0) : kTileRows;
        int d = 0;
        if (t < nr) {
            d = g.deg[r0 + t];
            if (d > kBlockMaxDeg) d = 0;
        }
        int x = d;   // inclusive prefix within the wavefront
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(x, o, kWave);
            if (lane >= o) x += y;
        }
        if (lane == kWave - 1) wsum[w] = x;
        __syncthreads();
        int base = 0, total = 0;
        for (int q = 0; q < kBlock / kWave; q++) {
            base += q < w ? wsum[q] : 0;
            total += wsum[q];
        }
        pre[t] = base + x - d;
        if (t == kBlock - 1) pre[kTileRows] = total;
        acc[t] = 0;
        __syncthreads();
        int carry = 0;   // FILL: kept entries of the tile before this step (the same in every thread)
        for (int v0 = 0; v0 < total; v0 += kBlock) {
            const int v = v0 + t;
            int j = 0;
            bool keep = false;
            int64_t e = 0;
            if (v < total) {
                int lo = 0, hi = nr - 1;   // the last row j with pre[j] <= v
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (pre[mid] <= v) lo = mid; else hi = mid - 1;
                }
                j = lo;
                e = g.off[r0 + j] + (v - pre[j]);
                if constexpr (FILL)
                    keep = kept[e] != 0;
                else
                    keep = bound[g.col[e]] == bound[r0 + j];
            }
            if constexpr (!FILL) {
                if (v < total) kept[e] = keep ? 1 : 0;
                if (keep) atomicAdd(&acc[j], 1);
            } else {
                const unsigned long long m = __ballot(keep);
                if (lane == 0) wsum[w] = __popcll(m);
                __syncthreads();
                int before = carry, step = 0;
                for (int q = 0; q < kBlock / kWave; q++) {
                    before += q < w ? wsum[q] : 0;
                    step += wsum[q];
                }
                before += __popcll(m & ((1ull << lane) - 1));
                if (v < total && v == pre[j]) acc[j] = before;
                __syncthreads();
                if (keep) put_entry<WT>(g, e, offR[r0 + j] + (before - acc[j]), colR, wR);
                carry += step;
            }
        }
        __syncthreads();
        if constexpr (!FILL) {
            if (t < nr) cnt[r0 + t] = acc[t];
        }
        __syncthreads();   // pre, acc and wsum are rewritten by the next tile
    }
}

// Hub rows, chunk c = [ch_beg[c], ch_beg[c] + kHubChunk) of row ch_vert[c]:
// FILL = false writes the chunk's kept count to ch_cnt[c] and adds it to the
// row's count; FILL = true copies the kept entries, in order, after those
// of the row's earlier chunks (hub_ch0[i] is the row's first chunk).
template <int WT, bool FILL>
__global__ void __launch_bounds__(kBlock) k_bound_chunks(Level g, const int32_t *bound, uint8_t *kept,
                                                        const int32_t *ch_vert,
                                                        const int64_t *ch_beg, int64_t nch, const int32_t *hub_ch0,
                                                        int64_t *ch_cnt, int32_t *cnt, const int64_t *offR,
                                                        int32_t *colR, double *wR) {
    __shared__ int64_t wsum[kBlock / kWave];
    __shared__ int64_t base;
    const int lane = lane_id(), w = threadIdx.x / kWave;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const int32_t i = ch_vert[c];
        const int b = bound[i];
        const int64_t beg = ch_beg[c];
        const int64_t row_end = g.off[i] + g.deg[i];
        const int64_t end = beg + kHubChunk < row_end ? beg + kHubChunk : row_end;
        if constexpr (!FILL) {
            int64_t k = 0;
            for (int64_t e = beg + threadIdx.x; e < end; e += kBlock) {
                const bool keep = bound[g.col[e]] == b;
                kept[e] = keep ? 1 : 0;
                k += keep;
            }
            k = group_sum_ll<kWave>(k);
            if (lane == 0) wsum[w] = k;
            __syncthreads();
            if (threadIdx.x == 0) {
                int64_t t = 0;
                for (int q = 0; q < kBlock / kWave; q++) t += wsum[q];
                ch_cnt[c] = t;
                if (t) atomicAdd(&cnt[i], (int32_t)t);
            }
            __syncthreads();
        } else {
            // where this chunk's entries start in row i of the subgraph
            int64_t k = 0;
            for (int64_t q = hub_ch0[i] + threadIdx.x; q < c; q += kBlock) k += ch_cnt[q];
            k = group_sum_ll<kWave>(k);
            if (lane == 0) wsum[w] = k;
            __syncthreads();
            if (threadIdx.x == 0) {
                int64_t t = offR[i];
                for (int q = 0; q < kBlock / kWave; q++) t += wsum[q];
                base = t;
            }
            __syncthreads();
            int64_t at = base;
            for (int64_t e0 = beg; e0 < end; e0 += kBlock) {
                const int64_t e = e0 + threadIdx.x;
                const bool keep = e < end && kept[e] != 0;
                const unsigned long long m = __ballot(keep);
                __syncthreads();   // the previous round's wsum reads are done
                if (lane == 0) wsum[w] = __popcll(m);
                __syncthreads();
                int64_t before = 0, total = 0;
                for (int q = 0; q < kBlock / kWave; q++) {
                    before += q < w ? wsum[q] : 0;
                    total += wsum[q];
                }
                if (keep) put_entry<WT>(g, e, at + before + __popcll(m & ((1ull << lane) - 1)), colR, wR);
                at += total;
            }
            __syncthreads();
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_bound_start(const int32_t *sub, const int32_t *bound, int64_t n,
                                                       int32_t *start) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        start[sub[i]] = bound[i];
}

// Sets *err if two vertices of one sub-community lie in different bound
// communities (home[c]: the bound its first-seen member claimed, -1 before).
__global__ void __launch_bounds__(kBlock) k_bound_check(const int32_t *sub, const int32_t *bound, int64_t n,
                                                       int32_t *home, int *err) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const int32_t b = bound[i];
        const int32_t prev = atomicCAS(&home[sub[i]], -1, b);
        if (prev != -1 && prev != b) atomicOr(err, 1);
    }
}

inline unsigned grid_of(int64_t n, int64_t per_block, unsigned cap) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (int64_t)cap) g = cap;
    return (unsigned)g;
}

template <int WT>
void bound_subgraph_t(const Level &g, const WorkLists &wl, const int32_t *bound, int32_t *deg, int64_t *off,
                      int32_t *col, double *w, int64_t *ch_cnt, uint8_t *kept, void *scan_tmp, hipStream_t s) {
    const unsigned gr = grid_of(g.n, kTileRows, 16384);
    const int64_t nch = wl.nchunks;
    const unsigned gc = grid_of(nch, 1, 65536);
    k_bound_tile<WT, false><<<gr, kBlock, 0, s>>>(g, bound, kept, deg, nullptr, nullptr, nullptr);
    if (nch > 0)
        k_bound_chunks<WT, false><<<gc, kBlock, 0, s>>>(g, bound, kept, wl.ch_vert, wl.ch_beg, nch, wl.hub_ch0,
                                                        ch_cnt, deg, nullptr, nullptr, nullptr);
    scan_exclusive_i32_to_i64(deg, off, g.n, scan_tmp, s);
    k_bound_tile<WT, true><<<gr, kBlock, 0, s>>>(g, bound, kept, nullptr, off, col, w);
    if (nch > 0)
        k_bound_chunks<WT, true><<<gc, kBlock, 0, s>>>(g, bound, kept, wl.ch_vert, wl.ch_beg, nch, wl.hub_ch0,
                                                       ch_cnt, nullptr, off, col, w);
}

}  // namespace

hipError_t bound_subgraph(const Level &g, const WorkLists &wl, const int32_t *bound, int32_t *deg, int64_t *off,
                          int32_t *col, double *w, int64_t *ch_cnt, uint8_t *kept, void *scan_tmp,
                          hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    if (g.wt == W_UNIT)
        bound_subgraph_t<W_UNIT>(g, wl, bound, deg, off, col, w, ch_cnt, kept, scan_tmp, s);
    else if (g.wt == W_F32)
        bound_subgraph_t<W_F32>(g, wl, bound, deg, off, col, w, ch_cnt, kept, scan_tmp, s);
    else
        bound_subgraph_t<W_F64>(g, wl, bound, deg, off, col, w, ch_cnt, kept, scan_tmp, s);
    return hipGetLastError();
}

void launch_bound_check(const int32_t *sub, const int32_t *bound, int64_t n, int32_t *home, int *err,
                        hipStream_t s) {
    if (n == 0) return;
    launch_fill_i32(home, -1, n, s);
    k_bound_check<<<grid_of(n, kBlock * 4, 8192), kBlock, 0, s>>>(sub, bound, n, home, err);
}

void launch_bound_start(const int32_t *sub, const int32_t *bound, int64_t n, int32_t *start, hipStream_t s) {
    if (n > 0) k_bound_start<<<grid_of(n, kBlock * 4, 8192), kBlock, 0, s>>>(sub, bound, n, start);
}

}  // namespace gsp
