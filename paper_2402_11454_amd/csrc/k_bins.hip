// k_bins.hip - per-level work lists: every vertex with at least one entry is
// put in bucket (bin of its degree, its sub-round); hubs are cut into chunks
// and get a slot range in the global hub-table pool.
#include <vector>

#include "gsp_internal.h"

namespace gsp {

namespace {

constexpr int kBinTile = kBlock * 4;

// Sub-round of vertex v: by its id within its graph when the level holds a
// batch of graphs (gid: graph of each vertex, vbase: first vertex of each
// graph), so every graph of a batch sees the groups it would see alone; by
// its caller's id orig[v] when the level is stored in degree order.
__device__ __forceinline__ int vertex_round(int64_t v, int shift, const int32_t *gid, const int64_t *vbase,
                                            const int32_t *orig) {
    if (orig) return sub_round_of(orig[v], shift);
    return sub_round_of(gid ? v - vbase[gid[v]] : v, shift);
}

__global__ void __launch_bounds__(kBlock) k_bin_count(const int32_t *deg, int64_t n, int rounds, int shift,
                                                     const int32_t *gid, const int64_t *vbase, const int32_t *orig,
                                                     unsigned long long *cnt, unsigned long long *ent) {
    __shared__ unsigned int lcnt[kNumBuckets];
    __shared__ unsigned long long lent[kNumBuckets];
    int nb = kNumBins * rounds;
    for (int k = threadIdx.x; k < nb; k += kBlock) { lcnt[k] = 0; lent[k] = 0; }
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)kBinTile + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBinTile) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
            int64_t v = i + (int64_t)r * kBlock;
            if (v >= n) break;
            int d = deg[v];
            int b = bin_of_degree(d);
            if (b < 0) continue;
            int k = b * rounds + vertex_round(v, shift, gid, vbase, orig);
            atomicAdd(&lcnt[k], 1u);
            atomicAdd(&lent[k], (unsigned long long)d);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nb; k += kBlock)
        if (lcnt[k]) {
            atomicAdd(&cnt[k], (unsigned long long)lcnt[k]);
            atomicAdd(&ent[k], lent[k]);
        }
}

// Places vertex ids into their buckets.  cursor[k] starts at the bucket's
// begin; each block reserves its slots with one atomic per bucket.
__global__ void __launch_bounds__(kBlock) k_bin_fill(const int32_t *deg, int64_t n, int rounds, int shift,
                                                    const int32_t *gid, const int64_t *vbase, const int32_t *orig,
                                                    unsigned long long *cursor, int32_t *bl) {
    __shared__ unsigned int lcnt[kNumBuckets];
    __shared__ unsigned long long lbase[kNumBuckets];
    int nb = kNumBins * rounds;
    for (int64_t t0 = blockIdx.x * (int64_t)kBinTile; t0 < n; t0 += (int64_t)gridDim.x * kBinTile) {
        for (int k = threadIdx.x; k < nb; k += kBlock) lcnt[k] = 0;
        __syncthreads();
        int bk[4];
        unsigned rk[4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            int64_t v = t0 + (int64_t)r * kBlock + threadIdx.x;
            bk[r] = -1;
            if (v < n) {
                int b = bin_of_degree(deg[v]);
                if (b >= 0) {
                    bk[r] = b * rounds + vertex_round(v, shift, gid, vbase, orig);
                    rk[r] = atomicAdd(&lcnt[bk[r]], 1u);
                }
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nb; k += kBlock)
            if (lcnt[k]) lbase[k] = atomicAdd(&cursor[k], (unsigned long long)lcnt[k]);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; r++) {
            int64_t v = t0 + (int64_t)r * kBlock + threadIdx.x;
            if (bk[r] >= 0) bl[lbase[bk[r]] + rk[r]] = (int32_t)v;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kBlock) k_hub_sizes(const int32_t *bl, int64_t hb, int64_t H, const int32_t *deg,
                                                     int64_t *tsize, int64_t *nch, int64_t *bsz) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < H; k += (int64_t)gridDim.x * kBlock) {
        int d = deg[bl[hb + k]];
        tsize[k] = (int64_t)hub_table_size(d);
        int64_t c = (d + kHubChunk - 1) / kHubChunk;
        nch[k] = c;
        bsz[k] = c <= kMaxParts ? c * c : 0;   // partition words of the hub
    }
}

__global__ void __launch_bounds__(kBlock) k_hub_fill(const int32_t *bl, int64_t hb, int64_t H, const int32_t *deg,
                                                    const int64_t *off, const int64_t *toff, const int64_t *coff,
                                                    const int64_t *boff, int64_t *hub_off, int32_t *hub_ch0,
                                                    int64_t *hub_b0, int32_t *ch_vert, int64_t *ch_beg) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < H; k += (int64_t)gridDim.x * kBlock) {
        int32_t i = bl[hb + k];
        hub_off[i] = toff[k];
        hub_b0[i] = boff[k];
        hub_ch0[i] = (int32_t)coff[k];
        int64_t nc = coff[k + 1] - coff[k];
        for (int64_t c = 0; c < nc; c++) {
            ch_vert[coff[k] + c] = i;
            ch_beg[coff[k] + c] = off[i] + c * kHubChunk;
        }
    }
}

}  // namespace

hipError_t bin_vertices(const int32_t *deg, int64_t n, int rounds, WorkLists &wl, Scratch &sc, hipStream_t s,
                        const int32_t *gid, const int64_t *vbase, const int32_t *orig) {
    int shift = 0;
    while ((1 << shift) < rounds) shift++;
    wl.rounds = rounds;
    wl.shift = shift;
    int nb = kNumBins * rounds;
    unsigned long long *cnt = sc.u64;          // nb counters at u64[0..nb)
    unsigned long long *ent = sc.u64 + kNumBuckets;
    hipError_t e = hipMemsetAsync(sc.u64, 0, sizeof(unsigned long long) * 2 * kNumBuckets, s);
    if (e != hipSuccess) return e;
    if (n > 0) {
        int64_t gr = (n + kBinTile - 1) / kBinTile;
        if (gr > 4096) gr = 4096;
        k_bin_count<<<(unsigned)gr, kBlock, 0, s>>>(deg, n, rounds, shift, gid, vbase, orig, cnt, ent);
    }
    unsigned long long hc[2 * kNumBuckets];
    e = hipMemcpyAsync(hc, sc.u64, sizeof(unsigned long long) * 2 * kNumBuckets, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    wl.boff[0] = 0;
    for (int k = 0; k < nb; k++) {
        wl.boff[k + 1] = wl.boff[k] + (int64_t)hc[k];
        wl.bucket_entries[k] = (int64_t)hc[kNumBuckets + k];
    }
    // cursors = bucket begins
    unsigned long long hcur[kNumBuckets];
    for (int k = 0; k < nb; k++) hcur[k] = (unsigned long long)wl.boff[k];
    e = hipMemcpyAsync(sc.u64, hcur, sizeof(unsigned long long) * nb, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);  // hcur lives on this stack frame
    if (e != hipSuccess) return e;
    if (n > 0) {
        int64_t gr = (n + kBinTile - 1) / kBinTile;
        if (gr > 4096) gr = 4096;
        k_bin_fill<<<(unsigned)gr, kBlock, 0, s>>>(deg, n, rounds, shift, gid, vbase, orig, sc.u64, wl.bl);
    }
    return hipGetLastError();
}

hipError_t build_work_lists(const Level &g, int rounds, WorkLists &wl, Scratch &sc, hipStream_t s) {
    hipError_t e = bin_vertices(g.deg, g.n, rounds, wl, sc, s, g.gid, g.vbase, g.orig);
    if (e != hipSuccess) return e;
    // hubs
    int64_t hb = wl.bin_begin(BIN_HUB), H = wl.bin_size(BIN_HUB);
    wl.nchunks = 0;
    wl.hub_table_total = 0;
    for (int p = 0; p <= rounds; p++) wl.ch_poff[p] = 0;
    if (H > 0) {
        unsigned gr = (unsigned)((H + kBlock - 1) / kBlock);
        if (gr > 4096) gr = 4096;
        // table sizes -> offsets
        k_hub_sizes<<<gr, kBlock, 0, s>>>(wl.bl, hb, H, g.deg, sc.i64a, sc.i64c, sc.i64d);
        scan_exclusive_i64(sc.i64a, sc.i64b, H, sc.scan_tmp, s);   // i64b = table offsets
        scan_exclusive_i64(sc.i64c, sc.i64a, H, sc.scan_tmp, s);   // i64a = chunk offsets
        scan_exclusive_i64(sc.i64d, sc.i64e, H, sc.scan_tmp, s);   // i64e = partition word offsets
        std::vector<int64_t> tmp(H + 1);
        int64_t ttot = 0, btot = 0;
        e = hipMemcpyAsync(&ttot, sc.i64b + H, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(&btot, sc.i64e + H, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(tmp.data(), sc.i64a, sizeof(int64_t) * (H + 1), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        wl.nchunks = tmp[H];
        wl.hub_table_total = (uint64_t)ttot;
        wl.bucket_total = (uint64_t)btot;
        if (wl.nchunks > sc.ch_cap) return hipErrorInvalidValue;
        for (int p = 0; p <= rounds; p++) {
            int64_t pos = (p < rounds ? wl.bucket_begin(BIN_HUB, p) : wl.bin_begin(BIN_HUB) + H) - hb;
            wl.ch_poff[p] = tmp[pos];
        }
        e = ensure_hub_tables(sc, wl.hub_table_total, s);
        if (e != hipSuccess) return e;
        e = ensure_hub_buckets(sc, wl.bucket_total, s);
        if (e != hipSuccess) return e;
        k_hub_fill<<<gr, kBlock, 0, s>>>(wl.bl, hb, H, g.deg, g.off, sc.i64b, sc.i64a, sc.i64e, wl.hub_off,
                                         wl.hub_ch0, wl.hub_b0, sc.ch_vert, sc.ch_beg);
    }
    wl.ch_vert = sc.ch_vert;
    wl.ch_beg = sc.ch_beg;
    return hipGetLastError();
}

}  // namespace gsp
