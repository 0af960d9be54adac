// k_batch.hip - per-graph bookkeeping for a batch of independent graphs run
// side by side as one block-diagonal level: the graph of each vertex, each
// graph's 2m, the first community id of each graph after a renumbering, and
// each graph's modularity (Eq. 1 with that graph's 2m).
//
// Vertices (and, after aggregation, communities) of graph g occupy the
// contiguous id range [vbase[g], vbase[g+1]); renumbering labels in
// ascending order keeps that property, because every label of graph g lies
// in g's range.
#include "gsp_internal.h"

namespace gsp {

namespace {

// gid[v] = g with vbase[g] <= v < vbase[g+1] (binary search over G+1 bases).
__global__ void __launch_bounds__(kBlock) k_batch_gid(const int64_t *vbase, int64_t G, int64_t n, int32_t *gid) {
    for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
        int64_t lo = 0, hi = G - 1;
        while (lo < hi) {
            int64_t mid = (lo + hi + 1) / 2;
            if (vbase[mid] <= v) lo = mid; else hi = mid - 1;
        }
        gid[v] = (int32_t)lo;
    }
}

// One block per graph: 2m_g = sum of K over the graph's vertices, in a
// fixed order (strided per thread, then a tree), so the value is
// reproducible.
__global__ void __launch_bounds__(kBlock) k_batch_m2(const double *K, const int64_t *vbase, int64_t G, double *M2g) {
    __shared__ double part[kBlock];
    for (int64_t g = blockIdx.x; g < G; g += gridDim.x) {
        double s = 0.0;
        for (int64_t v = vbase[g] + threadIdx.x; v < vbase[g + 1]; v += kBlock) s += K[v];
        part[threadIdx.x] = s;
        __syncthreads();
        for (int off = kBlock / 2; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) M2g[g] = part[0];
        __syncthreads();
    }
}

// First community id of each graph after a renumbering: rank = exclusive
// scan of the label-in-use flags, so graph g's ids start at rank[vbase[g]].
__global__ void __launch_bounds__(kBlock) k_batch_cfirst(const int32_t *rank, const int64_t *vbase, int64_t G,
                                                        const int64_t *count, int64_t *cfirst) {
    for (int64_t g = blockIdx.x * (int64_t)kBlock + threadIdx.x; g <= G; g += (int64_t)gridDim.x * kBlock)
        cfirst[g] = g < G ? (int64_t)rank[vbase[g]] : *count;
}

// Intra-community entry weight per graph: a wavefront takes 64 consecutive
// rows and flushes its running sum whenever the graph changes.
template <int WT>
__global__ void __launch_bounds__(kBlock) k_batch_qin(Level g, const int32_t *memb, double *qin) {
    const int lane = lane_id();
    const int64_t wid = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t r0 = wid * kWave; r0 < g.n; r0 += nw * kWave) {
        int64_t r1 = r0 + kWave < g.n ? r0 + kWave : g.n;
        int cur = g.gid[r0];
        double run = 0.0;
        for (int64_t i = r0; i < r1; i++) {
            int gi = g.gid[i];
            if (gi != cur) {
                if (lane == 0 && run != 0.0) unsafeAtomicAdd(&qin[cur], run);
                run = 0.0;
                cur = gi;
            }
            int32_t c = memb[i];
            double s = 0.0;
            for (int64_t k = g.off[i] + lane; k < g.off[i] + g.deg[i]; k += kWave)
                if (memb[g.col[k]] == c) s += edge_weight<WT>(g.w, k);
            run += group_sum<kWave>(s);
        }
        if (lane == 0 && run != 0.0) unsafeAtomicAdd(&qin[cur], run);
    }
}

// One block per graph: Q_g = qin_g / 2m_g - sum over g's communities of
// (Sigma_c / 2m_g)^2 (0 for 2m_g = 0).
__global__ void __launch_bounds__(kBlock) k_batch_q(const double *sig, const int64_t *cfirst, int64_t G,
                                                   const double *M2g, const double *qin, double *q) {
    __shared__ double part[kBlock];
    for (int64_t g = blockIdx.x; g < G; g += gridDim.x) {
        double m2 = M2g[g];
        double s = 0.0;
        if (m2 > 0.0)
            for (int64_t c = cfirst[g] + threadIdx.x; c < cfirst[g + 1]; c += kBlock) {
                double x = sig[c] / m2;
                s += x * x;
            }
        part[threadIdx.x] = s;
        __syncthreads();
        for (int off = kBlock / 2; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) q[g] = m2 > 0.0 ? qin[g] / m2 - part[0] : 0.0;
        __syncthreads();
    }
}

// A graph's confirming sweep starts with every vertex unprocessed.
__global__ void __launch_bounds__(kBlock) k_batch_flag_confirm(const int32_t *gid, const uint8_t *gconfirm, int64_t n,
                                                              uint8_t *flag) {
    for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock)
        if (gconfirm[gid[v]]) flag[v] = 1;
}

__global__ void __launch_bounds__(kBlock) k_add_i32(int32_t *p, int64_t n, int32_t delta) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] += delta;
}

inline unsigned grid_of(int64_t n, int64_t per, int64_t cap) {
    int64_t g = (n + per - 1) / per;
    if (g < 1) g = 1;
    return (unsigned)(g < cap ? g : cap);
}

}  // namespace

void launch_batch_gid(const int64_t *vbase, int64_t G, int64_t n, int32_t *gid, hipStream_t s) {
    if (n > 0) k_batch_gid<<<grid_of(n, kBlock, 8192), kBlock, 0, s>>>(vbase, G, n, gid);
}

void launch_batch_m2(const double *K, const int64_t *vbase, int64_t G, double *M2g, hipStream_t s) {
    if (G > 0) k_batch_m2<<<grid_of(G, 1, 4096), kBlock, 0, s>>>(K, vbase, G, M2g);
}

void launch_batch_cfirst(const int32_t *rank, const int64_t *vbase, int64_t G, const int64_t *count,
                         int64_t *cfirst, hipStream_t s) {
    k_batch_cfirst<<<grid_of(G + 1, kBlock, 1024), kBlock, 0, s>>>(rank, vbase, G, count, cfirst);
}

void launch_batch_modularity(const Level &g, const int32_t *memb, const double *sig, const int64_t *cfirst,
                             double *qin, double *q, hipStream_t s) {
    launch_fill_f64(qin, 0.0, g.graphs, s);
    if (g.n > 0) {
        unsigned gr = grid_of(g.n, (int64_t)kWave * (kBlock / kWave), 4096);
        if (g.wt == W_UNIT)
            k_batch_qin<W_UNIT><<<gr, kBlock, 0, s>>>(g, memb, qin);
        else if (g.wt == W_F32)
            k_batch_qin<W_F32><<<gr, kBlock, 0, s>>>(g, memb, qin);
        else
            k_batch_qin<W_F64><<<gr, kBlock, 0, s>>>(g, memb, qin);
    }
    k_batch_q<<<grid_of(g.graphs, 1, 4096), kBlock, 0, s>>>(sig, cfirst, g.graphs, g.M2g, qin, q);
}

void launch_batch_flag_confirm(const int32_t *gid, const uint8_t *gconfirm, int64_t n, uint8_t *flag, hipStream_t s) {
    if (n > 0) k_batch_flag_confirm<<<grid_of(n, kBlock * 4, 4096), kBlock, 0, s>>>(gid, gconfirm, n, flag);
}

void launch_add_i32(int32_t *p, int64_t n, int32_t delta, hipStream_t s) {
    if (n > 0 && delta != 0) k_add_i32<<<grid_of(n, kBlock * 4, 4096), kBlock, 0, s>>>(p, n, delta);
}

}  // namespace gsp
