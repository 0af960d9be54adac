// k_order.hip - the input graph stored in degree order (a layout only).
//
// Most CSR entries of a skewed graph point at a few high-degree vertices.
// Stored in the order they were loaded (often random), those vertices'
// membership and community-total words each sit in a different cache line,
// and every scan of an entry pulls a whole line for one 4- or 8-byte word.
// Here the vertices are renumbered by degree class, largest first, so that
// the words most entries gather share lines and stay in the caches; the
// shorter rows are grouped by sub-round first, so that a sub-round reads
// its vertices' rows and per-vertex words as contiguous ranges.  The
// method's results do not change: wherever it orders vertex or community ids
// (ties, the singleton rule, sub-rounds, traces, the numbering of
// communities) it compares the caller's ids, orig[v].
//
// Layout of the ordered copy: vertex p is the caller's vertex orig[p];
// rank[orig[p]] = p; row p holds row orig[p]'s entries, in the same order,
// with every column v replaced by rank[v] and the same weights.  Rows with
// at least kLongRow entries come first (p < nlong, by degree class), so the
// long rows are one contiguous entry range; then, for each sub-round in
// turn, its other rows by degree class.
#include <vector>

#include "gsp_internal.h"

namespace gsp {

namespace {

constexpr int kOrderClasses = 128;
constexpr int kOrderTile = kBlock * 4;
constexpr int kLongChunk = 8192;   // entries per workgroup on the long rows
constexpr int kShortCopy = 32;     // rows up to this length are copied by one lane

// Degree class: four per octave of the degree (the two bits after the
// leading one), largest degrees first, empty rows last.  d >= kLongRow =
// 2^kLongLog exactly when the class is at most kLongClass.
constexpr int kLongClass = kOrderClasses - 2 - 4 * kLongLog;
constexpr int kOrderBuckets = kOrderClasses * (kMaxRounds + 1);   // at most
static_assert(kOrderBuckets == kOrderBucketsMax, "bucket bound");

__device__ __forceinline__ int degree_class(int d) {
    if (d <= 0) return kOrderClasses - 1;
    const int e = 31 - __clz(d);
    const int q = e >= 2 ? (d >> (e - 2)) & 3 : (e == 1 ? (d & 1) << 1 : 0);
    return kOrderClasses - 2 - (4 * e + q);
}

// Bucket of vertex v (the caller's id) with d entries: its degree class if
// the row is long, else kOrderClasses * (1 + its sub-round) + its class.
__device__ __forceinline__ int order_bucket(int64_t v, int d, int shift) {
    const int c = degree_class(d);
    return c <= kLongClass ? c : kOrderClasses * (1 + sub_round_of(v, shift)) + c;
}

__global__ void __launch_bounds__(kBlock) k_order_count(const int32_t *deg, int64_t n, int shift, int nb,
                                                       unsigned long long *hist) {
    __shared__ unsigned int h[kOrderBuckets];
    for (int k = threadIdx.x; k < nb; k += kBlock) h[k] = 0;
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        atomicAdd(&h[order_bucket(i, deg[i], shift)], 1u);
    __syncthreads();
    for (int k = threadIdx.x; k < nb; k += kBlock)
        if (h[k]) atomicAdd(&hist[k], (unsigned long long)h[k]);
}

// Places every vertex in its class: cursor[k] starts at class k's first
// position; each tile reserves its positions with one atomic per class.
// (The order inside a class depends on the atomics' order; nothing but
// cache behaviour depends on it.)
__global__ void __launch_bounds__(kBlock) k_order_place(const int32_t *deg, int64_t n, int shift, int nb,
                                                       unsigned long long *cursor, int32_t *orig, int32_t *rank) {
    __shared__ unsigned int lcnt[kOrderBuckets];
    __shared__ unsigned long long lbase[kOrderBuckets];
    for (int64_t t0 = blockIdx.x * (int64_t)kOrderTile; t0 < n; t0 += (int64_t)gridDim.x * kOrderTile) {
        for (int k = threadIdx.x; k < nb; k += kBlock) lcnt[k] = 0;
        __syncthreads();
        int cls[4];
        unsigned int r[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t v = t0 + u * kBlock + threadIdx.x;
            cls[u] = v < n ? order_bucket(v, deg[v], shift) : 0;
            r[u] = v < n ? atomicAdd(&lcnt[cls[u]], 1u) : 0u;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nb; k += kBlock)
            if (lcnt[k]) lbase[k] = atomicAdd(&cursor[k], (unsigned long long)lcnt[k]);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t v = t0 + u * kBlock + threadIdx.x;
            if (v < n) {
                const int64_t p = (int64_t)(lbase[cls[u]] + r[u]);
                orig[p] = (int32_t)v;
                rank[v] = (int32_t)p;
            }
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kBlock) k_order_degrees(const int32_t *orig, const int32_t *deg, int64_t n,
                                                         int32_t *degp) {
    for (int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x; p < n; p += (int64_t)gridDim.x * kBlock)
        degp[p] = deg[orig[p]];
}

template <int WT>
__device__ __forceinline__ void copy_entry(const Level &g, const int32_t *rank, int64_t from, int64_t to,
                                           int32_t *colp, void *wp) {
    colp[to] = rank[g.col[from]];
    if constexpr (WT == W_F32) ((float *)wp)[to] = ((const float *)g.w)[from];
    if constexpr (WT == W_F64) ((double *)wp)[to] = ((const double *)g.w)[from];
}

// Rows p >= first (all shorter than kLongRow): a wavefront takes 64
// consecutive rows; a lane copies its own row if it has at most kShortCopy
// entries, the whole wavefront copies the others one by one.
template <int WT>
__global__ void __launch_bounds__(kBlock) k_order_rows(Level g, const int32_t *orig, const int32_t *rank,
                                                      const int64_t *offp, int64_t first, int32_t *colp,
                                                      void *wp) {
    const int lane = lane_id(), w = threadIdx.x / kWave;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t r0 = first + (int64_t)blockIdx.x * kBlock + w * kWave; r0 < g.n; r0 += stride) {
        const int64_t p = r0 + lane;
        int64_t src = 0, dst = 0, d = 0;
        if (p < g.n) {
            const int v = orig[p];
            src = g.off[v];
            d = g.deg[v];
            dst = offp[p];
        }
        const bool own = d <= kShortCopy;
        if (own)
            for (int64_t k = 0; k < d; k++) copy_entry<WT>(g, rank, src + k, dst + k, colp, wp);
        unsigned long long rest = __ballot(!own);
        while (rest) {
            const int l = __ffsll((long long)rest) - 1;
            rest &= rest - 1;
            const int64_t s0 = __shfl(src, l), t0 = __shfl(dst, l), dl = __shfl(d, l);
            for (int64_t k = lane; k < dl; k += kWave) copy_entry<WT>(g, rank, s0 + k, t0 + k, colp, wp);
        }
    }
}

// First row p < nlong whose entries reach past e (offp non-decreasing).
__device__ __forceinline__ int64_t row_of_entry(const int64_t *offp, int64_t nlong, int64_t e) {
    int64_t lo = 0, hi = nlong - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (offp[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Rows p < nlong: workgroup k copies the ordered entries [k C, (k+1) C)
// (C = kLongChunk), row segment by row segment.
template <int WT>
__global__ void __launch_bounds__(kBlock) k_order_long(Level g, const int32_t *orig, const int32_t *rank,
                                                      const int64_t *offp, int64_t nlong, int32_t *colp,
                                                      void *wp) {
    const int64_t total = offp[nlong];
    for (int64_t e0 = blockIdx.x * (int64_t)kLongChunk; e0 < total; e0 += (int64_t)gridDim.x * kLongChunk) {
        const int64_t e1 = e0 + kLongChunk < total ? e0 + kLongChunk : total;
        for (int64_t p = row_of_entry(offp, nlong, e0); p < nlong && offp[p] < e1; p++) {
            const int64_t s0 = offp[p] > e0 ? offp[p] : e0;
            const int64_t s1 = offp[p + 1] < e1 ? offp[p + 1] : e1;
            const int64_t shift = g.off[orig[p]] - offp[p];   // caller's entry = ordered entry + shift
            for (int64_t e = s0 + threadIdx.x; e < s1; e += kBlock)
                copy_entry<WT>(g, rank, e + shift, e, colp, wp);
        }
    }
}

// K_p of the long rows (p < nlong, K zeroed before): each workgroup sums its
// entry range row segment by row segment and adds the segment sums to K_p
// and to 2m.  Weights lie on the exact-sum grid, so the result does not
// depend on how the rows are cut.
template <int WT>
__global__ void __launch_bounds__(kBlock) k_vertex_weights_long(Level g, double *K, double *M2) {
    __shared__ double part[kBlock / kWave];
    const int64_t nlong = g.nlong;
    const int64_t total = g.off[nlong];
    const int lane = lane_id(), w = threadIdx.x / kWave;
    double blk = 0.0;
    for (int64_t e0 = blockIdx.x * (int64_t)kLongChunk; e0 < total; e0 += (int64_t)gridDim.x * kLongChunk) {
        const int64_t e1 = e0 + kLongChunk < total ? e0 + kLongChunk : total;
        for (int64_t p = row_of_entry(g.off, nlong, e0); p < nlong && g.off[p] < e1; p++) {
            const int64_t s0 = g.off[p] > e0 ? g.off[p] : e0;
            const int64_t s1 = g.off[p + 1] < e1 ? g.off[p + 1] : e1;
            double t = 0.0;
            for (int64_t e = s0 + threadIdx.x; e < s1; e += kBlock) t += edge_weight<WT>(g.w, e);
            t = group_sum<kWave>(t);
            if (lane == 0) part[w] = t;
            __syncthreads();
            if (threadIdx.x == 0) {
                double s = 0.0;
                for (int k = 0; k < kBlock / kWave; k++) s += part[k];
                unsafeAtomicAdd(&K[p], s);
                blk += s;
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0 && blk != 0.0) unsafeAtomicAdd(M2, blk);
}

// minorig[l] = min orig[v] over lab[v] = l.  The values only decrease, so a
// plain read that already shows a value at most orig[v] makes the atomic
// unnecessary; this keeps the atomics on a large community's word few.
__global__ void __launch_bounds__(kBlock) k_min_orig_of_label(const int32_t *lab, const int32_t *orig, int64_t n,
                                                             int32_t *minorig) {
    for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
        const int l = lab[v], o = orig[v];
        if (o < __hip_atomic_load(&minorig[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(&minorig[l], o);
    }
}

__global__ void __launch_bounds__(kBlock) k_label_lookup(int32_t *lab, const int32_t *table, int64_t n) {
    for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock)
        lab[v] = table[lab[v]];
}

__global__ void __launch_bounds__(kBlock) k_orig_of_label(const int32_t *lab, const int32_t *orig, int64_t n,
                                                         int32_t *out) {
    for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock)
        out[v] = orig[lab[v]];
}

__global__ void __launch_bounds__(kBlock) k_scatter_by_orig(const int32_t *in, const int32_t *orig, int64_t n,
                                                           int32_t *out) {
    for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock)
        out[orig[v]] = in[v];
}

inline unsigned grid_of(int64_t n, int64_t per_block, unsigned cap) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (int64_t)cap) g = cap;
    return (unsigned)g;
}

}  // namespace

hipError_t order_by_degree(const Level &g, Scratch &sc, DegreeOrder &o, int rounds, hipStream_t s) {
    const int64_t n = g.n;
    o.nlong = 0;
    o.rounds = rounds;
    if (n == 0) return hipSuccess;
    int shift = 0;
    while ((1 << shift) < rounds) shift++;
    const int nb = kOrderClasses * (rounds + 1);
    unsigned long long *hist = o.hist, *cursor = o.hist + kOrderBuckets;
    hipError_t e = hipMemsetAsync(hist, 0, sizeof(unsigned long long) * nb, s);
    if (e != hipSuccess) return e;
    k_order_count<<<grid_of(n, kBlock * 16, 4096), kBlock, 0, s>>>(g.deg, n, shift, nb, hist);
    std::vector<unsigned long long> h(nb), cur(nb);
    if ((e = hipMemcpyAsync(h.data(), hist, sizeof(unsigned long long) * nb, hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    unsigned long long at = 0;
    for (int k = 0; k < nb; k++) {
        cur[k] = at;
        at += h[k];
        if (k == kLongClass) o.nlong = (int64_t)at;
    }
    if ((e = hipMemcpyAsync(cursor, cur.data(), sizeof(unsigned long long) * nb, hipMemcpyHostToDevice, s)) !=
        hipSuccess)
        return e;
    k_order_place<<<grid_of(n, kOrderTile, 4096), kBlock, 0, s>>>(g.deg, n, shift, nb, cursor, o.orig, o.rank);
    k_order_degrees<<<grid_of(n, kBlock * 4, 8192), kBlock, 0, s>>>(o.orig, g.deg, n, o.deg);
    scan_exclusive_i32_to_i64(o.deg, o.off, n, sc.scan_tmp, s);
    int64_t long_entries = 0;
    if ((e = hipMemcpyAsync(&long_entries, o.off + o.nlong, sizeof(int64_t), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;   // cur and long_entries live on this frame
    if (o.nlong > 0) {
        const unsigned gl = grid_of(long_entries, kLongChunk, 65536);
        if (g.wt == W_UNIT)
            k_order_long<W_UNIT><<<gl, kBlock, 0, s>>>(g, o.orig, o.rank, o.off, o.nlong, o.col, o.w);
        else if (g.wt == W_F32)
            k_order_long<W_F32><<<gl, kBlock, 0, s>>>(g, o.orig, o.rank, o.off, o.nlong, o.col, o.w);
        else
            k_order_long<W_F64><<<gl, kBlock, 0, s>>>(g, o.orig, o.rank, o.off, o.nlong, o.col, o.w);
    }
    if (o.nlong < n) {
        const unsigned gr = grid_of(n - o.nlong, kBlock, 16384);
        if (g.wt == W_UNIT)
            k_order_rows<W_UNIT><<<gr, kBlock, 0, s>>>(g, o.orig, o.rank, o.off, o.nlong, o.col, o.w);
        else if (g.wt == W_F32)
            k_order_rows<W_F32><<<gr, kBlock, 0, s>>>(g, o.orig, o.rank, o.off, o.nlong, o.col, o.w);
        else
            k_order_rows<W_F64><<<gr, kBlock, 0, s>>>(g, o.orig, o.rank, o.off, o.nlong, o.col, o.w);
    }
    return hipGetLastError();
}

void launch_vertex_weights_long(const Level &g, double *K, double *M2, hipStream_t s) {
    if (g.nlong <= 0) return;
    launch_fill_f64(K, 0.0, g.nlong, s);
    // an upper bound of the long rows' entries is not known on the host:
    // the grid strides over them
    const unsigned gr = 4096;
    if (g.wt == W_UNIT)
        k_vertex_weights_long<W_UNIT><<<gr, kBlock, 0, s>>>(g, K, M2);
    else if (g.wt == W_F32)
        k_vertex_weights_long<W_F32><<<gr, kBlock, 0, s>>>(g, K, M2);
    else
        k_vertex_weights_long<W_F64><<<gr, kBlock, 0, s>>>(g, K, M2);
}

void launch_labels_min_orig(int32_t *lab, const int32_t *orig, int64_t n, int32_t *tmp, hipStream_t s) {
    if (n == 0) return;
    launch_fill_i32(tmp, 0x7fffffff, n, s);
    k_min_orig_of_label<<<grid_of(n, kBlock * 4, 8192), kBlock, 0, s>>>(lab, orig, n, tmp);
    k_label_lookup<<<grid_of(n, kBlock * 4, 8192), kBlock, 0, s>>>(lab, tmp, n);
}

void launch_labels_orig(const int32_t *lab, const int32_t *orig, int64_t n, int32_t *out, hipStream_t s) {
    if (n > 0) k_orig_of_label<<<grid_of(n, kBlock * 4, 8192), kBlock, 0, s>>>(lab, orig, n, out);
}

void launch_scatter_by_orig(const int32_t *in, const int32_t *orig, int64_t n, int32_t *out, hipStream_t s) {
    if (n > 0) k_scatter_by_orig<<<grid_of(n, kBlock * 4, 8192), kBlock, 0, s>>>(in, orig, n, out);
}

}  // namespace gsp
