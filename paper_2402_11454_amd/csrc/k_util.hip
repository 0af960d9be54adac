// k_util.hip - fills, device-wide exclusive scans, input validation, vertex
// weights (Section 3: K_i = sum_j w_ij) and the parts of modularity (Eq. 1).
#include <math.h>

#include "gsp_internal.h"

namespace gsp {

namespace {

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

inline unsigned grid_for(int64_t n, int64_t per_block, unsigned cap = 1u << 20) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (int64_t)cap) g = cap;
    return (unsigned)g;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_fill(T *p, T v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = v;
}

__global__ void __launch_bounds__(kBlock) k_iota(int32_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = (int32_t)i;
}

__global__ void __launch_bounds__(kBlock) k_copy_i32(int32_t *d, const int32_t *s, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) d[i] = s[i];
}

// Exclusive scan of the 256 values of a block (one per thread); returns the
// exclusive prefix of this thread and sets *total.
template <class T>
__device__ T block_exclusive_scan(T x, T *total) {
    __shared__ T wsum[kBlock / kWave];
    int lane = lane_id(), w = threadIdx.x / kWave;
    T inc = x;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        T y = __shfl_up(inc, off);
        if (lane >= off) inc += y;
    }
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kBlock / kWave; k++) {
        if (k < w) before += wsum[k];
        all += wsum[k];
    }
    __syncthreads();
    *total = all;
    return before + inc - x;
}

template <class TIn, class TAcc>
__global__ void __launch_bounds__(kBlock) k_scan_tile_sums(const TIn *in, int64_t n, TAcc *bsum) {
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    TAcc s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
        if (i < n) s += (TAcc)in[i];
    }
    TAcc tot;
    block_exclusive_scan<TAcc>(s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

template <class TAcc>
__global__ void __launch_bounds__(kBlock) k_scan_block_sums(TAcc *bsum, int64_t nb) {
    TAcc carry = 0;
    for (int64_t base = 0; base < nb; base += kBlock) {
        int64_t i = base + threadIdx.x;
        TAcc x = i < nb ? bsum[i] : 0;
        TAcc tot;
        TAcc ex = block_exclusive_scan<TAcc>(x, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

template <class TIn, class TOut>
__global__ void __launch_bounds__(kBlock) k_scan_down(const TIn *in, TOut *out, int64_t n, const TOut *bsum,
                                                    int64_t nb) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    TOut v[kScanItems];
    TOut s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        int64_t i = base + k;
        v[k] = i < n ? (TOut)in[i] : 0;
        s += v[k];
    }
    TOut tot;
    TOut ex = block_exclusive_scan<TOut>(s, &tot) + bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        int64_t i = base + k;
        if (i < n) out[i] = ex;
        ex += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = bsum[nb];
}

template <class TIn, class TOut>
void scan_exclusive(const TIn *in, TOut *out, int64_t n, void *tmp, hipStream_t s) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb < 1) nb = 1;
    TOut *bsum = (TOut *)tmp;
    k_scan_tile_sums<TIn, TOut><<<(unsigned)nb, kBlock, 0, s>>>(in, n, bsum);
    k_scan_block_sums<TOut><<<1, kBlock, 0, s>>>(bsum, nb);
    k_scan_down<TIn, TOut><<<(unsigned)nb, kBlock, 0, s>>>(in, out, n, bsum, nb);
}

__global__ void __launch_bounds__(kBlock) k_validate_offsets(const int64_t *off, int64_t n, int64_t nnz, int *err) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        int64_t a = off[i], b = off[i + 1];
        if (a > b || a < 0 || b > nnz || b - a > 0x7fffffffLL) atomicOr(err, 1);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        if (off[0] != 0 || off[n] != nnz) atomicOr(err, 1);
}

template <int WT>
__global__ void __launch_bounds__(kBlock) k_validate_entries(const int32_t *col, const void *w, int64_t n,
                                                            int64_t nnz, int *err) {
    int bad = 0;
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kBlock) {
        int32_t c = col[e];
        if (c < 0 || (int64_t)c >= n) bad |= 2;
        if constexpr (WT != W_UNIT) {
            double x = edge_weight<WT>(w, e);
            if (!(x >= 0.0) || isinf(x)) bad |= 4;
        }
    }
    if (bad) atomicOr(err, bad);
}

__global__ void __launch_bounds__(kBlock) k_offsets_from_i32(const int32_t *in, int64_t *out, int64_t n1) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n1; i += (int64_t)gridDim.x * kBlock)
        out[i] = (int64_t)in[i];
}

__global__ void __launch_bounds__(kBlock) k_degrees(const int64_t *off, int32_t *deg, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        deg[i] = (int32_t)(off[i + 1] - off[i]);
}

__global__ void __launch_bounds__(kBlock) k_weights_to_f64(const float *in, double *out, int64_t nnz) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * kBlock)
        out[i] = (double)in[i];
}

// K_i = sum of row i, *M2 += sum_i K_i.  A wavefront takes 64 consecutive
// rows: each lane sums its own row if it has at most kShortRow entries (most
// rows of sparse graphs), then the wavefront sums the longer ones together,
// one at a time.  Sums of weights are exact (weight grid), so the order of
// the additions does not matter.  On a level in degree order the first
// g.nlong rows (the long ones, side by side) are left to
// launch_vertex_weights_long, which cuts them into equal entry chunks.
constexpr int kShortRow = 32;

template <int WT>
__global__ void __launch_bounds__(kBlock) k_vertex_weights(Level g, double *K, double *M2) {
    __shared__ double part[kBlock / kWave];
    const int lane = lane_id(), w = threadIdx.x / kWave;
    double blk = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t r0 = g.nlong + (int64_t)blockIdx.x * kBlock + w * kWave; r0 < g.n; r0 += stride) {
        const int64_t i = r0 + lane;
        int64_t b = 0, d = 0;
        if (i < g.n) {
            b = g.off[i];
            d = g.deg[i];   // rows may be gapped
        }
        double s = 0.0;
        const bool shortrow = d <= kShortRow;
        if (shortrow)
            for (int64_t k = b; k < b + d; k++) s += edge_weight<WT>(g.w, k);
        unsigned long long longs = __ballot(!shortrow);
        while (longs) {
            const int src = __ffsll((long long)longs) - 1;
            longs &= longs - 1;
            const int64_t lb = __shfl(b, src), ld = __shfl(d, src);
            double t = 0.0;
            for (int64_t k = lb + lane; k < lb + ld; k += kWave) t += edge_weight<WT>(g.w, k);
            t = group_sum<kWave>(t);
            if (lane == src) s = t;
        }
        if (i < g.n) K[i] = s;
        blk += group_sum<kWave>(s);
    }
    if (lane == 0) part[w] = blk;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kBlock / kWave; k++) t += part[k];
        unsafeAtomicAdd(M2, t);
    }
}

// The short rows of a level in degree order (rows [nlong, n), dense CSR):
// a workgroup takes 256 consecutive rows and reads their entries as one
// contiguous range, 256 at a time (coalesced), each thread finding its
// entry's row by a binary search over the rows' offsets in LDS and adding
// the weight to the row's LDS sum (exact sums, so the order of the atomics
// does not matter).
template <int WT>
__global__ void __launch_bounds__(kBlock) k_vertex_weights_rows(Level g, double *K, double *M2) {
    __shared__ int64_t so[kBlock + 1];
    __shared__ double acc[kBlock];
    __shared__ double part[kBlock / kWave];
    const int tid = threadIdx.x;
    double blk = 0.0;
    for (int64_t r0 = g.nlong + (int64_t)blockIdx.x * kBlock; r0 < g.n; r0 += (int64_t)gridDim.x * kBlock) {
        const int nr = g.n - r0 < kBlock ? (int)(g.n - r0) : kBlock;
        so[tid] = g.off[r0 + (tid < nr ? tid : nr)];
        if (tid == 0) so[kBlock] = g.off[r0 + nr];
        acc[tid] = 0.0;
        __syncthreads();
        const int64_t e0 = so[0], e1 = so[kBlock];
        const int lane = lane_id();
        for (int64_t eb = e0; eb < e1; eb += kBlock) {   // the same trip count in every lane
            const int64_t e = eb + tid;
            int r = -1;   // the row r with so[r] <= e < so[r + 1]
            double v = 0.0;
            if (e < e1) {
                int lo = 0, hi = nr - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (so[mid] <= e) lo = mid; else hi = mid - 1;
                }
                r = lo;
                v = edge_weight<WT>(g.w, e);
            }
            // consecutive lanes hold consecutive entries, so a row's entries
            // are a run of lanes: sum each run into its first lane (exact on
            // the grid's weights), which adds it to the row
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const double y = __shfl_down(v, o, kWave);
                const int ry = __shfl_down(r, o, kWave);
                if (lane + o < kWave && ry == r) v += y;
            }
            const int rp = __shfl_up(r, 1, kWave);
            if (r >= 0 && (lane == 0 || rp != r)) atomicAdd(&acc[r], v);
        }
        __syncthreads();
        if (tid < nr) {
            K[r0 + tid] = acc[tid];
            blk += acc[tid];
        }
        __syncthreads();
    }
    blk = group_sum<kWave>(blk);
    if (lane_id() == 0) part[tid / kWave] = blk;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int k = 0; k < kBlock / kWave; k++) t += part[k];
        if (t != 0.0) unsafeAtomicAdd(M2, t);
    }
}

// One wavefront per row: *sigma_in += entries of row i whose column shares
// i's community (the community totals come from launch_community_totals).
template <int WT>
__global__ void __launch_bounds__(kBlock) k_modularity_parts(Level g, const int32_t *memb, const double *K,
                                                            double *sig, double *sigma_in) {
    __shared__ double part[kBlock / kWave];
    int lane = lane_id(), w = threadIdx.x / kWave;
    double blk = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * (kBlock / kWave) + w; i < g.n; i += (int64_t)gridDim.x * (kBlock / kWave)) {
        int64_t b = g.off[i], e = b + g.deg[i];   // rows may be gapped
        int32_t c = memb[i];
        double s = 0.0;
        for (int64_t k = b + lane; k < e; k += kWave)
            if (memb[g.col[k]] == c) s += edge_weight<WT>(g.w, k);
        s = group_sum<kWave>(s);
        if (lane == 0) blk += s;
    }
    if (lane == 0) part[w] = blk;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kBlock / kWave; k++) t += part[k];
        unsafeAtomicAdd(sigma_in, t);
    }
}

// *out += sum_c (Sigma_c / M2)^2 in fixed point: each term rounded to the
// nearest multiple of 2^-62 (the sum of the terms is at most 1), so the
// total is an exact integer sum, the same in any order of the atomics.
__global__ void __launch_bounds__(kBlock) k_sum_squares(const double *sig, int64_t n, double M2,
                                                       unsigned long long *out) {
    unsigned long long s = 0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double x = sig[i] / M2;
        s += (unsigned long long)(long long)rint(ldexp(x * x, 62));
    }
    s = (unsigned long long)group_sum_ll<kWave>((long long)s);
    if (lane_id() == 0 && s) atomicAdd(out, s);
}

// Weight grid (exact sums).  Non-negative doubles order like their bit
// patterns, so the largest weight is an atomic max over the bits.
template <int WT>
__global__ void __launch_bounds__(kBlock) k_weight_max(const void *w, int64_t nnz, unsigned long long *out) {
    double m = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kBlock) {
        const double x = edge_weight<WT>(w, e);
        m = x > m ? x : m;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double o = __shfl_xor(m, off);
        m = o > m ? o : m;
    }
    if (lane_id() == 0 && m > 0.0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

// *U += max(1, ceil(w 2^T)) over the positive weights: an exact integer
// bound of 2^T times the weight total (T chosen so that it stays below 2^63).
template <int WT>
__global__ void __launch_bounds__(kBlock) k_weight_bound(const void *w, int64_t nnz, int T, unsigned long long *U) {
    unsigned long long s = 0;
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kBlock) {
        const double x = edge_weight<WT>(w, e);
        if (!(x > 0.0)) continue;
        const double t = ceil(ldexp(x, T));
        s += t < 1.0 ? 1ull : (unsigned long long)t;
    }
    s = (unsigned long long)group_sum_ll<kWave>((long long)s);
    if (lane_id() == 0 && s) atomicAdd(U, s);
}

// w <- nearest multiple of 2^-S (ties to even), in place; *moved counts the
// weights that changed.  A weight rounded to a coarser grid needs no more
// significand bits than it had, so an fp32 weight stays exact in fp32.
template <int WT>
__global__ void __launch_bounds__(kBlock) k_weight_grid(void *w, int64_t nnz, int S, unsigned long long *moved) {
    unsigned long long c = 0;
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kBlock) {
        const double x = edge_weight<WT>(w, e);
        const double q = ldexp(rint(ldexp(x, S)), -S);
        if (q == x) continue;
        c++;
        if constexpr (WT == W_F32)
            ((float *)w)[e] = (float)q;
        else
            ((double *)w)[e] = q;
    }
    c = (unsigned long long)group_sum_ll<kWave>((long long)c);
    if (lane_id() == 0 && c) atomicAdd(moved, c);
}

__global__ void __launch_bounds__(kBlock) k_check_labels(const int32_t *memb, int64_t n, int *err) {
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        if (memb[i] < 0 || (int64_t)memb[i] >= n) bad = 1;
    if (bad) atomicOr(err, 1);
}

}  // namespace

void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n > 0) k_fill<int32_t><<<grid_for(n, kBlock * 4, 8192), kBlock, 0, s>>>(p, v, n);
}
void launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s) {
    if (n > 0) k_fill<uint8_t><<<grid_for(n, kBlock * 4, 8192), kBlock, 0, s>>>(p, v, n);
}
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t s) {
    if (n > 0) k_fill<double><<<grid_for(n, kBlock * 4, 8192), kBlock, 0, s>>>(p, v, n);
}
void launch_fill_f32(float *p, float v, int64_t n, hipStream_t s) {
    if (n > 0) k_fill<float><<<grid_for(n, kBlock * 4, 8192), kBlock, 0, s>>>(p, v, n);
}
void launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s) {
    if (n > 0) k_fill<unsigned long long><<<grid_for(n, kBlock * 4, 8192), kBlock, 0, s>>>(p, v, n);
}
void launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) {
    if (n > 0) k_fill<int64_t><<<grid_for(n, kBlock * 4, 8192), kBlock, 0, s>>>(p, v, n);
}
void launch_iota_i32(int32_t *p, int64_t n, hipStream_t s) {
    if (n > 0) k_iota<<<grid_for(n, kBlock * 4, 8192), kBlock, 0, s>>>(p, n);
}
void launch_copy_i32(int32_t *dst, const int32_t *src, int64_t n, hipStream_t s) {
    if (n > 0) k_copy_i32<<<grid_for(n, kBlock * 4, 8192), kBlock, 0, s>>>(dst, src, n);
}

size_t scan_tmp_bytes(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile + 2) * sizeof(int64_t); }

void scan_exclusive_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, void *tmp, hipStream_t s) {
    scan_exclusive<int32_t, int64_t>(in, out, n, tmp, s);
}
void scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, void *tmp, hipStream_t s) {
    scan_exclusive<int64_t, int64_t>(in, out, n, tmp, s);
}
void scan_exclusive_i32(const int32_t *in, int32_t *out, int64_t n, void *tmp, hipStream_t s) {
    scan_exclusive<int32_t, int32_t>(in, out, n, tmp, s);
}

void launch_validate(const int64_t *off, const int32_t *col, const void *w, int wt, int64_t n, int64_t nnz,
                     int *err, hipStream_t s) {
    k_validate_offsets<<<grid_for(n, kBlock * 4, 8192), kBlock, 0, s>>>(off, n, nnz, err);
    if (nnz == 0) return;
    unsigned gr = grid_for(nnz, kBlock * 8, 16384);
    if (wt == W_UNIT)
        k_validate_entries<W_UNIT><<<gr, kBlock, 0, s>>>(col, w, n, nnz, err);
    else if (wt == W_F32)
        k_validate_entries<W_F32><<<gr, kBlock, 0, s>>>(col, w, n, nnz, err);
    else
        k_validate_entries<W_F64><<<gr, kBlock, 0, s>>>(col, w, n, nnz, err);
}

void launch_offsets_from_i32(const int32_t *in, int64_t *out, int64_t n1, hipStream_t s) {
    k_offsets_from_i32<<<grid_for(n1, kBlock * 4, 8192), kBlock, 0, s>>>(in, out, n1);
}

void launch_degrees(const int64_t *off, int32_t *deg, int64_t n, hipStream_t s) {
    if (n > 0) k_degrees<<<grid_for(n, kBlock * 4, 8192), kBlock, 0, s>>>(off, deg, n);
}

void launch_weights_to_f64(const float *in, double *out, int64_t nnz, hipStream_t s) {
    if (nnz > 0) k_weights_to_f64<<<grid_for(nnz, kBlock * 4, 16384), kBlock, 0, s>>>(in, out, nnz);
}

void launch_vertex_weights(const Level &g, double *K, double *M2, hipStream_t s) {
    if (g.n == 0) return;
    launch_vertex_weights_long(g, K, M2, s);
    if (g.nlong >= g.n) return;
    unsigned gr = grid_for(g.n - g.nlong, kBlock, 8192);
    if (g.orig) {   // degree order: dense rows of similar length side by side
        if (g.wt == W_UNIT)
            k_vertex_weights_rows<W_UNIT><<<gr, kBlock, 0, s>>>(g, K, M2);
        else if (g.wt == W_F32)
            k_vertex_weights_rows<W_F32><<<gr, kBlock, 0, s>>>(g, K, M2);
        else
            k_vertex_weights_rows<W_F64><<<gr, kBlock, 0, s>>>(g, K, M2);
        return;
    }
    if (g.wt == W_UNIT)
        k_vertex_weights<W_UNIT><<<gr, kBlock, 0, s>>>(g, K, M2);
    else if (g.wt == W_F32)
        k_vertex_weights<W_F32><<<gr, kBlock, 0, s>>>(g, K, M2);
    else
        k_vertex_weights<W_F64><<<gr, kBlock, 0, s>>>(g, K, M2);
}

void launch_modularity_parts(const Level &g, const int32_t *memb, const double *K, double *sig, double *sigma_in,
                             hipStream_t s) {
    if (g.n == 0) return;
    unsigned gr = grid_for(g.n, kBlock / kWave, 65536);
    if (g.wt == W_UNIT)
        k_modularity_parts<W_UNIT><<<gr, kBlock, 0, s>>>(g, memb, K, sig, sigma_in);
    else if (g.wt == W_F32)
        k_modularity_parts<W_F32><<<gr, kBlock, 0, s>>>(g, memb, K, sig, sigma_in);
    else
        k_modularity_parts<W_F64><<<gr, kBlock, 0, s>>>(g, memb, K, sig, sigma_in);
}

void launch_sum_squares(const double *sig, int64_t n, double M2, unsigned long long *out, hipStream_t s) {
    if (n > 0) k_sum_squares<<<grid_for(n, kBlock * 4, 4096), kBlock, 0, s>>>(sig, n, M2, out);
}

void launch_weight_max(const void *w, int wt, int64_t nnz, unsigned long long *out, hipStream_t s) {
    if (nnz == 0 || wt == W_UNIT) return;
    unsigned gr = grid_for(nnz, kBlock * 8, 8192);
    if (wt == W_F32)
        k_weight_max<W_F32><<<gr, kBlock, 0, s>>>(w, nnz, out);
    else
        k_weight_max<W_F64><<<gr, kBlock, 0, s>>>(w, nnz, out);
}

void launch_weight_bound(const void *w, int wt, int64_t nnz, int T, unsigned long long *U, hipStream_t s) {
    if (nnz == 0 || wt == W_UNIT) return;
    unsigned gr = grid_for(nnz, kBlock * 8, 8192);
    if (wt == W_F32)
        k_weight_bound<W_F32><<<gr, kBlock, 0, s>>>(w, nnz, T, U);
    else
        k_weight_bound<W_F64><<<gr, kBlock, 0, s>>>(w, nnz, T, U);
}

void launch_weight_grid(void *w, int wt, int64_t nnz, int S, unsigned long long *moved, hipStream_t s) {
    if (nnz == 0 || wt == W_UNIT) return;
    unsigned gr = grid_for(nnz, kBlock * 8, 8192);
    if (wt == W_F32)
        k_weight_grid<W_F32><<<gr, kBlock, 0, s>>>(w, nnz, S, moved);
    else
        k_weight_grid<W_F64><<<gr, kBlock, 0, s>>>(w, nnz, S, moved);
}

void launch_check_labels(const int32_t *memb, int64_t n, int *err, hipStream_t s) {
    if (n > 0) k_check_labels<<<grid_for(n, kBlock * 4, 8192), kBlock, 0, s>>>(memb, n, err);
}

}  // namespace gsp
