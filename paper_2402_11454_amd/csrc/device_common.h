// device_common.h - device-side building blocks shared by the GSP-Louvain
// kernels: degree bins, the sub-round hash, edge-weight loads, open-addressing
// tables keyed by community id (in LDS and in global memory), and
// wavefront-group reductions.  gfx950 (CDNA4), wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsp {

constexpr int kWave = 64;
constexpr int kBlock = 256;            // threads per block for every kernel here
constexpr int kEmpty = -1;             // empty table key (community ids are >= 0)
constexpr int kIntMax = 0x7fffffff;     // "no community" in an argmax

// Degree bins.  A vertex (or a community, for aggregation) with d entries is
// processed by:
//   d <= 4, 8, 16, 32, 64 : a group of 4/8/16/32/64 lanes, one entry per lane,
//                           table of 2*group slots in LDS;
//   d <= 512              : one wavefront, table in LDS (1024 slots on unit
//                           weights, 768 otherwise);
//   d <= 2048             : one 256-thread workgroup, table in LDS (4096 slots
//                           on unit weights, 3072 otherwise);
//   d > 2048              : several workgroups, table of nextpow2(2d) slots in
//                           global memory ("hub").
// Every table is at most half full (the local-moving scan's wave and
// workgroup tables on weighted graphs two thirds), so linear probing always
// terminates.
constexpr int kNumBins = 8;
enum { BIN_G4 = 0, BIN_G8, BIN_G16, BIN_G32, BIN_G64, BIN_WAVE, BIN_BLOCK, BIN_HUB };
constexpr int kNumSmallBins = 5;
constexpr int kWaveMaxDeg = 512;
constexpr int kWaveTable = 1024;
constexpr int kBlockMaxDeg = 2048;
constexpr int kBlockTable = 4096;
constexpr int kHubChunk = 2048;        // entries per workgroup in the hub kernels

__host__ __device__ inline int bin_of_degree(int64_t d) {
    if (d <= 0) return -1;
    if (d <= 4) return BIN_G4;
    if (d <= 8) return BIN_G8;
    if (d <= 16) return BIN_G16;
    if (d <= 32) return BIN_G32;
    if (d <= 64) return BIN_G64;
    if (d <= kWaveMaxDeg) return BIN_WAVE;
    if (d <= kBlockMaxDeg) return BIN_BLOCK;
    return BIN_HUB;
}

__host__ __device__ inline uint64_t hub_table_size(int64_t d) {
    uint64_t t = 1;
    while (t < (uint64_t)(2 * d)) t <<= 1;
    return t;
}

// Sub-round of vertex i when an iteration has 2^shift ordered sub-rounds:
// the top `shift` bits of i * 0x9E3779B97F4A7C15 (Fibonacci hashing).
__host__ __device__ inline int sub_round_of(int64_t i, int shift) {
    if (shift == 0) return 0;
    uint64_t x = (uint64_t)i * 0x9E3779B97F4A7C15ull;
    return (int)(x >> (64 - shift));
}

enum WType { W_UNIT = 0, W_F32 = 1, W_F64 = 2 };

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

template <int WT>
__device__ __forceinline__ double edge_weight(const void *w, int64_t e) {
    if constexpr (WT == W_UNIT) {
        return 1.0;
    } else if constexpr (WT == W_F32) {
        return (double)((const float *)w)[e];
    } else {
        return ((const double *)w)[e];
    }
}

__device__ __forceinline__ int32_t load_col(const int32_t *col, int64_t e) {
    return col[e];
}

__device__ __forceinline__ uint32_t key_hash(int32_t k) {
    uint32_t h = (uint32_t)k * 0x9E3779B1u;
    return h ^ (h >> 15);
}

// Adds w to the value of `key` in an LDS table of mask+1 slots.
__device__ __forceinline__ void lds_table_add(int *keys, double *vals, uint32_t mask, int key, double w) {
    uint32_t s = key_hash(key) & mask;
    while (true) {
        int prev = atomicCAS(&keys[s], kEmpty, key);
        if (prev == kEmpty || prev == key) {
            atomicAdd(&vals[s], w);
            return;
        }
        s = (s + 1) & mask;
    }
}

// Slot of `key` in an LDS table of mask+1 slots (claimed if absent).
__device__ __forceinline__ int lds_table_slot(int *keys, uint32_t mask, int key) {
    uint32_t s = key_hash(key) & mask;
    while (true) {
        int prev = atomicCAS(&keys[s], kEmpty, key);
        if (prev == kEmpty || prev == key) return (int)s;
        s = (s + 1) & mask;
    }
}

// Same on a table in global memory (device-scope atomics).
__device__ __forceinline__ void gbl_table_add(int *keys, double *vals, uint64_t mask, int key, double w) {
    uint64_t s = key_hash(key) & mask;
    while (true) {
        int prev = atomicCAS(&keys[s], kEmpty, key);
        if (prev == kEmpty || prev == key) {
            unsafeAtomicAdd(&vals[s], w);
            return;
        }
        s = (s + 1) & mask;
    }
}

// Partition of community c among P (high bits of a second mix, independent
// of the LDS slot hash).
__device__ __forceinline__ int part_of(int c, int P) {
    uint32_t h = (uint32_t)c;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return (int)(((uint64_t)h * (uint64_t)(uint32_t)P) >> 32);
}

// Exclusive scan of v[0..P) in place over a block of kBlock threads, v[P] =
// total: each thread sums a run of ceil(P / kBlock) entries, the run sums
// are scanned across each wavefront with shuffles and across the
// wavefronts through LDS, then each thread rewrites its run.
__device__ __forceinline__ void block_scan_excl(int *v, int P) {
    __shared__ int wtot[kBlock / kWave];
    const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave;
    const int per = (P + kBlock - 1) / kBlock;
    const int b0 = tid * per, b1 = b0 + per < P ? b0 + per : P;
    int sum = 0;
    for (int b = b0; b < b1; b++) sum += v[b];
    int inc = sum;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        int y = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += y;
    }
    if (lane == kWave - 1) wtot[w] = inc;
    __syncthreads();
    int run = inc - sum, all = 0;
#pragma unroll
    for (int q = 0; q < kBlock / kWave; q++) {
        if (q < w) run += wtot[q];
        all += wtot[q];
    }
    for (int b = b0; b < b1; b++) {
        int x = v[b];
        v[b] = run;
        run += x;
    }
    if (tid == 0) v[P] = all;
    __syncthreads();
}

// Largest s in [0, n) with v[s] <= t (v non-decreasing, v[0] = 0 <= t).
__device__ __forceinline__ int last_le(const int *v, int n, int t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (v[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// (g, c) beats (g2, c2): larger score, ties to the lower community id.
// Community ids are vertex ids of the level; on a level stored in degree
// order (orig != nullptr) they are compared as the caller's vertex ids,
// orig[c], which are read on exact ties only.
__device__ __forceinline__ bool better(double g, int c, double g2, int c2, const int32_t *orig) {
    if (g != g2) return g > g2;
    if (!orig || c == kIntMax || c2 == kIntMax) return c < c2;
    return orig[c] < orig[c2];
}

// Argmax over the W lanes of an aligned lane group (W power of two <= 64).
template <int W>
__device__ __forceinline__ void group_argmax(double &g, int &c, const int32_t *orig) {
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) {
        double og = __shfl_xor(g, off, W);
        int oc = __shfl_xor(c, off, W);
        if (better(og, oc, g, c, orig)) {
            g = og;
            c = oc;
        }
    }
}

template <int W>
__device__ __forceinline__ double group_sum(double x) {
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, W);
    return x;
}

template <int W>
__device__ __forceinline__ long long group_sum_ll(long long x) {
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, W);
    return x;
}

// Wave-aggregated atomics keyed by an index: lanes of one wavefront that hit
// the same element are combined into one atomic (a popular community would
// otherwise serialise thousands of same-address atomics).  Lanes are taken
// one distinct key at a time; at most 64 rounds.
__device__ __forceinline__ void wave_add_i32_by_key(int *base, int key, int val, bool pred) {
    unsigned long long pending = __ballot(pred);
    while (pending) {
        int leader = __ffsll((long long)pending) - 1;
        int lk = __shfl(key, leader);
        bool mine = pred && key == lk && ((pending >> lane_id()) & 1ull);
        unsigned long long m = __ballot(mine);
        int sum = mine ? val : 0;
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
        if (lane_id() == leader) atomicAdd(&base[lk], sum);
        pending &= ~m;
    }
}

__device__ __forceinline__ void wave_add_u64_by_key(unsigned long long *base, int key, unsigned long long val,
                                                    bool pred) {
    unsigned long long pending = __ballot(pred);
    while (pending) {
        int leader = __ffsll((long long)pending) - 1;
        int lk = __shfl(key, leader);
        bool mine = pred && key == lk && ((pending >> lane_id()) & 1ull);
        unsigned long long m = __ballot(mine);
        long long sum = mine ? (long long)val : 0;
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
        if (lane_id() == leader) atomicAdd(&base[lk], (unsigned long long)sum);
        pending &= ~m;
    }
}

__device__ __forceinline__ void wave_add_f64_by_key(double *base, int key, double val, bool pred) {
    unsigned long long pending = __ballot(pred);
    while (pending) {
        int leader = __ffsll((long long)pending) - 1;
        int lk = __shfl(key, leader);
        bool mine = pred && key == lk && ((pending >> lane_id()) & 1ull);
        unsigned long long m = __ballot(mine);
        double sum = mine ? val : 0.0;
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
        if (lane_id() == leader && sum != 0.0) unsafeAtomicAdd(&base[lk], sum);
        pending &= ~m;
    }
}

// Each lane with `pred` gets a distinct slot of cursor[key].
__device__ __forceinline__ int wave_reserve_by_key(int *cursor, int key, bool pred) {
    unsigned long long pending = __ballot(pred);
    int pos = -1;
    while (pending) {
        int leader = __ffsll((long long)pending) - 1;
        int lk = __shfl(key, leader);
        bool mine = pred && key == lk && ((pending >> lane_id()) & 1ull);
        unsigned long long m = __ballot(mine);
        int base = 0;
        if (lane_id() == leader) base = atomicAdd(&cursor[lk], __popcll(m));
        base = __shfl(base, leader);
        if (mine) pos = base + __popcll(m & ((1ull << lane_id()) - 1ull));
        pending &= ~m;
    }
    return pos;
}

// Wave-aggregated append: every lane with `pred` gets a distinct slot of
// counter *ctr; returns the slot (or -1).
__device__ __forceinline__ int wave_append(bool pred, int *ctr) {
    unsigned long long m = __ballot(pred);
    if (m == 0) return -1;
    int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(ctr, __popcll(m));
    base = __shfl(base, leader);
    unsigned long long below = m & ((1ull << lane_id()) - 1ull);
    return pred ? base + __popcll(below) : -1;
}

}  // namespace gsp
