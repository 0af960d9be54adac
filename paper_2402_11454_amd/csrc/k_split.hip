// k_split.hip - splitting internally-disconnected communities (Section 4.1)
// and the renumber / dendrogram-lookup steps of Algorithm "louvain".
//
// The paper splits with a BFS per community (Algorithm "splitDisconnectedBfs")
// or minimum-label propagation (Algorithm "splitDisconnectedLp"); both give
// the connected components of the subgraph whose edges join vertices of the
// same community.  Here the components come from concurrent union-find over
// those edges: roots are hooked larger-under-smaller with a compare-and-swap,
// so every root is the smallest vertex of its set and the final label of a
// vertex is the smallest vertex id of its component -- the label the
// one-thread BFS from the lowest unvisited vertex gives.  Parent pointers
// only decrease, so path halving with plain (agent-scope) stores is safe
// while hooking; the final compression walks without halving (see there).
//
// Most of a community is usually one component, so the edges are taken in
// the order of the sampling scheme of Sutton et al. ("Optimizing parallel
// graph connectivity computation via subgraph sampling", IPDPS 2018): each
// vertex first links to those of its first kSample neighbours that share its
// community,
// the forest is compressed, and one root per community is picked by a
// vertex of it at random (usually that of its largest component).  A vertex
// already in the picked root's tree then skips its row: an edge from it to
// a vertex outside that tree is linked from the other end, whose row is
// scanned in full (every edge is stored in both rows); an edge inside the
// tree joins nothing new.  The components, hence the labels, are the same
// as with every edge linked.
#include "gsp_internal.h"

namespace gsp {

namespace {

__device__ __forceinline__ int ld(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st(int32_t *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ int find_root(int32_t *parent, int x) {
    while (true) {
        int p = ld(parent + x);
        if (p == x) return x;
        int gp = ld(parent + p);
        if (gp != p) st(parent + x, gp);
        x = gp;
    }
}

__device__ void unite(int32_t *parent, int a, int b) {
    while (true) {
        a = find_root(parent, a);
        b = find_root(parent, b);
        if (a == b) return;
        if (a < b) {
            int t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(parent + a, a, b) == a) return;
    }
}

__device__ __forceinline__ void hook_entry(int32_t *parent, const int32_t *cm, int i, int ci, int j) {
    if (j != i && cm[j] == ci) unite(parent, i, j);
}

// Sampling: every vertex links to those of its first kSample neighbours that
// share its community.  (With few entries inside communities, as on
// power-law graphs after a first local-moving phase, eight leave about 5 %
// of the vertices outside the picked trees.)
constexpr int kSample = 8;

__global__ void __launch_bounds__(kBlock) k_split_sample(Level g, const int32_t *cm, int32_t *parent) {
    // one thread per (vertex, sample): the unions of a vertex run side by side
    const int64_t total = g.n * kSample;
    for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < total; t += (int64_t)gridDim.x * kBlock) {
        const int i = (int)(t / kSample), r = (int)(t % kSample);
        if (r >= g.deg[i]) continue;
        const int j = g.col[g.off[i] + r];
        if (j != i && cm[j] == cm[i]) unite(parent, i, j);
    }
}

// The picked root of each community: first that of some vertex of it
// (racing plain stores; any winner will do), then, where a sampled vertex of
// the community votes, the root whose tree holds the most sampled degree
// (vote below).
__global__ void __launch_bounds__(kBlock) k_split_pick(const int32_t *parent, const int32_t *cm, int64_t n,
                                                      int32_t *dom) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        dom[cm[i]] = parent[i];
}

// Vote for the picked roots: every kVoteStride-th vertex adds deg + 1 to
// its root's count (summed per tile in LDS first: big trees draw many
// votes); then each sampled vertex offers (count of its root, root) for its
// community and the largest wins (packed in 64 bits, summed per tile in LDS
// first; a tie goes to the larger root id); then the winners become the
// picked roots.  Counts below 2^32: a vertex's deg + 1 summed over at most
// all vertices.
constexpr int kVoteStride = 16;
constexpr int kVoteTile = 4 * kBlock;
constexpr int kVoteTable = 2 * kVoteTile;

__global__ void __launch_bounds__(kBlock) k_split_vote_count(Level g, const int32_t *parent, uint32_t *cnt) {
    __shared__ int tk[kVoteTable];
    __shared__ unsigned tv[kVoteTable];
    for (int q = threadIdx.x; q < kVoteTable; q += kBlock) {
        tk[q] = kEmpty;
        tv[q] = 0;
    }
    __syncthreads();
    const int64_t ns = (g.n + kVoteStride - 1) / kVoteStride;
    for (int64_t t0 = blockIdx.x * (int64_t)kVoteTile; t0 < ns; t0 += (int64_t)gridDim.x * kVoteTile) {
        for (int64_t t = t0 + threadIdx.x; t < t0 + kVoteTile && t < ns; t += kBlock) {
            const int64_t i = t * kVoteStride;
            int sl = lds_table_slot(tk, kVoteTable - 1, parent[i]);
            atomicAdd(&tv[sl], (unsigned)g.deg[i] + 1u);
        }
        __syncthreads();
        for (int q = threadIdx.x; q < kVoteTable; q += kBlock) {
            if (tk[q] != kEmpty) atomicAdd(&cnt[tk[q]], tv[q]);
            tk[q] = kEmpty;
            tv[q] = 0;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kBlock) k_split_vote_best(int64_t n, const int32_t *parent, const int32_t *cm,
                                                           const uint32_t *cnt, unsigned long long *best) {
    __shared__ int tk[kVoteTable];
    __shared__ unsigned long long tv[kVoteTable];
    for (int q = threadIdx.x; q < kVoteTable; q += kBlock) {
        tk[q] = kEmpty;
        tv[q] = 0;
    }
    __syncthreads();
    const int64_t ns = (n + kVoteStride - 1) / kVoteStride;
    for (int64_t t0 = blockIdx.x * (int64_t)kVoteTile; t0 < ns; t0 += (int64_t)gridDim.x * kVoteTile) {
        for (int64_t t = t0 + threadIdx.x; t < t0 + kVoteTile && t < ns; t += kBlock) {
            const int64_t i = t * kVoteStride;
            const int r = parent[i];
            const unsigned long long v = ((unsigned long long)cnt[r] << 32) | (unsigned)r;
            int sl = lds_table_slot(tk, kVoteTable - 1, cm[i]);
            atomicMax(&tv[sl], v);
        }
        __syncthreads();
        for (int q = threadIdx.x; q < kVoteTable; q += kBlock) {
            if (tk[q] != kEmpty) atomicMax(&best[tk[q]], tv[q]);
            tk[q] = kEmpty;
            tv[q] = 0;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kBlock) k_split_vote_apply(int64_t n, const int32_t *cm,
                                                            const unsigned long long *best, int32_t *dom) {
    const int64_t ns = (n + kVoteStride - 1) / kVoteStride;
    for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < ns; t += (int64_t)gridDim.x * kBlock) {
        const int c = cm[t * kVoteStride];
        dom[c] = (int32_t)(best[c] & 0xffffffffull);
    }
}

// Vertex i may skip its row: it hangs directly under its community's picked
// root (parents only move to ancestors, so it stays in that tree).
__device__ __forceinline__ bool settled(const int32_t *parent, const int32_t *dom, int i, int ci) {
    return ld(parent + i) == dom[ci];
}

// All vertices of the level through its work lists: groups of G lanes for
// bins up to 64 entries, a wavefront per vertex up to 2048, a workgroup per
// hub chunk beyond.  Unit ranges: [0, us) small, [us, us+uw) wave, then hubs.
struct BinRanges {
    int64_t beg[kNumBins], n[kNumBins];
};

__global__ void __launch_bounds__(kBlock) k_split_hook(Level g, const int32_t *bl, BinRanges br,
                                                      const int32_t *ch_vert,
                                                      const int64_t *ch_beg, int64_t nchunks, const int32_t *cm,
                                                      const int32_t *dom, int32_t *parent) {
    const int64_t *binb = br.beg, *binn = br.n;
    int64_t pre[kNumSmallBins + 1];
    pre[0] = 0;
#pragma unroll
    for (int b = 0; b < kNumSmallBins; b++) {
        int vpb = kBlock / (4 << b);
        pre[b + 1] = pre[b] + (binn[b] + vpb - 1) / vpb;
    }
    int64_t nwave = binn[BIN_WAVE] + binn[BIN_BLOCK];
    int64_t uw = (nwave + (kBlock / kWave) - 1) / (kBlock / kWave);
    int64_t total = pre[kNumSmallBins] + uw + nchunks;
    for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
        if (u < pre[kNumSmallBins]) {
            int b = 0;
            while (u >= pre[b + 1]) b++;
            int G = 4 << b;
            int64_t qi = (u - pre[b]) * (kBlock / G) + threadIdx.x / G;
            int gl = threadIdx.x % G;
            if (qi < binn[b]) {
                int i = bl[binb[b] + qi];
                int ci = cm[i];
                if (gl < g.deg[i] && !settled(parent, dom, i, ci)) hook_entry(parent, cm, i, ci, g.col[g.off[i] + gl]);
            }
        } else if (u < pre[kNumSmallBins] + uw) {
            int64_t qi = (u - pre[kNumSmallBins]) * (kBlock / kWave) + threadIdx.x / kWave;
            if (qi < nwave) {
                // wave and block bins are adjacent in the lists
                int i = bl[binb[BIN_WAVE] + qi];
                int ci = cm[i];
                int64_t beg = g.off[i];
                if (!settled(parent, dom, i, ci))
                    for (int e = lane_id(); e < g.deg[i]; e += kWave) hook_entry(parent, cm, i, ci, g.col[beg + e]);
            }
        } else {
            int64_t k = u - pre[kNumSmallBins] - uw;
            int i = ch_vert[k];
            int ci = cm[i];
            int64_t beg = ch_beg[k];
            int64_t end = g.off[i] + g.deg[i];
            if (end > beg + kHubChunk) end = beg + kHubChunk;
            if (!settled(parent, dom, i, ci))
                for (int64_t e = beg + threadIdx.x; e < end; e += kBlock) hook_entry(parent, cm, i, ci, g.col[e]);
        }
    }
}

// Read-only walk to the root (no path halving): used once the forest no
// longer changes.
__device__ int find_root_ro(const int32_t *parent, int x) {
    while (true) {
        int p = ld(parent + x);
        if (p == x) return x;
        x = p;
    }
}

// Final labels.  Each thread writes only parent[i] (its root); a halving
// store from another thread's walk could otherwise overwrite that root with
// an older, non-root ancestor read before it.
__global__ void __launch_bounds__(kBlock) k_split_compress(int32_t *parent, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        int r = find_root_ro(parent, (int)i);
        st(parent + i, r);
    }
}

// flag[l] = 1 for every label in use (all writers store 1).
__global__ void __launch_bounds__(kBlock) k_mark_present(const int32_t *labels, int64_t n, int32_t *flag) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        flag[labels[i]] = 1;
}

__global__ void __launch_bounds__(kBlock) k_renumber_apply(const int32_t *labels, int64_t n, const int32_t *rank,
                                                          int32_t *out, int64_t *count) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        out[i] = rank[labels[i]];
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = rank[n];
}

__global__ void __launch_bounds__(kBlock) k_lookup(int32_t *top, int64_t n, const int32_t *cm) {
    for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock)
        top[v] = cm[top[v]];
}

__global__ void __launch_bounds__(kBlock) k_roots_per_comm(const int32_t *labels, const int32_t *memb, int64_t n,
                                                          int32_t *cnt) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        if (labels[i] == (int32_t)i) atomicAdd(&cnt[memb[i]], 1);
}

__global__ void __launch_bounds__(kBlock) k_count_gt1(const int32_t *cnt, int64_t n, unsigned long long *out) {
    unsigned long long c = 0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        c += cnt[i] > 1 ? 1 : 0;
    c = (unsigned long long)group_sum_ll<kWave>((long long)c);
    if (lane_id() == 0 && c) atomicAdd(out, c);
}

__global__ void __launch_bounds__(kBlock) k_min_vertex(const int32_t *memb, int64_t n, int32_t *first) {
    for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock)
        atomicMin(&first[memb[v]], (int32_t)v);
}

__global__ void __launch_bounds__(kBlock) k_gather(const int32_t *tab, const int32_t *idx, int64_t n, int32_t *out) {
    for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock)
        out[v] = tab[idx[v]];
}

// ---- split by minimum-label propagation with pruning (LPP) ----
//
// Algorithm "splitDisconnectedLp" with its pruning: labels start as the
// vertex ids, and a vertex whose label dropped pushes it to its neighbours
// in the same community, which become active when theirs drops in turn;
// at the fixed point every label is the smallest id of its component (the
// same labels as the BFS and union-find).  A round is one push from every
// active vertex (all of them in the first round), then a pointer jump
// lab[i] <- lab[lab[i]] for the vertices that changed: a label is always the
// id of a vertex of the same component (a push copies one along a
// same-community edge, a jump copies the label of such a vertex), so the
// jump keeps that and shortens long chains (road-like graphs) from their
// diameter to far fewer rounds.  Active vertices are queued in two lists:
// rows of at most kLpThreadDeg entries are pushed by one thread, longer rows
// by a wavefront (a hub's row is long but rare).

constexpr int kLpThreadDeg = 32;

// Round r: push from the queued vertices.  lab_now is read and lowered with
// atomicMin; a neighbour whose label dropped is flagged (next[j] = 1).
__global__ void __launch_bounds__(kBlock) k_lp_push(Level g, const int32_t *cm, int32_t *lab, const int32_t *q_small,
                                                   const int *n_small, const int32_t *q_large, const int *n_large,
                                                   uint8_t *next) {
    const int ns = *n_small, nl = *n_large;
    const int64_t nthr = (int64_t)gridDim.x * kBlock;
    for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < ns; t += nthr) {
        const int i = q_small[t];
        const int li = ld(lab + i), ci = cm[i];
        const int64_t b = g.off[i], e = b + g.deg[i];
        for (int64_t k = b; k < e; k++) {
            const int j = g.col[k];
            if (j == i || cm[j] != ci) continue;
            if (ld(lab + j) > li && atomicMin(lab + j, li) > li) next[j] = 1;
        }
    }
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t t = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; t < nl; t += nw) {
        const int i = q_large[t];
        const int li = ld(lab + i), ci = cm[i];
        const int64_t b = g.off[i], e = b + g.deg[i];
        for (int64_t k = b + lane_id(); k < e; k += kWave) {
            const int j = g.col[k];
            if (j == i || cm[j] != ci) continue;
            if (ld(lab + j) > li && atomicMin(lab + j, li) > li) next[j] = 1;
        }
    }
}

// After a round: every flagged vertex jumps (lab[i] <- lab[lab[i]] while that
// is smaller) and is queued for the next round; flags cleared.
__global__ void __launch_bounds__(kBlock) k_lp_collect(const int32_t *deg, int64_t n, int32_t *lab, uint8_t *next,
                                                      int32_t *q_small, int *n_small, int32_t *q_large,
                                                      int *n_large) {
    for (int64_t i0 = blockIdx.x * (int64_t)kBlock; i0 < n; i0 += (int64_t)gridDim.x * kBlock) {
        const int64_t i = i0 + threadIdx.x;
        bool act = false;
        int d = 0;
        if (i < n && next[i]) {
            next[i] = 0;
            int l = ld(lab + i);
            int l2 = ld(lab + l);
            while (l2 < l) {   // labels only decrease: the walk ends
                l = l2;
                l2 = ld(lab + l);
            }
            atomicMin(lab + i, l);
            d = deg[i];
            act = d > 0;
        }
        const bool small = act && d <= kLpThreadDeg, large = act && d > kLpThreadDeg;
        const int ps = wave_append(small, n_small);
        const int pl = wave_append(large, n_large);
        if (small) q_small[ps] = (int32_t)i;
        if (large) q_large[pl] = (int32_t)i;
    }
}

// First round's queues: every vertex with a non-empty row.
__global__ void __launch_bounds__(kBlock) k_lp_init(const int32_t *deg, int64_t n, int32_t *lab, uint8_t *next,
                                                   int32_t *q_small, int *n_small, int32_t *q_large, int *n_large) {
    for (int64_t i0 = blockIdx.x * (int64_t)kBlock; i0 < n; i0 += (int64_t)gridDim.x * kBlock) {
        const int64_t i = i0 + threadIdx.x;
        int d = 0;
        if (i < n) {
            lab[i] = (int32_t)i;
            next[i] = 0;
            d = deg[i];
        }
        const bool small = i < n && d > 0 && d <= kLpThreadDeg, large = i < n && d > kLpThreadDeg;
        const int ps = wave_append(small, n_small);
        const int pl = wave_append(large, n_large);
        if (small) q_small[ps] = (int32_t)i;
        if (large) q_large[pl] = (int32_t)i;
    }
}

// ---- the context-free disconnected count (caller's CSR, fixed scratch) ----
//
// flags[0]: communities with more than one component; flags[1]: nonzero if
// the input was malformed (an offset, a column or a label out of range).
// Every kernel checks what it indexes, so a malformed input gives -1 and no
// access outside the caller's arrays or the scratch.

__global__ void __launch_bounds__(kBlock) k_na_init(int32_t *parent, int32_t *roots, int64_t n,
                                                   unsigned long long *flags) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        parent[i] = (int32_t)i;
        roots[i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x < 2) flags[threadIdx.x] = 0;
}

// One wavefront per row: unite i with every neighbour in its community.
__global__ void __launch_bounds__(kBlock) k_na_hook(const int64_t *off, const int32_t *col, int64_t n, int64_t nnz,
                                                   const int32_t *memb, int32_t *parent,
                                                   unsigned long long *flags) {
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t i = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; i < n; i += nw) {
        const int64_t beg = off[i], end = off[i + 1];
        const int ci = memb[i];
        bool bad = beg < 0 || end < beg || end > nnz || ci < 0 || (int64_t)ci >= n;
        if (!bad)
            for (int64_t e = beg + lane_id(); e < end; e += kWave) {
                const int j = col[e];
                if (j < 0 || (int64_t)j >= n) {
                    bad = true;
                    continue;
                }
                if (j != (int)i && memb[j] == ci) unite(parent, (int)i, j);
            }
        if (bad) atomicOr(&flags[1], 1ull);
    }
}

__global__ void __launch_bounds__(kBlock) k_na_roots(const int32_t *parent, const int32_t *memb, int64_t n,
                                                    int32_t *roots) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const int c = memb[i];
        if (c >= 0 && (int64_t)c < n && parent[i] == (int32_t)i) atomicAdd(&roots[c], 1);
    }
}

__global__ void __launch_bounds__(kBlock) k_na_finish(const unsigned long long *flags, int64_t *out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *out = flags[1] ? -1 : (int64_t)flags[0];
}

inline unsigned grid1(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (unsigned)g;
}

}  // namespace

void launch_split(const Level &g, const WorkLists &wl, const int32_t *cm, int32_t *labels, int32_t *dom,
                  uint32_t *vote_cnt, unsigned long long *vote_best, hipStream_t s) {
    if (g.n == 0) return;
    launch_iota_i32(labels, g.n, s);
    k_split_sample<<<grid1(g.n * kSample), kBlock, 0, s>>>(g, cm, labels);
    k_split_compress<<<grid1(g.n), kBlock, 0, s>>>(labels, g.n);
    k_split_pick<<<grid1(g.n), kBlock, 0, s>>>(labels, cm, g.n, dom);
    const int64_t ns = (g.n + kVoteStride - 1) / kVoteStride;
    const unsigned gv = (unsigned)std::min<int64_t>((ns + kVoteTile - 1) / kVoteTile, 4096);
    launch_fill_i32(reinterpret_cast<int32_t *>(vote_cnt), 0, g.n, s);
    launch_fill_u64(vote_best, 0, g.n, s);
    k_split_vote_count<<<gv, kBlock, 0, s>>>(g, labels, vote_cnt);
    k_split_vote_best<<<gv, kBlock, 0, s>>>(g.n, labels, cm, vote_cnt, vote_best);
    k_split_vote_apply<<<grid1(ns), kBlock, 0, s>>>(g.n, cm, vote_best, dom);
    // per-bin begin/size over all sub-rounds (buckets of a bin are adjacent)
    BinRanges br;
    for (int b = 0; b < kNumBins; b++) {
        br.beg[b] = wl.bin_begin(b);
        br.n[b] = wl.bin_size(b);
    }
    int64_t units = 0;
    for (int b = 0; b < kNumSmallBins; b++) {
        int vpb = kBlock / (4 << b);
        units += (wl.bin_size(b) + vpb - 1) / vpb;
    }
    units += (wl.bin_size(BIN_WAVE) + wl.bin_size(BIN_BLOCK) + 3) / 4 + wl.nchunks;
    if (units > 0) {
        unsigned gr = (unsigned)(units < 65536 ? units : 65536);
        k_split_hook<<<gr, kBlock, 0, s>>>(g, wl.bl, br, wl.ch_vert, wl.ch_beg, wl.nchunks, cm, dom, labels);
    }
    k_split_compress<<<grid1(g.n), kBlock, 0, s>>>(labels, g.n);
}

void launch_renumber(const int32_t *labels, int64_t n, int32_t *out, int32_t *flag, int32_t *rank, int64_t *count,
                     void *tmp, hipStream_t s) {
    launch_fill_i32(flag, 0, n, s);
    k_mark_present<<<grid1(n), kBlock, 0, s>>>(labels, n, flag);
    scan_exclusive_i32(flag, rank, n, tmp, s);
    k_renumber_apply<<<grid1(n), kBlock, 0, s>>>(labels, n, rank, out, count);
}

void launch_lookup(int32_t *top, int64_t n, const int32_t *cm, hipStream_t s) {
    if (n > 0) k_lookup<<<grid1(n), kBlock, 0, s>>>(top, n, cm);
}

void launch_count_disconnected(const int32_t *labels, const int32_t *memb, int64_t n, int32_t *roots_per_comm,
                               unsigned long long *out, hipStream_t s) {
    launch_fill_i32(roots_per_comm, 0, n, s);
    k_roots_per_comm<<<grid1(n), kBlock, 0, s>>>(labels, memb, n, roots_per_comm);
    k_count_gt1<<<grid1(n), kBlock, 0, s>>>(roots_per_comm, n, out);
}

int launch_split_lp(const Level &g, const int32_t *cm, int32_t *labels, uint8_t *next, int32_t *q_small,
                    int32_t *q_large, int *counts, int *counts_h, hipStream_t s) {
    if (g.n == 0) return 0;
    const unsigned gn = grid1(g.n);
    launch_fill_i32(counts, 0, 4, s);
    k_lp_init<<<gn, kBlock, 0, s>>>(g.deg, g.n, labels, next, q_small, counts, q_large, counts + 1);
    int rounds = 0;
    for (int cur = 0;; cur ^= 1) {
        // queues of this round: counts[2 cur], counts[2 cur + 1]; the next
        // round's counters are cleared before its collection
        if (hipMemcpyAsync(counts_h, counts + 2 * cur, 2 * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return -1;
        const int ns = counts_h[0], nl = counts_h[1];
        if (ns + nl == 0) break;
        rounds++;
        const int64_t units = std::max<int64_t>((ns + kBlock - 1) / kBlock, (nl + 3) / 4);
        k_lp_push<<<(unsigned)std::min<int64_t>(std::max<int64_t>(units, 1), 65536), kBlock, 0, s>>>(
            g, cm, labels, q_small, counts + 2 * cur, q_large + 0, counts + 2 * cur + 1, next);
        launch_fill_i32(counts + 2 * (cur ^ 1), 0, 2, s);
        k_lp_collect<<<gn, kBlock, 0, s>>>(g.deg, g.n, labels, next, q_small, counts + 2 * (cur ^ 1), q_large,
                                           counts + 2 * (cur ^ 1) + 1);
    }
    return rounds;
}

void launch_count_disconnected_csr(const int64_t *off, const int32_t *col, int64_t n, int64_t nnz,
                                   const int32_t *memb, int32_t *parent, int32_t *roots, unsigned long long *flags,
                                   int64_t *out, hipStream_t s) {
    k_na_init<<<grid1(n), kBlock, 0, s>>>(parent, roots, n, flags);
    if (n > 0) {
        const int64_t wg = (n + kBlock / kWave - 1) / (kBlock / kWave);
        k_na_hook<<<(unsigned)std::min<int64_t>(wg, 65536), kBlock, 0, s>>>(off, col, n, nnz, memb, parent, flags);
        k_split_compress<<<grid1(n), kBlock, 0, s>>>(parent, n);
        k_na_roots<<<grid1(n), kBlock, 0, s>>>(parent, memb, n, roots);
        k_count_gt1<<<grid1(n), kBlock, 0, s>>>(roots, n, flags);
    }
    k_na_finish<<<1, kBlock, 0, s>>>(flags, out);
}

void launch_canonical_labels(const int32_t *memb, int64_t n, int32_t *first, int32_t *lab, hipStream_t s) {
    launch_fill_i32(first, 0x7fffffff, n, s);
    k_min_vertex<<<grid1(n), kBlock, 0, s>>>(memb, n, first);
    k_gather<<<grid1(n), kBlock, 0, s>>>(first, memb, n, lab);
}

}  // namespace gsp
