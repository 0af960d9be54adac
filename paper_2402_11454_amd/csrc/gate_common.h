// gate_common.h - device pieces of the learned vertex-pruning gate shared by
// the local-moving kernels (history, trace capture) and the gate kernels:
// the bf16 format, the piecewise-linear log2, the 8 per-vertex features and
// the trace sampling hash.
//
// The gate is not part of the paper.  It sits in front of the scan of
// Algorithm "louvainMove": an unprocessed vertex (Section 4.1's pruning
// flag) is scanned only if a small network predicts that it may move.  Its
// features use only O(1) state per vertex, never the vertex's row:
//   x0 = plog2(1 + deg_i) / 16     row length at this level
//   x1 = K_{i->d} / K_i             at i's last scan in this pass (0 before)
//   x2 = (G(best) - G(stay)) / (M2 K_i), clipped to [-1, 1], at that scan
//        (-1 if i had no candidate community, 0 for K_i = 0)
//   x3 = min(pass, 8) / 8
//   x4 = min(l, 20) / 20           l = counted iterations so far in the pass
//   x5 = K_i / Sigma_d             from the sub-round's snapshot
//   x6 = 0 if not scanned yet in this pass, 1/2 if it stayed at its last
//        scan, 1 if it moved
//   x7 = min(D_i / K_i, 1), D_i = weight of the entries (i, j) whose j moved
//        since i's last scan (or since the pass began; pruning keeps it)
// each computed in fp64, rounded to fp32, then to bf16 (round to nearest
// even).  Every step is an IEEE operation, so the values are reproducible
// bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsp {

constexpr int kGateFeatures = 8;
constexpr int kGateHidden = 64;
constexpr int kGateParams = (kGateFeatures * kGateHidden + kGateHidden) + (kGateHidden * kGateHidden + kGateHidden) +
                            (kGateHidden + 1);  // 4801
// Offsets of the parameter blocks in the flat fp32 vector.
constexpr int kPW1 = 0;
constexpr int kPB1 = kPW1 + kGateHidden * kGateFeatures;
constexpr int kPW2 = kPB1 + kGateHidden;
constexpr int kPB2 = kPW2 + kGateHidden * kGateHidden;
constexpr int kPW3 = kPB2 + kGateHidden;
constexpr int kPB3 = kPW3 + kGateHidden;

// History bits per vertex.
constexpr uint8_t kHistScanned = 1, kHistMoved = 2;

// bf16 bits of an fp32 value, round to nearest even (no NaN reaches here).
__host__ __device__ inline uint16_t bf16_bits(float x) {
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_value(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }
__host__ __device__ inline float bf16_round(float x) { return bf16_value(bf16_bits(x)); }

// Feature value: fp64 -> fp32 -> bf16.
__device__ __forceinline__ uint16_t feature_bits(double v) { return bf16_bits((float)v); }

// e + (x / 2^e - 1) for an integer x >= 1 with 2^e <= x < 2^(e+1): exact.
__device__ __forceinline__ double plog2_int(uint64_t x) {
    int e = 63 - __builtin_clzll(x);
    return (double)e + ((double)x / (double)(1ull << e) - 1.0);
}

__device__ __forceinline__ void gate_features(int64_t deg, double ki, double sig_d, float hfrac, float hgain,
                                              uint8_t hbits, double dmoved, int pass, int iter, uint16_t *x) {
    x[0] = feature_bits(plog2_int((uint64_t)deg + 1) / 16.0);
    x[1] = feature_bits((double)hfrac);
    x[2] = feature_bits((double)hgain);
    x[3] = feature_bits((double)(pass < 8 ? pass : 8) / 8.0);
    x[4] = feature_bits((double)(iter < 20 ? iter : 20) / 20.0);
    x[5] = feature_bits(ki > 0.0 && sig_d > 0.0 ? ki / sig_d : 0.0);
    x[6] = feature_bits((hbits & kHistScanned) ? ((hbits & kHistMoved) ? 1.0 : 0.5) : 0.0);
    double r = ki > 0.0 ? dmoved / ki : 0.0;
    x[7] = feature_bits(r < 1.0 ? r : 1.0);
}

// SplitMix64's output step (Steele, Lea and Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// A scan of vertex i in sweep `sweep` of pass `pass` is recorded iff
// mix64(seed ^ pass << 56 ^ sweep << 48 ^ i) < threshold.
__device__ __forceinline__ bool trace_keep(uint64_t seed, int pass, int sweep, int64_t i, uint64_t thr) {
    uint64_t key = seed ^ ((uint64_t)(uint32_t)pass << 56) ^ ((uint64_t)(uint32_t)sweep << 48) ^ (uint64_t)i;
    return mix64(key) < thr;
}

// The network in its inference formats: bf16 weight matrices (as bits),
// fp32 biases, the output weights rounded to bf16 and kept as fp32.
struct GateNet {
    const uint16_t *w1;  // [64][8]
    const uint16_t *w2;  // [64][64], row = output unit
    const float *b1;     // [64]
    const float *b2;     // [64]
    const float *w3;     // [64]
    float b3;
};

}  // namespace gsp
