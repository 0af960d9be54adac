// k_gate.hip - the learned vertex-pruning gate: its inference kernel (bf16
// matrix cores, fp32 accumulation) in front of the local-moving scan, and
// the fp32 training kernels (forward, backward, Adam) of its network.
//
// Network: z = w3 . relu(W2 relu(W1 x + b1) + b2) + b3, 8 -> 64 -> 64 -> 1,
// p = sigmoid(z); a vertex is scanned iff z >= logit(theta).
//
// Inference on CDNA4 matrix cores.  A wavefront takes 64 candidates as two
// batches of 32 columns and computes the transposed layers H^T = W X^T with
// v_mfma_f32_32x32x8_bf16: operand A is a 32x8 weight tile (lane l holds row
// l%32, columns 4(l/32)..+3), operand B an 8x32 activation tile (lane l holds
// rows 4(l/32)..+3 of column l%32), and the 32x32 fp32 result leaves lane l
// with column l%32, rows 8r + 4(l/32) + q (register 4r + q).  Those rows are
// exactly the B operand of the next layer's k-step 4t + r, so the hidden
// layer goes from the accumulators to bf16 operands inside each lane: no LDS
// round trip between layers.  Per 32 columns: 2 MFMAs for layer 1, 16 for
// layer 2; the 64 -> 1 output layer is a per-lane fp32 dot product plus one
// cross-half shuffle.
#include <math.h>

#include "gsp_internal.h"

namespace gsp {

namespace {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Weight operands of one lane, loaded once per wavefront.
struct NetRegs {
    s16x4 a1[2];     // W1 rows 32t + l%32, columns 4(l/32)..+3
    s16x4 a2[2][8];  // W2 rows 32t + l%32, columns 8s + 4(l/32)..+3
};

__device__ __forceinline__ void load_net(const GateNet &net, NetRegs &r) {
    const int lane = lane_id(), row = lane & 31, kq = (lane >> 5) * 4;
#pragma unroll
    for (int t = 0; t < 2; t++)
#pragma unroll
        for (int j = 0; j < 4; j++) r.a1[t][j] = (short)net.w1[(32 * t + row) * kGateFeatures + kq + j];
#pragma unroll
    for (int t = 0; t < 2; t++)
#pragma unroll
        for (int s = 0; s < 8; s++)
#pragma unroll
            for (int j = 0; j < 4; j++) r.a2[t][s][j] = (short)net.w2[(32 * t + row) * kGateHidden + 8 * s + kq + j];
}

// Logit of column l%32 of a 32-column batch whose features the lanes hold
// as B operands (bx); identical in lanes l and l^32.  The whole wavefront
// must execute this (matrix instructions need every lane).
__device__ __forceinline__ float mlp_columns(const NetRegs &r, s16x4 bx, const float *b1, const float *b2,
                                             const float *w3, float b3) {
    const int hi = lane_id() >> 5;
    f32x16 zero;
#pragma unroll
    for (int k = 0; k < 16; k++) zero[k] = 0.0f;
    s16x4 bh[8];
#pragma unroll
    for (int t = 0; t < 2; t++) {
        f32x16 c = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(r.a1[t], bx, zero, 0, 0, 0);
#pragma unroll
        for (int rr = 0; rr < 4; rr++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                int h = 32 * t + 8 * rr + 4 * hi + q;
                float v = c[4 * rr + q] + b1[h];
                v = v > 0.0f ? v : 0.0f;
                bh[4 * t + rr][q] = (short)bf16_bits(v);
            }
    }
    float part = 0.0f;
#pragma unroll
    for (int t = 0; t < 2; t++) {
        f32x16 c = zero;
#pragma unroll
        for (int s = 0; s < 8; s++) c = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(r.a2[t][s], bh[s], c, 0, 0, 0);
#pragma unroll
        for (int rr = 0; rr < 4; rr++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                int o = 32 * t + 8 * rr + 4 * hi + q;
                float v = c[4 * rr + q] + b2[o];
                v = v > 0.0f ? v : 0.0f;
                part += w3[o] * v;
            }
    }
    part += __shfl_xor(part, 32);
    return part + b3;
}

// Logits of the 64 rows fx[0..63][8] (bf16 bits) of a wavefront: the lane's
// own row's logit.
__device__ __forceinline__ float mlp_rows64(const NetRegs &r, const uint16_t (*fx)[kGateFeatures], const float *b1,
                                           const float *b2, const float *w3, float b3) {
    const int lane = lane_id(), col = lane & 31, hi = lane >> 5;
    s16x4 bx0 = *reinterpret_cast<const s16x4 *>(&fx[col][4 * hi]);
    s16x4 bx1 = *reinterpret_cast<const s16x4 *>(&fx[32 + col][4 * hi]);
    float z0 = mlp_columns(r, bx0, b1, b2, w3, b3);
    float z1 = mlp_columns(r, bx1, b1, b2, w3, b3);
    return lane < 32 ? z0 : z1;
}

__device__ __forceinline__ void load_biases(const GateNet &net, float *b1, float *b2, float *w3) {
    for (int k = threadIdx.x; k < kGateHidden; k += blockDim.x) {
        b1[k] = net.b1[k];
        b2[k] = net.b2[k];
        w3[k] = net.w3[k];
    }
}

constexpr int kGateSpan = 4096;   // candidates per workgroup, at most

// Gated sweep of one sub-round: candidates -> features -> network -> queue.
// Workgroup k takes the k-th of gridDim.x equal ranges of the candidates (at
// most kGateSpan), stages the vertices it keeps in LDS with their rank in
// their bin and reserves their queue slots with one atomic per bin.
__global__ void __launch_bounds__(kBlock) k_gate(MoveArgs a, GateNet net, float theta) {
    __shared__ float sb1[kGateHidden], sb2[kGateHidden], sw3[kGateHidden];
    __shared__ uint16_t fx[kBlock / kWave][kWave][kGateFeatures];
    __shared__ int lcnt[kNumBins], lbase[kNumBins];
    __shared__ unsigned long long spr[kBlock / kWave];
    __shared__ int32_t sv[kGateSpan];      // kept vertex
    __shared__ uint32_t sbr[kGateSpan];    // its bin (top 4 bits) and rank in the bin
    __shared__ int nst;
    load_biases(net, sb1, sb2, sw3);
    NetRegs r;
    load_net(net, r);
    int64_t pre[kNumBins + 1];
    pre[0] = 0;
#pragma unroll
    for (int b = 0; b < kNumBins; b++) pre[b + 1] = pre[b] + a.ctr->ccnt[a.round][b];
    const int64_t total = pre[kNumBins];
    int64_t span = (total + gridDim.x - 1) / gridDim.x;
    span = (span + kBlock - 1) / kBlock * kBlock;
    const int64_t lo = blockIdx.x * span;
    const int64_t hi = lo + span < total ? lo + span : total;
    const int w = threadIdx.x / kWave, lane = lane_id();
    unsigned long long pruned = 0;
    if (threadIdx.x < kNumBins) lcnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) nst = 0;
    __syncthreads();
    for (int64_t t0 = lo; t0 < hi; t0 += kBlock) {   // uniform over the workgroup
        int64_t t = t0 + threadIdx.x;
        bool valid = t < hi;
        int b = 0, i = -1;
        uint16_t x[kGateFeatures] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (valid) {
            while (t >= pre[b + 1]) b++;
            i = a.cand[a.qbase[b] + (t - pre[b])];
            const int li = a.giter ? a.giter[a.g.gid[i]] : (a.iter_dev ? (int)*a.iter_dev : a.iter);
            gate_features(a.g.deg[i], a.K[i], a.sig[a.cm[i]], a.hfrac[i], a.hgain[i], a.hbits[i], a.dsnap[i], a.pass,
                          li, x);
        }
#pragma unroll
        for (int f = 0; f < kGateFeatures; f++) fx[w][lane][f] = x[f];
        __syncthreads();
        float z = mlp_rows64(r, fx[w], sb1, sb2, sw3, net.b3);
        // a batch graph outside its gated sweeps keeps every candidate
        bool keep = valid && (z >= theta || (a.ggated && !a.ggated[a.g.gid[i]]));
        if (keep) {
            const int rank = atomicAdd(&lcnt[b], 1);
            const int slot = atomicAdd(&nst, 1);
            sv[slot] = i;
            sbr[slot] = ((uint32_t)b << 28) | (uint32_t)rank;
        } else if (valid) {
            pruned++;
            if (b == BIN_HUB) a.hub_act[i] = 0;
        }
        __syncthreads();   // fx is rewritten by the next pass
    }
    if (threadIdx.x < kNumBins && lcnt[threadIdx.x] > 0)
        lbase[threadIdx.x] = atomicAdd(&a.ctr->qcnt[a.round][threadIdx.x], lcnt[threadIdx.x]);
    __syncthreads();
    for (int k = threadIdx.x; k < nst; k += kBlock) {
        const uint32_t br = sbr[k];
        const int b = (int)(br >> 28);
        a.queue[a.qbase[b] + lbase[b] + (int64_t)(br & 0x0FFFFFFFu)] = sv[k];
    }
    long long pw = group_sum_ll<kWave>((long long)pruned);
    if (lane == 0) spr[w] = (unsigned long long)pw;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int q = 0; q < kBlock / kWave; q++) tot += spr[q];
        if (tot) atomicAdd(&a.ctr->st[blockIdx.x % kStripes].pruned, tot);
    }
}

// Logits of given feature rows (test hook of the inference kernel).
__global__ void __launch_bounds__(kBlock) k_gate_eval(GateNet net, const float *x, int64_t rows, float *logit) {
    __shared__ float sb1[kGateHidden], sb2[kGateHidden], sw3[kGateHidden];
    __shared__ uint16_t fx[kBlock / kWave][kWave][kGateFeatures];
    load_biases(net, sb1, sb2, sw3);
    NetRegs r;
    load_net(net, r);
    const int w = threadIdx.x / kWave, lane = lane_id();
    __syncthreads();
    for (int64_t t0 = blockIdx.x * (int64_t)kBlock; t0 < rows; t0 += (int64_t)gridDim.x * kBlock) {
        int64_t t = t0 + threadIdx.x;
#pragma unroll
        for (int f = 0; f < kGateFeatures; f++) fx[w][lane][f] = t < rows ? bf16_bits(x[t * kGateFeatures + f]) : 0;
        __syncthreads();
        float z = mlp_rows64(r, fx[w], sb1, sb2, sw3, net.b3);
        if (t < rows) logit[t] = z;
        __syncthreads();
    }
}

// ------------------------------------------------------------- training

constexpr int kR = kMlpRowsPerBlock;  // rows per block, one thread per row
constexpr int kH = kGateHidden;
constexpr int kF = kGateFeatures;
constexpr int kPad = kH + 1;         // row stride of the per-row LDS arrays

__device__ __forceinline__ float softplus_f(float t) { return (t > 0.0f ? t : 0.0f) + log1pf(expf(-fabsf(t))); }
__device__ __forceinline__ float sigmoid_f(float t) {
    return t >= 0.0f ? 1.0f / (1.0f + expf(-t)) : expf(t) / (1.0f + expf(t));
}

// One block = kR rows.  Phase A: thread r runs row r forward and backward to
// the hidden layers' deltas (kept in LDS).  Phase B: thread t sums, over the
// block's rows, the gradient entries of hidden unit t (column t of W2, row t
// of W1, b1[t], b2[t], w3[t]; thread 0 also b3), and writes the block's
// partial gradient in the parameter layout.
__global__ void __launch_bounds__(kR) k_mlp_grad(const float *params, const float *x, const uint8_t *y,
                                                 int64_t rows, float pw, float inv_b, float *part,
                                                 double *part_loss) {
    __shared__ float sW2[kH][kH];
    __shared__ float sW1[kH][kF];
    __shared__ float sb1[kH], sb2[kH], sw3[kH];
    __shared__ float sx[kR][kF];
    __shared__ float sh1[kR][kPad], sh2[kR][kPad], sd2[kR][kPad], sd1[kR][kPad];
    __shared__ float sdz[kR], sloss[kR];
    const int tid = threadIdx.x;
    for (int k = tid; k < kH * kH; k += kR) sW2[k / kH][k % kH] = params[kPW2 + k];
    for (int k = tid; k < kH * kF; k += kR) sW1[k / kF][k % kF] = params[kPW1 + k];
    for (int k = tid; k < kH; k += kR) {
        sb1[k] = params[kPB1 + k];
        sb2[k] = params[kPB2 + k];
        sw3[k] = params[kPW3 + k];
    }
    const float b3 = params[kPB3];
    const int64_t row = (int64_t)blockIdx.x * kR + tid;
    const bool valid = row < rows;
#pragma unroll
    for (int f = 0; f < kF; f++) sx[tid][f] = valid ? x[row * kF + f] : 0.0f;
    __syncthreads();
    // ---- phase A
    for (int h = 0; h < kH; h++) {
        float s = 0.0f;
#pragma unroll
        for (int f = 0; f < kF; f++) s += sW1[h][f] * sx[tid][f];
        float a1 = s + sb1[h];
        sh1[tid][h] = a1 > 0.0f ? a1 : 0.0f;
    }
    float z = 0.0f;
    for (int o = 0; o < kH; o++) {
        float s = 0.0f;
        for (int h = 0; h < kH; h++) s += sW2[o][h] * sh1[tid][h];
        float a2 = s + sb2[o];
        float h2 = a2 > 0.0f ? a2 : 0.0f;
        sh2[tid][o] = h2;
        z += sw3[o] * h2;
    }
    z += b3;
    float yr = valid && y[row] ? 1.0f : 0.0f;
    float dz = 0.0f, loss = 0.0f;
    if (valid) {
        loss = pw * yr * softplus_f(-z) + (1.0f - yr) * softplus_f(z);
        dz = (sigmoid_f(z) * (pw * yr + 1.0f - yr) - pw * yr) * inv_b;
    }
    sdz[tid] = dz;
    sloss[tid] = loss;
    for (int o = 0; o < kH; o++) sd2[tid][o] = sh2[tid][o] > 0.0f ? dz * sw3[o] : 0.0f;
    for (int h = 0; h < kH; h++) {
        float s = 0.0f;
        for (int o = 0; o < kH; o++) s += sW2[o][h] * sd2[tid][o];
        sd1[tid][h] = sh1[tid][h] > 0.0f ? s : 0.0f;
    }
    __syncthreads();
    // ---- phase B: hidden unit t = tid
    const int t = tid;
    float *pp = part + (int64_t)blockIdx.x * kGateParams;
    float acc[kH];
#pragma unroll
    for (int o = 0; o < kH; o++) acc[o] = 0.0f;
    float g1[kF] = {0, 0, 0, 0, 0, 0, 0, 0};
    float db1 = 0.0f, db2 = 0.0f, dw3 = 0.0f, db3 = 0.0f;
    for (int r = 0; r < kR; r++) {
        float hv = sh1[r][t];
#pragma unroll
        for (int o = 0; o < kH; o++) acc[o] += sd2[r][o] * hv;   // dW2[o][t]
        float d1 = sd1[r][t];
#pragma unroll
        for (int f = 0; f < kF; f++) g1[f] += d1 * sx[r][f];      // dW1[t][f]
        db1 += d1;
        db2 += sd2[r][t];
        dw3 += sdz[r] * sh2[r][t];
        db3 += sdz[r];
    }
#pragma unroll
    for (int o = 0; o < kH; o++) pp[kPW2 + o * kH + t] = acc[o];
#pragma unroll
    for (int f = 0; f < kF; f++) pp[kPW1 + t * kF + f] = g1[f];
    pp[kPB1 + t] = db1;
    pp[kPB2 + t] = db2;
    pp[kPW3 + t] = dw3;
    if (t == 0) {
        pp[kPB3] = db3;
        double L = 0.0;
        for (int r = 0; r < kR; r++) L += (double)sloss[r];
        part_loss[blockIdx.x] = L * (double)inv_b;
    }
}

// Sum of the blocks' partial gradients (in block order), then one Adam step
// (beta1 0.9, beta2 0.999, eps 1e-8) or the gradient itself.
__global__ void __launch_bounds__(kBlock) k_mlp_reduce(const float *part, const double *part_loss, int nblocks,
                                                       float *params, float *m, float *v, int adam, float lr,
                                                       float c1, float c2, float *grad, double *loss) {
    int k = blockIdx.x * kBlock + threadIdx.x;
    if (k < kGateParams) {
        float g = 0.0f;
        for (int b = 0; b < nblocks; b++) g += part[(int64_t)b * kGateParams + k];
        if (adam) {
            float mk = 0.9f * m[k] + 0.1f * g;
            float vk = 0.999f * v[k] + 0.001f * (g * g);
            m[k] = mk;
            v[k] = vk;
            float mh = mk / c1, vh = vk / c2;
            params[k] -= lr * mh / (sqrtf(vh) + 1e-8f);
        } else {
            grad[k] = g;
        }
    }
    if (k == 0 && loss) {
        double L = 0.0;
        for (int b = 0; b < nblocks; b++) L += part_loss[b];
        *loss += L;
    }
}

inline unsigned grid_cap(int64_t units, int64_t cap) {
    if (units < 1) units = 1;
    return (unsigned)(units < cap ? units : cap);
}

}  // namespace

void launch_gate(const MoveArgs &a, const GateNet &net, float theta_logit, int64_t cap, hipStream_t s) {
    if (cap == 0) return;
    // the candidates (at most cap) are split over the grid in equal ranges of
    // at most kGateSpan
    int64_t blocks = (cap + kBlock - 1) / kBlock;
    if (blocks > 1024) blocks = 1024;
    if (blocks < (cap + kGateSpan - 1) / kGateSpan) blocks = (cap + kGateSpan - 1) / kGateSpan;
    k_gate<<<(unsigned)blocks, kBlock, 0, s>>>(a, net, theta_logit);
}

void launch_gate_eval(const GateNet &net, const float *x, int64_t rows, float *logit, hipStream_t s) {
    if (rows == 0) return;
    k_gate_eval<<<grid_cap((rows + kBlock - 1) / kBlock, 4096), kBlock, 0, s>>>(net, x, rows, logit);
}

void launch_mlp_grad(const float *params, const float *x, const uint8_t *y, int64_t rows, float pos_weight,
                     float inv_batch, float *part, double *part_loss, hipStream_t s) {
    if (rows == 0) return;
    unsigned nb = (unsigned)((rows + kR - 1) / kR);
    k_mlp_grad<<<nb, kR, 0, s>>>(params, x, y, rows, pos_weight, inv_batch, part, part_loss);
}

void launch_mlp_reduce(const float *part, const double *part_loss, int nblocks, float *params, float *m, float *v,
                       bool adam, float lr, float c1, float c2, float *grad, double *loss, hipStream_t s) {
    k_mlp_reduce<<<(kGateParams + kBlock - 1) / kBlock, kBlock, 0, s>>>(part, part_loss, nblocks, params, m, v,
                                                                        adam ? 1 : 0, lr, c1, c2, grad, loss);
}

}  // namespace gsp
