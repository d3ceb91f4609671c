// Triplet network inference on the matrix cores over a list of triplets
// (the per-tile arithmetic and its register layout are in mlp_tile.h), and
// the training step of the same network.
#include "mlp_tile.h"

namespace tpcca {

// Logits of triplets [0, n): X is [n][16] BF16 (row-major), z out FP32.
__global__ __launch_bounds__(256) void k_mlp_infer(MlpDev W, const uint16_t *__restrict__ X,
                                                   const int32_t *n_dev, int32_t n_cap, float *__restrict__ z) {
    const int lane = threadIdx.x & 63;
    const int q = lane >> 4, c = lane & 15;
    MlpTile M;
    M.load(W, lane);
    const int n = n_dev ? min(*n_dev, n_cap) : n_cap;
    const int ntiles = (n + 15) >> 4;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int tile = wave; tile < ntiles; tile += nwaves) {
        const int t = tile * 16 + c;
        v4s bx = pack4(0, 0, 0, 0);
        if (t < n) bx = pack4(*reinterpret_cast<const uint2 *>(X + (int64_t)t * kMlpInP + 4 * q));
        const float zz = M.logit(bx);
        if (q == 0 && t < n) z[t] = zz;
    }
}

void launch_mlp_infer(const MlpDev &W, const uint16_t *X, const int32_t *n_dev, int32_t n_cap, float *z, int grid,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_infer, dim3(max(grid, 1)), dim3(256), 0, s, W, X, n_dev, n_cap, z);
}

// ------------------------------------------------------------ training
// One workgroup of kTrainWaves waves runs a whole step on a minibatch of
// n <= kMlpMaxBatch examples: every wave takes tiles of 16 examples,
// recomputes the forward pass in registers, and accumulates
//   dL/dw3 = sum dz h2, dL/db2 = sum dh2, dL/dW2 = dh2^T h1 (MFMA, K = examples),
//   dh1 = W2^T dh2 (MFMA, the register layout of dh2 is its B operand),
//   dL/db1 = sum dh1, dL/dW1 = dh1^T x (MFMA, K = examples),
// with dz = w (sigmoid(z) - y) / n, dh2 = dz w3 [h2 > 0], dh1 = (W2^T dh2)
// [h1 > 0]. Matrix operands are BF16, accumulation FP32. The two batch
// reductions read their operands through a per-wave LDS transpose; the
// waves' partial gradients are summed in LDS in a fixed wave order, then the same
// workgroup applies AdamW to the FP32 master parameters and rewrites the
// BF16 copies (or, gradient-only, writes the gradient out).
constexpr int kTrainWaves = 8;
constexpr int kOffW1 = 0, kOffB1 = 1024, kOffW2 = 1088, kOffB2 = 5184, kOffW3 = 5248, kOffB3 = 5312;

__device__ inline v4s lds4(const uint16_t *p) {
    const uint2 v = *reinterpret_cast<const uint2 *>(p);
    return pack4((uint16_t)(v.x & 0xffff), (uint16_t)(v.x >> 16), (uint16_t)(v.y & 0xffff), (uint16_t)(v.y >> 16));
}

__global__ __launch_bounds__(64 * kTrainWaves) void k_mlp_train(MlpTrainArgs T) {
    __shared__ uint16_t sW1[kMlpH * kMlpInP];
    __shared__ uint16_t sW2[kMlpH * kMlpH];
    __shared__ float sb1[kMlpH], sb2[kMlpH], sw3[kMlpH];
    __shared__ float sg[kMlpNParam];
    __shared__ __attribute__((aligned(16))) uint16_t sH1[kTrainWaves][kMlpH * 16];   // [unit][example]
    __shared__ __attribute__((aligned(16))) uint16_t sD2[kTrainWaves][kMlpH * 16];   // dh2, [unit][example]
    __shared__ __attribute__((aligned(16))) uint16_t sD1[kTrainWaves][kMlpH * 16];   // dh1, [unit][example]
    __shared__ __attribute__((aligned(16))) uint16_t sX[kTrainWaves][16 * 16];       // x, [feature][example]
    __shared__ float s_loss;
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63, q = lane >> 4, c = lane & 15;
    for (int i = tid; i < kMlpH * kMlpInP; i += blockDim.x) sW1[i] = T.w1[i];
    for (int i = tid; i < kMlpH * kMlpH; i += blockDim.x) sW2[i] = T.w2[i];
    for (int i = tid; i < kMlpH; i += blockDim.x) {
        sb1[i] = T.b1[i];
        sb2[i] = T.b2[i];
        sw3[i] = bf2f(T.w3[i]);
    }
    for (int i = tid; i < kMlpNParam; i += blockDim.x) sg[i] = 0.f;
    if (tid == 0) s_loss = 0.f;
    __syncthreads();
    const float b3 = *T.b3;
    const int n = T.n;
    const float inv_n = 1.0f / (float)max(n, 1);
    const int ntiles = (n + 15) >> 4;
    const int per_wave = (ntiles + kTrainWaves - 1) / kTrainWaves;
    v4f aW2[4][4], aW1[4];
    float g3[4][4], gb2[4][4], gb1[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        aW1[i] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < 4; j++) {
            aW2[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
            g3[i][j] = gb2[i][j] = gb1[i][j] = 0.f;
        }
    }
    float gb3 = 0.f, loss = 0.f;
    uint16_t *h1s = sH1[w], *d2s = sD2[w], *d1s = sD1[w], *xs = sX[w];
    for (int it = 0; it < per_wave; it++) {
        const int tile = w + it * kTrainWaves;
        const int t = tile * 16 + c;
        const bool valid = tile < ntiles && t < n;
        // x tile: B operand of layer 1, and x^T into LDS for dL/dW1
        uint16_t xv[4] = {0, 0, 0, 0};
        if (valid) {
            const uint2 v = *reinterpret_cast<const uint2 *>(T.X + (int64_t)t * kMlpInP + 4 * q);
            xv[0] = (uint16_t)(v.x & 0xffff);
            xv[1] = (uint16_t)(v.x >> 16);
            xv[2] = (uint16_t)(v.y & 0xffff);
            xv[3] = (uint16_t)(v.y >> 16);
        }
#pragma unroll
        for (int e = 0; e < 4; e++) xs[(4 * q + e) * 16 + c] = xv[e];
        const v4s bx = pack4(xv[0], xv[1], xv[2], xv[3]);
        // forward
        v4s h1b[4];
        bool m1[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            const v4s A = lds4(sW1 + (16 * mt + c) * kMlpInP + 4 * q);
            v4f C = {sb1[16 * mt + 4 * q], sb1[16 * mt + 4 * q + 1], sb1[16 * mt + 4 * q + 2], sb1[16 * mt + 4 * q + 3]};
            const v4f d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, bx, C, 0, 0, 0);
            uint16_t hv[4];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                m1[mt][r] = d[r] > 0.f;
                hv[r] = f2bf(fmaxf(d[r], 0.f));
                h1s[(16 * mt + 4 * q + r) * 16 + c] = hv[r];
            }
            h1b[mt] = pack4(hv[0], hv[1], hv[2], hv[3]);
        }
        float h2[4][4];
        bool m2[4][4];
        float part = 0.f;
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            v4f d = {sb2[16 * mt + 4 * q], sb2[16 * mt + 4 * q + 1], sb2[16 * mt + 4 * q + 2], sb2[16 * mt + 4 * q + 3]};
#pragma unroll
            for (int ks = 0; ks < 4; ks++)
                d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lds4(sW2 + (16 * mt + c) * kMlpH + 16 * ks + 4 * q),
                                                               h1b[ks], d, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; r++) {
                m2[mt][r] = d[r] > 0.f;
                h2[mt][r] = bf2f(f2bf(fmaxf(d[r], 0.f)));
                part = __fmaf_rn(sw3[16 * mt + 4 * q + r], h2[mt][r], part);
            }
        }
        part = __fadd_rn(part, __shfl_xor(part, 16));
        part = __fadd_rn(part, __shfl_xor(part, 32));
        const float z = __fadd_rn(part, b3);
        float dz = 0.f;
        if (valid) {
            const float yv = T.Y[t];
            const float wgt = yv > 0.5f ? T.pos_weight : 1.0f;
            const float sig = 1.0f / (1.0f + __expf(-z));
            dz = wgt * (sig - yv) * inv_n;
            if (q == 0) {
                const float sp = z > 0.f ? z + log1pf(__expf(-z)) : log1pf(__expf(z));
                loss += wgt * (sp - yv * z);
                gb3 += dz;
            }
        }
        // dh2 (registers: unit 16 mt + 4 q + r, example c) and its BF16 copy
        v4s d2b[4];
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            uint16_t dv[4];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const float g = m2[mt][r] ? dz * sw3[16 * mt + 4 * q + r] : 0.f;
                g3[mt][r] += dz * h2[mt][r];
                gb2[mt][r] += g;
                dv[r] = f2bf(g);
                d2s[(16 * mt + 4 * q + r) * 16 + c] = dv[r];
            }
            d2b[mt] = pack4(dv[0], dv[1], dv[2], dv[3]);
        }
        // dh1 = W2^T dh2, masked by h1 > 0
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4; ks++) {
                const int nn = 16 * ks + 4 * q;
                const v4s A = pack4(sW2[(nn + 0) * kMlpH + 16 * mt + c], sW2[(nn + 1) * kMlpH + 16 * mt + c],
                                    sW2[(nn + 2) * kMlpH + 16 * mt + c], sW2[(nn + 3) * kMlpH + 16 * mt + c]);
                d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, d2b[ks], d, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const float g = m1[mt][r] ? d[r] : 0.f;
                gb1[mt][r] += g;
                d1s[(16 * mt + 4 * q + r) * 16 + c] = f2bf(g);
            }
        }
        __syncthreads();
        // dL/dW2[n][k] += sum_ex dh2[n][ex] h1[k][ex]; dL/dW1[h][f] += sum_ex dh1[h][ex] x[ex][f]
#pragma unroll
        for (int nt = 0; nt < 4; nt++) {
            const v4s A = lds4(d2s + (16 * nt + c) * 16 + 4 * q);
#pragma unroll
            for (int kt = 0; kt < 4; kt++)
                aW2[nt][kt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, lds4(h1s + (16 * kt + c) * 16 + 4 * q),
                                                                         aW2[nt][kt], 0, 0, 0);
        }
        const v4s Bx = lds4(xs + c * 16 + 4 * q);
#pragma unroll
        for (int mt = 0; mt < 4; mt++)
            aW1[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lds4(d1s + (16 * mt + c) * 16 + 4 * q), Bx, aW1[mt],
                                                               0, 0, 0);
        __syncthreads();
    }
    // combine the waves' partial gradients in LDS in a fixed order (wave 0
    // writes, then waves 1..7 add theirs one after another), so that a step
    // is bit-reproducible and the gradient-only mode gives exactly the
    // gradient the update uses
    for (int i = 0; i < 4; i++)
        for (int r = 0; r < 4; r++) {
            float a3 = g3[i][r], ab2 = gb2[i][r], ab1 = gb1[i][r];
            for (int off = 1; off < 16; off <<= 1) {
                a3 = __fadd_rn(a3, __shfl_xor(a3, off));
                ab2 = __fadd_rn(ab2, __shfl_xor(ab2, off));
                ab1 = __fadd_rn(ab1, __shfl_xor(ab1, off));
            }
            g3[i][r] = a3;
            gb2[i][r] = ab2;
            gb1[i][r] = ab1;
        }
    for (int off = 1; off < 64; off <<= 1) {
        gb3 = __fadd_rn(gb3, __shfl_xor(gb3, off));
        loss = __fadd_rn(loss, __shfl_xor(loss, off));
    }
    for (int ww = 0; ww < kTrainWaves; ww++) {
        if (w == ww) {
            const bool first = ww == 0;
#pragma unroll
            for (int nt = 0; nt < 4; nt++)
#pragma unroll
                for (int kt = 0; kt < 4; kt++)
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        float &d = sg[kOffW2 + (16 * nt + 4 * q + r) * kMlpH + 16 * kt + c];
                        d = first ? aW2[nt][kt][r] : __fadd_rn(d, aW2[nt][kt][r]);
                    }
#pragma unroll
            for (int mt = 0; mt < 4; mt++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    float &d = sg[kOffW1 + (16 * mt + 4 * q + r) * kMlpInP + c];
                    d = first ? aW1[mt][r] : __fadd_rn(d, aW1[mt][r]);
                    if (c == 0) {
                        const int u = 16 * mt + 4 * q + r;
                        float &d3 = sg[kOffW3 + u], &d2 = sg[kOffB2 + u], &d1 = sg[kOffB1 + u];
                        d3 = first ? g3[mt][r] : __fadd_rn(d3, g3[mt][r]);
                        d2 = first ? gb2[mt][r] : __fadd_rn(d2, gb2[mt][r]);
                        d1 = first ? gb1[mt][r] : __fadd_rn(d1, gb1[mt][r]);
                    }
                }
            if (lane == 0) {
                sg[kOffB3] = first ? gb3 : __fadd_rn(sg[kOffB3], gb3);
                s_loss = first ? loss : __fadd_rn(s_loss, loss);
            }
        }
        __syncthreads();
    }
    __syncthreads();
    if (T.loss_out && tid == 0) *T.loss_out = s_loss * inv_n;
    if (!T.update) {
        for (int i = tid; i < kMlpNParam; i += blockDim.x) T.grad_out[i] = sg[i];
        return;
    }
    // AdamW on the FP32 master parameters (decoupled weight decay on weights only)
    const int step = *T.step + 1;
    const float bc1 = 1.0f - powf(T.beta1, (float)step), bc2 = 1.0f - powf(T.beta2, (float)step);
    for (int i = tid; i < kMlpNParam; i += blockDim.x) {
        const float g = sg[i];
        const float m = T.beta1 * T.adam_m[i] + (1.0f - T.beta1) * g;
        const float v = T.beta2 * T.adam_v[i] + (1.0f - T.beta2) * g * g;
        T.adam_m[i] = m;
        T.adam_v[i] = v;
        const bool is_w = (i < kOffB1) || (i >= kOffW2 && i < kOffB2) || (i >= kOffW3 && i < kOffB3);
        const bool pad = i < kOffB1 && (i % kMlpInP) >= kMlpIn;
        float pv = T.master[i];
        if (is_w) pv -= T.lr * T.weight_decay * pv;
        pv -= T.lr * (m / bc1) / (sqrtf(v / bc2) + T.eps);
        if (pad) pv = 0.f;
        T.master[i] = pv;
        if (i < kOffB1) T.w1[i] = f2bf(pv);
        else if (i < kOffW2) T.b1[i - kOffB1] = pv;
        else if (i < kOffB2) T.w2[i - kOffW2] = f2bf(pv);
        else if (i < kOffW3) T.b2[i - kOffB2] = pv;
        else if (i < kOffB3) T.w3[i - kOffW3] = f2bf(pv);
        else *T.b3 = pv;
    }
    if (tid == 0) *T.step = step;
}

void launch_mlp_train(const MlpTrainArgs &t, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(64 * kTrainWaves), 0, s, t);
}

}  // namespace tpcca
