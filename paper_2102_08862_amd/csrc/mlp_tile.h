// The triplet network on one tile of 16 triplets with the matrix cores:
// z = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 (12 features padded to 16, 64
// and 64 hidden units, BF16 weights and activations, FP32 accumulation).
//
// Each layer is computed transposed, H^T = W X^T, with
// v_mfma_f32_16x16x16_bf16 (A = a 16x16 weight tile held in registers, B =
// 16 triplets): lane l = 16 q + c holds column c (one triplet) and rows
// 4q..4q+3 of every tile, which is exactly the B-operand layout of the next
// layer, so activations never leave registers. The last layer (64 -> 1) is
// a dot product finished with two cross-lane shuffles. The stand-alone
// inference kernel and the pruned neighbour search share this code, so both
// produce the same logit for the same features.
#pragma once
#include "tpcca_internal.h"

namespace tpcca {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (finite values)
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline v4s pack4(uint16_t a, uint16_t b, uint16_t c, uint16_t d) {
    v4s r;
    r.x = (short)a;
    r.y = (short)b;
    r.z = (short)c;
    r.w = (short)d;
    return r;
}

// BF16 (round to nearest even, the hardware conversion) of two values,
// then relu on the packed halves as signed 16-bit integers (a BF16 with the
// sign bit set becomes +0, the rest keep their bits): for finite values this
// is f2bf(max(x, 0)); a NaN keeps its sign, as in the plain definition.
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef short v2s __attribute__((ext_vector_type(2)));
__device__ inline uint32_t relu_pk_bf16(float a, float b) {
    const v2f v = {a, b};
    const v2s h = __builtin_bit_cast(v2s, __builtin_convertvector(v, v2bf));
    const v2s z = {0, 0};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(h, z));
}
__device__ inline v4s relu_bf16x4(v4f d) {
    const uint2 u = make_uint2(relu_pk_bf16(d[0], d[1]), relu_pk_bf16(d[2], d[3]));
    return __builtin_bit_cast(v4s, u);
}

// Two packed BF16 pairs (features 4q..4q+3 of one triplet) as a B operand.
__device__ inline v4s pack4(uint2 v) {
    return pack4((uint16_t)(v.x & 0xffff), (uint16_t)(v.x >> 16), (uint16_t)(v.y & 0xffff), (uint16_t)(v.y >> 16));
}

// The network on one tile, with the weights from any source W providing
// a1(mt), c1(mt), a2(mt, ks), c2(mt), w3(mt) (4 FP32 values) and b3().
template <class Wt>
__device__ inline float mlp_logit(const Wt &W, v4s bx) {
    v4s h1[4];
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        h1[mt] = relu_bf16x4(__builtin_amdgcn_mfma_f32_16x16x16bf16_1k(W.a1(mt), bx, W.c1(mt), 0, 0, 0));
    }
    float part = 0.f;
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        v4f d = W.c2(mt);
#pragma unroll
        for (int ks = 0; ks < 4; ks++) d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(W.a2(mt, ks), h1[ks], d, 0, 0, 0);
        const v4f w3 = W.w3(mt);
        const v4s h = relu_bf16x4(d);
#pragma unroll
        for (int r = 0; r < 4; r++) part = __fmaf_rn(w3[r], bf2f((uint16_t)h[r]), part);
    }
    part = __fadd_rn(part, __shfl_xor(part, 16));
    part = __fadd_rn(part, __shfl_xor(part, 32));
    return __fadd_rn(part, W.b3());
}

// The network on nt <= 4 tiles at once (bx[t]: features of tile t): every
// weight operand is read once and used for all tiles, so few registers hold
// weights. Each tile's arithmetic is that of mlp_logit.
template <class Wt>
__device__ inline void mlp_logit4(const Wt &W, const v4s (&bx)[4], int nt, float (&z)[4]) {
    v4s h1[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        const v4s A = W.a1(mt);
        const v4f C = W.c1(mt);
#pragma unroll
        for (int t = 0; t < 4; t++) {
            if (t >= nt) break;
            h1[t][mt] = relu_bf16x4(__builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, bx[t], C, 0, 0, 0));
        }
    }
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        v4f d[4];
        const v4f C = W.c2(mt);
#pragma unroll
        for (int t = 0; t < 4; t++) d[t] = C;
#pragma unroll
        for (int ks = 0; ks < 4; ks++) {
            const v4s A = W.a2(mt, ks);
#pragma unroll
            for (int t = 0; t < 4; t++) {
                if (t >= nt) break;
                d[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, h1[t][ks], d[t], 0, 0, 0);
            }
        }
        const v4f w3 = W.w3(mt);
#pragma unroll
        for (int t = 0; t < 4; t++) {
            if (t >= nt) break;
            const v4s h = relu_bf16x4(d[t]);
#pragma unroll
            for (int r = 0; r < 4; r++) part[t] = __fmaf_rn(w3[r], bf2f((uint16_t)h[r]), part[t]);
        }
    }
    const float b3 = W.b3();
#pragma unroll
    for (int t = 0; t < 4; t++) {
        float p = part[t];
        p = __fadd_rn(p, __shfl_xor(p, 16));
        p = __fadd_rn(p, __shfl_xor(p, 32));
        z[t] = __fadd_rn(p, b3);
    }
}

// Loads from global memory (the weights are device buffers): explicit so that
// the compiler keeps global (not flat) loads when the pointer is opaque.
__device__ inline uint2 gload2(const void *p) {
    const unsigned long long v = *(__attribute__((address_space(1))) const unsigned long long *)p;
    return make_uint2((unsigned)v, (unsigned)(v >> 32));
}
__device__ inline v4f gload4f(const void *p) { return *(__attribute__((address_space(1))) const v4f *)p; }

// Weights read from memory where they are used (few registers; every
// operand of a lane is 8 or 16 contiguous bytes).
struct MlpStream {
    MlpDev W;
    int q, c;
    __device__ MlpStream(const MlpDev &w, int lane) : W(w), q(lane >> 4), c(lane & 15) {}
    __device__ v4s a1(int mt) const { return pack4(gload2(W.w1 + (16 * mt + c) * kMlpInP + 4 * q)); }
    __device__ v4s a2(int mt, int ks) const { return pack4(gload2(W.w2 + (16 * mt + c) * kMlpH + 16 * ks + 4 * q)); }
    __device__ v4f c1(int mt) const { return gload4f(W.b1 + 16 * mt + 4 * q); }
    __device__ v4f c2(int mt) const { return gload4f(W.b2 + 16 * mt + 4 * q); }
    __device__ v4f w3(int mt) const {
        const uint2 v = gload2(W.w3 + 16 * mt + 4 * q);
        return v4f{bf2f((uint16_t)(v.x & 0xffff)), bf2f((uint16_t)(v.x >> 16)), bf2f((uint16_t)(v.y & 0xffff)),
                   bf2f((uint16_t)(v.y >> 16))};
    }
    __device__ float b3() const { return *W.b3; }
};

// Weights held in registers (loaded once, for a kernel that only scores).
struct MlpTile {
    v4s A1[4], A2[4][4];
    v4f C1[4], C2[4], W3[4];
    float B3;

    __device__ void load(const MlpDev &W, int lane) {
        const MlpStream S(W, lane);
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            A1[mt] = S.a1(mt);
#pragma unroll
            for (int ks = 0; ks < 4; ks++) A2[mt][ks] = S.a2(mt, ks);
            C1[mt] = S.c1(mt);
            C2[mt] = S.c2(mt);
            W3[mt] = S.w3(mt);
        }
        B3 = S.b3();
    }
    __device__ v4s a1(int mt) const { return A1[mt]; }
    __device__ v4s a2(int mt, int ks) const { return A2[mt][ks]; }
    __device__ v4f c1(int mt) const { return C1[mt]; }
    __device__ v4f c2(int mt) const { return C2[mt]; }
    __device__ v4f w3(int mt) const { return W3[mt]; }
    __device__ float b3() const { return B3; }
    // Logit of the triplet in column (lane & 15); bx holds its features
    // 4q..4q+3. Every lane of a column returns the same value.
    __device__ float logit(v4s bx) const { return mlp_logit(*this, bx); }
};

}  // namespace tpcca
