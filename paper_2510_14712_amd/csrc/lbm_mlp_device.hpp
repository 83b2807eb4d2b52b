// Wave-level inference of the 2 -> 64 -> 64 -> 3 equation-of-state surrogate
// without LDS.  One wavefront evaluates 64 samples (one per lane).
//
// The hidden layer is computed transposed, Z2^T = W2 H1^T, with
// v_mfma_f32_32x32x16_bf16: A = W2 (rows: output neurons, loaded as 8
// contiguous BF16 per lane), B = H1^T (rows: input neurons, columns: samples).
// For the B operand lane l holds input neurons 16 ks + 8 (l / 32) + j of
// samples 32 nt + l % 32, so each lane evaluates its own first-layer
// activations; no transpose through memory is needed.  The accumulator gives
// lane l the output neurons 32 mt + 8 (v / 4) + 4 (l / 32) + v % 4 of the same
// samples; the output layer is a per-lane partial dot product completed with
// the partner lane l ^ 32.
#pragma once

#include "lbm_device.hpp"

namespace lbm {
namespace mlp {

constexpr int H = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 128, OFF_W2 = 192, OFF_B2 = 4288, OFF_W3 = 4352, OFF_B3 = 4544;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// hidden activation: ReLU, max(z, 0), taken on the bit pattern: a set sign bit reads as a negative
// integer and gives +0, a positive value passes unchanged.  One integer max
// per value; the float max would first quiet its input (a second
// instruction per value on matrix-core results).  Differs from fmaxf only
// for a NaN input, which the residual check sends to the fallback anyway.
__device__ __forceinline__ float relu(float z) { return __int_as_float(max(__float_as_int(z), 0)); }

// ReLU of two BF16 values packed in a word, as a 16-bit integer max with 0
// on each half.  Rounding to BF16 is monotone and keeps the sign, so this
// equals rounding relu(a), relu(b): bit for bit, also for -0 and NaN.
typedef short s16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t p) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, p), (s16x2){0, 0}));
}

__device__ __forceinline__ __bf16 to_bf16(float v) { return __builtin_bit_cast(__bf16, bf16_hw(v)); }

__device__ __forceinline__ void normalise(const float *norm, float rho, float e, float &x0, float &x1) {
    x0 = 2.0f * (rho - norm[0]) / (norm[1] - norm[0]) - 1.0f;
    x1 = 2.0f * (e - norm[2]) / (norm[3] - norm[2]) - 1.0f;
}

// Parameter pointers of one forward pass: the small layers may live in LDS,
// the 64 x 64 hidden weights are read as BF16 (w2b, rows of w2_ld elements,
// global memory or LDS) or rounded on the fly from FP32 (w2b null: w2).
struct Net {
    const float *w1, *b1;  // [64][2], [64]
    const uint16_t *w2b;   // [64][w2_ld] BF16, row-major [out][in], or null
    const float *w2;       // [64][64] FP32 (when w2b is null)
    const float *b2, *w3, *b3;  // [64], [NOUT][64], [NOUT]
    int w2_ld;
};
__device__ __forceinline__ Net net_of(const float *P, const uint16_t *W2b) {
    return Net{P + OFF_W1, P + OFF_B1, W2b, P + OFF_W2, P + OFF_B2, P + OFF_W3, P + OFF_B3, H};
}

// Returns the normalised outputs 0..NOUT-1 of this lane's sample.  Every lane
// of the wavefront must call with uniform control flow.  The 32-sample halves
// of the wavefront go through the hidden layer one after the other and each
// k-step's B operand is formed just before its MFMA, which keeps the live
// registers low.  HALVES = 1 evaluates only the samples of lanes 0..31 (the
// outputs of lanes 32..63 are left unset).
template <int NOUT, int HALVES = 2>
__device__ __forceinline__ void forward_wave(float x0, float x1, const Net &p, float y[NOUT]) {
    static_assert(HALVES == 1 || HALVES == 2, "one or two 32-sample halves");
    const int lane = threadIdx.x & 63;
    const int hh = lane >> 5, c = lane & 31;
    // byte offset of this lane's A-operand row segment in the BF16 weights
    // (uniform base + 32-bit lane offset + constant per (mt, ks))
    const unsigned a_off = (unsigned)(c * p.w2_ld + 8 * hh) * 2u;
#pragma unroll
    for (int nt = 0; nt < HALVES; nt++) {
        // inputs of the sample this lane serves in the B operand
        const float xs0 = __shfl(x0, 32 * nt + c, 64), xs1 = __shfl(x1, 32 * nt + c, 64);
        f32x16 acc[2];
#pragma unroll
        for (int mt = 0; mt < 2; mt++)
#pragma unroll
            for (int v = 0; v < 16; v++) acc[mt][v] = 0.0f;
#pragma unroll
        for (int ks = 0; ks < 4; ks++) {
            float hv[8];
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int k = 16 * ks + 8 * hh + j;
                hv[j] = relu(fmaf(p.w1[2 * k], xs0, fmaf(p.w1[2 * k + 1], xs1, p.b1[k])));
            }
            // two activations per convert
            uint4 bp;
            bp.x = bf16x2_hw(hv[0], hv[1]);
            bp.y = bf16x2_hw(hv[2], hv[3]);
            bp.z = bf16x2_hw(hv[4], hv[5]);
            bp.w = bf16x2_hw(hv[6], hv[7]);
            const bf16x8 b = __builtin_bit_cast(bf16x8, bp);
#pragma unroll
            for (int mt = 0; mt < 2; mt++) {
                bf16x8 a;
                if (p.w2b) {
                    const uint4 raw =
                        *(const uint4 *)((const char *)p.w2b + a_off + (unsigned)((32 * mt * p.w2_ld + 16 * ks) * 2));
                    a = __builtin_bit_cast(bf16x8, raw);
                } else {
                    const float *row = p.w2 + (32 * mt + c) * H + 16 * ks + 8 * hh;
#pragma unroll
                    for (int j = 0; j < 8; j++) a[j] = to_bf16(row[j]);
                }
                acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[mt], 0, 0, 0);
            }
            // keep the next k-step's parameter loads from being hoisted here:
            // bounds the live registers of the first layer to one k-step
            __builtin_amdgcn_sched_barrier(0);
        }
        float ys[NOUT];
#pragma unroll
        for (int k = 0; k < NOUT; k++) ys[k] = 0.0f;
#pragma unroll
        for (int mt = 0; mt < 2; mt++) {
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int o = 32 * mt + 8 * (v >> 2) + 4 * hh + (v & 3);
                const float h2 = relu(acc[mt][v] + p.b2[o]);
#pragma unroll
                for (int k = 0; k < NOUT; k++) ys[k] = fmaf(p.w3[k * H + o], h2, ys[k]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int k = 0; k < NOUT; k++) {
            ys[k] += __shfl_xor(ys[k], 32, 64);
            // lane l's own sample is 32 nt + c with nt = l / 32
            if (hh == nt) y[k] = ys[k] + p.b3[k];
        }
    }
}

// ---------------------------------------------------------------------------
// Both hidden layers on MFMA (the surrogate pass's form).  Layer 1 is the
// contraction of [w1_0, w1_1, b1] with [x0, x1, 1] padded to K = 16: one
// v_mfma_f32_32x32x16_bf16 per 32 neurons and 32 samples, its operands
// rounded to BF16.  Its accumulator gives lane l (h = l / 32) neurons
// 32 mt + 8 q + 4 h + r (q, r < 4) of its sample; the layer-2 B operand of
// k-step ks wants 8 consecutive k-indices 16 ks + 8 h + j.  Numbering the
// layer-2 inputs by
//   sigma(16 ks + 8 h + j) = 32 (ks / 2) + 8 (2 (ks % 2) + j / 4) + 4 h + j % 4
// makes that operand the accumulator entries 8 (ks % 2) + j of tile ks / 2,
// so no value crosses lanes; the A operand reads W2 with its columns in the
// same order (w2_perm_col).  Layer 2 starts its accumulators at b2.
__host__ __device__ constexpr int w2_perm_col(int k) {
    return 32 * ((k >> 4) >> 1) + 8 * (2 * ((k >> 4) & 1) + ((k & 7) >> 2)) + 4 * ((k >> 3) & 1) + (k & 3);
}
// per-lane layer-1 A operands (neurons 32 mt + l % 32 in lanes 0..31: their
// w1 row and bias; zero in lanes 32..63)
struct L1Ops {
    bf16x8 a[2];
};
__device__ __forceinline__ L1Ops l1_operands(const float *w1, const float *b1) {
    const int lane = threadIdx.x & 63, c = lane & 31;
    L1Ops o;
#pragma unroll
    for (int mt = 0; mt < 2; mt++) {
        uint4 u = {0u, 0u, 0u, 0u};
        if (lane < 32) {
            const int m = 32 * mt + c;
            u.x = bf16x2_hw(w1[2 * m], w1[2 * m + 1]);
            u.y = bf16x2_hw(b1[m], 0.0f);
        }
        o.a[mt] = __builtin_bit_cast(bf16x8, u);
    }
    return o;
}
// normalised outputs 0..NOUT-1 of this lane's sample; uniform control flow.
// p.w2b: BF16 W2 with permuted columns (row stride p.w2_ld elements).
template <int NOUT>
__device__ __forceinline__ void forward_wave_l1mfma(float x0, float x1, const Net &p, const L1Ops &l1, float y[NOUT]) {
    const int lane = threadIdx.x & 63;
    const int hh = lane >> 5, c = lane & 31;
    const unsigned a_off = (unsigned)(c * p.w2_ld + 8 * hh) * 2u;
#pragma unroll
    for (int nt = 0; nt < 2; nt++) {
        const float xs0 = __shfl(x0, 32 * nt + c, 64), xs1 = __shfl(x1, 32 * nt + c, 64);
        uint4 bu = {0u, 0u, 0u, 0u};
        if (hh == 0) {
            bu.x = bf16x2_hw(xs0, xs1);
            bu.y = bf16x2_hw(1.0f, 0.0f);
        }
        const bf16x8 b1 = __builtin_bit_cast(bf16x8, bu);
        f32x16 z1[2];
#pragma unroll
        for (int mt = 0; mt < 2; mt++) {
#pragma unroll
            for (int v = 0; v < 16; v++) z1[mt][v] = 0.0f;
            z1[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(l1.a[mt], b1, z1[mt], 0, 0, 0);
        }
        // layer 2, accumulators seeded with b2 of the output neurons
        f32x16 acc[2];
#pragma unroll
        for (int mt = 0; mt < 2; mt++)
#pragma unroll
            for (int v = 0; v < 16; v++) acc[mt][v] = p.b2[32 * mt + 8 * (v >> 2) + 4 * hh + (v & 3)];
#pragma unroll
        for (int ks = 0; ks < 4; ks++) {
            const int t = ks >> 1, o = 8 * (ks & 1);
            uint4 bp;
            bp.x = relu_bf16x2(bf16x2_hw(z1[t][o + 0], z1[t][o + 1]));
            bp.y = relu_bf16x2(bf16x2_hw(z1[t][o + 2], z1[t][o + 3]));
            bp.z = relu_bf16x2(bf16x2_hw(z1[t][o + 4], z1[t][o + 5]));
            bp.w = relu_bf16x2(bf16x2_hw(z1[t][o + 6], z1[t][o + 7]));
            const bf16x8 b = __builtin_bit_cast(bf16x8, bp);
#pragma unroll
            for (int mt = 0; mt < 2; mt++) {
                const uint4 raw =
                    *(const uint4 *)((const char *)p.w2b + a_off + (unsigned)((32 * mt * p.w2_ld + 16 * ks) * 2));
                acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, raw), b, acc[mt], 0, 0, 0);
            }
        }
        float ys[NOUT];
#pragma unroll
        for (int k = 0; k < NOUT; k++) ys[k] = 0.0f;
#pragma unroll
        for (int mt = 0; mt < 2; mt++)
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int o = 32 * mt + 8 * (v >> 2) + 4 * hh + (v & 3);
                const float h2 = relu(acc[mt][v]);
#pragma unroll
                for (int k = 0; k < NOUT; k++) ys[k] = fmaf(p.w3[k * H + o], h2, ys[k]);
            }
#pragma unroll
        for (int k = 0; k < NOUT; k++) {
            ys[k] += __shfl_xor(ys[k], 32, 64);
            if (hh == nt) y[k] = ys[k] + p.b3[k];
        }
    }
}

}  // namespace mlp
}  // namespace lbm
