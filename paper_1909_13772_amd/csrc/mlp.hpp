// mlp.hpp -- learned relaxation-time closure: a 7 -> 32 -> 32 -> 1 MLP per
// cell, evaluated by one wavefront for its 64 cells with bf16 matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulate).
//
// The paper lets the relaxation rate vary per cell, read from a field or set
// by a turbulence model (Sec. 5.1.1); here a small network predicts the
// correction tau - tau0 = softplus(o) from the cell's non-equilibrium stress
// and density.  Inputs x_k = (raw_k - mean_k) * inv_std_k with raw =
// (Pi_xx, Pi_yy, Pi_zz, Pi_xy, Pi_xz, Pi_yz, rho - 1); h1 = GELU(W1 x + b1),
// h2 = GELU(W2 h1 + b2), o = w3 . h2 + b3, GELU with the exact erf.  GEMM
// operands (weights, x, h1, h2) are rounded to bf16 (nearest even); sums,
// biases and activations are FP32.
//
// Matrix-core layout (32x32x16 bf16): A operand lane l = row l % 32, k
// 8 (l / 32) + 0..7; B operand lane l = column l % 32, same k; result lane l =
// column l % 32, rows 8 (j / 4) + 4 (l / 32) + j % 4 for its 16 registers j.
// Each layer computes hidden x cells (transposed) so a lane keeps the column
// of its own cell: tile A holds cells 0..31 (fed by lanes 0..31 through k
// 0..7), tile B cells 32..63 (fed by lanes 32..63 through k 8..15), so no
// data moves between lanes before the last layer.  Layer 2 consumes layer 1's
// registers directly; the k order this implies is folded into the layout of
// W2 prepared on the host (MlpDev).
#pragma once

#include "lattice.hpp"
#include "wlb_internal.hpp"

namespace wlb {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

// Device copy of the network, laid out per lane (built by mlp_prepare).
struct MlpDev {
    float mean[8];
    float istd[8];
    uint16_t w1[64][8];     // layer-1 A operand per lane (bf16 bits)
    uint16_t w2[2][64][8];  // layer-2 A operand per k-chunk and lane
    float b1[2][16];        // bias of result register j for lane half h
    float b2[2][16];
    float w3[2][16];        // bf16-rounded output weights per register
    float b3;
    float pad[7];
};

// Host-side: hidden unit held in result register j by lane half h.
__host__ __device__ constexpr int mlp_unit(int j, int h) { return 8 * (j / 4) + 4 * h + (j % 4); }

__device__ __forceinline__ uint16_t bf16_bits(float v)
{
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0x007fffffu) ? 0x40u : 0u));
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_round(float v) { return __uint_as_float((uint32_t)bf16_bits(v) << 16); }

__device__ __forceinline__ float gelu_erf(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ bf16x8_t load_bf16x8(const uint16_t *p)
{
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    bf16x8_t r;
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        r[2 * t] = __builtin_bit_cast(__bf16, (uint16_t)(w[t] & 0xffffu));
        r[2 * t + 1] = __builtin_bit_cast(__bf16, (uint16_t)(w[t] >> 16));
    }
    return r;
}

__device__ __forceinline__ bf16x8_t pack_bf16x8(const float *v)
{
    bf16x8_t r;
#pragma unroll
    for (int t = 0; t < 8; ++t) r[t] = __builtin_bit_cast(__bf16, bf16_bits(v[t]));
    return r;
}

// Wave-collective forward pass: every lane of the wavefront must call it
// (inactive lanes pass zeros).  x[7] are the standardised features of the
// lane's own cell.  Returns the network output o for the lane's cell.
__device__ __forceinline__ float mlp_forward_wave(const MlpDev *__restrict__ P, const float x[7])
{
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5;
    float xv[8];
#pragma unroll
    for (int t = 0; t < 7; ++t) xv[t] = x[t];
    xv[7] = 0.f;
    const bf16x8_t xb = pack_bf16x8(xv);
    bf16x8_t zero;
#pragma unroll
    for (int t = 0; t < 8; ++t) zero[t] = __builtin_bit_cast(__bf16, (uint16_t)0);
    const bf16x8_t bA = h ? zero : xb;
    const bf16x8_t bB = h ? xb : zero;
    const bf16x8_t w1 = load_bf16x8(P->w1[lane]);
    f32x16_t cA = {}, cB = {};
    cA = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1, bA, cA, 0, 0, 0);
    cB = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1, bB, cB, 0, 0, 0);
    float gA[16], gB[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const float b = P->b1[h][j];
        gA[j] = gelu_erf(cA[j] + b);
        gB[j] = gelu_erf(cB[j] + b);
    }
    f32x16_t dA = {}, dB = {};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const bf16x8_t w2 = load_bf16x8(P->w2[c][lane]);
        dA = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w2, pack_bf16x8(gA + 8 * c), dA, 0, 0, 0);
        dB = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w2, pack_bf16x8(gB + 8 * c), dB, 0, 0, 0);
    }
    float pA = 0.f, pB = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const float b = P->b2[h][j], w = P->w3[h][j];
        pA += w * bf16_round(gelu_erf(dA[j] + b));
        pB += w * bf16_round(gelu_erf(dB[j] + b));
    }
    // lane l < 32 owns cell l (tile A), lane l >= 32 owns cell l (tile B);
    // the other half of each dot product sits in lane l ^ 32.
    const float send = h ? pA : pB;
    const float recv = __shfl_xor(send, 32, 64);
    return (h ? pB : pA) + recv + P->b3;
}

__device__ __forceinline__ float softplus_f(float o) { return o > 20.f ? o : log1pf(expf(o)); }

}  // namespace wlb
