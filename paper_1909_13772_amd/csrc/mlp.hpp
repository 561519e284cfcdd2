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
struct alignas(16) MlpDev {
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
static_assert(sizeof(MlpDev) % 16 == 0, "MlpDev is copied in 16-byte units");

// Copy the network into a workgroup's shared memory (all threads call it).
__device__ __forceinline__ void mlp_stage(MlpDev *dst, const void *src)
{
    const uint4 *s = static_cast<const uint4 *>(src);
    uint4 *d = reinterpret_cast<uint4 *>(dst);
    for (int k = threadIdx.x; k < (int)(sizeof(MlpDev) / 16); k += blockDim.x) d[k] = s[k];
    __syncthreads();
}

// Host-side: hidden unit held in result register j by lane half h.
__host__ __device__ constexpr int mlp_unit(int j, int h) { return 8 * (j / 4) + 4 * h + (j % 4); }

// Round to bf16, nearest even (the hardware conversion of gfx950; a NaN
// stays a quiet NaN).
__device__ __forceinline__ uint16_t bf16_bits(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
__device__ __forceinline__ float bf16_round(float v) { return __uint_as_float((uint32_t)bf16_bits(v) << 16); }

// Phi(-|z|) = erfc(|z| / sqrt 2) / 2 without branches, as t * e: erfc(u)
// for u >= 0 from the Chebyshev-fitted form t exp(-u^2 + P(t)), t = 1 / (1 +
// u / 2), of Numerical Recipes (2nd ed., Sec. 6.2), whose fractional error is
// below 1.2e-7 for every u >= 0.  The exponential is the hardware base-2 one:
// P's coefficients below are NR's times log2(e), with the factor 1/2 folded
// into the constant term (-1), and u^2 log2(e) = (|z| sqrt(log2(e) / 2))^2.
// One reciprocal, one exp2 and a degree-9 polynomial, the same for every
// lane.  t and e are returned apart so that GELU can fold |z| into t.
struct HalfErfc {
    float t, e;
};
__device__ __forceinline__ HalfErfc half_erfc_parts(float z)
{
    const float az = fabsf(z);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.35355339059327376f, az, 1.0f));  // 1 / (1 + u/2), u = |z|/sqrt2
    const float v = az * 0.8493218003f;
    float p = 2.465172979e-01f;
    p = fmaf(p, t, -1.186114945e+00f);
    p = fmaf(p, t, 2.147474464e+00f);
    p = fmaf(p, t, -1.637753152e+00f);
    p = fmaf(p, t, 4.023215817e-01f);
    p = fmaf(p, t, -2.687568603e-01f);
    p = fmaf(p, t, 1.396300565e-01f);
    p = fmaf(p, t, 5.397006155e-01f);
    p = fmaf(p, t, 1.442729204e+00f);
    p = fmaf(p, t, -2.825748218e+00f);
    return HalfErfc{t, __builtin_amdgcn_exp2f(fmaf(-v, v, p))};
}

// Standard normal CDF: Phi(z) = 1 - Phi(-z) for z >= 0.
__device__ __forceinline__ float norm_cdf(float z)
{
    const HalfErfc h = half_erfc_parts(z);
    const float half_erfc = h.t * h.e;
    return z >= 0.f ? 1.0f - half_erfc : half_erfc;
}

// GELU with the exact Gaussian CDF, z Phi(z) = max(z, 0) - |z| Phi(-|z|):
// one multiply, one max and one fused multiply-add after the CDF's parts.
__device__ __forceinline__ float gelu_erf(float z)
{
    const HalfErfc h = half_erfc_parts(z);
    return fmaf(-(fabsf(z) * h.t), h.e, fmaxf(z, 0.f));
}

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
    for (int t = 0; t < 8; ++t) r[t] = (__bf16)v[t];
    return r;
}

// Sixteen floats from a 16-byte aligned address (four 128-bit reads).
__device__ __forceinline__ f32x16_t load_f32x16(const float *p)
{
    const float4 *q = reinterpret_cast<const float4 *>(p);
    f32x16_t r;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float4 v = q[k];
        r[4 * k] = v.x;
        r[4 * k + 1] = v.y;
        r[4 * k + 2] = v.z;
        r[4 * k + 3] = v.w;
    }
    return r;
}

// Layers 1-3 for one 32-cell tile: b1op is the layer-1 B operand (the
// lane's features in its k half, zeros in the other), the result is this
// lane's half of the output dot product for the tile's cell in its column.
// The biases enter as the accumulators' initial values.
__device__ __forceinline__ float mlp_tile(const MlpDev *__restrict__ P, int lane, int h, const bf16x8_t b1op)
{
    // An opaque zero in the weight indices keeps these reads inside the
    // tile loop: hoisted, they would hold ~60 registers for the whole sweep.
    int z = 0;
    asm volatile("" : "+v"(z));
    h += z;
    f32x16_t c = load_f32x16(P->b1[h]);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load_bf16x8(P->w1[lane]), b1op, c, 0, 0, 0);
    bf16x8_t g[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        float v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            v[t] = gelu_erf(c[8 * q + t]);
            // evaluate the activations a few at a time: all sixteen in
            // flight need ~80 registers for their temporaries
            if (t % 4 == 3) __builtin_amdgcn_sched_barrier(0);
        }
        g[q] = pack_bf16x8(v);
    }
    f32x16_t d = load_f32x16(P->b2[h]);
#pragma unroll
    for (int q = 0; q < 2; ++q) d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load_bf16x8(P->w2[q][lane]), g[q], d, 0, 0, 0);
    const f32x16_t w3 = load_f32x16(P->w3[h]);
    float part = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        part = fmaf(w3[j], bf16_round(gelu_erf(d[j])), part);
        if (j % 4 == 3) __builtin_amdgcn_sched_barrier(0);
    }
    return part;
}

// Wave-collective forward pass: every lane of the wavefront must call it
// (inactive lanes pass zeros).  x[7] are the standardised features of the
// lane's own cell.  Returns the network output o for the lane's cell.  The
// two 32-cell tiles are evaluated one after the other so their
// accumulators share registers.
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
    float part[2];
#pragma unroll 1
    for (int tile = 0; tile < 2; ++tile) part[tile] = mlp_tile(P, lane, h, (h == tile) ? xb : zero);
    const float pA = part[0], pB = part[1];
    // lane l < 32 owns cell l (tile A), lane l >= 32 owns cell l (tile B);
    // the other half of each dot product sits in lane l ^ 32.
    const float send = h ? pA : pB;
    const float recv = __shfl_xor(send, 32, 64);
    return (h ? pB : pA) + recv + P->b3;
}

__device__ __forceinline__ float softplus_f(float o) { return o > 20.f ? o : log1pf(expf(o)); }

}  // namespace wlb
