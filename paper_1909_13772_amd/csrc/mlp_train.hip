// mlp_train.hip -- training kernels of the learned closure network and the
// standalone forward evaluation.
//
// Loss over a minibatch of n samples: L = (1/n) sum_s ((softplus(o_s) - t_s)
// * inv_scale)^2, o = network output for the sample's raw features (see
// mlp.hpp for the network).  The forward/backward pass runs one sample per
// thread in FP32 with the GEMM operands (weights, x, h1, h2) rounded to bf16
// exactly where the matrix-core forward rounds them; the rounding has the
// straight-through gradient.  Parameter gradients are summed per workgroup
// through LDS in a fixed order, then over workgroups in a fixed order
// (deterministic).  Adam keeps FP32 master weights; mean / inv_std are not
// trained.
#include <cstring>
#include <mutex>

#include "mlp.hpp"
#include "wlb_internal.hpp"

namespace wlb {

constexpr int kIn = 7, kH = 32;
constexpr int kOffMean = 0, kOffIstd = 7, kOffW1 = 14, kOffB1 = kOffW1 + kH * kIn, kOffW2 = kOffB1 + kH,
              kOffB2 = kOffW2 + kH * kH, kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH, kNParam = kOffB3 + 1;
static_assert(kNParam == 1359, "parameter count");
constexpr int kChunk = 64;  // samples staged in LDS at a time

__device__ __forceinline__ float gelu_grad(float z)
{
    return norm_cdf(z) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}
__device__ __forceinline__ float sigmoid_f(float o) { return 1.0f / (1.0f + expf(-o)); }

// One sample per thread; per-workgroup gradient partials [gridDim.x][kNParam + 1]
// (last entry: sum of squared residuals).
__global__ __launch_bounds__(kWG) void mlp_grad_kernel(const float *__restrict__ P, const float *__restrict__ raw,
                                                        const float *__restrict__ target, int64_t n, float inv_scale,
                                                        float *__restrict__ partial)
{
    __shared__ float sw[kNParam];  // bf16-rounded weights, FP32 biases
    __shared__ float s_xb[kChunk][8];
    __shared__ float s_h1b[kChunk][kH];
    __shared__ float s_gz1[kChunk][kH];
    __shared__ float s_h2b[kChunk][kH];
    __shared__ float s_gz2[kChunk][kH];
    __shared__ float s_go[kChunk];
    __shared__ float s_loss[kWG];
    for (int k = threadIdx.x; k < kNParam; k += kWG) {
        const bool is_w = (k >= kOffW1 && k < kOffB1) || (k >= kOffW2 && k < kOffB2) || (k >= kOffW3 && k < kOffB3);
        sw[k] = is_w ? bf16_round(P[k]) : P[k];
    }
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * kWG + threadIdx.x;
    const bool act = s < n;
    // ---- forward
    float xb[8], z1[kH], h1b[kH], z2[kH], h2b[kH];
    for (int k = 0; k < kIn; ++k) {
        const float r = act ? raw[s * kIn + k] : 0.f;
        xb[k] = bf16_round((r - sw[kOffMean + k]) * sw[kOffIstd + k]);
    }
    xb[7] = 0.f;
    for (int j = 0; j < kH; ++j) {
        float a = 0.f;
        for (int k = 0; k < kIn; ++k) a += sw[kOffW1 + j * kIn + k] * xb[k];
        z1[j] = a + sw[kOffB1 + j];
        h1b[j] = bf16_round(gelu_erf(z1[j]));
    }
    for (int j = 0; j < kH; ++j) {
        float a = 0.f;
        for (int k = 0; k < kH; ++k) a += sw[kOffW2 + j * kH + k] * h1b[k];
        z2[j] = a + sw[kOffB2 + j];
        h2b[j] = bf16_round(gelu_erf(z2[j]));
    }
    float o = 0.f;
    for (int k = 0; k < kH; ++k) o += sw[kOffW3 + k] * h2b[k];
    o += sw[kOffB3];
    // ---- backward
    const float res = act ? (softplus_f(o) - target[s]) * inv_scale : 0.f;
    const float go = act ? 2.f * res * inv_scale * sigmoid_f(o) / (float)n : 0.f;
    float gz2[kH], gz1[kH];
    for (int j = 0; j < kH; ++j) gz2[j] = go * sw[kOffW3 + j] * gelu_grad(z2[j]);
    for (int k = 0; k < kH; ++k) {
        float a = 0.f;
        for (int j = 0; j < kH; ++j) a += gz2[j] * sw[kOffW2 + j * kH + k];
        gz1[k] = a * gelu_grad(z1[k]);
    }
    s_loss[threadIdx.x] = res * res;
    // ---- parameter sums over the workgroup's samples, kChunk at a time
    float acc[(kNParam + kWG - 1) / kWG];
    for (int r = 0; r < (kNParam + kWG - 1) / kWG; ++r) acc[r] = 0.f;
    for (int c0 = 0; c0 < kWG; c0 += kChunk) {
        __syncthreads();
        const int ls = (int)threadIdx.x - c0;
        if (ls >= 0 && ls < kChunk) {
            for (int k = 0; k < 8; ++k) s_xb[ls][k] = xb[k];
            for (int j = 0; j < kH; ++j) {
                s_h1b[ls][j] = h1b[j];
                s_gz1[ls][j] = gz1[j];
                s_h2b[ls][j] = h2b[j];
                s_gz2[ls][j] = gz2[j];
            }
            s_go[ls] = go;
        }
        __syncthreads();
        for (int r = 0; r < (kNParam + kWG - 1) / kWG; ++r) {
            const int p = (int)threadIdx.x + r * kWG;
            if (p < kOffW1 || p >= kNParam) continue;
            float a = 0.f;
            if (p < kOffB1) {
                const int j = (p - kOffW1) / kIn, k = (p - kOffW1) % kIn;
                for (int q = 0; q < kChunk; ++q) a += s_gz1[q][j] * s_xb[q][k];
            } else if (p < kOffW2) {
                const int j = p - kOffB1;
                for (int q = 0; q < kChunk; ++q) a += s_gz1[q][j];
            } else if (p < kOffB2) {
                const int j = (p - kOffW2) / kH, k = (p - kOffW2) % kH;
                for (int q = 0; q < kChunk; ++q) a += s_gz2[q][j] * s_h1b[q][k];
            } else if (p < kOffW3) {
                const int j = p - kOffB2;
                for (int q = 0; q < kChunk; ++q) a += s_gz2[q][j];
            } else if (p < kOffB3) {
                const int k = p - kOffW3;
                for (int q = 0; q < kChunk; ++q) a += s_go[q] * s_h2b[q][k];
            } else {
                for (int q = 0; q < kChunk; ++q) a += s_go[q];
            }
            acc[r] += a;
        }
    }
    float *out = partial + (int64_t)blockIdx.x * (kNParam + 1);
    for (int r = 0; r < (kNParam + kWG - 1) / kWG; ++r) {
        const int p = (int)threadIdx.x + r * kWG;
        if (p < kNParam) out[p] = p < kOffW1 ? 0.f : acc[r];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float l = 0.f;
        for (int k = 0; k < kWG; ++k) l += s_loss[k];
        out[kNParam] = l;
    }
}

// grad[p] = sum over workgroups (fixed order); loss = sum of squares / n.
__global__ __launch_bounds__(kWG) void mlp_grad_reduce_kernel(const float *__restrict__ partial, int nwg, int64_t n,
                                                               float *__restrict__ grad, float *__restrict__ loss)
{
    const int p = blockIdx.x * kWG + threadIdx.x;
    if (p > kNParam) return;
    float a = 0.f;
    for (int w = 0; w < nwg; ++w) a += partial[(int64_t)w * (kNParam + 1) + p];
    if (p < kNParam)
        grad[p] = a;
    else
        *loss = a / (float)n;
}

__global__ __launch_bounds__(kWG) void mlp_adam_kernel(float *__restrict__ P, const float *__restrict__ g,
                                                        float *__restrict__ m, float *__restrict__ v, float lr,
                                                        float b1, float b2, float eps, float bc1, float bc2)
{
    const int p = blockIdx.x * kWG + threadIdx.x;
    if (p < kOffW1 || p >= kNParam) return;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.f - b1) * gi;
    const float vi = b2 * v[p] + (1.f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    P[p] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// Standalone evaluation of the closure network with the same wavefront code
// (for parity tests): raw[n][7] -> out[n], flag[n] = 1 where the sweep would
// fall back to Smagorinsky.
__global__ __launch_bounds__(kWG) void mlp_forward_kernel(const MlpDev *net, const float *raw, int64_t n, float *out,
                                                          int32_t *flag)
{
    for (int64_t base = (int64_t)blockIdx.x * kWG; base < n; base += (int64_t)gridDim.x * kWG) {
        const int64_t s = base + threadIdx.x;
        const bool act = s < n;
        float x[7];
        bool bad = false;
        for (int k = 0; k < 7; ++k) {
            const float r = act ? raw[s * 7 + k] : 0.f;
            x[k] = (r - net->mean[k]) * net->istd[k];
            bad |= !(fabsf(x[k]) <= 8.f);
            if (!act) x[k] = 0.f;
        }
        const float o = mlp_forward_wave(net, x);
        if (act) {
            out[s] = o;
            flag[s] = (bad || !isfinite(o)) ? 1 : 0;
        }
    }
}

hipError_t launch_mlp_forward(const void *net, const float *raw, int64_t n, float *out, int32_t *flag, hipStream_t st)
{
    int64_t g = (n + kWG - 1) / kWG;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((int)g), dim3(kWG), 0, st, reinterpret_cast<const MlpDev *>(net), raw,
                       n, out, flag);
    return hipGetLastError();
}

size_t mlp_grad_workspace_bytes(int64_t n)
{
    const int64_t nwg = (n + kWG - 1) / kWG;
    return (size_t)nwg * (kNParam + 1) * sizeof(float);
}

hipError_t launch_mlp_grad(const float *P, const float *raw, const float *target, int64_t n, float inv_scale,
                           float *grad, float *loss, float *work, hipStream_t st)
{
    const int64_t nwg = (n + kWG - 1) / kWG;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((int)nwg), dim3(kWG), 0, st, P, raw, target, n, inv_scale, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp_grad_reduce_kernel, dim3((kNParam + 1 + kWG - 1) / kWG), dim3(kWG), 0, st, work, (int)nwg, n,
                       grad, loss);
    return hipGetLastError();
}

// Gradient pass without a caller workspace: the per-workgroup partials live in
// a library-owned device array of fixed size, one copy per GPU (each device
// gets its own instance of a __device__ variable).  Every workgroup writes its
// whole partial row before the reduction reads it, so nothing needs clearing
// between calls; calls that overlap on one GPU share the array and race.
constexpr int64_t kNoAllocMaxWG = kMlpNoAllocMaxSamples / kWG;
static_assert(kMlpNoAllocMaxSamples % kWG == 0, "whole workgroups");
static __device__ __align__(256) float scratch[kNoAllocMaxWG * (kNParam + 1)];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t mlp_scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        // the array's name is a host-side stand-in: the device address of
        // this GPU's copy comes from the runtime, with this device current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_mlp_adam(float *P, const float *g, float *m, float *v, int64_t step, float lr, float b1, float b2,
                           float eps, hipStream_t st)
{
    const float bc1 = 1.f - powf(b1, (float)step), bc2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kNParam + kWG - 1) / kWG), dim3(kWG), 0, st, P, g, m, v, lr, b1, b2, eps,
                       bc1, bc2);
    return hipGetLastError();
}

}  // namespace wlb

namespace wlb {

static uint16_t host_bf16_bits(float v)
{
    uint32_t u;
    std::memcpy(&u, &v, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0x007fffffu) ? 0x40u : 0u));
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
static float host_bf16_round(float v)
{
    uint32_t u = (uint32_t)host_bf16_bits(v) << 16;
    float r;
    std::memcpy(&r, &u, 4);
    return r;
}

size_t mlp_dev_bytes() { return sizeof(MlpDev); }

// Per-lane operand layout for mlp_forward_wave (see mlp.hpp): layer-1 A
// operand = W1 row (lane % 32) in both k halves; layer-2 A operand for
// k-chunk c = W2 row (lane % 32) at the hidden units that the B operand's
// k slots hold, unit(k = 8 h + t) = 16 c + 8 (t / 4) + 4 h + t % 4.
void mlp_prepare(const float *P, void *out)
{
    MlpDev d;
    std::memset(&d, 0, sizeof d);
    for (int k = 0; k < kIn; ++k) {
        d.mean[k] = P[kOffMean + k];
        d.istd[k] = P[kOffIstd + k];
    }
    for (int lane = 0; lane < 64; ++lane) {
        const int m = lane % 32, h = lane / 32;
        for (int t = 0; t < 8; ++t) {
            d.w1[lane][t] = t < kIn ? host_bf16_bits(P[kOffW1 + m * kIn + t]) : 0;
            for (int c = 0; c < 2; ++c) {
                const int unit = 16 * c + 8 * (t / 4) + 4 * h + (t % 4);
                d.w2[c][lane][t] = host_bf16_bits(P[kOffW2 + m * kH + unit]);
            }
        }
    }
    for (int h = 0; h < 2; ++h)
        for (int j = 0; j < 16; ++j) {
            const int u = mlp_unit(j, h);
            d.b1[h][j] = P[kOffB1 + u];
            d.b2[h][j] = P[kOffB2 + u];
            d.w3[h][j] = host_bf16_round(P[kOffW3 + u]);
        }
    d.b3 = P[kOffB3];
    std::memcpy(out, &d, sizeof d);
}

}  // namespace wlb
