// misc.hip -- storage-independent kernels: geometry masks, the second pass of
// the deterministic FP64 conservation reduction, and a bandwidth probe copy.
#include "lattice.hpp"
#include "wlb_internal.hpp"

namespace wlb {

// Mask word per interior cell of every block that has solid cells nearby:
// bit 31 = the cell is solid, bit i = the neighbour x + c_i is solid
// (periodic axes wrap; beyond a non-periodic face the bit stays clear, the
// sweep handles those faces from coordinates).  solid = global u8 array.
__global__ __launch_bounds__(kWG) void masks_kernel(const SweepArgs a, const uint8_t *solid, int q)
{
    uint32_t *masks = const_cast<uint32_t *>(a.masks);
    for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const int4 tv = a.tiles[t];
        const int ex = tv.y >> 16, ey = tv.z >> 16, ez = tv.w >> 16;
        const int l = threadIdx.x;
        if (l >= ex * ey * ez) continue;
        const DevBlock &B = a.blocks[tv.x];
        if (B.mask < 0) continue;
        const int x = (tv.y & 0xffff) + l % ex;
        const int y = (tv.z & 0xffff) + (l / ex) % ey;
        const int z = (tv.w & 0xffff) + l / (ex * ey);
        const int g[3] = {B.g[0] + x, B.g[1] + y, B.g[2] + z};
        const int64_t nx = a.dom[0], ny = a.dom[1];
        uint32_t m = solid[(g[2] * ny + g[1]) * nx + g[0]] ? kSolidBit : 0u;
        for (int i = 1; i < q; ++i) {
            int n[3];
            bool inside = true;
            for (int ax = 0; ax < 3; ++ax) {
                n[ax] = g[ax] + cc(i, ax);
                if (n[ax] < 0 || n[ax] >= a.dom[ax]) {
                    if ((a.periodic >> ax) & 1)
                        n[ax] = (n[ax] + a.dom[ax]) % a.dom[ax];
                    else
                        inside = false;
                }
            }
            if (inside && solid[(n[2] * ny + n[1]) * nx + n[0]]) m |= 1u << i;
        }
        masks[B.mask + (int64_t)z * B.mplane + y * B.mpitch + x] = m;
    }
}

hipError_t launch_masks(const SweepArgs &a, const uint8_t *solid, int q, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(masks_kernel, dim3(grid), dim3(kWG), 0, st, a, solid, q);
    return hipGetLastError();
}

// Second pass of the conservation reduction over per-tile partials
// [n][8] = (sum drho, px, py, pz, kinetic energy, max|u|, n_fluid, -).
// One workgroup, fixed summation order: the result does not depend on the
// launch configuration of the first pass.
__global__ __launch_bounds__(kWG) void reduce_totals_kernel(const double *p, int n, double *out)
{
    __shared__ double s[kWG][7];
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int k = threadIdx.x; k < n; k += kWG)
        for (int j = 0; j < 7; ++j) {
            const double v = p[(int64_t)k * 8 + j];
            acc[j] = (j == 5) ? fmax(acc[j], v) : acc[j] + v;
        }
    for (int j = 0; j < 7; ++j) s[threadIdx.x][j] = acc[j];
    __syncthreads();
    for (int w = kWG / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int j = 0; j < 7; ++j) {
                const double o = s[threadIdx.x + w][j];
                s[threadIdx.x][j] = (j == 5) ? fmax(s[threadIdx.x][j], o) : s[threadIdx.x][j] + o;
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s[0][6] + s[0][0];  // mass = n_fluid + sum (rho - 1)
        for (int j = 1; j < 7; ++j) out[j] = s[0][j];
        out[7] = 0.0;
    }
}

hipError_t launch_reduce_totals(const double *partials, int n, double *out8, hipStream_t st)
{
    hipLaunchKernelGGL(reduce_totals_kernel, dim3(1), dim3(kWG), 0, st, partials, n, out8);
    return hipGetLastError();
}

// Plain streaming copy (16-byte vectors, grid-stride): the library's own
// measure of achievable HBM bandwidth.
__global__ __launch_bounds__(kWG) void copy_kernel(uint4 *__restrict__ dst, const uint4 *__restrict__ src, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG) dst[i] = src[i];
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    const int64_t n = (int64_t)(bytes / 16);
    const int64_t want = (n + kWG - 1) / kWG;
    const int grid = (int)(want < 65536 ? (want > 0 ? want : 1) : 65536);
    hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(kWG), 0, st, reinterpret_cast<uint4 *>(dst),
                       reinterpret_cast<const uint4 *>(src), n);
    return hipGetLastError();
}

}  // namespace wlb
