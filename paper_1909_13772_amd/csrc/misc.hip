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
                n[ax] = g[ax] + ccq(q, i, ax);
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

// Second pass of a plain 8-component sum over per-tile partials [n][8], in a
// fixed order (independent of the first pass's launch configuration).
__global__ __launch_bounds__(kWG) void reduce_sum8_kernel(const double *p, int n, double *out)
{
    __shared__ double s[kWG][8];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = threadIdx.x; k < n; k += kWG)
        for (int j = 0; j < 8; ++j) acc[j] += p[(int64_t)k * 8 + j];
    for (int j = 0; j < 8; ++j) s[threadIdx.x][j] = acc[j];
    __syncthreads();
    for (int w = kWG / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int j = 0; j < 8; ++j) s[threadIdx.x][j] += s[threadIdx.x + w][j];
        __syncthreads();
    }
    if (threadIdx.x < 8) out[threadIdx.x] = s[0][threadIdx.x];
}

hipError_t launch_reduce_sum8(const double *partials, int n, double *out8, hipStream_t st)
{
    hipLaunchKernelGGL(reduce_sum8_kernel, dim3(1), dim3(kWG), 0, st, partials, n, out8);
    return hipGetLastError();
}

// Streaming copy, one 16-byte vector per thread over a grid that covers the
// buffer, non-temporal loads and stores (the fastest simple copy form
// measured on MI355X): the library's own measure of achievable HBM
// bandwidth.
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kWG) void copy_kernel(u32x4_t *__restrict__ dst, const u32x4_t *__restrict__ src, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    const int64_t n = (int64_t)(bytes / 16);
    const int64_t grid = (n + kWG - 1) / kWG;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)(grid > 0 ? grid : 1)), dim3(kWG), 0, st,
                       reinterpret_cast<u32x4_t *>(dst), reinterpret_cast<const u32x4_t *>(src), n);
    return hipGetLastError();
}

// Training pairs of the learned closure from box-filtered fine fields
// filt[10][Nc] (rho, u, u_a u_b averages) on a periodic coarse grid (spacing
// 1, acoustic scaling keeps velocities):
//   S_ab = (d_a u_b + d_b u_a) / 2 with central differences of the filtered u;
//   tau_sgs = avg(u u) - u u; nu_t = max(0, -dev(tau_sgs) : S / (2 S : S + 1e-30));
//   target dtau = 3 nu_t; features raw = (Pi = -(2/3) rho (tau0 + dtau) S, rho - 1)
//   in the order xx, yy, zz, xy, xz, yz.
__global__ __launch_bounds__(kWG) void les_targets_kernel(const double *__restrict__ F, int nx, int ny, int nz,
                                                          double tau0, float *__restrict__ raw,
                                                          float *__restrict__ target)
{
    const int64_t N = (int64_t)nx * ny * nz;
    for (int64_t c = (int64_t)blockIdx.x * kWG + threadIdx.x; c < N; c += (int64_t)gridDim.x * kWG) {
        const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((int64_t)nx * ny));
        const int xp = (x + 1) % nx, xm = (x + nx - 1) % nx, yp = (y + 1) % ny, ym = (y + ny - 1) % ny,
                  zp = (z + 1) % nz, zm = (z + nz - 1) % nz;
        auto at = [&](int k, int X, int Y, int Z) { return F[k * N + ((int64_t)Z * ny + Y) * nx + X]; };
        double g[3][3];  // g[a][b] = d_a u_b
        for (int b = 0; b < 3; ++b) {
            g[0][b] = 0.5 * (at(1 + b, xp, y, z) - at(1 + b, xm, y, z));
            g[1][b] = 0.5 * (at(1 + b, x, yp, z) - at(1 + b, x, ym, z));
            g[2][b] = 0.5 * (at(1 + b, x, y, zp) - at(1 + b, x, y, zm));
        }
        double S[6] = {g[0][0], g[1][1], g[2][2], 0.5 * (g[0][1] + g[1][0]), 0.5 * (g[0][2] + g[2][0]),
                       0.5 * (g[1][2] + g[2][1])};
        const double rho = at(0, x, y, z);
        const double u[3] = {at(1, x, y, z), at(2, x, y, z), at(3, x, y, z)};
        double t[6] = {at(4, x, y, z) - u[0] * u[0], at(5, x, y, z) - u[1] * u[1], at(6, x, y, z) - u[2] * u[2],
                       at(7, x, y, z) - u[0] * u[1], at(8, x, y, z) - u[0] * u[2], at(9, x, y, z) - u[1] * u[2]};
        const double tr = (t[0] + t[1] + t[2]) / 3.0;
        t[0] -= tr;
        t[1] -= tr;
        t[2] -= tr;
        const double tS = t[0] * S[0] + t[1] * S[1] + t[2] * S[2] + 2.0 * (t[3] * S[3] + t[4] * S[4] + t[5] * S[5]);
        const double SS = S[0] * S[0] + S[1] * S[1] + S[2] * S[2] + 2.0 * (S[3] * S[3] + S[4] * S[4] + S[5] * S[5]);
        double nu = -tS / (2.0 * SS + 1e-30);
        if (!(nu > 0.0)) nu = 0.0;
        const double dtau = 3.0 * nu;
        for (int k = 0; k < 6; ++k) raw[c * 7 + k] = (float)(-(2.0 / 3.0) * rho * (tau0 + dtau) * S[k]);
        raw[c * 7 + 6] = (float)(rho - 1.0);
        target[c] = (float)dtau;
    }
}

hipError_t launch_les_targets(const double *filt, const int32_t nc[3], double tau0, float *raw, float *target,
                              hipStream_t st)
{
    const int64_t N = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t g = (N + kWG - 1) / kWG;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(les_targets_kernel, dim3((int)g), dim3(kWG), 0, st, filt, nc[0], nc[1], nc[2], tau0, raw,
                       target);
    return hipGetLastError();
}

}  // namespace wlb
