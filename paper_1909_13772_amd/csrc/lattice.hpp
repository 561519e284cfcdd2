// lattice.hpp -- compile-time D3Q19 / D3Q27 velocity sets for the HIP kernels.
//
// Direction order: rest; (+-1,0,0), (0,+-1,0), (0,0,+-1); twelve edges; eight
// corners (D3Q27), each odd direction followed by its opposite.  Weights are
// the textbook ones for these sets (the paper names the sets in Sec. 5.1.1 and
// refers to Krueger et al. 2017 for them): D3Q19 1/3, 1/18, 1/36 and D3Q27
// 8/27, 2/27, 1/54, 1/216 for |c|^2 = 0, 1, 2, 3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace wlb {

// Components packed 2 bits per direction (0 -> 0, 1 -> +1, 3 -> -1).
__host__ __device__ constexpr uint64_t pack_axis(const int (&v)[27])
{
    uint64_t r = 0;
    for (int i = 0; i < 27; ++i) r |= (uint64_t)(v[i] & 3) << (2 * i);
    return r;
}

struct Dirs {
    static constexpr int X[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                                  1, -1, 1, -1, 1, -1, -1, 1};
    static constexpr int Y[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                                  1, -1, 1, -1, -1, 1, 1, -1};
    static constexpr int Z[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                                  1, -1, -1, 1, 1, -1, 1, -1};
};

constexpr uint64_t kPX = pack_axis(Dirs::X);
constexpr uint64_t kPY = pack_axis(Dirs::Y);
constexpr uint64_t kPZ = pack_axis(Dirs::Z);

__host__ __device__ constexpr int unpack(uint64_t p, int i)
{
    int v = (int)((p >> (2 * i)) & 3);
    return v == 3 ? -1 : v;
}
__host__ __device__ constexpr int cx(int i) { return unpack(kPX, i); }
__host__ __device__ constexpr int cy(int i) { return unpack(kPY, i); }
__host__ __device__ constexpr int cz(int i) { return unpack(kPZ, i); }
__host__ __device__ constexpr int cc(int i, int a) { return a == 0 ? cx(i) : (a == 1 ? cy(i) : cz(i)); }
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr int c2(int i) { return cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i); }

// Weight as an exact ratio num / den (den = 36 for D3Q19, 216 for D3Q27).
template <int Q>
__host__ __device__ constexpr int wnum(int i)
{
    if (Q == 19) return c2(i) == 0 ? 12 : (c2(i) == 1 ? 2 : 1);
    return c2(i) == 0 ? 64 : (c2(i) == 1 ? 16 : (c2(i) == 2 ? 4 : 1));
}
template <int Q>
__host__ __device__ constexpr int wden() { return Q == 19 ? 36 : 216; }

template <int Q, typename T>
__host__ __device__ constexpr T weight(int i) { return (T)wnum<Q>(i) / (T)wden<Q>(); }

// Links whose target x + c_i lies beyond the low (sign -1) or high (+1) face
// of axis a.
template <int Q>
__host__ __device__ constexpr uint32_t face_links(int a, int sign)
{
    uint32_t m = 0;
    for (int i = 0; i < Q; ++i)
        if (cc(i, a) == sign) m |= 1u << i;
    return m;
}

// Compile-time loop: f(std::integral_constant<int, I>) for I = 0 .. N-1.
template <typename F, int... Is>
__device__ __forceinline__ void sfor_impl(F &&f, std::integer_sequence<int, Is...>)
{
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void sfor(F &&f)
{
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

}  // namespace wlb
