// lattice.hpp -- compile-time velocity sets D2Q9, D3Q15, D3Q19, D3Q27 for the
// HIP kernels.
//
// Directions are numbered once, in the D3Q27 order: rest; (+-1,0,0),
// (0,+-1,0), (0,0,+-1); twelve edges; eight corners, each odd direction
// followed by its opposite.  A velocity set stores its q populations in slots
// 0..q-1, and slot i holds direction dir<Q>(i): the identity for D3Q19 and
// D3Q27 (D3Q19 is the first 19 directions); D3Q15 takes the rest, the six
// faces and the eight corners; D2Q9 the rest, the four x/y faces and the four
// xy edges.  Each set keeps the odd/opposite pairing of its slots.  Weights
// are the textbook ones (the paper names the four sets in Sec. 5.1.1 and
// refers to Krueger et al. 2017 for them): D2Q9 4/9, 1/9, 1/36; D3Q15 2/9,
// 1/9, 1/72; D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27, 1/54, 1/216, by |c|^2.
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
// Components of direction d.
__host__ __device__ constexpr int dcx(int d) { return unpack(kPX, d); }
__host__ __device__ constexpr int dcy(int d) { return unpack(kPY, d); }
__host__ __device__ constexpr int dcz(int d) { return unpack(kPZ, d); }

// Direction held by slot i of a q-population set.
__host__ __device__ constexpr int dir_of(int q, int i)
{
    return q == 15 ? (i < 7 ? i : i + 12) : (q == 9 ? (i < 5 ? i : i + 2) : i);
}
template <int Q>
__host__ __device__ constexpr int dir(int i) { return dir_of(Q, i); }

// Velocity of slot i.
template <int Q>
__host__ __device__ constexpr int cx(int i) { return dcx(dir<Q>(i)); }
template <int Q>
__host__ __device__ constexpr int cy(int i) { return dcy(dir<Q>(i)); }
template <int Q>
__host__ __device__ constexpr int cz(int i) { return dcz(dir<Q>(i)); }
template <int Q>
__host__ __device__ constexpr int cc(int i, int a) { return a == 0 ? cx<Q>(i) : (a == 1 ? cy<Q>(i) : cz<Q>(i)); }
template <int Q>
__host__ __device__ constexpr int c2(int i) { return cx<Q>(i) * cx<Q>(i) + cy<Q>(i) * cy<Q>(i) + cz<Q>(i) * cz<Q>(i); }
// Component a of slot i for a set chosen at run time (host code, masks).
__host__ __device__ constexpr int ccq(int q, int i, int a)
{
    const int d = dir_of(q, i);
    return a == 0 ? dcx(d) : (a == 1 ? dcy(d) : dcz(d));
}
// Slot of the opposite velocity (the same in every set).
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Weight as an exact ratio num / den.
template <int Q>
__host__ __device__ constexpr int wnum(int i)
{
    if (Q == 9) return c2<Q>(i) == 0 ? 16 : (c2<Q>(i) == 1 ? 4 : 1);
    if (Q == 15) return c2<Q>(i) == 0 ? 16 : (c2<Q>(i) == 1 ? 8 : 1);
    if (Q == 19) return c2<Q>(i) == 0 ? 12 : (c2<Q>(i) == 1 ? 2 : 1);
    return c2<Q>(i) == 0 ? 64 : (c2<Q>(i) == 1 ? 16 : (c2<Q>(i) == 2 ? 4 : 1));
}
template <int Q>
__host__ __device__ constexpr int wden() { return Q == 9 ? 36 : (Q == 15 ? 72 : (Q == 19 ? 36 : 216)); }

template <int Q, typename T>
__host__ __device__ constexpr T weight(int i) { return (T)wnum<Q>(i) / (T)wden<Q>(); }

// Links whose target x + c_i lies beyond the low (sign -1) or high (+1) face
// of axis a.
template <int Q>
__host__ __device__ constexpr uint32_t face_links(int a, int sign)
{
    uint32_t m = 0;
    for (int i = 0; i < Q; ++i)
        if (cc<Q>(i, a) == sign) m |= 1u << i;
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
