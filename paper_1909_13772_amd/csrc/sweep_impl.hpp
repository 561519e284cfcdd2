// sweep_impl.hpp -- HIP kernels of the lattice Boltzmann sweep for one
// storage type (included by sweep_f64.hip, sweep_f32.hip, sweep_f16.hip,
// sweep_bf16.hip with WLB_STORAGE set).
//
// Method (paper Sec. 5.1.1): moments rho = sum f, rho u = sum c f (Eq. 1);
// update f_i(x + c_i, t + 1) = f_i(x, t) + Omega_i (Eq. 2), collision then
// streaming; MRT collision Omega = -M^{-1} S (M f - m_eq) (Eq. 3) with SRT /
// TRT as special relaxation matrices; relaxation time per cell from a
// closure; bounce-back and pressure (anti-bounce-back) boundaries; Guo body
// force.  Populations are stored as deviations d_i = f_i - w_i.
//
// Streaming uses the in-place AA pattern on one array per block:
//   even sweep: read slot i of x, collide, write f*_i into slot opp(i) of x
//               (no neighbour access);
//   odd sweep : read the incoming f_i from slot opp(i) of x - c_i (the ghost
//               layer when outside the block), collide, write f*_i into slot
//               i of x + c_i.
// Each cell of the odd sweep reads and writes exactly the set
// {(x + c_j, j)}, so the update is race-free in place.  Bounce-back links
// (solid neighbour or wall) use the cell's own slots; anti-bounce-back links
// get their value written by the collision that knows the cell's velocity.
#pragma once

#include <hip/hip_fp16.h>

#include <type_traits>

#include "lattice.hpp"
#include "mlp.hpp"
#include "wlb_internal.hpp"

namespace wlb {

// ---------------------------------------------------------------------------
// Storage codecs: load a deviation as the compute type, store with
// round-to-nearest-even.  Raw is the bit container used by the exchange.
// ---------------------------------------------------------------------------
struct bf16_t {
    uint16_t v;
};
// Write-coverage check: a 4-byte "storage" whose every population store adds
// one to a counter in the population's place (loads read zero), so a sweep
// run with it counts the writes each (cell, slot) receives.
struct cover_t {
    uint32_t v;
};

template <typename ST> struct Codec;

// Populations are streamed once per sweep with no reuse inside the sweep, so
// aligned (full-line) accesses carry the non-temporal hint; accesses that
// share cache lines with neighbouring waves (single-lane halo accesses) use
// ordinary loads / stores.  Measured on MI355X: non-temporal aligned
// accesses raise the sweep from ~4.7 to ~5.4 TB/s (FP64).
template <bool NT, typename V>
__device__ __forceinline__ V mem_ld(const V *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    return *p;
}
template <bool NT, typename V>
__device__ __forceinline__ void mem_st(V *p, V v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Codec: Raw is the storage bit pattern (used by LDS staging and the
// exchange); dec / enc convert between Raw and the compute type T (enc
// rounds to nearest even).
template <> struct Codec<double> {
    using T = double;
    using Raw = uint64_t;
    static __device__ __forceinline__ T dec(Raw r) { return __longlong_as_double((long long)r); }
    static __device__ __forceinline__ Raw enc(T v) { return (Raw)__double_as_longlong(v); }
};
template <> struct Codec<float> {
    using T = float;
    using Raw = uint32_t;
    static __device__ __forceinline__ T dec(Raw r) { return __uint_as_float(r); }
    static __device__ __forceinline__ Raw enc(T v) { return __float_as_uint(v); }
};
template <> struct Codec<_Float16> {
    using T = float;
    using Raw = uint16_t;
    static __device__ __forceinline__ T dec(Raw r) { return (float)__builtin_bit_cast(_Float16, r); }
    static __device__ __forceinline__ Raw enc(T v) { return __builtin_bit_cast(Raw, (_Float16)v); }
};
template <> struct Codec<cover_t> {
    using T = float;
    using Raw = uint32_t;
    static __device__ __forceinline__ T dec(Raw) { return 0.0f; }
    static __device__ __forceinline__ Raw enc(T) { return 0u; }
};
template <> struct Codec<bf16_t> {
    using T = float;
    using Raw = uint16_t;
    static __device__ __forceinline__ T dec(Raw r) { return __uint_as_float((uint32_t)r << 16); }
    // round to nearest even in the hardware conversion (inf stays inf, a NaN
    // stays a quiet NaN)
    static __device__ __forceinline__ Raw enc(T v) { return __builtin_bit_cast(Raw, (__bf16)v); }
};

// FP16 deviations are stored multiplied by a power of two per weight class
// (the same for slot i and its opposite, which the AA pattern exchanges):
// the largest S with 16 w_i S <= 65504, so |d_i| up to 16 w_i stays finite
// and deviations down to 2^-14 / S (about 5e-10 for the smallest weights)
// stay normal instead of losing their low bits as subnormals.  Scaling by a
// power of two is exact both ways.  Other storage types use no scale.
// The scale of weight class c (|c|^2 = c) is evaluated at compile time only
// (its loop must never reach the device code), and a slot picks the value of
// its class.
template <int Q>
__host__ __device__ constexpr float f16_class_scale(int c)
{
    int num = 0;
    for (int i = 0; i < Q && num == 0; ++i)
        if (c2<Q>(i) == c) num = wnum<Q>(i);
    if (num == 0) return 1.0f;
    const double lim = 65504.0 * (double)wden<Q>() / (16.0 * (double)num);
    double s = 1.0;
    while (s * 2.0 <= lim) s *= 2.0;
    return (float)s;
}
template <int Q, bool INV = false>
__host__ __device__ __forceinline__ float f16_scale(int i)
{
    constexpr float s0 = INV ? 1.0f / f16_class_scale<Q>(0) : f16_class_scale<Q>(0);
    constexpr float s1 = INV ? 1.0f / f16_class_scale<Q>(1) : f16_class_scale<Q>(1);
    constexpr float s2 = INV ? 1.0f / f16_class_scale<Q>(2) : f16_class_scale<Q>(2);
    constexpr float s3 = INV ? 1.0f / f16_class_scale<Q>(3) : f16_class_scale<Q>(3);
    const int k = c2<Q>(i);
    return k == 0 ? s0 : (k == 1 ? s1 : (k == 2 ? s2 : s3));
}

// Decode / encode one population of slot class i (round to nearest even).
template <int Q, typename ST>
__device__ __forceinline__ typename Codec<ST>::T dec_slot(typename Codec<ST>::Raw r, int i)
{
    if constexpr (std::is_same_v<ST, _Float16>)
        return Codec<ST>::dec(r) * f16_scale<Q, true>(i);
    else
        return Codec<ST>::dec(r);
}
template <int Q, typename ST>
__device__ __forceinline__ typename Codec<ST>::Raw enc_slot(typename Codec<ST>::T v, int i)
{
    if constexpr (std::is_same_v<ST, _Float16>)
        return Codec<ST>::enc(v * f16_scale<Q>(i));
    else
        return Codec<ST>::enc(v);
}

// Stochastic rounding of the 16-bit stores: the value goes to one of its
// two neighbours in the storage format with probabilities that make the
// stored value's expectation the value itself (rnd: 32 uniform bits).  A
// population changes by a nearly constant amount per step while it stays in
// one binade (a body force, a slowly growing flow), so rounding to nearest
// would commit the same error every step and the state would drift by up to
// half an ulp per step; the unbiased rounding turns that drift into a random
// walk.  gfx950 converts FP32 to FP16 / BF16 with stochastic rounding in
// one instruction (v_cvt_sr_f16_f32, v_cvt_sr_bf16_f32), which takes the
// random bits as an operand.  FP32 and FP64 round to nearest.
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
template <int Q, typename ST>
__device__ __forceinline__ typename Codec<ST>::Raw enc_slot_sr(typename Codec<ST>::T v, int i, uint32_t rnd)
{
    if constexpr (std::is_same_v<ST, _Float16>) {
        const f16x2_t r = __builtin_amdgcn_cvt_sr_f16_f32(f16x2_t{}, v * f16_scale<Q>(i), rnd, false);
        return __builtin_bit_cast(uint16_t, r[0]);
    } else if constexpr (std::is_same_v<ST, bf16_t>) {
        const bf16x2_t r = __builtin_amdgcn_cvt_sr_bf16_f32(bf16x2_t{}, v, rnd, false);
        return __builtin_bit_cast(uint16_t, r[0]);
    } else {
        return Codec<ST>::enc(v);
    }
}
template <typename ST>
constexpr bool kStochastic = std::is_same_v<ST, _Float16> || std::is_same_v<ST, bf16_t>;
// Type in which a collision accumulates each new population before it is
// rounded for storage: FP64 for FP32 storage (a final FP32 rounding of the
// same sum would be the only rounding), the compute type otherwise.
template <typename ST>
using AccOf = std::conditional_t<std::is_same_v<ST, float>, double, typename Codec<ST>::T>;

// Random bits of a cell for the stochastic rounding of its stores: a hash
// of four of the cell's incoming populations (which change every step) and
// its global index, so that the rounding is reproducible and the same
// whatever the tiles, blocks, launch order or kernel variant.  Per
// population the bits are mixed once more with the population's index.
__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
template <int Q, typename T>
__device__ __forceinline__ uint32_t state_hash(const T (&f)[Q], uint32_t gcell)
{
    uint32_t h = gcell * 0x9e3779b1u;
    if constexpr (sizeof(T) == 4) {
        // the rest population and one per axis (slots 1, 3, 5 exist in every set)
        h += __float_as_uint((float)f[0]);
        h += __builtin_rotateleft32(__float_as_uint((float)f[1]), 7);
        h += __builtin_rotateleft32(__float_as_uint((float)f[3]), 14);
        h += __builtin_rotateleft32(__float_as_uint((float)f[5]), 21);
    }
    return mix32(h);
}
__device__ __forceinline__ uint32_t pop_bits(uint32_t h, int i)
{
    // 24-bit multiply: full rate, where a 32-bit integer multiply issues at
    // a quarter of the rate; the cell hash is uniform in every bit, so its
    // low 24 bits carry the mix.  The conversions take their random bits
    // from the high end of the word (a value half an ulp above a
    // representable one is lifted by bit 31 alone and by no lower bit, as
    // measured on gfx950), which is where a multiply mixes best.
    return __umul24(h ^ (0x9e3779b9u * (uint32_t)(i + 1)), 0xebca6bu);
}

// Raw bits of a collision result for storage (stochastic rounding for
// 16-bit storage).
template <int Q, typename ST>
__device__ __forceinline__ typename Codec<ST>::Raw enc_result(typename Codec<ST>::T v, int i, uint32_t h)
{
    if constexpr (kStochastic<ST>)
        return enc_slot_sr<Q, ST>(v, i, pop_bits(h, i));
    else
        return enc_slot<Q, ST>(v, i);
}
// Global cell index (x fastest) that seeds the rounding hash.
__device__ __forceinline__ uint32_t global_cell(const SweepArgs &a, const DevBlock &B, int x, int y, int z)
{
    return (uint32_t)(B.g[0] + x) + (uint32_t)a.dom[0] * ((uint32_t)(B.g[1] + y) + (uint32_t)a.dom[1] * (uint32_t)(B.g[2] + z));
}

// Typed loads / stores of one population of slot class i through the codec.
template <int Q, typename ST, bool NT = true>
__device__ __forceinline__ typename Codec<ST>::T ldv(const ST *p, int i)
{
    using Raw = typename Codec<ST>::Raw;
    return dec_slot<Q, ST>(mem_ld<NT>(reinterpret_cast<const Raw *>(p)), i);
}
template <int Q, typename ST, bool NT = true>
__device__ __forceinline__ void stv(ST *p, typename Codec<ST>::T v, int i)
{
    using Raw = typename Codec<ST>::Raw;
    if constexpr (std::is_same_v<ST, cover_t>)
        atomicAdd(reinterpret_cast<uint32_t *>(p), 1u);
    else
        mem_st<NT>(reinterpret_cast<Raw *>(p), enc_slot<Q, ST>(v, i));
}
// Store of a collision result (stochastic rounding for 16-bit storage).
template <int Q, typename ST, bool NT = true>
__device__ __forceinline__ void stv_sr(ST *p, typename Codec<ST>::T v, int i, uint32_t h)
{
    using Raw = typename Codec<ST>::Raw;
    if constexpr (std::is_same_v<ST, cover_t>)
        atomicAdd(reinterpret_cast<uint32_t *>(p), 1u);
    else if constexpr (kStochastic<ST>)
        mem_st<NT>(reinterpret_cast<Raw *>(p), enc_slot_sr<Q, ST>(v, i, pop_bits(h, i)));
    else
        mem_st<NT>(reinterpret_cast<Raw *>(p), enc_slot<Q, ST>(v, i));
}
template <typename ST, bool NT = true>
__device__ __forceinline__ typename Codec<ST>::Raw ldraw(const ST *p)
{
    return mem_ld<NT>(reinterpret_cast<const typename Codec<ST>::Raw *>(p));
}
template <typename ST, bool NT = true>
__device__ __forceinline__ void straw(ST *p, typename Codec<ST>::Raw r)
{
    if constexpr (std::is_same_v<ST, cover_t>)
        atomicAdd(reinterpret_cast<uint32_t *>(p), 1u);
    else
        mem_st<NT>(reinterpret_cast<typename Codec<ST>::Raw *>(p), r);
}

// ---------------------------------------------------------------------------
// Collision (deviation form).  In: d[Q] = f - w.  Out: post-collision d[Q],
// density rho and velocity u (Guo: u = (j + F/2) / rho).
// ---------------------------------------------------------------------------
template <int Q, typename T>
struct Macro {
    T drho, rho, u[3], uu;
    T j[3];  // sum c d (without the force half-step)
};

// 1/x: exact division in FP64; the hardware reciprocal (1 ulp) in FP32,
// where an IEEE division costs about ten instructions per call.
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// a * b + c with one rounding.  The library is compiled without
// floating-point contraction, so that every kernel variant (direct or
// LDS-staged sweep, any tile mode) evaluates the collision with the same
// roundings and results stay bitwise independent of the launch choice; the
// fused operations of the hot path are written out here.
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <int Q, typename T>
__device__ __forceinline__ Macro<Q, T> moments_of(const T (&d)[Q], const T F[3])
{
    T drho = 0, jx = 0, jy = 0, jz = 0;
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        drho += d[i];
        if constexpr (cx<Q>(i) == 1) jx += d[i];
        if constexpr (cx<Q>(i) == -1) jx -= d[i];
        if constexpr (cy<Q>(i) == 1) jy += d[i];
        if constexpr (cy<Q>(i) == -1) jy -= d[i];
        if constexpr (cz<Q>(i) == 1) jz += d[i];
        if constexpr (cz<Q>(i) == -1) jz -= d[i];
    });
    Macro<Q, T> m;
    m.j[0] = jx;
    m.j[1] = jy;
    m.j[2] = jz;
    m.drho = drho;
    m.rho = T(1) + drho;
    const T inv = recip(m.rho);
    m.u[0] = fmadd(T(0.5), F[0], jx) * inv;
    m.u[1] = fmadd(T(0.5), F[1], jy) * inv;
    m.u[2] = fmadd(T(0.5), F[2], jz) * inv;
    m.uu = fmadd(m.u[0], m.u[0], fmadd(m.u[1], m.u[1], m.u[2] * m.u[2]));
    return m;
}

template <int Q, int i, typename T>
__device__ __forceinline__ T cdot(const T v[3])
{
    T r = T(0);
    if constexpr (cx<Q>(i) == 1) r += v[0];
    if constexpr (cx<Q>(i) == -1) r -= v[0];
    if constexpr (cy<Q>(i) == 1) r += v[1];
    if constexpr (cy<Q>(i) == -1) r -= v[1];
    if constexpr (cz<Q>(i) == 1) r += v[2];
    if constexpr (cz<Q>(i) == -1) r -= v[2];
    return r;
}

// Smagorinsky relaxation time: tau = (tau0 + sqrt(tau0^2 + k sqrt(Pi:Pi) / rho)) / 2,
// k = 18 sqrt(2) C_s^2 (from nu_t = C_s^2 |S| and Pi = -2 rho c_s^2 tau S).
template <typename T>
__device__ __forceinline__ T tau_smagorinsky(const T P[6], T rho, T tau0, T k)
{
    const T Q = P[0] * P[0] + P[1] * P[1] + P[2] * P[2] + T(2) * (P[3] * P[3] + P[4] * P[4] + P[5] * P[5]);
    return T(0.5) * (tau0 + sqrt(tau0 * tau0 + k * sqrt(Q) * recip(rho)));
}

// Raw-moment transform along one axis of a 3x3x3 array v[z][y][x] (index
// 9 z + 3 y + x, velocity component c = index - 1): replaces (v(-1), v(0),
// v(+1)) by the moments of order 0, 1, 2.
template <int AX, typename T>
__device__ __forceinline__ void tmoments(T (&v)[27])
{
    constexpr int s = AX == 0 ? 1 : (AX == 1 ? 3 : 9);
    sfor<9>([&](auto L) {
        constexpr int l = decltype(L)::value;
        constexpr int a = l % 3, b = l / 3;
        constexpr int base = AX == 0 ? (3 * a + 9 * b) : (AX == 1 ? (a + 9 * b) : (a + 3 * b));
        const T m = v[base], z = v[base + s], p = v[base + 2 * s];
        v[base] = m + z + p;
        v[base + s] = p - m;
        v[base + 2 * s] = p + m;
    });
}
// Inverse of tmoments along one axis.
template <int AX, typename T>
__device__ __forceinline__ void tvalues(T (&v)[27])
{
    constexpr int s = AX == 0 ? 1 : (AX == 1 ? 3 : 9);
    sfor<9>([&](auto L) {
        constexpr int l = decltype(L)::value;
        constexpr int a = l % 3, b = l / 3;
        constexpr int base = AX == 0 ? (3 * a + 9 * b) : (AX == 1 ? (a + 9 * b) : (a + 3 * b));
        const T m0 = v[base], m1 = v[base + s], m2 = v[base + 2 * s];
        v[base] = T(0.5) * (m2 - m1);
        v[base + s] = m0 - m2;
        v[base + 2 * s] = T(0.5) * (m2 + m1);
    });
}
template <int Q>
__host__ __device__ constexpr int tpos(int i) { return 9 * (cz<Q>(i) + 1) + 3 * (cy<Q>(i) + 1) + (cx<Q>(i) + 1); }

// Lattice moment numerator sum_i wnum_i c_x^a c_y^b c_z^c (divide by wden):
// compile-time constants of the stencil.
template <int Q>
__host__ __device__ constexpr int lmom_num(int a, int b, int c)
{
    int s = 0;
    for (int i = 0; i < Q; ++i) {
        int t = wnum<Q>(i);
        for (int k = 0; k < a; ++k) t *= cx<Q>(i);
        for (int k = 0; k < b; ++k) t *= cy<Q>(i);
        for (int k = 0; k < c; ++k) t *= cz<Q>(i);
        s += t;
    }
    return s;
}

// Per-cell inputs of the closed-form equilibrium and source moments.
template <typename T>
struct MomentSources {
    T A;       // drho - 3/2 rho u.u
    T ru[3];   // rho u
    T ruu[6];  // rho u_j u_l: xx yy zz xy xz yz
    T uF;      // u.F
    T F[3];
    T uFs[6];  // u_j F_j (diagonal), u_j F_l + u_l F_j (off-diagonal)
};

template <int Q, typename T>
__device__ __forceinline__ MomentSources<T> moment_sources(const Macro<Q, T> &m, const T F[3])
{
    MomentSources<T> s;
    s.A = fmadd(T(-1.5) * m.rho, m.uu, m.drho);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        s.ru[k] = m.rho * m.u[k];
        s.F[k] = F[k];
    }
    s.ruu[0] = s.ru[0] * m.u[0];
    s.ruu[1] = s.ru[1] * m.u[1];
    s.ruu[2] = s.ru[2] * m.u[2];
    s.ruu[3] = s.ru[0] * m.u[1];
    s.ruu[4] = s.ru[0] * m.u[2];
    s.ruu[5] = s.ru[1] * m.u[2];
    s.uF = fmadd(m.u[0], F[0], fmadd(m.u[1], F[1], m.u[2] * F[2]));
    s.uFs[0] = m.u[0] * F[0];
    s.uFs[1] = m.u[1] * F[1];
    s.uFs[2] = m.u[2] * F[2];
    s.uFs[3] = fmadd(m.u[0], F[1], m.u[1] * F[0]);
    s.uFs[4] = fmadd(m.u[0], F[2], m.u[2] * F[0]);
    s.uFs[5] = fmadd(m.u[1], F[2], m.u[2] * F[1]);
    return s;
}

// Raw moment of order (a, b, c) of the equilibrium deviation
// w (drho + rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)) (EQ) or of the Guo term
// w (3 (c - u).F + 9 (c.u)(c.F)) (!EQ): expanding (c.u)^2 and (c.u)(c.F)
// leaves sums sum w c^(a,b,c) c_j c_l, i.e. lattice moments of higher order,
// most of which vanish; what remains is a few FMAs per moment.
template <int Q, bool EQ, int a, int b, int c, typename T>
__device__ __forceinline__ T source_moment(const MomentSources<T> &s)
{
    constexpr double D = wden<Q>();
    constexpr int L0 = lmom_num<Q>(a, b, c);
    constexpr int L1[3] = {lmom_num<Q>(a + 1, b, c), lmom_num<Q>(a, b + 1, c), lmom_num<Q>(a, b, c + 1)};
    constexpr int L2[6] = {lmom_num<Q>(a + 2, b, c),     lmom_num<Q>(a, b + 2, c),     lmom_num<Q>(a, b, c + 2),
                           lmom_num<Q>(a + 1, b + 1, c), lmom_num<Q>(a + 1, b, c + 1), lmom_num<Q>(a, b + 1, c + 1)};
    T r = T(0);
    if constexpr (L0 != 0) {
        if constexpr (EQ)
            r = T(L0 / D) * s.A;
        else
            r = T(-3.0 * L0 / D) * s.uF;
    }
    sfor<3>([&](auto J) {
        constexpr int j = decltype(J)::value;
        if constexpr (L1[j] != 0) r = fmadd(T(3.0 * L1[j] / D), EQ ? s.ru[j] : s.F[j], r);
    });
    sfor<6>([&](auto J) {
        constexpr int j = decltype(J)::value;
        // (c.u)^2 counts each off-diagonal product twice; (c.u)(c.F) is
        // already summed over both orders in uFs
        constexpr double k = EQ ? (j < 3 ? 4.5 : 9.0) : 9.0;
        if constexpr (L2[j] != 0) r = fmadd(T(k * L2[j] / D), EQ ? s.ruu[j] : s.uFs[j], r);
    });
    return r;
}

// MRT in the raw-moment basis sum c_x^a c_y^b c_z^c (a, b, c <= 2) through
// the tensor-product transform; the three diagonal second-order moments are
// relaxed as x2-y2, x2-z2 (rate omega) and x2+y2+z2 (omega_bulk), xy/xz/yz
// with omega, order >= 3 with omega_higher, conserved moments with 0.  The
// Guo source enters as M^{-1} (I - S/2) M F.  Only the populations are
// transformed: the equilibrium's and the source's moments are closed forms.
// D3Q19 uses the same transform with the eight corner populations held at
// zero: D3Q19 distributions are exactly those whose moments with a factor
// xyz vanish, a subspace that the relaxation maps into itself.  With the
// Smagorinsky closure omega comes from the non-equilibrium second moments.
// KBC (Sec. 5.1.1: entropic stabilisation, Boesch, Chikatamarla and Karlin):
// the same transform; f - f_eq splits by moment class into the conserved
// part, the shear part s (deviatoric second moments, relaxed at
// 2 beta = omega) and the rest h (trace of the second moments and every
// moment of order >= 3), which relaxes at gamma beta with
//   gamma = 1/beta - (2 - 1/beta) <ds|dh> / <dh|dh>,  <x|y> = sum x_i y_i / f_eq_i,
// the stationary point of the quadratic entropy of the post-collision state
// (gamma = 2 when dh vanishes).  ds and dh are taken back to populations by
// the inverse transform for the two entropic products.
template <int Q, typename T, bool KBC = false, typename A = T>
__device__ __forceinline__ void mrt_collide(T (&d)[Q], const Macro<Q, T> &m, const T F[3], T om, T omb, T omh,
                                            int closure, T tau0, T smag_k)
{
    T mn[27];
#pragma unroll
    for (int k = 0; k < 27; ++k) mn[k] = T(0);
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        mn[tpos<Q>(i)] = d[i];
    });
    tmoments<0>(mn);
    tmoments<1>(mn);
    tmoments<2>(mn);
    const MomentSources<T> src = moment_sources<Q, T>(m, F);
    // after the transform, index a + 3 b + 9 c holds the moment of order (a, b, c)
    sfor<27>([&](auto K) {
        constexpr int k = decltype(K)::value;
        mn[k] -= source_moment<Q, true, k % 3, (k / 3) % 3, k / 9>(src);
    });
    constexpr int XX = 2, YY = 6, ZZ = 18, XY = 4, XZ = 10, YZ = 12;
    if (closure == 1) {
        const T P[6] = {mn[XX], mn[YY], mn[ZZ], mn[XY], mn[XZ], mn[YZ]};
        om = recip(tau_smagorinsky<T>(P, m.rho, tau0, smag_k));
    }
    if constexpr (KBC) {
        static_assert(Q == 27, "KBC runs on D3Q27");
        T vs[27], vh[27];
#pragma unroll
        for (int k = 0; k < 27; ++k) vs[k] = vh[k] = T(0);
        const T t3 = (mn[XX] + mn[YY] + mn[ZZ]) * (T(1) / T(3));
        vs[XX] = mn[XX] - t3;
        vs[YY] = mn[YY] - t3;
        vs[ZZ] = mn[ZZ] - t3;
        vs[XY] = mn[XY];
        vs[XZ] = mn[XZ];
        vs[YZ] = mn[YZ];
        vh[XX] = vh[YY] = vh[ZZ] = t3;
        sfor<27>([&](auto K) {
            constexpr int k = decltype(K)::value;
            if constexpr (k % 3 + (k / 3) % 3 + k / 9 >= 3) vh[k] = mn[k];
        });
        tvalues<2>(vs);
        tvalues<1>(vs);
        tvalues<0>(vs);
        tvalues<2>(vh);
        tvalues<1>(vh);
        tvalues<0>(vh);
        // f_eq_i = w_i (1 + A + rho c.u (3 + 9/2 c.u)), A = drho - 3/2 rho u.u
        const T A1 = T(1) + m.drho - T(1.5) * m.rho * m.uu;
        T sh = T(0), hh = T(0);
        sfor<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr T w = weight<Q, T>(i);
            const T cu = cdot<Q, i>(m.u);
            const T r = recip(w * (A1 + m.rho * cu * (T(3) + T(4.5) * cu)));
            const T h = vh[tpos<Q>(i)];
            sh += vs[tpos<Q>(i)] * h * r;
            hh += h * h * r;
        });
        const T beta = T(0.5) * om, ib = recip(beta);
        const T gamma = hh > T(1e-30) ? ib - (T(2) - ib) * sh * recip(hh) : T(2);
        omh = gamma * beta;
        omb = omh;
    }
    T g[27];
    sfor<27>([&](auto K) {
        constexpr int k = decltype(K)::value;
        constexpr int a = k % 3, b = (k / 3) % 3, c = k / 9;
        constexpr int ord = a + b + c;
        if constexpr (ord <= 1) {
            g[k] = -source_moment<Q, false, a, b, c>(src);
        } else if constexpr (ord == 2 && (a == 2 || b == 2 || c == 2)) {
            g[k] = T(0);  // diagonal: below
        } else if constexpr (ord == 2) {
            g[k] = fmadd(om, mn[k], -(T(1) - T(0.5) * om) * source_moment<Q, false, a, b, c>(src));
        } else {
            g[k] = fmadd(omh, mn[k], -(T(1) - T(0.5) * omh) * source_moment<Q, false, a, b, c>(src));
        }
    });
    {
        const T fxx = source_moment<Q, false, 2, 0, 0>(src), fyy = source_moment<Q, false, 0, 2, 0>(src),
                fzz = source_moment<Q, false, 0, 0, 2>(src);
        const T An = mn[XX] - mn[YY], Bn = mn[XX] - mn[ZZ], Tn = mn[XX] + mn[YY] + mn[ZZ];
        const T Af = fxx - fyy, Bf = fxx - fzz, Tf = fxx + fyy + fzz;
        const T gA = fmadd(om, An, -(T(1) - T(0.5) * om) * Af);
        const T gB = fmadd(om, Bn, -(T(1) - T(0.5) * om) * Bf);
        const T gT = fmadd(omb, Tn, -(T(1) - T(0.5) * omb) * Tf);
        const T third = T(1) / T(3);
        g[XX] = (gA + gB + gT) * third;
        g[YY] = (gT - T(2) * gA + gB) * third;
        g[ZZ] = (gT + gA - T(2) * gB) * third;
    }
    tvalues<2>(g);
    tvalues<1>(g);
    tvalues<0>(g);
    // the change g contains the force, a nearly constant amount per step:
    // subtracted in A (FP64 for FP32 storage) and rounded once
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        d[i] = T(A(d[i]) - A(g[tpos<Q>(i)]));
    });
}

// Central moments to raw moments along one axis of the 3 x 3 x 3 moment
// array (index a + 3 b + 9 c): with the shift u, r0 = k0, r1 = k1 + u k0,
// r2 = k2 + 2 u k1 + u^2 k0.
template <int AX, typename T>
__device__ __forceinline__ void central_to_raw(T (&v)[27], T u)
{
    constexpr int s = AX == 0 ? 1 : (AX == 1 ? 3 : 9);
    sfor<9>([&](auto L) {
        constexpr int l = decltype(L)::value;
        constexpr int a = l % 3, b = l / 3;
        constexpr int base = AX == 0 ? (3 * a + 9 * b) : (AX == 1 ? (a + 9 * b) : (a + 3 * b));
        const T k0 = v[base], k1 = v[base + s], k2 = v[base + 2 * s];
        v[base + s] = k1 + u * k0;
        v[base + 2 * s] = k2 + u * (T(2) * k1 + u * k0);
    });
}

// Raw moment (a, b, c) of rho times the factorised three-velocity
// distribution at u (per axis: moments 1, u, 1/3 + u^2) minus that of the
// lattice weights (u = 0, rho = 1), written in small quantities only.
template <int a, int b, int c, typename T>
__device__ __forceinline__ T factorised_moment_dev(const T u[3], const T u2[3], T drho)
{
    const int e[3] = {a, b, c};
    T P = T(1);
    bool odd = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (e[k] == 1) {
            P *= u[k];
            odd = true;
        } else if (e[k] == 2) {
            P *= T(1) / T(3) + u2[k];
        }
    }
    if (odd) return (T(1) + drho) * P;  // the weights' moment is zero
    // prod over the axes with exponent 2 of (1/3 + u_k^2) minus (1/3)^n
    T diff = T(0), lower = T(1);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (e[k] == 2) {  // diff' = (1/3 + s) (prev product) - (1/3)^n = diff/3 + s * prev
            diff = diff * (T(1) / T(3)) + u2[k] * lower;
            lower *= T(1) / T(3) + u2[k];
        }
    }
    return drho * P + diff;
}

// Cumulant collision (Sec. 5.1.1: cumulants relaxed instead of moments;
// Geier et al. 2015) on D3Q27, every cumulant of order >= 3 relaxed at rate
// 1 (to zero).  With u = (j + F/2)/rho the covariance S of the populations
// about u (the second-order cumulants) has its deviatoric part relaxed at
// omega and its trace at omega_bulk towards 1; afterwards the populations
// have density rho, first-order central moments F/2 (sum c f* = j + F) and
// the central moments of rho times a zero-mean Gaussian with covariance S*.
// Computed as S^ = S - I/3 so that nothing of order one is formed: the
// central moments split into a part in S^ and F (shifted to raw moments
// axis by axis) and the factorised rest distribution at u, whose raw moments
// minus the weights' moments have a closed form; the difference is the raw
// moment array of the deviations, which the inverse transform turns into
// populations.
template <int Q, typename T>
__device__ __forceinline__ void cumulant_collide(T (&d)[Q], const Macro<Q, T> &m, const T F[3], T om, T omb)
{
    static_assert(Q == 27, "the cumulant collision runs on D3Q27");
    constexpr int XX = 2, YY = 6, ZZ = 18, XY = 4, XZ = 10, YZ = 12;
    T mn[27];
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        mn[tpos<Q>(i)] = d[i];
    });
    tmoments<0>(mn);
    tmoments<1>(mn);
    tmoments<2>(mn);
    const T ir = recip(m.rho), r = m.rho;
    const T *u = m.u;
    const T d3 = m.drho * (T(1) / T(3));
    // S^ = S - I/3 from the raw second moments of the deviations
    T sxx = (mn[XX] - r * u[0] * u[0] + u[0] * F[0] - d3) * ir;
    T syy = (mn[YY] - r * u[1] * u[1] + u[1] * F[1] - d3) * ir;
    T szz = (mn[ZZ] - r * u[2] * u[2] + u[2] * F[2] - d3) * ir;
    T sxy = (mn[XY] - r * u[0] * u[1] + T(0.5) * (u[0] * F[1] + u[1] * F[0])) * ir;
    T sxz = (mn[XZ] - r * u[0] * u[2] + T(0.5) * (u[0] * F[2] + u[2] * F[0])) * ir;
    T syz = (mn[YZ] - r * u[1] * u[2] + T(0.5) * (u[1] * F[2] + u[2] * F[1])) * ir;
    {
        const T kd = T(1) - om, kb = T(1) - omb;
        const T A = kd * (sxx - syy), B = kd * (sxx - szz), Tr = kb * (sxx + syy + szz);
        sxx = (A + B + Tr) * (T(1) / T(3));
        syy = (Tr - T(2) * A + B) * (T(1) / T(3));
        szz = (Tr + A - T(2) * B) * (T(1) / T(3));
        sxy *= kd;
        sxz *= kd;
        syz *= kd;
    }
    const T t = T(1) / T(3);
    const T Sxx = sxx + t, Syy = syy + t, Szz = szz + t;
    // central moments minus those of rho x (Gaussian with covariance I/3)
    T k[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) k[q] = T(0);
    k[1] = T(0.5) * F[0];
    k[3] = T(0.5) * F[1];
    k[9] = T(0.5) * F[2];
    k[XX] = r * sxx;
    k[YY] = r * syy;
    k[ZZ] = r * szz;
    k[XY] = r * sxy;
    k[XZ] = r * sxz;
    k[YZ] = r * syz;
    k[8] = r * (sxx * syy + t * (sxx + syy) + T(2) * sxy * sxy);    // (2,2,0)
    k[20] = r * (sxx * szz + t * (sxx + szz) + T(2) * sxz * sxz);   // (2,0,2)
    k[24] = r * (syy * szz + t * (syy + szz) + T(2) * syz * syz);   // (0,2,2)
    k[14] = r * (Sxx * syz + T(2) * sxy * sxz);                     // (2,1,1)
    k[16] = r * (Syy * sxz + T(2) * sxy * syz);                     // (1,2,1)
    k[22] = r * (Szz * sxy + T(2) * sxz * syz);                     // (1,1,2)
    k[26] = r * (sxx * syy * szz + t * (sxx * syy + sxx * szz + syy * szz) + t * t * (sxx + syy + szz) +
                 T(2) * (Sxx * syz * syz + Syy * sxz * sxz + Szz * sxy * sxy) + T(8) * sxy * sxz * syz);  // (2,2,2)
    central_to_raw<0>(k, u[0]);
    central_to_raw<1>(k, u[1]);
    central_to_raw<2>(k, u[2]);
    const T u2[3] = {u[0] * u[0], u[1] * u[1], u[2] * u[2]};
    sfor<27>([&](auto K) {
        constexpr int q = decltype(K)::value;
        k[q] += factorised_moment_dev<q % 3, (q / 3) % 3, q / 9, T>(u, u2, m.drho);
    });
    tvalues<2>(k);
    tvalues<1>(k);
    tvalues<0>(k);
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        d[i] = k[tpos<Q>(i)];
    });
}

template <typename T>
struct CollParams {
    T om, omm, magic, omb, omh, F[3], tau0, smag_k;
    int closure;
};

// Uniform value the compiler may not treat as loop-invariant: the parameters
// are re-read through it once per tile so that constants derived from them
// (force projections per direction, rates, their FP32 conversions) are
// recomputed where used instead of being hoisted out of the tile loop, where
// they would occupy ~50 vector registers for the whole kernel.
__device__ __forceinline__ double opaque(double v)
{
    asm volatile("" : "+s"(v));
    return v;
}

template <typename T>
__device__ __forceinline__ CollParams<T> coll_params(const SweepArgs &a)
{
    CollParams<T> c;
    c.om = (T)opaque(a.omega);
    c.omm = (T)opaque(a.omega_minus);
    c.magic = (T)opaque(a.magic);
    c.omb = (T)opaque(a.omega_bulk);
    c.omh = (T)opaque(a.omega_higher);
    c.F[0] = (T)opaque(a.force[0]);
    c.F[1] = (T)opaque(a.force[1]);
    c.F[2] = (T)opaque(a.force[2]);
    c.tau0 = (T)opaque(a.tau0);
    c.smag_k = (T)opaque(a.smag_k);
    c.closure = a.closure;
    return c;
}

// Non-equilibrium stress from the symmetric pair parts:
// Pi = sum over pairs of c c (d_i + d_opp - 2 e+), e+ = w (A + 9/2 rho cu^2),
// A = drho - 3/2 rho uu.
template <int Q, typename T>
__device__ __forceinline__ void pi_pairs(const T (&d)[Q], const Macro<Q, T> &m, T P[6])
{
    const T A = m.drho - T(1.5) * m.rho * m.uu;
    for (int k = 0; k < 6; ++k) P[k] = T(0);
    sfor<(Q - 1) / 2>([&](auto K) {
        constexpr int i = 2 * decltype(K)::value + 1, o = i + 1;
        constexpr T w = weight<Q, T>(i);
        const T cu = cdot<Q, i>(m.u);
        const T n = d[i] + d[o] - T(2) * w * (A + T(4.5) * m.rho * cu * cu);
        if constexpr (cx<Q>(i) != 0) P[0] += n;
        if constexpr (cy<Q>(i) != 0) P[1] += n;
        if constexpr (cz<Q>(i) != 0) P[2] += n;
        if constexpr (cx<Q>(i) * cy<Q>(i) == 1) P[3] += n;
        if constexpr (cx<Q>(i) * cy<Q>(i) == -1) P[3] -= n;
        if constexpr (cx<Q>(i) * cz<Q>(i) == 1) P[4] += n;
        if constexpr (cx<Q>(i) * cz<Q>(i) == -1) P[4] -= n;
        if constexpr (cy<Q>(i) * cz<Q>(i) == 1) P[5] += n;
        if constexpr (cy<Q>(i) * cz<Q>(i) == -1) P[5] -= n;
    });
}

// Antisymmetric pair constants t_i ~ 3 w_i of the SRT / TRT update, as
// values of the compute type T whose lattice sum sum_i t_i c_ia c_ib = delta_ab
// holds exactly (no rounding): with the textbook weights rounded to T that
// sum misses 1 by about one ulp, and the collision then multiplies the
// momentum by 1 + omega- eps every step (a drift of 1e-4 over 2000 steps in
// FP32 for a flow that is only accelerated).  Every class but the faces is
// rounded to a multiple of U = ulp(t_face) / 4 (twice that where its count
// along an axis is not a multiple of 8, and never finer than its own ulp in
// T), and t_face takes what the identity
// leaves, 1 - sum, which is then a multiple of ulp(t_face): exact.  The
// symmetric part keeps the plain weights (their rounding only perturbs the
// mass, by omega+ eps A per step, A = drho - 3/2 rho u.u).
template <int Q>
__host__ __device__ constexpr int n_xclass(int c2v)
{
    int n = 0;
    for (int i = 0; i < Q; ++i) n += (c2<Q>(i) == c2v && cx<Q>(i) != 0);
    return n;
}
template <int Q>
__host__ __device__ constexpr int first_of_class(int c2v)
{
    for (int i = 0; i < Q; ++i)
        if (c2<Q>(i) == c2v) return i;
    return 0;
}
template <int Q, typename T>
__host__ __device__ constexpr T pair_t(int i)
{
    constexpr int P = sizeof(T) == 8 ? 53 : 24;
    const double tf = 3.0 * (double)wnum<Q>(1) / (double)wden<Q>();
    double g = 1.0;  // 2^floor(log2 tf)
    while (g > tf) g *= 0.5;
    while (g * 2.0 <= tf) g *= 2.0;
    for (int k = 1; k < P; ++k) g *= 0.5;  // ulp(tf)
    long long inv_u = 4;  // 1 / U in powers of two: U = g / 4
    for (double x = g; x < 1.0; x *= 2.0) inv_u *= 2;
    const double U = 1.0 / (double)inv_u;
    long long rest = inv_u;  // 1 / U - sum over non-face classes of count * n
    long long ni = 0;
    for (int k = 2; k <= 3; ++k) {
        const int cnt = n_xclass<Q>(k);
        if (cnt == 0) continue;
        const double tk = 3.0 * (double)wnum<Q>(first_of_class<Q>(k)) / (double)wden<Q>();
        long long step = (cnt % 8 == 0) ? 1 : 2;
        double uk = 1.0;  // ulp(tk): the multiple must also be a value of T
        while (uk > tk) uk *= 0.5;
        for (int b = 1; b < P; ++b) uk *= 0.5;
        while ((double)step * U < uk) step *= 2;
        const long long nk = (long long)(tk / U / (double)step + 0.5) * step;
        rest -= (long long)cnt * nk;
        if (c2<Q>(i) == k) ni = nk;
    }
    if (c2<Q>(i) == 1) ni = rest / 2;
    if (c2<Q>(i) == 0) ni = 0;
    return (T)((double)ni * U);
}

template <int Q, typename T>
__host__ __device__ constexpr bool pair_t_exact()
{
    // summed in integer units of 2^-60 (every t_i is a multiple of 2^-58 or
    // coarser), so the check itself does not round
    long long s = 0;
    double unit = 1.0;
    for (int k = 0; k < 60; ++k) unit *= 2.0;
    for (int i = 0; i < Q; ++i) s += (long long)((double)pair_t<Q, T>(i) * unit) * (cx<Q>(i) * cx<Q>(i));
    return s == (long long)unit;
}
static_assert(pair_t_exact<19, float>() && pair_t_exact<27, float>() && pair_t_exact<15, float>() &&
                  pair_t_exact<9, float>() && pair_t_exact<19, double>() && pair_t_exact<27, double>() &&
                  pair_t_exact<15, double>() && pair_t_exact<9, double>(),
              "pair constants must sum exactly to the identity");

// SRT / TRT relaxation evaluated pair by pair (i, opp(i)) on the pair parts
// s = d_i + d_opp and a = d_i - d_opp:
//   s' = (1 - omega+) s + 2 z+,  a' = (1 - omega-) a + 2 z-,
//   d_i' = (s' + a')/2,  d_opp' = (s' - a')/2,
//   z+ = omega+ e+ + (1 - omega+/2) F+ = w (K + cu c.V),
//        K = omega+ A - 3 (1 - omega+/2) u.F,  V = 9/2 omega+ rho u + 9 (1 - omega+/2) F,
//        e+ = w (A + 9/2 rho cu^2),  A = drho - 3/2 rho u.u,  F+ = w (9 cu cF - 3 u.F),
//   z- = omega- e- + (1 - omega-/2) F- = t (omega- c.j + c.F),
//        e- = 3 w c.(rho u) = 3 w c.(j + F/2),  F- = 3 w c.F,  t = 3 w,
// where j = sum c d is the momentum without the half force, so that the
// constant force never enters a sum with the much larger momentum in the
// compute type (rounding j + F/2 to FP32 would round the same way every step
// while j grows by F).  Each new population is accumulated in A (FP64 for
// FP32 storage, the storage's compute type otherwise) from the pair parts
// and the force part t c.F and rounded once: with t_i summing exactly to the
// identity (pair_t) the momentum then changes by exactly F per step up to
// one rounding per population.
template <int Q, typename T, bool SRT = false, typename A = T>
__device__ __forceinline__ void relax_pairs(T (&d)[Q], const Macro<Q, T> &m, const T F[3], T om, T omm)
{
    const T fop = fmadd(T(-0.5), om, T(1));
    const T A0 = fmadd(T(-1.5) * m.rho, m.uu, m.drho);
    const T uF = fmadd(m.u[0], F[0], fmadd(m.u[1], F[1], m.u[2] * F[2]));
    const T K = fmadd(om, A0, T(-3) * fop * uF);
    const T kv = T(4.5) * om * m.rho, fv = T(9) * fop;
    T V[3], J[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        V[k] = fmadd(kv, m.u[k], fv * F[k]);
        J[k] = (SRT ? om : omm) * m.j[k];
    }
    // (1 - omega)/2, exact for omega in [1/2, 2]
    const A hp = A(fmadd(T(-0.5), om, T(0.5))), hm = SRT ? hp : A(fmadd(T(-0.5), omm, T(0.5)));
    {
        constexpr T w0 = weight<Q, T>(0);
        d[0] = fmadd(T(1) - om, d[0], w0 * K);
    }
    sfor<(Q - 1) / 2>([&](auto I) {
        constexpr int i = 2 * decltype(I)::value + 1, o = i + 1;
        constexpr T w = weight<Q, T>(i);
        constexpr T t = pair_t<Q, T>(i);
        const T cu = cdot<Q, i>(m.u);
        const T zp = w * fmadd(cu, cdot<Q, i>(V), K);
        const T zj = t * cdot<Q, i>(J);
        const A sh = fmadd(hp, A(d[i] + d[o]), A(zp));
        const A ah = fmadd(hm, A(d[i] - d[o]), A(zj) + A(t) * A(cdot<Q, i>(F)));
        d[i] = T(sh + ah);
        d[o] = T(sh - ah);
    });
}

// Collide one cell in place.  Returns the macroscopic state used.
template <int Q, int COLL, typename T, typename A = T>
__device__ __forceinline__ Macro<Q, T> collide(T (&d)[Q], const CollParams<T> &p)
{
    const Macro<Q, T> m = moments_of<Q, T>(d, p.F);
    T om = p.om, omm = p.omm;
    if constexpr (COLL == 4) {
        if (p.closure == 1) {
            T P[6];
            pi_pairs<Q, T>(d, m, P);
            om = recip(tau_smagorinsky<T>(P, m.rho, p.tau0, p.smag_k));
        }
        cumulant_collide<Q, T>(d, m, p.F, om, p.omb);
    } else if constexpr (COLL == 2 || COLL == 3) {
        mrt_collide<Q, T, COLL == 3, A>(d, m, p.F, om, p.omb, p.omh, p.closure, p.tau0, p.smag_k);
    } else {
        if (p.closure == 1) {
            T P[6];
            pi_pairs<Q, T>(d, m, P);
            const T tau = tau_smagorinsky<T>(P, m.rho, p.tau0, p.smag_k);
            om = recip(tau);
            omm = recip(T(0.5) + p.magic * recip(tau - T(0.5)));
        }
        if constexpr (COLL == 0) omm = om;
        relax_pairs<Q, T, COLL == 0, A>(d, m, p.F, om, omm);
    }
    return m;
}

// ---------------------------------------------------------------------------
// Cell addressing and boundary classification
// ---------------------------------------------------------------------------
struct CellPos {
    int x, y, z;
    bool valid;
};

// Item handled by workgroup b when a launch gives every item (tile,
// exchange chunk) its own workgroup.  Workgroups are dispatched round-robin
// over the 8 XCDs, each with its own L2; this mapping hands every XCD one
// contiguous range of items, so that neighbouring tiles, which share cache
// lines at their edges (packed short rows, row ends), meet in the same L2.
__device__ __forceinline__ int xcd_item(int b, int n)
{
    constexpr int kXcd = 8;
    const int q = n / kXcd, r = n % kXcd;
    const int k = b % kXcd, j = b / kXcd;
    return k * q + (k < r ? k : r) + j;
}
__device__ __forceinline__ int first_tile(const SweepArgs &a)
{
    return (a.xcd_map && (int)gridDim.x == a.nstiles) ? xcd_item(blockIdx.x, a.nstiles) : (int)blockIdx.x;
}

__device__ __forceinline__ CellPos tile_cell(const int4 tv, int l)
{
    const int ex = tv.y >> 16, ey = tv.z >> 16, ez = tv.w >> 16;
    CellPos c;
    c.valid = l < ex * ey * ez;
    const int lx = l % ex, r = l / ex;
    c.x = (tv.y & 0xffff) + lx;
    c.y = (tv.z & 0xffff) + r % ey;
    c.z = (tv.w & 0xffff) + r / ey;
    return c;
}

// Cell of lane l in a sweep tile: a box tile, or a list tile of fluid cells
// (porous media: no lanes spent on solid cells, full waves on short rows).
__device__ __forceinline__ CellPos sweep_cell(const SweepArgs &a, const int4 tv, int l)
{
    if (tv.w >= 0) return tile_cell(tv, l);
    CellPos c;
    c.valid = l < -tv.w;
    const uint32_t p = c.valid ? a.cells[tv.y + l] : 0u;
    c.x = (int)(p & 1023u);
    c.y = (int)((p >> 10) & 1023u);
    c.z = (int)(p >> 20);
    return c;
}

// Link classes of a fluid cell: bb = bounce-back links (solid neighbour or a
// wall face), alo / ahi = anti-bounce-back links through the low / high face
// of the pressure axis.  Walls take precedence over pressure faces.
template <int Q>
struct Links {
    uint32_t bb, alo, ahi;
};

template <int Q>
__device__ __forceinline__ Links<Q> classify(uint32_t mask, const DevBlock &B, int x, int y, int z,
                                             const SweepArgs &a)
{
    Links<Q> L;
    L.bb = mask & ((1u << Q) - 1u);
    L.alo = 0;
    L.ahi = 0;
    const int p[3] = {B.g[0] + x, B.g[1] + y, B.g[2] + z};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        if ((a.periodic >> ax) & 1) continue;
        const uint32_t lo = (p[ax] == 0) ? (ax == 0 ? face_links<Q>(0, -1) : ax == 1 ? face_links<Q>(1, -1)
                                                                                     : face_links<Q>(2, -1))
                                         : 0u;
        const uint32_t hi = (p[ax] == a.dom[ax] - 1) ? (ax == 0 ? face_links<Q>(0, 1) : ax == 1 ? face_links<Q>(1, 1)
                                                                                                : face_links<Q>(2, 1))
                                                     : 0u;
        if (ax == a.pressure_axis) {
            L.alo |= lo;
            L.ahi |= hi;
        } else {
            L.bb |= lo | hi;
        }
    }
    L.alo &= ~L.bb;
    L.ahi &= ~L.bb;
    return L;
}

// Anti-bounce-back value for the population entering the cell against
// direction i: -f*_i + 2 w_i rho_w (1 + 9/2 (c_i.u)^2 - 3/2 u.u), as deviation
// -d*_i + 2 w_i ((rho_w - 1) + rho_w (9/2 (c_i.u)^2 - 3/2 u.u)).  This form
// keeps every intermediate at the size of the result (rho_w - 1 comes exact
// from the FP64 parameters), so FP32 loses no digits to a term of order one.
template <int Q, int i, typename T>
__device__ __forceinline__ T abb_value(T post_i, const Macro<Q, T> &m, T rho_w, T drho_w)
{
    constexpr T w = weight<Q, T>(i);
    const T cu = cdot<Q, i>(m.u);
    const T X = fmadd(T(4.5) * cu, cu, T(-1.5) * m.uu);
    return fmadd(T(2) * w, fmadd(rho_w, X, drho_w), -post_i);
}

// Addressing: every access is (uniform 64-bit slot base) + (32-bit byte
// offset) so loads and stores use the scalar-base / vector-offset form and a
// cell's accesses share one offset register.  The runtime guarantees that a
// slot spans less than 2^31 bytes.
template <typename ST>
__device__ __forceinline__ const char *slot_base(const SweepArgs &a, const DevBlock &B, int i)
{
    return reinterpret_cast<const char *>(a.arena) + (B.pop + (int64_t)i * B.slot) * (int64_t)sizeof(ST);
}

template <typename ST>
__device__ __forceinline__ ST *at(const char *base, uint32_t byte_off)
{
    return reinterpret_cast<ST *>(const_cast<char *>(base) + (uint64_t)byte_off);
}

__device__ __forceinline__ uint32_t cell_off(const DevBlock &B, int x, int y, int z)
{
    return (uint32_t)((z + 1) * B.plane + (y + B.gy) * B.pitch + B.xoff + x);
}

// A copy of the descriptor whose addressing fields the compiler cannot
// relate to the original: the stores of a sweep then compute their slot
// bases after the collision instead of sharing the loads' bases, which
// would keep some 40-60 uniform registers live through the collision and
// spill them into vector lanes (a VALU instruction per spill and reload).
__device__ __forceinline__ DevBlock fresh_bases(const DevBlock &B)
{
    DevBlock C = B;
    int64_t z = 0;
    int32_t zi = 0;
    asm volatile("" : "+s"(z), "+s"(zi));
    C.pop += z;
    C.slot += z;
    C.pitch += zi;
    C.plane += zi;
    return C;
}

template <int Q, int i>
__device__ __forceinline__ int link_delta(const DevBlock &B)
{
    return cx<Q>(i) + cy<Q>(i) * B.pitch + cz<Q>(i) * B.plane;
}

// Odd-sweep access of link i as one uniform base plus a per-lane choice of
// two uniform addends (regular link / bounce-back or anti-bounce-back link).
// Incoming: regular = slot opp(i) of x - c_i, special = slot i of x.
// Outgoing: regular = slot i of x + c_i, special = slot opp(i) of x.
// Slots i and opp(i) are adjacent, so the lower address is known at compile
// time and both addends are non-negative.
template <typename ST>
struct Alt {
    const char *base;
    uint32_t add_reg, add_sp;
};

// regular access: slot sr shifted by dr elements; special access: slot ss.
template <typename ST>
__device__ __forceinline__ Alt<ST> pick_alt(const SweepArgs &a, const DevBlock &B, int sr, int dr, int ss)
{
    const int64_t er = (B.pop + (int64_t)sr * B.slot + dr) * (int64_t)sizeof(ST);
    const int64_t es = (B.pop + (int64_t)ss * B.slot) * (int64_t)sizeof(ST);
    Alt<ST> p;
    if (sr < ss) {  // regular access is lower (slots differ by one, |dr| < slot)
        p.base = reinterpret_cast<const char *>(a.arena) + er;
        p.add_reg = 0;
        p.add_sp = (uint32_t)(es - er);
    } else {
        p.base = reinterpret_cast<const char *>(a.arena) + es;
        p.add_reg = (uint32_t)(er - es);
        p.add_sp = 0;
    }
    return p;
}

template <int Q, typename ST, int i>
__device__ __forceinline__ Alt<ST> alt_in(const SweepArgs &a, const DevBlock &B)
{
    return pick_alt<ST>(a, B, opp(i), -link_delta<Q, i>(B), i);
}
template <int Q, typename ST, int i>
__device__ __forceinline__ Alt<ST> alt_out(const SweepArgs &a, const DevBlock &B)
{
    return pick_alt<ST>(a, B, i, link_delta<Q, i>(B), opp(i));
}

// Byte offsets of a cell for regular accesses shifted by 0, -1 and +1 cells
// along x.  Blocks of one x-run share their rows, so a shifted access across
// an x face inside the run is the next element of the row.  A run that spans
// a periodic axis has no x exchange: the odd sweep and every reader of the
// swapped layout wrap the shifted accesses of its end cells around the row
// instead, so that the sweep writes whole cache lines at both row ends.
struct XOff {
    uint32_t at, left, right;
};
template <typename ST>
__device__ __forceinline__ XOff xoffsets(const DevBlock &B, uint32_t off, int x)
{
    XOff o;
    o.at = off * (uint32_t)sizeof(ST);
    o.left = o.at + (x == 0 ? (uint32_t)B.wraplo * (uint32_t)sizeof(ST) : 0u);
    o.right = o.at - (x == B.n[0] - 1 ? (uint32_t)B.wraphi * (uint32_t)sizeof(ST) : 0u);
    return o;
}
// Offset of the regular access shifted by dx in {-1, 0, 1} cells along x.
template <int dx>
__device__ __forceinline__ uint32_t xshift(const XOff &o)
{
    return dx < 0 ? o.left : (dx > 0 ? o.right : o.at);
}

// Hint of an x-shifted (odd-sweep / swapped-layout) access of a population
// with x velocity cx.  AO (aligned only): the non-temporal hint goes to the
// accesses of populations with cx = 0, which cover whole lines per
// wavefront; those with cx != 0 sit one element off the row alignment and
// share their edge lines with the neighbouring wavefronts, which meet in L2
// only without the hint.
template <bool NT, int cx, bool AO>
__device__ __forceinline__ constexpr bool nt_shifted()
{
    return NT && (!AO || cx == 0);
}

// Gather the populations f_i(x) of a fluid cell for the current layout:
// natural (after an odd sweep / init) reads slot i of x; swapped (after an
// even sweep) reads slot opp(i) of x - c_i, or slot i of x on bounce-back /
// anti-bounce-back links.
template <int Q, typename ST, bool SWAPPED, bool NT = true, bool AO = false>
__device__ __forceinline__ void gather(const SweepArgs &a, const DevBlock &B, uint32_t off, int x, int y, int z,
                                       uint32_t special, typename Codec<ST>::T (&f)[Q])
{
    const XOff o = xoffsets<ST>(B, off, x);
    if constexpr (SWAPPED) {
        if (!__any(special != 0u)) {
            // no lane of the wave has a bounce-back link: every access is the
            // regular one, a uniform base and the lane's shifted offset
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                const Alt<ST> p = alt_in<Q, ST, i>(a, B);
                f[i] = ldv<Q, ST, nt_shifted<NT, cx<Q>(i), AO>()>(at<ST>(p.base + p.add_reg, xshift<-cx<Q>(i)>(o)), i);
            });
        } else {
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                const Alt<ST> p = alt_in<Q, ST, i>(a, B);
                f[i] = ldv<Q, ST, nt_shifted<NT, cx<Q>(i), AO>()>(at<ST>(p.base, ((special >> opp(i)) & 1u) ? o.at + p.add_sp
                                                                             : xshift<-cx<Q>(i)>(o) + p.add_reg),
                                      i);
            });
        }
    } else {
        sfor<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            f[i] = ldv<Q, ST, NT>(at<ST>(slot_base<ST>(a, B, i), o.at), i);
        });
    }
    if constexpr (SWAPPED) {
        // x faces shared with another block: populations entering through
        // the face come straight from the neighbour's cells (no x exchange;
        // the regular loads above read this block's unused ghost column)
        if (x == 0 && B.nbx[0] >= 0) {
            const DevBlock N = a.blocks[B.nbx[0]];
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                if constexpr (cx<Q>(i) == 1)
                    if (!((special >> opp(i)) & 1u))
                        f[i] = ldv<Q, ST, false>(at<ST>(slot_base<ST>(a, N, opp(i)),
                                                        cell_off(N, N.n[0] - 1, y - cy<Q>(i), z - cz<Q>(i)) * (uint32_t)sizeof(ST)),
                                                 i);
            });
        }
        if (x == B.n[0] - 1 && B.nbx[1] >= 0) {
            const DevBlock N = a.blocks[B.nbx[1]];
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                if constexpr (cx<Q>(i) == -1)
                    if (!((special >> opp(i)) & 1u))
                        f[i] = ldv<Q, ST, false>(
                            at<ST>(slot_base<ST>(a, N, opp(i)), cell_off(N, 0, y - cy<Q>(i), z - cz<Q>(i)) * (uint32_t)sizeof(ST)), i);
            });
        }
    }
}

// Store the post-collision populations of a fluid cell: even sweep into
// slot opp(i) of x; odd sweep into slot i of x + c_i, or slot opp(i) of x on
// bounce-back / anti-bounce-back links.
template <int Q, typename ST, bool ODD, bool NT = true, bool AO = false>
__device__ __forceinline__ void scatter(const SweepArgs &a, const DevBlock &B, uint32_t off, int x, int y, int z,
                                        uint32_t special, const typename Codec<ST>::T (&f)[Q], uint32_t h)
{
    const XOff o = xoffsets<ST>(B, off, x);
    if constexpr (ODD) {
        if (!__any(special != 0u)) {  // regular stores only (see gather)
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                const Alt<ST> p = alt_out<Q, ST, i>(a, B);
                stv_sr<Q, ST, nt_shifted<NT, cx<Q>(i), AO>()>(at<ST>(p.base + p.add_reg, xshift<cx<Q>(i)>(o)), f[i], i, h);
            });
        } else {
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                const Alt<ST> p = alt_out<Q, ST, i>(a, B);
                stv_sr<Q, ST, nt_shifted<NT, cx<Q>(i), AO>()>(at<ST>(p.base, ((special >> i) & 1u) ? o.at + p.add_sp : xshift<cx<Q>(i)>(o) + p.add_reg),
                                  f[i], i, h);
            });
        }
    } else {
        sfor<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            stv_sr<Q, ST, NT>(at<ST>(slot_base<ST>(a, B, opp(i)), o.at), f[i], i, h);
        });
    }
    if constexpr (ODD) {
        // populations leaving through an x face shared with another block go
        // straight into the neighbour's cells (the regular stores above
        // wrote this block's unused ghost column)
        if (x == B.n[0] - 1 && B.nbx[1] >= 0) {
            const DevBlock N = a.blocks[B.nbx[1]];
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                if constexpr (cx<Q>(i) == 1)
                    if (!((special >> i) & 1u))
                        stv_sr<Q, ST, false>(
                            at<ST>(slot_base<ST>(a, N, i), cell_off(N, 0, y + cy<Q>(i), z + cz<Q>(i)) * (uint32_t)sizeof(ST)), f[i],
                            i, h);
            });
        }
        if (x == 0 && B.nbx[0] >= 0) {
            const DevBlock N = a.blocks[B.nbx[0]];
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                if constexpr (cx<Q>(i) == -1)
                    if (!((special >> i) & 1u))
                        stv_sr<Q, ST, false>(
                            at<ST>(slot_base<ST>(a, N, i), cell_off(N, N.n[0] - 1, y + cy<Q>(i), z + cz<Q>(i)) * (uint32_t)sizeof(ST)),
                            f[i], i, h);
            });
        }
    }
}

// Regular incoming access of link i (slot opp(i) of x - c_i) as the direct
// odd sweep makes it, returned as raw storage bits.
template <int Q, typename ST, int i>
__device__ __forceinline__ typename Codec<ST>::Raw load_regular_in(const SweepArgs &a, const DevBlock &B, const XOff &o,
                                                                   int x, int y, int z)
{
    if constexpr (cx<Q>(i) == 1) {
        if (x == 0 && B.nbx[0] >= 0) {
            const DevBlock N = a.blocks[B.nbx[0]];
            return ldraw<ST, false>(at<ST>(slot_base<ST>(a, N, opp(i)),
                                           cell_off(N, N.n[0] - 1, y - cy<Q>(i), z - cz<Q>(i)) * (uint32_t)sizeof(ST)));
        }
    } else {
        if (x == B.n[0] - 1 && B.nbx[1] >= 0) {
            const DevBlock N = a.blocks[B.nbx[1]];
            return ldraw<ST, false>(
                at<ST>(slot_base<ST>(a, N, opp(i)), cell_off(N, 0, y - cy<Q>(i), z - cz<Q>(i)) * (uint32_t)sizeof(ST)));
        }
    }
    const Alt<ST> p = alt_in<Q, ST, i>(a, B);
    return ldraw<ST, false>(at<ST>(p.base, xshift<-cx<Q>(i)>(o) + p.add_reg));
}
// Regular outgoing access of link i (slot i of x + c_i) as the direct odd
// sweep makes it.
template <int Q, typename ST, int i>
__device__ __forceinline__ void store_regular_out(const SweepArgs &a, const DevBlock &B, const XOff &o, int x, int y,
                                                  int z, typename Codec<ST>::T v, uint32_t h)
{
    if constexpr (cx<Q>(i) == 1) {
        if (x == B.n[0] - 1 && B.nbx[1] >= 0) {
            const DevBlock N = a.blocks[B.nbx[1]];
            stv_sr<Q, ST, false>(at<ST>(slot_base<ST>(a, N, i), cell_off(N, 0, y + cy<Q>(i), z + cz<Q>(i)) * (uint32_t)sizeof(ST)), v,
                                 i, h);
            return;
        }
    } else {
        if (x == 0 && B.nbx[0] >= 0) {
            const DevBlock N = a.blocks[B.nbx[0]];
            stv_sr<Q, ST, false>(
                at<ST>(slot_base<ST>(a, N, i), cell_off(N, N.n[0] - 1, y + cy<Q>(i), z + cz<Q>(i)) * (uint32_t)sizeof(ST)), v, i,
                h);
            return;
        }
    }
    const Alt<ST> p = alt_out<Q, ST, i>(a, B);
    stv_sr<Q, ST, false>(at<ST>(p.base, xshift<cx<Q>(i)>(o) + p.add_reg), v, i, h);
}

// ---------------------------------------------------------------------------
// The sweep kernel (one launch covers every tile of every block)
// ---------------------------------------------------------------------------
#ifndef WLB_WAVES_PER_EU
#define WLB_WAVES_PER_EU 1
#endif
// NT: the population accesses carry the non-temporal hint (the autotuner
// chooses it per parity).
// AO: the odd sweep's hint on its aligned accesses only (nt_shifted).
template <int Q, int COLL, typename ST, bool ODD, bool NT, bool AO>
__device__ __forceinline__ void sweep_tiles(const SweepArgs &a)
{
    using T = typename Codec<ST>::T;
    for (int t = first_tile(a); t < a.nstiles; t += gridDim.x) {
        const CollParams<T> cp = coll_params<T>(a);
        const int4 tv = a.stiles[t];
        const CellPos c = sweep_cell(a, tv, threadIdx.x);
        if (!c.valid) continue;
        const DevBlock B = a.blocks[tv.x];
        uint32_t mask = 0;
        if (B.mask >= 0) mask = a.masks[B.mask + (int64_t)c.z * B.mplane + c.y * B.mpitch + c.x];
        // The even sweep loads and stores a solid cell's slots along with the
        // fluid cells' (no collision, each value back into its own slot), so
        // that every load and store of the wavefront covers whole lines in
        // one instruction, which the non-temporal hint needs (a line split
        // between two instructions is fetched twice).  The odd sweep, whose
        // stores go to the neighbours, leaves solid cells alone.
        constexpr bool kMoveSolid = !ODD && !std::is_same_v<ST, cover_t>;
        const bool solid = (mask & kSolidBit) != 0;
        if (!kMoveSolid && solid) continue;
        const Links<Q> L = classify<Q>(mask, B, c.x, c.y, c.z, a);
        const uint32_t off = cell_off(B, c.x, c.y, c.z);
        const uint32_t special = L.bb | L.alo | L.ahi;
        T f[Q];
        gather<Q, ST, ODD, NT, AO>(a, B, off, c.x, c.y, c.z, special, f);
        const uint32_t h = kStochastic<ST> ? state_hash<Q, T>(f, global_cell(a, B, c.x, c.y, c.z)) : 0u;
        if (!solid) {
            const Macro<Q, T> m = collide<Q, COLL, T, AccOf<ST>>(f, cp);
            if (L.alo | L.ahi) {
                const T rin = (T)a.rho_in, rout = (T)a.rho_out;
                const T drin = (T)(a.rho_in - 1.0), drout = (T)(a.rho_out - 1.0);
                sfor<Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    const bool lo = (L.alo >> i) & 1u, hi = (L.ahi >> i) & 1u;
                    if (lo | hi) f[i] = abb_value<Q, i, T>(f[i], m, lo ? rin : rout, lo ? drin : drout);
                });
            }
        } else {
            // the store of link i goes to slot opp(i): swap each pair so that
            // slot opp(i) gets its own value back (the codecs reproduce a
            // decoded value exactly, stochastic rounding included)
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                if constexpr (i < opp(i)) {
                    const T t = f[i];
                    f[i] = f[opp(i)];
                    f[opp(i)] = t;
                }
            });
        }
        scatter<Q, ST, ODD, NT, AO>(a, fresh_bases(B), off, c.x, c.y, c.z, special, f, h);
    }
}

template <int Q, int COLL, typename ST, bool ODD, bool NT>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(WLB_WAVES_PER_EU, 8))) void sweep_kernel(
    const SweepArgs a)
{
    sweep_tiles<Q, COLL, ST, ODD, NT, false>(a);
}

// Odd sweep with the non-temporal hint on its aligned accesses only (the
// populations with c_x = 0); an autotuner candidate beside the odd sweep
// with the hint on every access and the one without it.
template <int Q, int COLL, typename ST>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(WLB_WAVES_PER_EU, 8))) void sweep_odd_aligned_nt_kernel(
    const SweepArgs a)
{
    sweep_tiles<Q, COLL, ST, true, true, true>(a);
}

// ---------------------------------------------------------------------------
// Odd sweep with LDS staging of the x-shifted populations.  A tile is a box
// of whole x-row segments.  Populations whose link has c_x != 0 would be read
// from x - c_x and written to x + c_x, one element off the row alignment;
// instead every lane moves its own aligned element between memory and an
// LDS row buffer, and the one-cell shift happens in LDS.  Every global access
// of the sweep is then a full-line aligned access.
//  - A segment that is a whole row of a block wrapping onto itself along x
//    shifts around the row inside LDS: nothing leaves the row buffer.
//  - Any other segment keeps one halo element per row end, loaded from where
//    the direct sweep would read it (the next cell, the block's other end,
//    its ghost column, or an x-neighbour block), and stores the one target
//    outside the segment directly, to where the direct sweep would write it.
// One buffer serves the incoming and the outgoing populations.
// ---------------------------------------------------------------------------
template <int Q>
__host__ __device__ constexpr int n_xshift()
{
    int n = 0;
    for (int i = 0; i < Q; ++i) n += cx<Q>(i) != 0;
    return n;
}
template <int Q>
__host__ __device__ constexpr int xshift_index(int i)
{
    int n = 0;
    for (int j = 0; j < i; ++j) n += cx<Q>(j) != 0;
    return n;
}
// LDS bytes of the staged odd sweep for row buffers of `stride` elements.
template <int Q, typename Raw>
__host__ __device__ constexpr size_t lds_stage_bytes(int stride)
{
    return (((size_t)n_xshift<Q>() * stride * sizeof(Raw) + 15) & ~(size_t)15) + kWG * 4;
}

// RING: every tile is a whole row of a self-wrapping block (chosen on the
// host), so the halo and out-of-segment paths are compiled out.
template <int Q, int COLL, typename ST, bool RING, bool NT>
__global__ __launch_bounds__(kWG) void sweep_odd_lds_kernel(const SweepArgs a)
{
    using T = typename Codec<ST>::T;
    using Raw = typename Codec<ST>::Raw;
    constexpr int NSH = n_xshift<Q>();
    extern __shared__ __align__(16) unsigned char smem[];
    const int stride = a.lds_stride;
    Raw *buf = reinterpret_cast<Raw *>(smem);  // row buffers [NSH][stride], incoming then outgoing
    uint32_t *info = reinterpret_cast<uint32_t *>(smem + (((size_t)NSH * stride * sizeof(Raw) + 15) & ~(size_t)15));
    const CollParams<T> cp = coll_params<T>(a);
    const int l = threadIdx.x;
    for (int t = first_tile(a); t < a.nstiles; t += gridDim.x) {
        const int4 tv = a.stiles[t];
        const int ex = tv.y >> 16, ey = tv.z >> 16, ez = tv.w >> 16;
        const bool valid = l < ex * ey * ez;
        const int lx = l % ex, lr = l / ex;  // lr = row within the tile = ly + ey * lz
        const int x = (tv.y & 0xffff) + lx, y = (tv.z & 0xffff) + lr % ey, z = (tv.w & 0xffff) + lr / ey;
        const DevBlock B = a.blocks[tv.x];
        const bool ring = RING || (B.wrapx != 0 && ex == B.n[0]);  // whole row of a self-wrapping block
        uint32_t mask = 0;
        if (valid && B.mask >= 0) mask = a.masks[B.mask + (int64_t)z * B.mplane + y * B.mpitch + x];
        const bool active = valid && !(mask & kSolidBit);
        const Links<Q> L = classify<Q>(mask, B, x, y, z, a);
        const uint32_t special = L.bb | L.alo | L.ahi;
        const uint32_t off = valid ? cell_off(B, x, y, z) : 0u;
        const uint32_t boff = off * (uint32_t)sizeof(ST);
        const XOff o = xoffsets<ST>(B, off, x);
        const int row = lr * (ex + 2) + 1;  // element 0 of this lane's row segment in its buffer
        const int rb = row + lx;            // this lane's own element
        // lane of the same row segment dx cells along x (around the row on a ring)
        auto lane_at = [&](int dx) {
            int s = lx + dx;
            if (ring) s += s < 0 ? ex : (s >= ex ? -ex : 0);
            return s;
        };
        info[l] = active ? special : 0xffffffffu;
        // ---- all loads in one phase: the shifted incoming populations are
        // staged (aligned element at (x, y - c_y, z - c_z) of slot opp(i),
        // plus the halo one cell outside a segment that is not a ring), the
        // others are read directly (they are row-aligned either way).
        T f[Q];
        if (valid) {
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                if constexpr (cx<Q>(i) != 0) {
                    constexpr int k = xshift_index<Q>(i);
                    const char *base = slot_base<ST>(a, B, opp(i)) -
                                       (int64_t)(cy<Q>(i) * B.pitch + cz<Q>(i) * B.plane) * (int64_t)sizeof(ST);
                    buf[k * stride + rb] = ldraw<ST, NT>(at<ST>(base, boff));
                    if (!RING && !ring) {
                        if (cx<Q>(i) == 1 && lx == 0) buf[k * stride + rb - 1] = load_regular_in<Q, ST, i>(a, B, o, x, y, z);
                        if (cx<Q>(i) == -1 && lx == ex - 1)
                            buf[k * stride + rb + 1] = load_regular_in<Q, ST, i>(a, B, o, x, y, z);
                    }
                    if ((special >> opp(i)) & 1u) f[i] = ldv<Q, ST, NT>(at<ST>(slot_base<ST>(a, B, i), boff), i);
                } else {
                    const Alt<ST> p = alt_in<Q, ST, i>(a, B);
                    f[i] = ldv<Q, ST, NT>(at<ST>(p.base, boff + (((special >> opp(i)) & 1u) ? p.add_sp : p.add_reg)), i);
                }
            });
        }
        __syncthreads();
        if (active) {
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                if constexpr (cx<Q>(i) != 0) {
                    constexpr int k = xshift_index<Q>(i);
                    if (!((special >> opp(i)) & 1u)) f[i] = dec_slot<Q, ST>(buf[k * stride + row + lane_at(-cx<Q>(i))], i);
                }
            });
        }
        __syncthreads();  // the buffer now takes the outgoing populations
        if (active) {
            const uint32_t h = kStochastic<ST> ? state_hash<Q, T>(f, global_cell(a, B, x, y, z)) : 0u;
            const Macro<Q, T> m = collide<Q, COLL, T, AccOf<ST>>(f, cp);
            if (L.alo | L.ahi) {
                const T rin = (T)a.rho_in, rout = (T)a.rho_out;
                const T drin = (T)(a.rho_in - 1.0), drout = (T)(a.rho_out - 1.0);
                sfor<Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    const bool lo = (L.alo >> i) & 1u, hi = (L.ahi >> i) & 1u;
                    if (lo | hi) f[i] = abb_value<Q, i, T>(f[i], m, lo ? rin : rout, lo ? drin : drout);
                });
            }
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                const bool sp = (special >> i) & 1u;
                if constexpr (cx<Q>(i) == 0) {
                    const Alt<ST> p = alt_out<Q, ST, i>(a, B);
                    stv_sr<Q, ST, NT>(at<ST>(p.base, boff + (sp ? p.add_sp : p.add_reg)), f[i], i, h);
                } else {
                    constexpr int k = xshift_index<Q>(i);
                    if (sp) {
                        stv_sr<Q, ST, NT>(at<ST>(slot_base<ST>(a, B, opp(i)), boff), f[i], i, h);
                    } else if (!RING && !ring && ((cx<Q>(i) == 1 && lx == ex - 1) || (cx<Q>(i) == -1 && lx == 0))) {
                        store_regular_out<Q, ST, i>(a, B, o, x, y, z, f[i], h);  // target outside the segment
                    } else {
                        buf[k * stride + row + lane_at(cx<Q>(i))] = enc_result<Q, ST>(f[i], i, h);
                    }
                }
            });
        }
        __syncthreads();
        // ---- aligned stores of the shifted outgoing populations: this lane
        // stores the element at (x, y + c_y, z + c_z) of slot i when its
        // writer, the lane c_x cells back along the row segment, is a fluid
        // cell with a regular link i.
        if (valid) {
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                if constexpr (cx<Q>(i) != 0) {
                    constexpr int k = xshift_index<Q>(i);
                    const int lw = lane_at(-cx<Q>(i));
                    if (lw >= 0 && lw < ex && !((info[l - lx + lw] >> i) & 1u)) {
                        const char *base = slot_base<ST>(a, B, i) +
                                           (int64_t)(cy<Q>(i) * B.pitch + cz<Q>(i) * B.plane) * (int64_t)sizeof(ST);
                        straw<ST, NT>(at<ST>(base, boff), buf[k * stride + rb]);
                    }
                }
            });
        }
        // LDS and info are reused by the next tile of this workgroup (t is
        // the same in all its waves, so all or none of them wait)
        if (t + (int)gridDim.x < a.nstiles) __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Odd sweep over whole rows with V = 16 / (element bytes) consecutive cells
// per lane, so that every population access of a lane is one 16-byte vector.
// For blocks that wrap onto themselves along x and hold no solid cells: all
// cells of a row then share their link classes (walls and density faces lie
// on y / z faces), and a row's populations move as whole vectors.  A
// population with c_x != 0 is read from (written to) the aligned vector of
// the lane's own cells in the row shifted by c_y, c_z; the one-cell x shift
// is done with lane moves, each lane taking the element at the end of its
// neighbour lane's vector.  A row held by one wavefront rotates within its
// lanes (the x wrap); where a row spans several wavefronts, the lane at a
// wavefront edge reads (writes) the element that crosses the edge from
// (to) memory itself, and the lane on the other side leaves that element
// out of its vector store.  A workgroup takes floor(256 / (n0 / V)) rows
// (tiles built on the host, a.vtiles).
// ---------------------------------------------------------------------------
// Value of `v` held by lane `src` of the wavefront.
template <typename Raw>
__device__ __forceinline__ Raw lane_get(Raw v, int src)
{
    if constexpr (sizeof(Raw) == 8) {
        const uint64_t b = (uint64_t)v;
        const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)b);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)(b >> 32));
        return (Raw)(((uint64_t)hi << 32) | lo);
    } else {
        return (Raw)(uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)v);
    }
}

template <typename ST>
constexpr int kRowVec = 16 / (int)sizeof(typename Codec<ST>::Raw);

// A lane's row vector: 16 bytes as four 32-bit words, elements of the
// storage type packed in order (two 16-bit elements per word).
typedef uint32_t RowWords __attribute__((ext_vector_type(4)));
template <typename ST>
__device__ __forceinline__ typename Codec<ST>::Raw row_get(const RowWords &w, int k)
{
    using Raw = typename Codec<ST>::Raw;
    if constexpr (sizeof(Raw) == 8)
        return (Raw)w[2 * k] | ((Raw)w[2 * k + 1] << 32);
    else if constexpr (sizeof(Raw) == 4)
        return (Raw)w[k];
    else
        return (Raw)((w[k >> 1] >> (16 * (k & 1))) & 0xffffu);
}
template <typename ST>
__device__ __forceinline__ void row_set(RowWords &w, int k, typename Codec<ST>::Raw r)
{
    using Raw = typename Codec<ST>::Raw;
    if constexpr (sizeof(Raw) == 8) {
        w[2 * k] = (uint32_t)r;
        w[2 * k + 1] = (uint32_t)((uint64_t)r >> 32);
    } else if constexpr (sizeof(Raw) == 4) {
        w[k] = (uint32_t)r;
    } else {
        const uint32_t sh = 16u * (uint32_t)(k & 1);
        w[k >> 1] = (w[k >> 1] & ~(0xffffu << sh)) | ((uint32_t)r << sh);
    }
}
// The vector shifted by one element: towards higher x (cells x0 - 1 ..
// x0 + V - 2, `in` entering at element 0) or towards lower x (cells x0 + 1
// .. x0 + V, `in` entering at element V - 1).
template <typename ST>
__device__ __forceinline__ RowWords row_shift_up(const RowWords &w, typename Codec<ST>::Raw in)
{
    constexpr int V = kRowVec<ST>;
    RowWords o;
    row_set<ST>(o, 0, in);
#pragma unroll
    for (int k = 1; k < V; ++k) row_set<ST>(o, k, row_get<ST>(w, k - 1));
    return o;
}
template <typename ST>
__device__ __forceinline__ RowWords row_shift_down(const RowWords &w, typename Codec<ST>::Raw in)
{
    constexpr int V = kRowVec<ST>;
    RowWords o;
#pragma unroll
    for (int k = 0; k < V - 1; ++k) row_set<ST>(o, k, row_get<ST>(w, k + 1));
    row_set<ST>(o, V - 1, in);
    return o;
}

// Elements [k0, k1) of a row vector to memory (the counting storage adds one
// per element).
template <typename ST, bool NT>
__device__ __forceinline__ void store_elems(char *p, const RowWords &w, int k0, int k1)
{
    using Raw = typename Codec<ST>::Raw;
    constexpr int V = kRowVec<ST>;
    if constexpr (std::is_same_v<ST, cover_t>) {
        for (int k = k0; k < k1; ++k) atomicAdd(reinterpret_cast<uint32_t *>(p) + k, 1u);
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k)
            if (k >= k0 && k < k1) mem_st<false>(reinterpret_cast<Raw *>(p) + k, row_get<ST>(w, k));
    }
}
template <typename ST, bool NT>
__device__ __forceinline__ void store_vec(char *p, const RowWords &w)
{
    if constexpr (std::is_same_v<ST, cover_t>)
        store_elems<ST, NT>(p, w, 0, kRowVec<ST>);
    else
        mem_st<NT>(reinterpret_cast<RowWords *>(p), w);
}

template <int Q, int COLL, typename ST, bool NT>
__global__ __launch_bounds__(kWG) void sweep_odd_vec_kernel(const SweepArgs a)
{
    using T = typename Codec<ST>::T;
    using Raw = typename Codec<ST>::Raw;
    constexpr int V = kRowVec<ST>;
    constexpr uint32_t E = (uint32_t)sizeof(ST);
    const int tid = threadIdx.x, lane = tid & 63, wlo = tid & ~63;
    for (int t = blockIdx.x; t < a.nvtiles; t += gridDim.x) {
        const int4 tv = a.vtiles[t];
        const DevBlock B = a.blocks[tv.x];
        const int n0 = B.n[0], L = n0 / V;  // lanes per row (the host checks n0 % V == 0, L <= 256)
        const int ey = tv.z >> 16, ez = tv.w >> 16;
        const int r = tid / L;
        if (r >= ey * ez) continue;  // whole rows stay active together
        const int rlo = r * L, rhi = rlo + L;
        const int x0 = (tid - rlo) * V;
        const int y = (tv.z & 0xffff) + r % ey, z = (tv.w & 0xffff) + r / ey;
        const bool inwave = rlo >= wlo && rhi <= wlo + 64;  // the row lies in this wavefront: rotate
        const bool has_prev = tid > rlo && tid > wlo, has_next = tid + 1 < rhi && tid + 1 < wlo + 64;
        const int src_prev = has_prev ? lane - 1 : (inwave ? ((rhi - 1) & 63) : lane);
        const int src_next = has_next ? lane + 1 : (inwave ? (rlo & 63) : lane);
        const bool edge_prev = !has_prev && !inwave, edge_next = !has_next && !inwave;
        // every access is a uniform base (slot and row shift) plus one of
        // three per-lane byte offsets: the lane's vector, and the elements
        // one cell before and after it (with the x wrap)
        const uint32_t row0 = cell_off(B, 0, y, z) * E;
        const uint32_t ov = row0 + (uint32_t)x0 * E;
        const uint32_t om1 = row0 + (uint32_t)(x0 == 0 ? n0 - 1 : x0 - 1) * E;
        const uint32_t opv = row0 + (uint32_t)(x0 + V == n0 ? 0 : x0 + V) * E;
        const Links<Q> Lk = classify<Q>(0u, B, 0, y, z, a);  // the same for every cell of the row
        const uint32_t special = Lk.bb | Lk.alo | Lk.ahi;
        // ---- incoming populations of the lane's cells
        RowWords v[Q];
        sfor<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if ((special >> opp(i)) & 1u) {
                // bounce-back / anti-bounce-back link: the cell's own slot i
                v[i] = mem_ld<NT>(reinterpret_cast<const RowWords *>(slot_base<ST>(a, B, i) + (uint64_t)ov));
            } else {
                const char *base = slot_base<ST>(a, B, opp(i)) -
                                   (int64_t)(cy<Q>(i) * B.pitch + cz<Q>(i) * B.plane) * (int64_t)E;
                const RowWords w = mem_ld<NT>(reinterpret_cast<const RowWords *>(base + (uint64_t)ov));
                if constexpr (cx<Q>(i) == 1) {  // cells x0 - 1 .. x0 + V - 2
                    Raw in = lane_get<Raw>(row_get<ST>(w, V - 1), src_prev);
                    if (edge_prev) in = mem_ld<false>(reinterpret_cast<const Raw *>(base + (uint64_t)om1));
                    v[i] = row_shift_up<ST>(w, in);
                } else if constexpr (cx<Q>(i) == -1) {  // cells x0 + 1 .. x0 + V
                    Raw in = lane_get<Raw>(row_get<ST>(w, 0), src_next);
                    if (edge_next) in = mem_ld<false>(reinterpret_cast<const Raw *>(base + (uint64_t)opv));
                    v[i] = row_shift_down<ST>(w, in);
                } else {
                    v[i] = w;
                }
            }
        });
        // ---- collide the V cells one after the other
        const T rin = (T)a.rho_in, rout = (T)a.rho_out;
        const T drin = (T)(a.rho_in - 1.0), drout = (T)(a.rho_out - 1.0);
        const CollParams<T> cp = coll_params<T>(a);
        sfor<V>([&](auto K) {
            constexpr int k = decltype(K)::value;
            T f[Q];
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                f[i] = dec_slot<Q, ST>(row_get<ST>(v[i], k), i);
            });
            const uint32_t h = kStochastic<ST> ? state_hash<Q, T>(f, global_cell(a, B, x0 + k, y, z)) : 0u;
            const Macro<Q, T> m = collide<Q, COLL, T, AccOf<ST>>(f, cp);
            if (Lk.alo | Lk.ahi) {
                sfor<Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    const bool lo = (Lk.alo >> i) & 1u, hi = (Lk.ahi >> i) & 1u;
                    if (lo | hi) f[i] = abb_value<Q, i, T>(f[i], m, lo ? rin : rout, lo ? drin : drout);
                });
            }
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                row_set<ST>(v[i], k, enc_result<Q, ST>(f[i], i, h));
            });
            __builtin_amdgcn_sched_barrier(0);  // one cell's collision at a time
        });
        // ---- outgoing populations
        sfor<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const RowWords w = v[i];
            if ((special >> i) & 1u) {
                // bounce-back / anti-bounce-back: slot opp(i) of the cell itself
                store_vec<ST, NT>(const_cast<char *>(slot_base<ST>(a, B, opp(i))) + (uint64_t)ov, w);
            } else {
                char *base = const_cast<char *>(slot_base<ST>(a, B, i)) +
                             (int64_t)(cy<Q>(i) * B.pitch + cz<Q>(i) * B.plane) * (int64_t)E;
                if constexpr (cx<Q>(i) == 1) {  // positions x0 .. x0 + V - 1 take cells x0 - 1 .. x0 + V - 2
                    const RowWords o = row_shift_up<ST>(w, lane_get<Raw>(row_get<ST>(w, V - 1), src_prev));
                    if (edge_prev)
                        store_elems<ST, NT>(base + (uint64_t)ov, o, 1, V);  // position x0 comes from the other wave
                    else
                        store_vec<ST, NT>(base + (uint64_t)ov, o);
                    if (edge_next) store_elems<ST, NT>(base + (uint64_t)opv - (V - 1) * E, w, V - 1, V);
                } else if constexpr (cx<Q>(i) == -1) {  // positions x0 .. x0 + V - 1 take cells x0 + 1 .. x0 + V
                    const RowWords o = row_shift_down<ST>(w, lane_get<Raw>(row_get<ST>(w, 0), src_next));
                    if (edge_next)
                        store_elems<ST, NT>(base + (uint64_t)ov, o, 0, V - 1);  // position x0 + V - 1 comes from the other wave
                    else
                        store_vec<ST, NT>(base + (uint64_t)ov, o);
                    if (edge_prev) store_elems<ST, NT>(base + (uint64_t)om1, w, 0, 1);
                } else {
                    store_vec<ST, NT>(base + (uint64_t)ov, w);
                }
            }
        });
    }
}

// ---------------------------------------------------------------------------
// Sweep with the learned closure (D3Q19, SRT/TRT, FP32 collision).  The MLP
// is evaluated by the whole wavefront, so every lane runs the tile body;
// lanes without a fluid cell compute on zeros and store nothing.  Falls back
// to the Smagorinsky time when a feature is outside |x| <= 8 or the output is
// not finite.
// ---------------------------------------------------------------------------
template <int COLL, typename ST, bool ODD>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(4, 8))) void sweep_mlp_kernel(const SweepArgs a)
{
    constexpr int Q = 19;
    using T = float;
    static_assert(std::is_same<typename Codec<ST>::T, float>::value, "MLP closure runs in FP32");
    const CollParams<T> cp = coll_params<T>(a);
    __shared__ MlpDev net_s;
    __shared__ T park[Q][kWG];
    mlp_stage(&net_s, a.mlp);
    const MlpDev *net = &net_s;
    for (int t = first_tile(a); t < a.nstiles; t += gridDim.x) {
        const int4 tv = a.stiles[t];
        const CellPos c = sweep_cell(a, tv, threadIdx.x);
        const DevBlock B = a.blocks[tv.x];
        uint32_t mask = 0;
        if (c.valid && B.mask >= 0) mask = a.masks[B.mask + (int64_t)c.z * B.mplane + c.y * B.mpitch + c.x];
        const bool active = c.valid && !(mask & kSolidBit);
        const Links<Q> L = classify<Q>(mask, B, c.x, c.y, c.z, a);
        const uint32_t special = L.bb | L.alo | L.ahi;
        const uint32_t off = active ? cell_off(B, c.x, c.y, c.z) : 0u;
        T f[Q];
        if (active) {
            gather<Q, ST, ODD>(a, B, off, c.x, c.y, c.z, special, f);
        } else {
            for (int i = 0; i < Q; ++i) f[i] = T(0);
        }
        const uint32_t h = kStochastic<ST> ? state_hash<Q, T>(f, global_cell(a, B, c.x, c.y, c.z)) : 0u;
        const Macro<Q, T> m0 = moments_of<Q, T>(f, cp.F);
        T P[6];
        pi_pairs<Q, T>(f, m0, P);
        float x[7];
        bool bad = false;
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const float raw = k < 6 ? P[k] : m0.drho;
            x[k] = (raw - net->mean[k]) * net->istd[k];
            bad |= !(fabsf(x[k]) <= 8.f);
        }
        if (!active)
            for (int k = 0; k < 7; ++k) x[k] = 0.f;
        // Park the populations in shared memory while the network runs and
        // rebuild the moments from them afterwards: otherwise the compiler
        // precomputes most of the relaxation before the network and keeps
        // ~64 values live through it, halving the occupancy.
#pragma unroll
        for (int i = 0; i < Q; ++i) park[i][threadIdx.x] = f[i];
        asm volatile("" ::: "memory");
        const float o = mlp_forward_wave(net, x);
        asm volatile("" ::: "memory");
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = park[i][threadIdx.x];
        const Macro<Q, T> m = moments_of<Q, T>(f, cp.F);
        T tau;
        if (bad || !isfinite(o)) {
            // Smagorinsky fallback (rare lanes): the same Pi and rho as above
            T Ps[6];
            pi_pairs<Q, T>(f, m, Ps);
            tau = tau_smagorinsky<T>(Ps, m.rho, cp.tau0, cp.smag_k);
        } else {
            tau = cp.tau0 + softplus_f(o);
        }
        const T om = recip(tau);
        const T omm = COLL == 1 ? recip(T(0.5) + cp.magic * recip(tau - T(0.5))) : om;
        relax_pairs<Q, T, COLL == 0, AccOf<ST>>(f, m, cp.F, om, omm);
        if (!active) continue;
        if (L.alo | L.ahi) {
            const T rin = (T)a.rho_in, rout = (T)a.rho_out;
            const T drin = (T)(a.rho_in - 1.0), drout = (T)(a.rho_out - 1.0);
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                const bool lo = (L.alo >> i) & 1u, hi = (L.ahi >> i) & 1u;
                if (lo | hi) f[i] = abb_value<Q, i, T>(f[i], m, lo ? rin : rout, lo ? drin : drout);
            });
        }
        scatter<Q, ST, ODD>(a, B, off, c.x, c.y, c.z, special, f, h);
    }
}

// ---------------------------------------------------------------------------
// Moments and conservation partials (FP64), optional per-cell output
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

template <int Q, typename ST, bool SWAPPED>
__global__ __launch_bounds__(kWG) void moments_kernel(const MomArgs ma)
{
    const SweepArgs &a = ma.s;
    __shared__ double red[kWG / 64][8];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const int4 tv = a.tiles[t];
        const CellPos c = tile_cell(tv, threadIdx.x);
        const DevBlock B = a.blocks[tv.x];
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // drho, px, py, pz, ke, umax, nfluid, -
        if (c.valid) {
            uint32_t mask = 0;
            if (B.mask >= 0) mask = a.masks[B.mask + (int64_t)c.z * B.mplane + c.y * B.mpitch + c.x];
            const int gx = B.g[0] + c.x, gy = B.g[1] + c.y, gz = B.g[2] + c.z;
            double rho = 0.0, u[3] = {0.0, 0.0, 0.0};
            if (!(mask & kSolidBit)) {
                const Links<Q> L = classify<Q>(mask, B, c.x, c.y, c.z, a);
                const uint32_t off = cell_off(B, c.x, c.y, c.z);
                typename Codec<ST>::T f[Q];
                gather<Q, ST, SWAPPED>(a, B, off, c.x, c.y, c.z, L.bb | L.alo | L.ahi, f);
                double drho = 0, j[3] = {0, 0, 0};
                sfor<Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    const double v = (double)f[i];
                    drho += v;
                    if constexpr (cx<Q>(i) != 0) j[0] += cx<Q>(i) * v;
                    if constexpr (cy<Q>(i) != 0) j[1] += cy<Q>(i) * v;
                    if constexpr (cz<Q>(i) != 0) j[2] += cz<Q>(i) * v;
                });
                rho = 1.0 + drho;
                double pu[3];
                for (int k = 0; k < 3; ++k) {
                    pu[k] = j[k] + 0.5 * a.force[k];
                    u[k] = pu[k] / rho;
                }
                const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                acc[0] = drho;
                acc[1] = pu[0];
                acc[2] = pu[1];
                acc[3] = pu[2];
                acc[4] = 0.5 * rho * uu;
                acc[5] = sqrt(uu);
                acc[6] = 1.0;
            }
            if (ma.out && gz >= ma.z0 && gz < ma.z1) {
                const int64_t S = (int64_t)(ma.z1 - ma.z0) * a.dom[1] * a.dom[0];
                const int64_t k = ((int64_t)(gz - ma.z0) * a.dom[1] + gy) * a.dom[0] + gx;
                ma.out[k] = rho;
                ma.out[S + k] = u[0];
                ma.out[2 * S + k] = u[1];
                ma.out[3 * S + k] = u[2];
            }
        }
        if (ma.partials) {
            for (int k = 0; k < 7; ++k) acc[k] = (k == 5) ? wave_max(acc[k]) : wave_sum(acc[k]);
            if (lane == 0)
                for (int k = 0; k < 7; ++k) red[wv][k] = acc[k];
            __syncthreads();
            if (threadIdx.x < 8) {
                double r = 0.0;
                const int k = threadIdx.x;
                for (int w = 0; w < kWG / 64; ++w) {
                    const double v = (k < 7) ? red[w][k] : 0.0;
                    r = (k == 5) ? fmax(r, v) : r + v;
                }
                ma.partials[(int64_t)t * 8 + k] = r;
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Box filter for LES training data: averages over factor^3 fine cells of
// rho, u (Guo velocity) and the products u_a u_b, one thread per coarse cell,
// fixed summation order.  Single-block handles; out[10][Nc] =
// (rho, ux, uy, uz, uxux, uyuy, uzuz, uxuy, uxuz, uyuz).
// ---------------------------------------------------------------------------
template <int Q, typename ST, bool SWAPPED>
__global__ __launch_bounds__(kWG) void filter_kernel(const SweepArgs a, int fac, double *out)
{
    const DevBlock B = a.blocks[0];
    const int ncx = B.n[0] / fac, ncy = B.n[1] / fac, ncz = B.n[2] / fac;
    const int64_t Nc = (int64_t)ncx * ncy * ncz;
    const double inv = 1.0 / ((double)fac * fac * fac);
    for (int64_t c = (int64_t)blockIdx.x * kWG + threadIdx.x; c < Nc; c += (int64_t)gridDim.x * kWG) {
        const int X = (int)(c % ncx), Y = (int)((c / ncx) % ncy), Z = (int)(c / ((int64_t)ncx * ncy));
        double acc[10];
        for (int k = 0; k < 10; ++k) acc[k] = 0.0;
        for (int dz = 0; dz < fac; ++dz)
            for (int dy = 0; dy < fac; ++dy)
                for (int dx = 0; dx < fac; ++dx) {
                    const int x = X * fac + dx, y = Y * fac + dy, z = Z * fac + dz;
                    uint32_t mask = 0;
                    if (B.mask >= 0) mask = a.masks[B.mask + (int64_t)z * B.mplane + y * B.mpitch + x];
                    if (mask & kSolidBit) continue;
                    const Links<Q> L = classify<Q>(mask, B, x, y, z, a);
                    typename Codec<ST>::T f[Q];
                    gather<Q, ST, SWAPPED>(a, B, cell_off(B, x, y, z), x, y, z, L.bb | L.alo | L.ahi, f);
                    double drho = 0, j[3] = {0, 0, 0};
                    sfor<Q>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        const double v = (double)f[i];
                        drho += v;
                        if constexpr (cx<Q>(i) != 0) j[0] += cx<Q>(i) * v;
                        if constexpr (cy<Q>(i) != 0) j[1] += cy<Q>(i) * v;
                        if constexpr (cz<Q>(i) != 0) j[2] += cz<Q>(i) * v;
                    });
                    const double rho = 1.0 + drho;
                    double u[3];
                    for (int k = 0; k < 3; ++k) u[k] = (j[k] + 0.5 * a.force[k]) / rho;
                    acc[0] += rho;
                    acc[1] += u[0];
                    acc[2] += u[1];
                    acc[3] += u[2];
                    acc[4] += u[0] * u[0];
                    acc[5] += u[1] * u[1];
                    acc[6] += u[2] * u[2];
                    acc[7] += u[0] * u[1];
                    acc[8] += u[0] * u[2];
                    acc[9] += u[1] * u[2];
                }
        for (int k = 0; k < 10; ++k) out[k * Nc + c] = acc[k] * inv;
    }
}

// ---------------------------------------------------------------------------
// Initialisation: d = f_eq(rho, u) - w from rho/u of a global z slab
// ---------------------------------------------------------------------------
template <int Q, typename ST>
__global__ __launch_bounds__(kWG) void init_kernel(const SweepArgs a, const double *rhou, int z0, int z1)
{
    using T = typename Codec<ST>::T;
    for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const int4 tv = a.tiles[t];
        const CellPos c = tile_cell(tv, threadIdx.x);
        if (!c.valid) continue;
        const DevBlock B = a.blocks[tv.x];
        const int gx = B.g[0] + c.x, gy = B.g[1] + c.y, gz = B.g[2] + c.z;
        if (gz < z0 || gz >= z1) continue;
        uint32_t mask = 0;
        if (B.mask >= 0) mask = a.masks[B.mask + (int64_t)c.z * B.mplane + c.y * B.mpitch + c.x];
        const uint32_t off = cell_off(B, c.x, c.y, c.z);
        if (mask & kSolidBit) {
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                stv<Q, ST>(at<ST>(slot_base<ST>(a, B, i), off * sizeof(ST)), T(0), i);
            });
            continue;
        }
        const int64_t S = (int64_t)(z1 - z0) * a.dom[1] * a.dom[0];
        const int64_t k = ((int64_t)(gz - z0) * a.dom[1] + gy) * a.dom[0] + gx;
        // equilibrium evaluated in FP64, then rounded once to the storage type
        const double rho = rhou[k];
        const double u[3] = {rhou[S + k], rhou[2 * S + k], rhou[3 * S + k]};
        const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        sfor<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double cu = cdot<Q, i>(u);
            const double v = weight<Q, double>(i) * ((rho - 1.0) + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
            stv<Q, ST>(at<ST>(slot_base<ST>(a, B, i), off * sizeof(ST)), (T)v, i);
        });
    }
}

// ---------------------------------------------------------------------------
// Population I/O (natural layout, FP64 [q][slab cells]) for get / set
// ---------------------------------------------------------------------------
template <int Q, typename ST, bool TO_DEVICE, bool SWAPPED>
__global__ __launch_bounds__(kWG) void pdfs_kernel(const SweepArgs a, double *buf, int z0, int z1)
{
    using T = typename Codec<ST>::T;
    for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const int4 tv = a.tiles[t];
        const CellPos c = tile_cell(tv, threadIdx.x);
        if (!c.valid) continue;
        const DevBlock B = a.blocks[tv.x];
        const int gx = B.g[0] + c.x, gy = B.g[1] + c.y, gz = B.g[2] + c.z;
        if (gz < z0 || gz >= z1) continue;
        uint32_t mask = 0;
        if (B.mask >= 0) mask = a.masks[B.mask + (int64_t)c.z * B.mplane + c.y * B.mpitch + c.x];
        const int64_t S = (int64_t)(z1 - z0) * a.dom[1] * a.dom[0];
        const int64_t k = ((int64_t)(gz - z0) * a.dom[1] + gy) * a.dom[0] + gx;
        const uint32_t off = cell_off(B, c.x, c.y, c.z);
        if (mask & kSolidBit) {
            if (!TO_DEVICE)
                for (int i = 0; i < Q; ++i) buf[i * S + k] = 0.0;
            continue;
        }
        if constexpr (TO_DEVICE) {
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                stv<Q, ST>(at<ST>(slot_base<ST>(a, B, i), off * sizeof(ST)), (T)buf[i * S + k], i);
            });
        } else {
            const Links<Q> L = classify<Q>(mask, B, c.x, c.y, c.z, a);
            T f[Q];
            gather<Q, ST, SWAPPED>(a, B, off, c.x, c.y, c.z, L.bb | L.alo | L.ahi, f);
            for (int i = 0; i < Q; ++i) buf[i * S + k] = (double)f[i];
        }
    }
}

// ---------------------------------------------------------------------------
// Ghost-layer exchange: bitwise copy of one population over a cell region
// between two blocks (device-local copy without buffers, Sec. 3.3).
// ---------------------------------------------------------------------------
// ADD (write-coverage check): add the source counter to the target instead
// of copying it.
template <typename Raw, bool ADD = false>
__global__ __launch_bounds__(kWG) void exchange_kernel(Raw *arena, const DevBlock *blocks, const uint32_t *masks,
                                                       const XItem *items, int xcd_map)
{
    const XItem &it = items[xcd_map ? xcd_item(blockIdx.x, gridDim.x) : (int)blockIdx.x];
    const DevBlock &S = blocks[it.sb];
    const DevBlock &D = blocks[it.db];
    // up to kXChunk / kWG cells per thread: every load is issued before the
    // first store, so one workgroup keeps several independent copies in flight
    constexpr int K = kXChunk / kWG;
    Raw v[K];
    Raw *dst[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int l = (int)threadIdx.x + k * kWG;
        dst[k] = nullptr;
        if (l >= it.count) continue;
        const int r = it.start + l;
        const int rx = r % it.ex, rq = r / it.ex;
        const int ry = rq % it.ey, rz = rq / it.ey;
        const int dx = it.d0[0] + rx, dy = it.d0[1] + ry, dz = it.d0[2] + rz;
        if (it.chk >= 0 && D.mask >= 0) {
            const uint32_t m = masks[D.mask + (int64_t)dz * D.mplane + dy * D.mpitch + dx];
            if (m & (kSolidBit | (1u << it.chk))) continue;
        }
        const Raw *src = arena + S.pop + (int64_t)it.slot * S.slot + cell_off(S, it.s0[0] + rx, it.s0[1] + ry, it.s0[2] + rz);
        dst[k] = arena + D.pop + (int64_t)it.slot * D.slot + cell_off(D, dx, dy, dz);
        v[k] = mem_ld<true>(src);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (!dst[k]) continue;
        if constexpr (ADD)
            atomicAdd(dst[k], v[k]);
        else
            mem_st<true>(dst[k], v[k]);
    }
}

// ---------------------------------------------------------------------------
// Force on obstacles by momentum exchange (section "Geometrically fully
// resolved simulations": momentum-exchange method after Ladd and Aidun).  A
// post-collision population f*_i of a fluid cell whose target x + c_i is a
// solid cell or lies beyond a wall is bounced back into the cell, handing
// 2 c_i f*_i to the obstacle.  In both AA layouts, after a step that value
// sits in slot opp(i) of the cell itself (the even sweep stores every f*_i
// there; the odd sweep stores bounced populations there), so this pass reads
// one element per bounce-back link and nothing else.  Per-tile partials:
// force on solid cells (x, y, z), on walls (x, y, z), solid links, wall
// links; a fixed-order second pass sums them.
// ---------------------------------------------------------------------------
template <int Q, typename ST>
__global__ __launch_bounds__(kWG) void force_kernel(const SweepArgs a, double *partials)
{
    __shared__ double red[kWG / 64][8];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const int4 tv = a.tiles[t];
        const CellPos c = tile_cell(tv, threadIdx.x);
        const DevBlock B = a.blocks[tv.x];
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (c.valid) {
            uint32_t mask = 0;
            if (B.mask >= 0) mask = a.masks[B.mask + (int64_t)c.z * B.mplane + c.y * B.mpitch + c.x];
            if (!(mask & kSolidBit)) {
                const Links<Q> L = classify<Q>(mask, B, c.x, c.y, c.z, a);
                const uint32_t to_solid = mask & ((1u << Q) - 1u);  // targets inside the domain that are solid
                const uint32_t off = cell_off(B, c.x, c.y, c.z) * (uint32_t)sizeof(ST);
                sfor<Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    if ((L.bb >> i) & 1u) {
                        const double f = weight<Q, double>(i) + (double)ldv<Q, ST, false>(at<ST>(slot_base<ST>(a, B, opp(i)), off), i);
                        const int k = ((to_solid >> i) & 1u) ? 0 : 3;
                        if constexpr (cx<Q>(i) != 0) acc[k + 0] += 2.0 * cx<Q>(i) * f;
                        if constexpr (cy<Q>(i) != 0) acc[k + 1] += 2.0 * cy<Q>(i) * f;
                        if constexpr (cz<Q>(i) != 0) acc[k + 2] += 2.0 * cz<Q>(i) * f;
                        acc[k == 0 ? 6 : 7] += 1.0;
                    }
                });
            }
        }
        for (int k = 0; k < 8; ++k) acc[k] = wave_sum(acc[k]);
        if (lane == 0)
            for (int k = 0; k < 8; ++k) red[wv][k] = acc[k];
        __syncthreads();
        if (threadIdx.x < 8) {
            double r = 0.0;
            for (int w = 0; w < kWG / 64; ++w) r += red[w][threadIdx.x];
            partials[(int64_t)t * 8 + threadIdx.x] = r;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int Q, int COLL, bool NT>
static hipError_t sweep_qn(bool odd, const SweepArgs &a, int grid, hipStream_t st)
{
    if (odd && a.vec_odd) {
        // FP64 only (and the counting storage of the write-coverage check,
        // 4 cells per lane): with 4- and 2-byte elements a lane would hold 4
        // or 8 cells, whose registers cut the occupancy to one or two waves
        if constexpr (sizeof(typename Codec<WLB_STORAGE>::Raw) == 8 || std::is_same_v<WLB_STORAGE, cover_t>) {
            hipLaunchKernelGGL((sweep_odd_vec_kernel<Q, COLL, WLB_STORAGE, NT>), dim3(grid), dim3(kWG), 0, st, a);
            return hipGetLastError();
        } else {
            return hipErrorNotSupported;
        }
    }
    if (odd && a.lds_stride > 0) {
        using Raw = typename Codec<WLB_STORAGE>::Raw;
        const size_t bytes = lds_stage_bytes<Q, Raw>(a.lds_stride);
        if (a.lds_ring)
            hipLaunchKernelGGL((sweep_odd_lds_kernel<Q, COLL, WLB_STORAGE, true, NT>), dim3(grid), dim3(kWG), bytes, st,
                               a);
        else
            hipLaunchKernelGGL((sweep_odd_lds_kernel<Q, COLL, WLB_STORAGE, false, NT>), dim3(grid), dim3(kWG), bytes, st,
                               a);
        return hipGetLastError();
    }
    if constexpr (NT && !std::is_same_v<WLB_STORAGE, cover_t>) {
        if (odd && a.nt == 2) {  // the hint on the aligned accesses only
            hipLaunchKernelGGL((sweep_odd_aligned_nt_kernel<Q, COLL, WLB_STORAGE>), dim3(grid), dim3(kWG), 0, st, a);
            return hipGetLastError();
        }
    }
    if (odd)
        hipLaunchKernelGGL((sweep_kernel<Q, COLL, WLB_STORAGE, true, NT>), dim3(grid), dim3(kWG), 0, st, a);
    else
        hipLaunchKernelGGL((sweep_kernel<Q, COLL, WLB_STORAGE, false, NT>), dim3(grid), dim3(kWG), 0, st, a);
    return hipGetLastError();
}

template <int Q, int COLL>
static hipError_t sweep_q(bool odd, const SweepArgs &a, int grid, hipStream_t st)
{
    // the counting stores of the write-coverage check ignore the hint
    if (a.nt || std::is_same_v<WLB_STORAGE, cover_t>) return sweep_qn<Q, COLL, true>(odd, a, grid, st);
    return sweep_qn<Q, COLL, false>(odd, a, grid, st);
}

template <int COLL>
static hipError_t sweep_mlp_q(bool odd, const SweepArgs &a, int grid, hipStream_t st)
{
    if constexpr (std::is_same<WLB_STORAGE, double>::value) {
        return hipErrorNotSupported;
    } else {
        if (odd)
            hipLaunchKernelGGL((sweep_mlp_kernel<COLL, WLB_STORAGE, true>), dim3(grid), dim3(kWG), 0, st, a);
        else
            hipLaunchKernelGGL((sweep_mlp_kernel<COLL, WLB_STORAGE, false>), dim3(grid), dim3(kWG), 0, st, a);
        return hipGetLastError();
    }
}

template <int Q>
static hipError_t sweep_c(int coll, bool odd, const SweepArgs &a, int grid, hipStream_t st)
{
    if (a.closure == 2) {
        if (Q != 19) return hipErrorNotSupported;
        return coll == 0 ? sweep_mlp_q<0>(odd, a, grid, st)
                         : (coll == 1 ? sweep_mlp_q<1>(odd, a, grid, st) : hipErrorNotSupported);
    }
    switch (coll) {
    case 0: return sweep_q<Q, 0>(odd, a, grid, st);
    case 1: return sweep_q<Q, 1>(odd, a, grid, st);
    case 2:
        if constexpr (Q == 19 || Q == 27) return sweep_q<Q, 2>(odd, a, grid, st);
        return hipErrorNotSupported;
    case 3:
        if constexpr (Q == 27) return sweep_q<Q, 3>(odd, a, grid, st);
        return hipErrorNotSupported;
    case 4:
        if constexpr (Q == 27) return sweep_q<Q, 4>(odd, a, grid, st);
        return hipErrorNotSupported;
    default: return hipErrorInvalidValue;
    }
}

template <int Q>
static hipError_t moments_q(const MomArgs &a, int grid, hipStream_t st)
{
    if (a.swapped)
        hipLaunchKernelGGL((moments_kernel<Q, WLB_STORAGE, true>), dim3(grid), dim3(kWG), 0, st, a);
    else
        hipLaunchKernelGGL((moments_kernel<Q, WLB_STORAGE, false>), dim3(grid), dim3(kWG), 0, st, a);
    return hipGetLastError();
}

template <int Q>
static hipError_t force_q(const SweepArgs &a, double *partials, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((force_kernel<Q, WLB_STORAGE>), dim3(grid), dim3(kWG), 0, st, a, partials);
    return hipGetLastError();
}

template <int Q>
static hipError_t pdfs_q(const SweepArgs &a, double *buf, int z0, int z1, bool to_dev, bool swapped, int grid,
                         hipStream_t st)
{
    if (to_dev)
        hipLaunchKernelGGL((pdfs_kernel<Q, WLB_STORAGE, true, false>), dim3(grid), dim3(kWG), 0, st, a, buf, z0, z1);
    else if (swapped)
        hipLaunchKernelGGL((pdfs_kernel<Q, WLB_STORAGE, false, true>), dim3(grid), dim3(kWG), 0, st, a, buf, z0, z1);
    else
        hipLaunchKernelGGL((pdfs_kernel<Q, WLB_STORAGE, false, false>), dim3(grid), dim3(kWG), 0, st, a, buf, z0, z1);
    return hipGetLastError();
}


#define WLB_CAT2(a, b) a##b
#define WLB_CAT(a, b) WLB_CAT2(a, b)

// Calls f(std::integral_constant<int, Q>{}) for the velocity set with q
// populations.
template <typename F>
static hipError_t by_set(int q, F &&f)
{
    switch (q) {
    case 9: return f(std::integral_constant<int, 9>{});
    case 15: return f(std::integral_constant<int, 15>{});
    case 19: return f(std::integral_constant<int, 19>{});
    case 27: return f(std::integral_constant<int, 27>{});
    default: return hipErrorInvalidValue;
    }
}

hipError_t WLB_CAT(sweep_, WLB_SUFFIX)(int q, int coll, bool odd, const SweepArgs &a, int grid, hipStream_t st)
{
    return by_set(q, [&](auto S) { return sweep_c<decltype(S)::value>(coll, odd, a, grid, st); });
}

hipError_t WLB_CAT(moments_, WLB_SUFFIX)(int q, const MomArgs &a, int grid, hipStream_t st)
{
    return by_set(q, [&](auto S) { return moments_q<decltype(S)::value>(a, grid, st); });
}

hipError_t WLB_CAT(force_, WLB_SUFFIX)(int q, const SweepArgs &a, double *partials, int grid, hipStream_t st)
{
    return by_set(q, [&](auto S) { return force_q<decltype(S)::value>(a, partials, grid, st); });
}

hipError_t WLB_CAT(init_, WLB_SUFFIX)(int q, const SweepArgs &a, const double *rhou, int z0, int z1, int grid,
                                      hipStream_t st)
{
    return by_set(q, [&](auto S) {
        constexpr int Q = decltype(S)::value;
        hipLaunchKernelGGL((init_kernel<Q, WLB_STORAGE>), dim3(grid), dim3(kWG), 0, st, a, rhou, z0, z1);
        return hipGetLastError();
    });
}

hipError_t WLB_CAT(pdfs_, WLB_SUFFIX)(int q, const SweepArgs &a, double *buf, int z0, int z1, bool to_device,
                                      bool swapped, int grid, hipStream_t st)
{
    return by_set(q, [&](auto S) {
        return pdfs_q<decltype(S)::value>(a, buf, z0, z1, to_device, swapped, grid, st);
    });
}

hipError_t WLB_CAT(filter_, WLB_SUFFIX)(int q, const SweepArgs &a, int fac, double *out, int64_t ncoarse,
                                        bool swapped, hipStream_t st)
{
    int64_t g = (ncoarse + kWG - 1) / kWG;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    return by_set(q, [&](auto S) {
        constexpr int Q = decltype(S)::value;
        if (swapped)
            hipLaunchKernelGGL((filter_kernel<Q, WLB_STORAGE, true>), dim3((int)g), dim3(kWG), 0, st, a, fac, out);
        else
            hipLaunchKernelGGL((filter_kernel<Q, WLB_STORAGE, false>), dim3((int)g), dim3(kWG), 0, st, a, fac, out);
        return hipGetLastError();
    });
}

hipError_t WLB_CAT(exchange_, WLB_SUFFIX)(void *arena, const DevBlock *blocks, const uint32_t *masks,
                                          const XItem *items, int nitems, int xcd_map, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    using Raw = typename Codec<WLB_STORAGE>::Raw;
    constexpr bool add = std::is_same_v<WLB_STORAGE, cover_t>;
    hipLaunchKernelGGL((exchange_kernel<Raw, add>), dim3(nitems), dim3(kWG), 0, st, reinterpret_cast<Raw *>(arena),
                       blocks, masks, items, xcd_map);
    return hipGetLastError();
}

}  // namespace wlb
