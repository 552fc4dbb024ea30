// Device-side building blocks for the gfx950 kernels: complex arithmetic,
// native field layouts, lattice geometry, the Z4 noise hash and wave64
// reductions.  Included only by the .hip translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>

#include "tm_types.h"

namespace tmq {

// ---------------------------------------------------------------------------
// complex numbers
// ---------------------------------------------------------------------------
template <typename R>
struct cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
// conj(a) * b
template <typename R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> times_i(cx<R> a) { return {-a.im, a.re}; }
template <typename R>
__device__ __forceinline__ cx<R> times_mi(cx<R> a) { return {a.im, -a.re}; }
template <typename R>
__device__ __forceinline__ R norm2(cx<R> a) { return a.re * a.re + a.im * a.im; }

// ---------------------------------------------------------------------------
// reduced-precision conversions (round to nearest even)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }
// Two floats to a packed pair, low half first, rounded to nearest even: one
// v_cvt_pk_bf16_f32 / v_cvt_pk_f16_f32 on gfx950.
typedef float tm_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 tm_bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 tm_f16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack2_bf16(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((tm_f32x2){lo, hi}, tm_bf16x2));
}
__device__ __forceinline__ uint32_t pack2_f16(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((tm_f32x2){lo, hi}, tm_f16x2));
}
#ifdef TM_F16_ASM_CVT
__device__ __forceinline__ uint32_t f32_to_f16(float f) {
    uint32_t h;
    asm volatile("v_cvt_f16_f32 %0, %1" : "=v"(h) : "v"(f));
    return h & 0xFFFFu;
}
__device__ __forceinline__ float f16_to_f32(uint32_t h) {
    float f;
    asm volatile("v_cvt_f32_f16 %0, %1" : "=v"(f) : "v"(h & 0xFFFFu));
    return f;
}
#else
__device__ __forceinline__ uint32_t f32_to_f16(float f) {
    _Float16 h = (_Float16)f;
    return (uint32_t)__builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_to_f32(uint32_t h) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(h & 0xFFFFu));
}
#endif

// ---------------------------------------------------------------------------
// native spinor storage: component planes of 16-byte vectors, stride Vs
//   F64 : 12 planes of double2 (one complex component each)
//   F32 :  6 planes of float4  (components 2k, 2k+1)
//   F16 :  3 planes of uint4   (components 4k..4k+3 as packed halves)
//   BF16:  3 planes of uint4   (same, bfloat16)
// A field of nrhs spinors is nrhs such blocks back to back.
// ---------------------------------------------------------------------------
struct SF64 {
    using V = double2;
    static constexpr int NV = 12;
};
struct SF32 {
    using V = float4;
    static constexpr int NV = 6;
};
struct SF16 {
    using V = uint4;
    static constexpr int NV = 3;
};
struct SBF16 {
    using V = uint4;
    static constexpr int NV = 3;
};

// Every native plane holds 16-byte elements and is read and written with
// buffer instructions: the field's base address lives in a descriptor in
// scalar registers, the plane offset k*Vs*16 is a scalar offset, and the
// only per-lane address is the 32-bit byte offset 16*site, shared by all
// planes of all fields.  (Offsets stay below 4 GiB: at most 36 planes sit
// behind one base, and tm_create rejects lattices with 576 * Vs >= 2^32.)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const void* base) {
    // raw buffer, no stride; dword3 = 0x00020000 is the gfx9-family format word
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, -1, 0x00020000);
}
// CP: cache-policy bits of the buffer instruction (0: default, kStream:
// non-temporal, for fields that are streamed once and would otherwise evict
// the stencil's neighbour data from L2)
constexpr int kStream = 2;
template <typename T, int CP = 0>
__device__ __forceinline__ T ld_plane(const void* base, long Vs, int k, uint32_t s) {
    auto v = __builtin_amdgcn_raw_buffer_load_b128(rsrc_of(base), s << 4, (uint32_t)((size_t)k * Vs * 16), CP);
    return __builtin_bit_cast(T, v);
}
// A 128-bit store reads its data registers after it issues; the compiler's
// hazard model adds wait states before those registers are rewritten only
// when the store's scalar offset is not a register, which it is here.  The
// guard below takes the data as operands of a few wait states placed after
// the store, so no instruction can overwrite them earlier.  (Without it,
// stores issued under memory pressure intermittently wrote the next values
// of the data registers for some lanes.)
template <typename T, int CP = 0>
__device__ __forceinline__ void st_plane(void* base, long Vs, int k, uint32_t s, T val) {
    using V4 = unsigned int __attribute__((ext_vector_type(4)));
    const V4 v = __builtin_bit_cast(V4, val);
    __builtin_amdgcn_raw_buffer_store_b128(v, rsrc_of(base), s << 4, (uint32_t)((size_t)k * Vs * 16), CP);
    asm volatile("s_nop 4" ::"v"(v) : "memory");
}

template <class S, typename R>
__device__ __forceinline__ void load_spinor(const void* base, long Vs, uint32_t s, cx<R> p[12]);
template <class S, typename R>
__device__ __forceinline__ void store_spinor(void* base, long Vs, uint32_t s, const cx<R> p[12]);

template <>
__device__ __forceinline__ void load_spinor<SF64, double>(const void* base, long Vs, uint32_t s, cx<double> p[12]) {
#pragma unroll
    for (int k = 0; k < 12; k++) {
        double2 v = ld_plane<double2>(base, Vs, k, s);
        p[k] = {v.x, v.y};
    }
}
template <>
__device__ __forceinline__ void store_spinor<SF64, double>(void* base, long Vs, uint32_t s, const cx<double> p[12]) {
#pragma unroll
    for (int k = 0; k < 12; k++) st_plane(base, Vs, k, s, make_double2(p[k].re, p[k].im));
}
template <typename R, int CP = 0>
__device__ __forceinline__ void load_f32_planes(const void* base, long Vs, uint32_t s, cx<R> p[12]) {
#pragma unroll
    for (int k = 0; k < 6; k++) {
        float4 v = ld_plane<float4, CP>(base, Vs, k, s);
        p[2 * k] = {(R)v.x, (R)v.y};
        p[2 * k + 1] = {(R)v.z, (R)v.w};
    }
}
template <>
__device__ __forceinline__ void load_spinor<SF32, float>(const void* base, long Vs, uint32_t s, cx<float> p[12]) {
    load_f32_planes<float>(base, Vs, s, p);
}
template <>
__device__ __forceinline__ void load_spinor<SF32, double>(const void* base, long Vs, uint32_t s, cx<double> p[12]) {
    load_f32_planes<double>(base, Vs, s, p);
}
template <>
__device__ __forceinline__ void store_spinor<SF32, float>(void* base, long Vs, uint32_t s, const cx<float> p[12]) {
#pragma unroll
    for (int k = 0; k < 6; k++)
        st_plane(base, Vs, k, s, make_float4(p[2 * k].re, p[2 * k].im, p[2 * k + 1].re, p[2 * k + 1].im));
}
template <>
__device__ __forceinline__ void store_spinor<SF32, double>(void* base, long Vs, uint32_t s, const cx<double> p[12]) {
#pragma unroll
    for (int k = 0; k < 6; k++)
        st_plane(base, Vs, k, s,
                 make_float4((float)p[2 * k].re, (float)p[2 * k].im, (float)p[2 * k + 1].re, (float)p[2 * k + 1].im));
}

template <bool BF, typename R, int CP = 0>
__device__ __forceinline__ void load_half_planes(const void* base, long Vs, uint32_t s, cx<R> p[12]) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
        uint4 v = ld_plane<uint4, CP>(base, Vs, k, s);
        uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; j++) {
            float re = BF ? bf16_to_f32(w[j] & 0xFFFFu) : f16_to_f32(w[j] & 0xFFFFu);
            float im = BF ? bf16_to_f32(w[j] >> 16) : f16_to_f32(w[j] >> 16);
            p[4 * k + j] = {(R)re, (R)im};
        }
    }
}
template <bool BF, int CP = 0>
__device__ __forceinline__ void store_half_planes(void* base, long Vs, uint32_t s, const cx<float> p[12]) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
        uint32_t w[4];
#pragma unroll
        for (int j = 0; j < 4; j++)
            w[j] = BF ? pack2_bf16(p[4 * k + j].re, p[4 * k + j].im) : pack2_f16(p[4 * k + j].re, p[4 * k + j].im);
        st_plane<uint4, CP>(base, Vs, k, s, make_uint4(w[0], w[1], w[2], w[3]));
    }
}
template <>
__device__ __forceinline__ void load_spinor<SF16, float>(const void* base, long Vs, uint32_t s, cx<float> p[12]) {
    load_half_planes<false, float>(base, Vs, s, p);
}
template <>
__device__ __forceinline__ void load_spinor<SF16, double>(const void* base, long Vs, uint32_t s, cx<double> p[12]) {
    load_half_planes<false, double>(base, Vs, s, p);
}
template <>
__device__ __forceinline__ void load_spinor<SBF16, float>(const void* base, long Vs, uint32_t s, cx<float> p[12]) {
    load_half_planes<true, float>(base, Vs, s, p);
}
template <>
__device__ __forceinline__ void load_spinor<SBF16, double>(const void* base, long Vs, uint32_t s, cx<double> p[12]) {
    load_half_planes<true, double>(base, Vs, s, p);
}
template <>
__device__ __forceinline__ void store_spinor<SF16, float>(void* base, long Vs, uint32_t s, const cx<float> p[12]) {
    store_half_planes<false>(base, Vs, s, p);
}
template <>
__device__ __forceinline__ void store_spinor<SBF16, float>(void* base, long Vs, uint32_t s, const cx<float> p[12]) {
    store_half_planes<true>(base, Vs, s, p);
}

// Round values to what the storage format holds (so norms can be taken of
// exactly the stored values).
template <class S, typename R>
__device__ __forceinline__ void round_storage(cx<R> p[12]);
template <>
__device__ __forceinline__ void round_storage<SF64, double>(cx<double>*) {}
template <>
__device__ __forceinline__ void round_storage<SF32, float>(cx<float>*) {}
template <>
__device__ __forceinline__ void round_storage<SF32, double>(cx<double>* p) {
#pragma unroll
    for (int k = 0; k < 12; k++) p[k] = {(double)(float)p[k].re, (double)(float)p[k].im};
}
template <>
__device__ __forceinline__ void round_storage<SF16, float>(cx<float>* p) {
#pragma unroll
    for (int k = 0; k < 12; k++) p[k] = {f16_to_f32(f32_to_f16(p[k].re)), f16_to_f32(f32_to_f16(p[k].im))};
}
template <>
__device__ __forceinline__ void round_storage<SBF16, float>(cx<float>* p) {
#pragma unroll
    for (int k = 0; k < 12; k++) p[k] = {bf16_to_f32(f32_to_bf16(p[k].re)), bf16_to_f32(f32_to_bf16(p[k].im))};
}

// Spinor load / store with a cache policy (see ld_plane).
template <class S, typename R, int CP>
__device__ __forceinline__ void load_spinor_cp(const void* base, long Vs, uint32_t s, cx<R> p[12]) {
    if constexpr (std::is_same<S, SF64>::value) {
#pragma unroll
        for (int k = 0; k < 12; k++) {
            double2 v = ld_plane<double2, CP>(base, Vs, k, s);
            p[k] = {(R)v.x, (R)v.y};
        }
    } else if constexpr (std::is_same<S, SF32>::value) {
        load_f32_planes<R, CP>(base, Vs, s, p);
    } else {
        load_half_planes<std::is_same<S, SBF16>::value, R, CP>(base, Vs, s, p);
    }
}
template <class S, typename R, int CP>
__device__ __forceinline__ void store_spinor_cp(void* base, long Vs, uint32_t s, const cx<R> p[12]) {
    if constexpr (std::is_same<S, SF64>::value) {
#pragma unroll
        for (int k = 0; k < 12; k++) st_plane<double2, CP>(base, Vs, k, s, make_double2(p[k].re, p[k].im));
    } else if constexpr (std::is_same<S, SF32>::value) {
#pragma unroll
        for (int k = 0; k < 6; k++)
            st_plane<float4, CP>(base, Vs, k, s,
                                 make_float4((float)p[2 * k].re, (float)p[2 * k].im, (float)p[2 * k + 1].re,
                                             (float)p[2 * k + 1].im));
    } else {
        static_assert(sizeof(R) == 4, "half storage is written from FP32");
        store_half_planes<std::is_same<S, SBF16>::value, CP>(base, Vs, s, p);
    }
}

template <class S>
__device__ __forceinline__ const void* field_rhs(const void* base, long Vs, int r) {
    return (const char*)base + (size_t)r * S::NV * Vs * 16;
}
template <class S>
__device__ __forceinline__ void* field_rhs(void* base, long Vs, int r) {
    return (char*)base + (size_t)r * S::NV * Vs * 16;
}

// ---------------------------------------------------------------------------
// native gauge storage (no boundary sign folded in)
//   GF64: double2 [4][9][Vs]   full 3x3 links
//   GF32: float4  [4][3][Vs]   rows 0 and 1 (12 reals); row 2 rebuilt as
//                              conj(row0 x row1), exact for SU(3) (measured:
//                              the 30 flops per link cost less than the 24
//                              bytes of a stored row 2)
// ---------------------------------------------------------------------------
struct GF64 {};
struct GF32 {};

template <class G, typename R>
__device__ __forceinline__ void load_link(const void* g, long Vs, int mu, uint32_t s, cx<R> U[3][3]);

template <>
__device__ __forceinline__ void load_link<GF64, double>(const void* g, long Vs, int mu, uint32_t s,
                                                        cx<double> U[3][3]) {
#pragma unroll
    for (int k = 0; k < 9; k++) {
        double2 v = ld_plane<double2>(g, Vs, mu * 9 + k, s);
        U[k / 3][k % 3] = {v.x, v.y};
    }
}
// the FP32 link from its two stored rows (three float4: row 0, then row 1)
__device__ __forceinline__ void link_from_rows(float4 a0, float4 a1, float4 a2, cx<float> U[3][3]) {
    U[0][0] = {a0.x, a0.y};
    U[0][1] = {a0.z, a0.w};
    U[0][2] = {a1.x, a1.y};
    U[1][0] = {a1.z, a1.w};
    U[1][1] = {a2.x, a2.y};
    U[1][2] = {a2.z, a2.w};
    // row2 = conj(row0 x row1): U[2][k] = conj(a b - c d) with (a, b, c, d)
    // the entries of the 2x2 cofactor, as FMA chains
    auto cof = [](cx<float> a, cx<float> b, cx<float> c, cx<float> d) -> cx<float> {
        float re = a.re * b.re;
        re = fmaf(-a.im, b.im, re);
        re = fmaf(-c.re, d.re, re);
        re = fmaf(c.im, d.im, re);
        float im = a.re * b.im;
        im = fmaf(a.im, b.re, im);
        im = fmaf(-c.re, d.im, im);
        im = fmaf(-c.im, d.re, im);
        return {re, -im};
    };
    U[2][0] = cof(U[0][1], U[1][2], U[0][2], U[1][1]);
    U[2][1] = cof(U[0][2], U[1][0], U[0][0], U[1][2]);
    U[2][2] = cof(U[0][0], U[1][1], U[0][1], U[1][0]);
}
template <>
__device__ __forceinline__ void load_link<GF32, float>(const void* g, long Vs, int mu, uint32_t s, cx<float> U[3][3]) {
    const float4 a0 = ld_plane<float4>(g, Vs, mu * 3 + 0, s);
    const float4 a1 = ld_plane<float4>(g, Vs, mu * 3 + 1, s);
    const float4 a2 = ld_plane<float4>(g, Vs, mu * 3 + 2, s);
    link_from_rows(a0, a1, a2, U);
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t fdiv(uint32_t n, uint32_t m) { return __umulhi(n, m); }

struct Site {
    int x, y, z, t;
};
__device__ __forceinline__ Site site_coords(const Geom& g, uint32_t s) {
    uint32_t q0 = fdiv(s, g.m[0]);
    uint32_t q1 = fdiv(q0, g.m[1]);
    uint32_t q2 = fdiv(q1, g.m[2]);
    Site c;
    c.x = (int)(s - q0 * (uint32_t)g.L[0]);
    c.y = (int)(q0 - q1 * (uint32_t)g.L[1]);
    c.z = (int)(q1 - q2 * (uint32_t)g.L[2]);
    c.t = (int)q2;
    return c;
}

// neighbour site index in direction mu (forward or backward)
__device__ __forceinline__ uint32_t nb_fwd(const Geom& g, uint32_t s, const Site& c, int mu) {
    const uint32_t L0 = g.L[0], L1 = g.L[1], L2 = g.L[2], L3 = g.L[3];
    switch (mu) {
    case 0: return (c.x + 1 == (int)L0) ? s - (L0 - 1) : s + 1;
    case 1: return (c.y + 1 == (int)L1) ? s - (L1 - 1) * L0 : s + L0;
    case 2: return (c.z + 1 == (int)L2) ? s - (L2 - 1) * L0 * L1 : s + L0 * L1;
    default: return (c.t + 1 == (int)L3) ? s - (L3 - 1) * L0 * L1 * L2 : s + L0 * L1 * L2;
    }
}
__device__ __forceinline__ uint32_t nb_bwd(const Geom& g, uint32_t s, const Site& c, int mu) {
    const uint32_t L0 = g.L[0], L1 = g.L[1], L2 = g.L[2], L3 = g.L[3];
    switch (mu) {
    case 0: return (c.x == 0) ? s + (L0 - 1) : s - 1;
    case 1: return (c.y == 0) ? s + (L1 - 1) * L0 : s - L0;
    case 2: return (c.z == 0) ? s + (L2 - 1) * L0 * L1 : s - L0 * L1;
    default: return (c.t == 0) ? s + (L3 - 1) * L0 * L1 * L2 : s - L0 * L1 * L2;
    }
}

// Blocks are dealt round-robin to the 8 XCDs; remap so that each XCD works
// on one contiguous range of the lattice (its neighbours then sit in that
// XCD's L2).
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
    uint32_t full = nb & ~7u;
    if (b >= full) return b;
    return (b & 7u) * (full >> 3) + (b >> 3);
}

// Stencil launches are 1-D grids of nsb site blocks x nch right-hand-side
// chunks.  After the XCD remap, consecutive logical blocks are the chunks of
// one site block, so every chunk of a site block runs back to back on the same
// XCD (its links and neighbours are served from that XCD's L2), and each XCD
// sweeps one contiguous range of sites.
struct BlockMap {
    uint32_t sb;   // site block
    uint32_t ch;   // right-hand-side chunk
    uint32_t nsb;  // number of site blocks
};
__device__ __forceinline__ BlockMap stencil_block(uint32_t nch) {
    const uint32_t L = xcd_block(blockIdx.x, gridDim.x);
    BlockMap m;
    m.nsb = gridDim.x / nch;
    m.sb = L / nch;
    m.ch = L - m.sb * nch;
    return m;
}

// ---------------------------------------------------------------------------
// Z4 noise: splitmix64 output mix (Steele, Lea & Flood 2014) applied to the
// counter 1 + j*V + site of a stream started at mix(seed); component c takes
// bits 2c, 2c+1 of the hash as k, eta = i^k.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t noise_bits(uint64_t seed_mixed, uint64_t j, uint64_t V, uint64_t s) {
    return sm64_mix(seed_mixed + 0x9E3779B97F4A7C15ULL * (1ULL + j * V + s));
}
template <typename R>
__device__ __forceinline__ cx<R> z4_value(uint32_t k) {
    // k = 0, 1, 2, 3 -> 1, i, -1, -i
    R a = (k & 2) ? (R)-1 : (R)1;
    return (k & 1) ? cx<R>{(R)0, a} : cx<R>{a, (R)0};
}

// ---------------------------------------------------------------------------
// reductions (wave64 butterflies, fixed order: bitwise reproducible)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of v over a 256-thread block; result valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double* sh /*[4]*/) {
    v = wave_sum(v);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0;
    if (threadIdx.x == 0) r = ((sh[0] + sh[1]) + (sh[2] + sh[3]));
    __syncthreads();
    return r;
}

// Occupancy target of the stencil kernels (waves per SIMD) for NR
// right-hand sides per lane; caps the registers the scheduler may spend on
// hoisting neighbour loads.
#ifndef TM_WAVES_NR1
#define TM_WAVES_NR1 4
#endif
#ifndef TM_WAVES_NR2
#define TM_WAVES_NR2 3
#endif
#ifndef TM_WAVES_NR4
#define TM_WAVES_NR4 2
#endif
template <int NR>
struct StencilOcc {
    static constexpr int waves = NR == 1 ? TM_WAVES_NR1 : (NR == 2 ? TM_WAVES_NR2 : (NR == 4 ? TM_WAVES_NR4 : 1));
};

}  // namespace tmq

#define TM_STENCIL(NR) __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(::tmq::StencilOcc<NR>::waves)))
// FP64 arithmetic needs twice the registers of FP32 per right-hand side
#define TM_STENCIL_R(NR, R) \
    __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(::tmq::StencilOcc<(sizeof(R) == 8 ? 2 * NR : NR)>::waves)))
