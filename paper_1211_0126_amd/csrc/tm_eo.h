// Even-odd building blocks shared by the half-hop kernels (gfx950): half-site
// coordinates and neighbours, the hops of one direction, the site-local
// twisted-mass block D = 1 + i tw g5 and its inverse, the Z4 source at a site.
//
// Half fields hold the sites of one parity (x + y + z + t even or odd),
// indexed h = x/2 + (Lx/2)(y + Ly(z + Lz t)); every extent is even, so each
// hop joins sites of opposite parity.
#pragma once

#include <type_traits>

#include "tm_device.h"
#include "tm_stencil.h"

namespace tmq {

struct EoSite {
    int xh, x, y, z, t;
};

// coordinates of half-site h of parity par (hg.m[0] divides by Lx/2; it is
// 0 for Lx = 2, where the row is h itself)
__device__ __forceinline__ EoSite eo_coords(const Geom& hg, uint32_t h, int par) {
    const uint32_t Lxh = (uint32_t)hg.L[0] >> 1;
    const uint32_t q0 = hg.m[0] ? fdiv(h, hg.m[0]) : h;
    const uint32_t q1 = fdiv(q0, hg.m[1]);
    const uint32_t q2 = fdiv(q1, hg.m[2]);
    EoSite c;
    c.xh = (int)(h - q0 * Lxh);
    c.y = (int)(q0 - q1 * (uint32_t)hg.L[1]);
    c.z = (int)(q1 - q2 * (uint32_t)hg.L[2]);
    c.t = (int)q2;
    c.x = 2 * c.xh + ((c.y + c.z + c.t + par) & 1);
    return c;
}

// Half-site of thread tid in site block sb.  Natural order: 256 consecutive
// half-sites.  Brick order (hg.brick = rows per wave, Lx/2 * hg.brick = 64):
// a wave covers hg.brick consecutive rows of one z plane (1 KiB per plane of
// an FP32 field, as in the natural order), the block's four waves four
// consecutive z planes of one time slice; the blocks run through the bricks
// of one z slab y-brick fastest, then time slice, so that the y neighbours
// of a block belong to the blocks dispatched just before and after it on the
// same XCD and its time neighbours to blocks a y row of bricks away (both
// served from that XCD's L2 instead of HBM).
__device__ __forceinline__ uint32_t eo_site(const Geom& hg, uint32_t sb, uint32_t tid) {
    if (hg.brick == 0) return sb * 256u + tid;
    const uint32_t Lxh = (uint32_t)hg.L[0] >> 1, by = hg.brick;
    const uint32_t Lt = (uint32_t)hg.L[3], nty = (uint32_t)hg.L[1] / by;
    const uint32_t ty = sb % nty, rest = sb / nty;
    const uint32_t t = rest % Lt, tz = rest / Lt;
    const uint32_t lane = tid & 63u;
    const uint32_t y = ty * by + lane / Lxh, z = tz * 4u + (tid >> 6);
    return lane % Lxh + Lxh * (y + (uint32_t)hg.L[1] * (z + (uint32_t)hg.L[2] * t));
}

// half index of the neighbour (opposite parity) in direction mu
__device__ __forceinline__ uint32_t eo_nb(const Geom& hg, uint32_t h, const EoSite& c, int mu, bool fwd) {
    const uint32_t L0 = hg.L[0], L1 = hg.L[1], L2 = hg.L[2], L3 = hg.L[3];
    const uint32_t Lxh = L0 >> 1;
    switch (mu) {
    case 0: {
        const int xn = fwd ? ((c.x + 1 == (int)L0) ? 0 : c.x + 1) : ((c.x == 0) ? (int)L0 - 1 : c.x - 1);
        return h - (uint32_t)c.xh + (uint32_t)(xn >> 1);
    }
    case 1:
        return fwd ? ((c.y + 1 == (int)L1) ? h - (L1 - 1) * Lxh : h + Lxh)
                   : ((c.y == 0) ? h + (L1 - 1) * Lxh : h - Lxh);
    case 2:
        return fwd ? ((c.z + 1 == (int)L2) ? h - (L2 - 1) * Lxh * L1 : h + Lxh * L1)
                   : ((c.z == 0) ? h + (L2 - 1) * Lxh * L1 : h - Lxh * L1);
    default:
        return fwd ? ((c.t + 1 == (int)L3) ? h - (L3 - 1) * Lxh * L1 * L2 : h + Lxh * L1 * L2)
                   : ((c.t == 0) ? h + (L3 - 1) * Lxh * L1 * L2 : h - Lxh * L1 * L2);
    }
}

// full-lattice site index of half-site h (parity par)
__device__ __forceinline__ uint32_t eo_full_site(uint32_t h, const EoSite& c) {
    return (h - (uint32_t)c.xh) * 2u + (uint32_t)c.x;  // x + Lx row with row = (h - xh) / (Lx/2)
}

// both hops in direction MU into half-site h: forward links from gout (the
// output parity's copy, at h), backward links from gin at the neighbour
template <int MU, bool DAG, typename R, class S, class G, int NR>
__device__ __forceinline__ void eo_hop_mu(const Geom& hg, const void* gout, const void* gin, const void* in,
                                          uint32_t h, const EoSite& c, cx<R> (&acc)[NR][12]) {
    constexpr int SF = DAG ? -1 : 1;
    const long Vs = hg.Vs;
    {
        const uint32_t y = eo_nb(hg, h, c, MU, true);
        const bool flip = (MU == 3) && (c.t + 1 == hg.L[3]) && (hg.t_bc < 0);
        cx<R> U[3][3];
        load_link<G, R>(gout, Vs, MU, h, U);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<R> p[12], hh[6], g[6];
            load_spinor<S, R>(field_rhs<S>(in, Vs, r), Vs, y, p);
            proj<MU, SF>(p, hh);
            if (flip) negate6(hh);
            su3_mul(U, hh, g);
            recon<MU, SF>(g, acc[r]);
        }
    }
    if (sizeof(R) == 8) {
        pin_acc<R, NR>(acc);
        TM_MEM_FENCE();
    }
    {
        const uint32_t y = eo_nb(hg, h, c, MU, false);
        const bool flip = (MU == 3) && (c.t == 0) && (hg.t_bc < 0);
        cx<R> U[3][3];
        load_link<G, R>(gin, Vs, MU, y, U);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<R> p[12], hh[6], g[6];
            load_spinor<S, R>(field_rhs<S>(in, Vs, r), Vs, y, p);
            proj<MU, -SF>(p, hh);
            if (flip) negate6(hh);
            su3_dag_mul(U, hh, g);
            recon<MU, -SF>(g, acc[r]);
        }
    }
}

// ---------------------------------------------------------------------------
// FP16 links for the FP16-storage hops (GH16): the nine entries of a link as
// (re, im) binary16 pairs, [mu][3][Vs] uint4 per parity (entries 0-3, 4-7, 8
// and padding).  A hop projects the FP16 input spinor in packed FP16 (one
// rounding of each sum), multiplies by the link with v_dot2_f32_f16 (FP16
// products, exact in FP32, summed in FP32) and reconstructs in FP32.
// ---------------------------------------------------------------------------
struct GH16 {};
#ifndef TM_H16_GROUP
#define TM_H16_GROUP 1
#endif
typedef _Float16 h2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ h2v as_h2(uint32_t u) { return __builtin_bit_cast(h2v, u); }
__device__ __forceinline__ uint32_t as_u32(h2v v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ uint32_t h2_swap(uint32_t u) { return __builtin_amdgcn_alignbit(u, u, 16); }

// c + a.lo b.lo + a.hi b.hi with FP16 operands and FP32 result
// (v_dot2_f32_f16, left to the compiler, which knows its hazards)
__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float c) {
    return __builtin_amdgcn_fdot2(as_h2(a), as_h2(b), c, false);
}
// (re, im) -> (re, -im) and (-re, im)
__device__ __forceinline__ uint32_t h2_neg_hi(uint32_t u) { return u ^ 0x80000000u; }
__device__ __forceinline__ uint32_t h2_neg_lo(uint32_t u) { return u ^ 0x00008000u; }

__device__ __forceinline__ void load_link16(const void* g, long Vs, int mu, uint32_t s, uint32_t U[9]) {
    const uint4 a = ld_plane<uint4>(g, Vs, mu * 3 + 0, s);
    const uint4 b = ld_plane<uint4>(g, Vs, mu * 3 + 1, s);
    const uint4 c = ld_plane<uint4>(g, Vs, mu * 3 + 2, s);
    U[0] = a.x; U[1] = a.y; U[2] = a.z; U[3] = a.w;
    U[4] = b.x; U[5] = b.y; U[6] = b.z; U[7] = b.w;
    U[8] = c.x;
}

__device__ __forceinline__ void load_spinor_h2(const void* base, long Vs, uint32_t s, h2v p[12]) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const uint4 v = ld_plane<uint4>(base, Vs, k, s);
        p[4 * k + 0] = as_h2(v.x);
        p[4 * k + 1] = as_h2(v.y);
        p[4 * k + 2] = as_h2(v.z);
        p[4 * k + 3] = as_h2(v.w);
    }
}

// packed FP16 spin projection for the hop with projector 1 - SG g_MU (the
// same signed permutations as proj<MU, SG>)
template <int MU, int SG>
__device__ __forceinline__ void proj_h2(const h2v p[12], h2v h[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const h2v u0 = p[c], u1 = p[3 + c], d0 = p[6 + c], d1 = p[9 + c];
        h2v b0, b1;
        if (MU == 0) {        // -i d1, -i d0
            b0 = (h2v){d1.y, -d1.x};
            b1 = (h2v){d0.y, -d0.x};
        } else if (MU == 1) { // -d1, d0
            b0 = -d1;
            b1 = d0;
        } else if (MU == 2) { // -i d0, i d1
            b0 = (h2v){d0.y, -d0.x};
            b1 = (h2v){-d1.y, d1.x};
        } else {
            b0 = d0;
            b1 = d1;
        }
        if (SG > 0) {
            h[c] = u0 - b0;
            h[3 + c] = u1 - b1;
        } else {
            h[c] = u0 + b0;
            h[3 + c] = u1 + b1;
        }
    }
}

// g = U h (forward) or U^dag h: both colour vectors of a half spinor, FP32
// out, from the link forms A and B (link_forms):
//   forward  U[i][j]:       re = (re, -im).h,  im = (im, re).h
//   adjoint  conj(U[j][i]): re = (re, im).h,   im = (-im, re).h
__device__ __forceinline__ void su3_h2(const uint32_t A[9], const uint32_t B[9], const uint32_t h[6],
                                       cx<float> g[6]) {
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int i = 0; i < 3; i++) {
            float re = dot2(A[3 * i + 0], h[3 * a + 0], 0.f);
            re = dot2(A[3 * i + 1], h[3 * a + 1], re);
            re = dot2(A[3 * i + 2], h[3 * a + 2], re);
            float im = dot2(B[3 * i + 0], h[3 * a + 0], 0.f);
            im = dot2(B[3 * i + 1], h[3 * a + 1], im);
            im = dot2(B[3 * i + 2], h[3 * a + 2], im);
            g[3 * a + i] = {re, im};
        }
}
// the two operand forms of a link for su3_h2 (once per link, shared by the
// right-hand sides of a lane)
template <bool DAGL>
__device__ __forceinline__ void link_forms(const uint32_t U[9], uint32_t A[9], uint32_t B[9]) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const uint32_t u = DAGL ? U[3 * j + i] : U[3 * i + j];
            const uint32_t w = h2_swap(u);
            A[3 * i + j] = DAGL ? u : h2_neg_hi(u);
            B[3 * i + j] = DAGL ? h2_neg_lo(w) : w;
        }
}

// both FP16 hops in direction MU (FP16 spinors and links, FP32 accumulators)
template <int MU, bool DAG, int NR>
__device__ __forceinline__ void eo_hop_mu_h16(const Geom& hg, const void* gout, const void* gin, const void* in,
                                              uint32_t h, const EoSite& c, cx<float> (&acc)[NR][12]) {
    constexpr int SF = DAG ? -1 : 1;
    const long Vs = hg.Vs;
    // the antiperiodic time boundary flips the sign of the projected spinor
    // (both halves of every FP16 pair)
    {
        const uint32_t y = eo_nb(hg, h, c, MU, true);
        const uint32_t sgn = ((MU == 3) && (c.t + 1 == hg.L[3]) && (hg.t_bc < 0)) ? 0x80008000u : 0u;
        uint32_t U[9], A[9], B[9];
        load_link16(gout, Vs, MU, h, U);
        link_forms<false>(U, A, B);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            h2v p[12], hh[6];
            uint32_t hu[6];
            cx<float> g[6];
            load_spinor_h2(field_rhs<SF16>(in, Vs, r), Vs, y, p);
            proj_h2<MU, SF>(p, hh);
#pragma unroll
            for (int k = 0; k < 6; k++) hu[k] = MU == 3 ? (as_u32(hh[k]) ^ sgn) : as_u32(hh[k]);
            su3_h2(A, B, hu, g);
            recon<MU, SF>(g, acc[r]);
        }
    }
    {
        const uint32_t y = eo_nb(hg, h, c, MU, false);
        const uint32_t sgn = ((MU == 3) && (c.t == 0) && (hg.t_bc < 0)) ? 0x80008000u : 0u;
        uint32_t U[9], A[9], B[9];
        load_link16(gin, Vs, MU, y, U);
        link_forms<true>(U, A, B);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            h2v p[12], hh[6];
            uint32_t hu[6];
            cx<float> g[6];
            load_spinor_h2(field_rhs<SF16>(in, Vs, r), Vs, y, p);
            proj_h2<MU, -SF>(p, hh);
#pragma unroll
            for (int k = 0; k < 6; k++) hu[k] = MU == 3 ? (as_u32(hh[k]) ^ sgn) : as_u32(hh[k]);
            su3_h2(A, B, hu, g);
            recon<MU, -SF>(g, acc[r]);
        }
    }
}

template <bool DAG, typename R, class S, class G, int NR>
__device__ __forceinline__ void eo_hop_all(const Geom& hg, const void* gout, const void* gin, const void* in,
                                           uint32_t h, const EoSite& c, cx<R> (&acc)[NR][12]) {
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int k = 0; k < 12; k++) acc[r][k] = {(R)0, (R)0};
    if constexpr (std::is_same<G, GH16>::value) {
        static_assert(std::is_same<S, SF16>::value && sizeof(R) == 4, "FP16 links go with FP16 spinors");
        // FP16 operands take half the registers: the loads of TM_H16_GROUP
        // directions may be in flight together
        eo_hop_mu_h16<0, DAG, NR>(hg, gout, gin, in, h, c, acc);
        if (TM_H16_GROUP < 2) {
            pin_acc<R, NR>(acc);
            TM_MEM_FENCE();
        }
        eo_hop_mu_h16<1, DAG, NR>(hg, gout, gin, in, h, c, acc);
        if (TM_H16_GROUP < 4) {
            pin_acc<R, NR>(acc);
            TM_MEM_FENCE();
        }
        eo_hop_mu_h16<2, DAG, NR>(hg, gout, gin, in, h, c, acc);
        if (TM_H16_GROUP < 2) {
            pin_acc<R, NR>(acc);
            TM_MEM_FENCE();
        }
        eo_hop_mu_h16<3, DAG, NR>(hg, gout, gin, in, h, c, acc);
    } else {
        eo_hop_mu<0, DAG, R, S, G, NR>(hg, gout, gin, in, h, c, acc);
        pin_acc<R, NR>(acc);
        TM_MEM_FENCE();
        eo_hop_mu<1, DAG, R, S, G, NR>(hg, gout, gin, in, h, c, acc);
        pin_acc<R, NR>(acc);
        TM_MEM_FENCE();
        eo_hop_mu<2, DAG, R, S, G, NR>(hg, gout, gin, in, h, c, acc);
        pin_acc<R, NR>(acc);
        TM_MEM_FENCE();
        eo_hop_mu<3, DAG, R, S, G, NR>(hg, gout, gin, in, h, c, acc);
    }
}

// v <- (1 + i tw g5) v, g5 = diag(1, 1, -1, -1) (components 0-5 upper spins)
template <typename R>
__device__ __forceinline__ void mul_diag(cx<R> v[12], R tw) {
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const R s = k < 6 ? tw : -tw;
        v[k] = {v[k].re - s * v[k].im, v[k].im + s * v[k].re};
    }
}
// v <- (1 + i tw g5)^{-1} v = (1 - i tw g5) v / (1 + tw^2)
template <typename R>
__device__ __forceinline__ void mul_diag_inv(cx<R> v[12], R tw, R inv) {
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const R s = k < 6 ? -tw : tw;
        v[k] = {inv * (v[k].re - s * v[k].im), inv * (v[k].im + s * v[k].re)};
    }
}

// Z4 source at full site s (the same hash as the full-lattice noise)
template <typename R>
__device__ __forceinline__ void noise_at(uint64_t seed_mixed, uint64_t id, uint64_t V, uint64_t s, cx<R> e[12]) {
    const uint64_t hb = noise_bits(seed_mixed, id, V, s);
#pragma unroll
    for (int k = 0; k < 12; k++) e[k] = z4_value<R>((uint32_t)(hb >> (2 * k)) & 3u);
}

// two spinors to the adjacent full-lattice sites s0 and s1 (the even and odd
// site of one half index), plane by plane, so that each plane's 32 bytes of
// a lane are written together
template <class X, typename R>
__device__ __forceinline__ void store_site_pair(void* base, long Vs, uint32_t s0, const cx<R> a[12], uint32_t s1,
                                                const cx<R> b[12]) {
    if constexpr (X::NV == 12) {
#pragma unroll
        for (int k = 0; k < 12; k++) {
            st_plane(base, Vs, k, s0, make_double2((double)a[k].re, (double)a[k].im));
            st_plane(base, Vs, k, s1, make_double2((double)b[k].re, (double)b[k].im));
        }
    } else {
        static_assert(X::NV == 6, "FP32 or FP64 solutions");
#pragma unroll
        for (int k = 0; k < 6; k++) {
            st_plane(base, Vs, k, s0,
                     make_float4((float)a[2 * k].re, (float)a[2 * k].im, (float)a[2 * k + 1].re, (float)a[2 * k + 1].im));
            st_plane(base, Vs, k, s1,
                     make_float4((float)b[2 * k].re, (float)b[2 * k].im, (float)b[2 * k + 1].re, (float)b[2 * k + 1].im));
        }
    }
}

}  // namespace tmq
