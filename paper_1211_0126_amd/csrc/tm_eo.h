// Even-odd building blocks shared by the half-hop kernels (gfx950): half-site
// coordinates and neighbours, the hops of one direction, the site-local
// twisted-mass block D = 1 + i tw g5 and its inverse, the Z4 source at a site.
//
// Half fields hold the sites of one parity (x + y + z + t even or odd),
// indexed h = x/2 + (Lx/2)(y + Ly(z + Lz t)); every extent is even, so each
// hop joins sites of opposite parity.
#pragma once

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

template <bool DAG, typename R, class S, class G, int NR>
__device__ __forceinline__ void eo_hop_all(const Geom& hg, const void* gout, const void* gin, const void* in,
                                           uint32_t h, const EoSite& c, cx<R> (&acc)[NR][12]) {
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int k = 0; k < 12; k++) acc[r][k] = {(R)0, (R)0};
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
