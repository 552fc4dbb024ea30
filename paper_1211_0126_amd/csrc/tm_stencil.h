// Stencil building blocks of the twisted-mass Wilson operator (gfx950):
// spin projection and reconstruction, SU(3) products, the hops of one
// direction and the diagonal term.  Shared by the site-per-lane kernels and
// the time-marching kernels.
//
// M = 1 - kappa H + 2 i kappa mu gamma_5 in the hopping normalisation, with
// H psi(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^dag
// psi(x-mu); H^dag swaps the two projectors.

#pragma once

#include "tm_device.h"

// Compiler-only barrier: memory operations are not moved across it.
#define TM_MEM_FENCE() asm volatile("" ::: "memory")

namespace tmq {

// Cache policies of the streamed accesses of the CG kernels (see ld_plane):
// K2's centre-site fields, K1's output, K3's inputs.
#ifndef TM_CP_K2
#define TM_CP_K2 kStream
#endif
#ifndef TM_CP_K1T
#define TM_CP_K1T kStream
#endif
#ifndef TM_CP_K3
#define TM_CP_K3 kStream
#endif

// ---------------------------------------------------------------------------
// spin projection for the hop in direction MU with projector 1 - SG g_MU.
// With g_MU = [[0, B], [B^dag, 0]] (2x2 spin blocks) the projected spinor is
// (h, -SG B^dag h) with h = u - SG B d, u and d the upper and lower halves.
// ---------------------------------------------------------------------------
template <int MU, int SG, typename R>
__device__ __forceinline__ void proj(const cx<R> p[12], cx<R> h[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        cx<R> u0 = p[c], u1 = p[3 + c], d0 = p[6 + c], d1 = p[9 + c];
        cx<R> b0, b1;
        if (MU == 0) {        // B = -i sigma_1
            b0 = times_mi(d1);
            b1 = times_mi(d0);
        } else if (MU == 1) { // B = -i sigma_2
            b0 = {-d1.re, -d1.im};
            b1 = d0;
        } else if (MU == 2) { // B = -i sigma_3
            b0 = times_mi(d0);
            b1 = times_i(d1);
        } else {              // B = 1
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

template <int MU, int SG, typename R>
__device__ __forceinline__ void recon(const cx<R> g[6], cx<R> acc[12]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        cx<R> g0 = g[c], g1 = g[3 + c];
        cx<R> e0, e1;  // B^dag g
        if (MU == 0) {
            e0 = times_i(g1);
            e1 = times_i(g0);
        } else if (MU == 1) {
            e0 = g1;
            e1 = {-g0.re, -g0.im};
        } else if (MU == 2) {
            e0 = times_i(g0);
            e1 = times_mi(g1);
        } else {
            e0 = g0;
            e1 = g1;
        }
        acc[c] = acc[c] + g0;
        acc[3 + c] = acc[3 + c] + g1;
        if (SG > 0) {
            acc[6 + c] = acc[6 + c] - e0;
            acc[9 + c] = acc[9 + c] - e1;
        } else {
            acc[6 + c] = acc[6 + c] + e0;
            acc[9 + c] = acc[9 + c] + e1;
        }
    }
}

// SU(3) times the two colour vectors of a half spinor, as chains of fused
// multiply-adds (a complex multiply-add is four FMAs; written out because the
// compiler may not fuse across the complex products without reassociating)
template <typename R>
__device__ __forceinline__ cx<R> cmul_f(cx<R> a, cx<R> b) {
    return {fma(-a.im, b.im, a.re * b.re), fma(a.im, b.re, a.re * b.im)};
}
template <typename R>
__device__ __forceinline__ void cmac_f(cx<R>& t, cx<R> a, cx<R> b) {
    t.re = fma(a.re, b.re, t.re);
    t.re = fma(-a.im, b.im, t.re);
    t.im = fma(a.re, b.im, t.im);
    t.im = fma(a.im, b.re, t.im);
}
// conj(a) * b, and t += conj(a) * b
template <typename R>
__device__ __forceinline__ cx<R> cmulc_f(cx<R> a, cx<R> b) {
    return {fma(a.im, b.im, a.re * b.re), fma(-a.im, b.re, a.re * b.im)};
}
template <typename R>
__device__ __forceinline__ void cmacc_f(cx<R>& t, cx<R> a, cx<R> b) {
    t.re = fma(a.re, b.re, t.re);
    t.re = fma(a.im, b.im, t.re);
    t.im = fma(a.re, b.im, t.im);
    t.im = fma(-a.im, b.re, t.im);
}

template <typename R>
__device__ __forceinline__ void su3_mul(const cx<R> U[3][3], const cx<R> h[6], cx<R> g[6]) {
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int i = 0; i < 3; i++) {
            cx<R> t = cmul_f(U[i][0], h[3 * a]);
            cmac_f(t, U[i][1], h[3 * a + 1]);
            cmac_f(t, U[i][2], h[3 * a + 2]);
            g[3 * a + i] = t;
        }
}
template <typename R>
__device__ __forceinline__ void su3_dag_mul(const cx<R> U[3][3], const cx<R> h[6], cx<R> g[6]) {
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int i = 0; i < 3; i++) {
            cx<R> t = cmulc_f(U[0][i], h[3 * a]);
            cmacc_f(t, U[1][i], h[3 * a + 1]);
            cmacc_f(t, U[2][i], h[3 * a + 2]);
            g[3 * a + i] = t;
        }
}

template <typename R>
__device__ __forceinline__ void negate6(cx<R> h[6]) {
#pragma unroll
    for (int k = 0; k < 6; k++) h[k] = {-h[k].re, -h[k].im};
}

// Materialise the accumulators here: the arithmetic of one direction then
// completes before the next direction's loads are issued.
template <typename R, int NR>
__device__ __forceinline__ void pin_acc(cx<R> (&acc)[NR][12]) {
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int k = 0; k < 12; k++) asm volatile("" : "+v"(acc[r][k].re), "+v"(acc[r][k].im));
}

// Both hops in direction MU for NR spinors (rhs r at field_rhs(in, r)).
template <int MU, bool DAG, typename R, class S, class G, int NR>
__device__ __forceinline__ void hop_mu(const Geom& geo, const void* gauge, const void* in, uint32_t s, const Site& c,
                                       cx<R> (&acc)[NR][12]) {
    constexpr int SF = DAG ? -1 : 1;
    const long Vs = geo.Vs;
    {
        const uint32_t y = nb_fwd(geo, s, c, MU);
        const bool flip = (MU == 3) && (c.t + 1 == geo.L[3]) && (geo.t_bc < 0);
        cx<R> U[3][3];
        load_link<G, R>(gauge, Vs, MU, s, U);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<R> p[12], h[6], g[6];
            load_spinor<S, R>(field_rhs<S>(in, Vs, r), Vs, y, p);
            proj<MU, SF>(p, h);
            if (flip) negate6(h);
            su3_mul(U, h, g);
            recon<MU, SF>(g, acc[r]);
        }
    }
    if (sizeof(R) == 8) {
        pin_acc<R, NR>(acc);
        TM_MEM_FENCE();
    }
    {
        const uint32_t y = nb_bwd(geo, s, c, MU);
        const bool flip = (MU == 3) && (c.t == 0) && (geo.t_bc < 0);
        cx<R> U[3][3];
        load_link<G, R>(gauge, Vs, MU, y, U);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<R> p[12], h[6], g[6];
            load_spinor<S, R>(field_rhs<S>(in, Vs, r), Vs, y, p);
            proj<MU, -SF>(p, h);
            if (flip) negate6(h);
            su3_dag_mul(U, h, g);
            recon<MU, -SF>(g, acc[r]);
        }
    }
}

template <bool DAG, typename R, class S, class G, int NR>
__device__ __forceinline__ void hop_all(const Geom& geo, const void* gauge, const void* in, uint32_t s, const Site& c,
                                        cx<R> (&acc)[NR][12]) {
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int k = 0; k < 12; k++) acc[r][k] = {(R)0, (R)0};
    // compiler barriers keep one direction's loads in flight at a time, so
    // the register budget of the occupancy target is not spent on hoisting
    hop_mu<0, DAG, R, S, G, NR>(geo, gauge, in, s, c, acc);
    pin_acc<R, NR>(acc);
    TM_MEM_FENCE();
    hop_mu<1, DAG, R, S, G, NR>(geo, gauge, in, s, c, acc);
    pin_acc<R, NR>(acc);
    TM_MEM_FENCE();
    hop_mu<2, DAG, R, S, G, NR>(geo, gauge, in, s, c, acc);
    pin_acc<R, NR>(acc);
    TM_MEM_FENCE();
    hop_mu<3, DAG, R, S, G, NR>(geo, gauge, in, s, c, acc);
}

// out = p - kappa acc + i tw gamma_5 p   (tw = +2 kappa mu for M, -2 kappa mu for M^dag)
template <typename R>
__device__ __forceinline__ void diag_combine(const cx<R> p[12], const cx<R> acc[12], R kappa, R tw, cx<R> out[12]) {
#pragma unroll
    for (int k = 0; k < 6; k++)
        out[k] = {p[k].re - kappa * acc[k].re - tw * p[k].im, p[k].im - kappa * acc[k].im + tw * p[k].re};
#pragma unroll
    for (int k = 6; k < 12; k++)
        out[k] = {p[k].re - kappa * acc[k].re + tw * p[k].im, p[k].im - kappa * acc[k].im - tw * p[k].re};
}

template <typename R>
__device__ __forceinline__ double spinor_norm2(const cx<R> v[12]) {
    double s = 0;
#pragma unroll
    for (int k = 0; k < 12; k++) s += (double)v[k].re * (double)v[k].re + (double)v[k].im * (double)v[k].im;
    return s;
}

}  // namespace tmq
