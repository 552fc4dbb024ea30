// Even-odd (Schur complement) form of the twisted-mass operator (gfx950).
//
// A site is even or odd by the parity of x + y + z + t.  With every extent
// even each hop of H joins sites of opposite parity, so M = 1 - kappa H +
// i tw g5 (tw = 2 kappa mu) splits into the site-local blocks D = 1 + i tw g5
// on either parity and the hops H_eo, H_oe.  CG runs on the normal
// equations of the Schur complement on the odd sites,
//   Mhat = D - kappa^2 H_oe D^{-1} H_eo,
// whose source is etahat_o = eta_o + kappa H_oe D^{-1} eta_e; the even half
// of the solution follows as x_e = D^{-1} (eta_e + kappa H_eo x_o).  Mhat^dag
// is the same construction on M^dag (D^dag = 1 - i tw g5, H^dag = g5 H g5:
// the two projectors swapped).  This reduction is not in the paper: it is an
// alternative inverter for the LP and HP solves of the TSM (section 2.2,
// Eq. 4), whose combination is unbiased for any fixed LP map.
//
// Half fields: the sites of one parity, indexed h = x/2 + (Lx/2)(y + Ly(z +
// Lz t)), stored like full native fields (component planes of 16-byte
// vectors) with their own plane stride.  The links are split the same way:
// each parity's copy holds the forward links U_mu(x) of its sites, so a
// half-hop reads the forward links from the output parity's copy and the
// backward links U_mu(x - mu) from the input parity's copy at the neighbour,
// and every link is read once per half-hop.
//
// Per CG iteration (k_eo_lin, k_eo_mp, k_eo_lin, k_eo_upd; the alpha and beta
// reductions and p = r + beta p are the full-lattice kernels on the half
// geometry):
//   y = D^{-1} H_eo p          t = D p - kappa^2 H_oe y,  |t|^2
//   y = D^{-dag} H_eo^dag t    q = D^dag t - kappa^2 H_oe^dag y,
//                              r -= alpha q, x += alpha p, |r|^2

#include <algorithm>

#include "tm_device.h"
#include "tm_kernels.h"
#include "tm_stencil.h"
#include "tm_eo.h"

namespace tmq {

// ---------------------------------------------------------------------------
// linear half-hop: out = POST(PRE(b) + c acc), acc = H (or H^dag if DAG) in,
// PRE = D (if PRE_D) or 1 applied to the centre term b (nullptr: none; with
// a.bnoise the Z4 source of the output site), POST = D^{-1} (if POST_DINV)
// or 1; D carries the twist of M (or M^dag if DAG).
// gate (nullable): only right-hand sides whose reliable flag is set (NR = 1,
// small grid striding over the site blocks).
// ---------------------------------------------------------------------------
template <bool DAG, bool PRE_D, bool POST_DINV, typename R, class Si, class So, class G, int NR>
__global__ TM_STENCIL_R(NR, R) void k_eo_lin(EoArgs a) {
    const Geom& hg = a.hg;
    const BlockMap bm = stencil_block((uint32_t)(a.nrhs / NR));
    const int r0 = bm.ch * NR;
    if (a.gate != nullptr) {
        bool any = false;
#pragma unroll
        for (int r = 0; r < NR; r++) any |= a.gate[r0 + r].rflag != 0;
        if (!any) return;  // (sources of the chunk without the flag are computed and not used)
    }
    if (a.act != nullptr) {
        bool any = false;
#pragma unroll
        for (int r = 0; r < NR; r++) any |= a.act[r0 + r].active != 0;
        if (!any) return;  // uniform over the chunk's blocks
    }
    const long Vs = hg.Vs;
    const R tw = (R)(DAG ? -a.twist : a.twist);
    const R inv = (R)(1.0 / (1.0 + a.twist * a.twist));
    const R cf = (R)a.c;
    const void* in0 = field_rhs<Si>(a.in, Vs, r0);
    const uint32_t nsb_all = (uint32_t)((hg.V + 255) / 256);
    for (uint32_t sb = bm.sb; sb < nsb_all; sb += bm.nsb) {
        const uint32_t h = eo_site(hg, sb, threadIdx.x);
        if (h >= hg.V) continue;
        const EoSite c = eo_coords(hg, h, a.pout);
        cx<R> acc[NR][12];
        eo_hop_all<DAG, R, Si, G, NR>(hg, a.gout, a.gin, in0, h, c, acc);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<R> o[12];
            if (a.bnoise) {
                noise_at<R>(a.seed_mixed, a.ids[r0 + r], (uint64_t)(2 * hg.V), eo_full_site(h, c), o);
                if (PRE_D) mul_diag(o, tw);
#pragma unroll
                for (int k = 0; k < 12; k++) o[k] = o[k] + cf * acc[r][k];
            } else if (a.b != nullptr) {
                load_spinor<So, R>(field_rhs<So>(a.b, Vs, r0 + r), Vs, h, o);
                if (PRE_D) mul_diag(o, tw);
#pragma unroll
                for (int k = 0; k < 12; k++) o[k] = o[k] + cf * acc[r][k];
            } else {
#pragma unroll
                for (int k = 0; k < 12; k++) o[k] = cf * acc[r][k];
            }
            if (POST_DINV) mul_diag_inv(o, tw, inv);
            store_spinor<So, R>(field_rhs<So>(a.out, Vs, r0 + r), Vs, h, o);
        }
    }
}

// Full-lattice index of the neighbour in direction MU of half-site h (the
// Z4 source of a site is a hash of its full index)
template <int MU>
__device__ __forceinline__ uint32_t eo_nb_full(const Geom& hg, uint32_t h, const EoSite& c, bool fwd) {
    const uint32_t L0 = hg.L[0], L1 = hg.L[1], L2 = hg.L[2], L3 = hg.L[3];
    const uint32_t row = (h - (uint32_t)c.xh) * 2u;  // Lx (y + Ly (z + Lz t))
    if (MU == 0) {
        const uint32_t xn = fwd ? ((c.x + 1 == (int)L0) ? 0u : (uint32_t)c.x + 1u)
                                : ((c.x == 0) ? L0 - 1u : (uint32_t)c.x - 1u);
        return row + xn;
    }
    const uint32_t s = row + (uint32_t)c.x;
    if (MU == 1) return fwd ? ((c.y + 1 == (int)L1) ? s - (L1 - 1u) * L0 : s + L0) : ((c.y == 0) ? s + (L1 - 1u) * L0 : s - L0);
    if (MU == 2)
        return fwd ? ((c.z + 1 == (int)L2) ? s - (L2 - 1u) * L0 * L1 : s + L0 * L1)
                   : ((c.z == 0) ? s + (L2 - 1u) * L0 * L1 : s - L0 * L1);
    return fwd ? ((c.t + 1 == (int)L3) ? s - (L3 - 1u) * L0 * L1 * L2 : s + L0 * L1 * L2)
               : ((c.t == 0) ? s + (L3 - 1u) * L0 * L1 * L2 : s - L0 * L1 * L2);
}

// Both hops of H (not H^dag) in direction MU into odd half-site h with the
// input D^{-1} eta generated at the even neighbours from the hash
template <int MU, typename R, class G, int NR>
__device__ __forceinline__ void src_hop_mu(const EoArgs& a, const uint64_t* ids, uint32_t h, const EoSite& c, R tw,
                                           R inv, cx<R> (&acc)[NR][12]) {
    const Geom& hg = a.hg;
    const long Vs = hg.Vs;
    const uint64_t Vf = 2 * (uint64_t)hg.V;
    {
        const uint32_t sy = eo_nb_full<MU>(hg, h, c, true);
        const bool flip = (MU == 3) && (c.t + 1 == hg.L[3]) && (hg.t_bc < 0);
        cx<R> U[3][3];
        load_link<G, R>(a.gout, Vs, MU, h, U);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<R> p[12], hh[6], g[6];
            noise_at<R>(a.seed_mixed, ids[r], Vf, sy, p);
            mul_diag_inv(p, tw, inv);
            proj<MU, 1>(p, hh);
            if (flip) negate6(hh);
            su3_mul(U, hh, g);
            recon<MU, 1>(g, acc[r]);
        }
    }
    {
        const uint32_t y = eo_nb(hg, h, c, MU, false);
        const uint32_t sy = eo_nb_full<MU>(hg, h, c, false);
        const bool flip = (MU == 3) && (c.t == 0) && (hg.t_bc < 0);
        cx<R> U[3][3];
        load_link<G, R>(a.gin, Vs, MU, y, U);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<R> p[12], hh[6], g[6];
            noise_at<R>(a.seed_mixed, ids[r], Vf, sy, p);
            mul_diag_inv(p, tw, inv);
            proj<MU, -1>(p, hh);
            if (flip) negate6(hh);
            su3_dag_mul(U, hh, g);
            recon<MU, -1>(g, acc[r]);
        }
    }
}

// Source of the Schur system on the odd sites, etahat = eta_o + kappa H_oe
// D^{-1} eta_e, with the Z4 source generated from the hash at each site it
// needs: no source field is written or read.  The chunk of right-hand sides
// r0 .. r0 + NR - 1 takes the ids a.ids[r0 ..].
template <typename R, class So, class G, int NR>
__global__ __launch_bounds__(256) void k_eo_src(EoArgs a) {
    const Geom& hg = a.hg;
    const BlockMap bm = stencil_block((uint32_t)(a.nrhs / NR));
    const int r0 = bm.ch * NR;
    const uint32_t h = eo_site(hg, bm.sb, threadIdx.x);
    if (h >= hg.V) return;
    const long Vs = hg.Vs;
    const R tw = (R)a.twist;
    const R inv = (R)(1.0 / (1.0 + a.twist * a.twist));
    const R kap = (R)a.kappa;
    const EoSite c = eo_coords(hg, h, 1);
    const uint64_t* ids = a.ids + r0;
    cx<R> acc[NR][12];
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int k = 0; k < 12; k++) acc[r][k] = {(R)0, (R)0};
    src_hop_mu<0, R, G, NR>(a, ids, h, c, tw, inv, acc);
    pin_acc<R, NR>(acc);
    TM_MEM_FENCE();
    src_hop_mu<1, R, G, NR>(a, ids, h, c, tw, inv, acc);
    pin_acc<R, NR>(acc);
    TM_MEM_FENCE();
    src_hop_mu<2, R, G, NR>(a, ids, h, c, tw, inv, acc);
    pin_acc<R, NR>(acc);
    TM_MEM_FENCE();
    src_hop_mu<3, R, G, NR>(a, ids, h, c, tw, inv, acc);
    const uint32_t so = eo_full_site(h, c);
#pragma unroll
    for (int r = 0; r < NR; r++) {
        cx<R> o[12];
        noise_at<R>(a.seed_mixed, ids[r], 2 * (uint64_t)hg.V, so, o);
#pragma unroll
        for (int k = 0; k < 12; k++) o[k] = o[k] + kap * acc[r][k];
        store_spinor<So, R>(field_rhs<So>(a.out, Vs, r0 + r), Vs, h, o);
    }
}

// The whole solution in the full native layout of X (stride g.Vs): the even
// site of half index h gets D^{-1} (eta_e + kappa H_eo x_o) with eta_e from
// the hash, the odd site of the same half index gets x_o(h); a.in = x_o
template <typename R, class X, class G, int NR>
__global__ TM_STENCIL_R(NR, R) void k_eo_rec_full(EoArgs a, Geom g, void* full) {
    const Geom& hg = a.hg;
    const BlockMap bm = stencil_block((uint32_t)(a.nrhs / NR));
    const int r0 = bm.ch * NR;
    const uint32_t h = eo_site(hg, bm.sb, threadIdx.x);
    if (h >= hg.V) return;
    const long Vs = hg.Vs;
    const R tw = (R)a.twist;
    const R inv = (R)(1.0 / (1.0 + a.twist * a.twist));
    const R kap = (R)a.kappa;
    const EoSite c = eo_coords(hg, h, 0);
    const uint32_t se = eo_full_site(h, c);
    const uint32_t so = se - (uint32_t)c.x + (uint32_t)(c.x ^ 1);
    const void* in0 = field_rhs<X>(a.in, Vs, r0);
    cx<R> acc[NR][12];
    eo_hop_all<false, R, X, G, NR>(hg, a.gout, a.gin, in0, h, c, acc);
#pragma unroll
    for (int r = 0; r < NR; r++) {
        cx<R> o[12], xo[12];
        noise_at<R>(a.seed_mixed, a.ids[r0 + r], (uint64_t)(2 * hg.V), se, o);
#pragma unroll
        for (int k = 0; k < 12; k++) o[k] = o[k] + kap * acc[r][k];
        mul_diag_inv(o, tw, inv);
        load_spinor<X, R>(field_rhs<X>(in0, Vs, r), Vs, h, xo);
        void* f = field_rhs<X>(full, g.Vs, r0 + r);
        if (c.x & 1)
            store_site_pair<X, R>(f, g.Vs, so, xo, se, o);
        else
            store_site_pair<X, R>(f, g.Vs, se, o, so, xo);
    }
}

// site-local out = D^{-1} in (D of M, or of M^dag if dag)
template <typename R, class S>
__global__ __launch_bounds__(256) void k_eo_dinv(Geom hg, double twist, int nrhs, const void* in, void* out) {
    const uint32_t h = blockIdx.x * 256u + threadIdx.x;
    const int r = blockIdx.y;
    if (h >= hg.V || r >= nrhs) return;
    cx<R> v[12];
    load_spinor<S, R>(field_rhs<S>(in, hg.Vs, r), hg.Vs, h, v);
    mul_diag_inv(v, (R)twist, (R)(1.0 / (1.0 + twist * twist)));
    store_spinor<S, R>(field_rhs<S>(out, hg.Vs, r), hg.Vs, h, v);
}

// ---------------------------------------------------------------------------
// CG steps on the odd sites (a.geo is the half geometry)
// ---------------------------------------------------------------------------

// K1b: t = D p - kappa^2 H_oe y, block partials of |t|^2
template <typename R, class S, class G, int NR>
__global__ TM_STENCIL_R(NR, R) void k_eo_mp(CgArgs a, EoCg e) {
    __shared__ double sh[4];
    const Geom& hg = a.geo;
    const BlockMap bm = stencil_block((uint32_t)(a.nrhs / NR));
    const uint32_t nb = bm.nsb;
    const uint32_t h = eo_site(hg, bm.sb, threadIdx.x);
    const int r0 = bm.ch * NR;
    const long Vs = hg.Vs;
    bool act[NR];
    bool any = false;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        act[r] = a.scal[r0 + r].active != 0;
        any |= act[r];
    }
    if (!any) return;
    double part[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) part[r] = 0;
    if (h < hg.V) {
        const EoSite c = eo_coords(hg, h, 1);
        cx<R> acc[NR][12];
        eo_hop_all<false, R, S, G, NR>(hg, e.godd, e.geven, field_rhs<S>(e.y, Vs, r0), h, c, acc);
        const R tw = (R)a.twist, k2 = (R)(-a.kappa * a.kappa);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (!act[r]) continue;
            cx<R> t[12];
            load_spinor<S, R>(field_rhs<S>(a.p, Vs, r0 + r), Vs, h, t);
            mul_diag(t, tw);
#pragma unroll
            for (int k = 0; k < 12; k++) t[k] = t[k] + k2 * acc[r][k];
            round_storage<S, R>(t);
            store_spinor_cp<S, R, TM_CP_K1T>(field_rhs<S>(a.t, Vs, r0 + r), Vs, h, t);
            part[r] = spinor_norm2(t);
        }
    }
#pragma unroll
    for (int r = 0; r < NR; r++) {
        double v = block_sum256(part[r], sh);
        if (threadIdx.x == 0) a.partials[(size_t)(r0 + r) * nb + bm.sb] = v;
    }
}

// K2b: q = D^dag t - kappa^2 H_oe^dag y, r -= alpha q, x += alpha p, |r|^2;
// with TRACK rho -= alpha t (rho = etahat - Mhat x) and |rho|^2; with XFREE
// no x update (the directions are kept, k_eo_xflush forms x)
template <typename R, class S, class G, class X, typename RX, int NR, bool TRACK, bool XFREE = false>
__global__ TM_STENCIL_R(NR, R) void k_eo_upd(CgArgs a, EoCg e) {
    __shared__ double sh[4];
    const Geom& hg = a.geo;
    const BlockMap bm = stencil_block((uint32_t)(a.nrhs / NR));
    const uint32_t nb = bm.nsb;
    const uint32_t h = eo_site(hg, bm.sb, threadIdx.x);
    const int r0 = bm.ch * NR;
    const long Vs = hg.Vs;
    bool act[NR];
    bool any = false;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        act[r] = a.scal[r0 + r].active != 0;
        any |= act[r];
    }
    if (!any) return;
    double prr[NR], prho[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) prr[r] = prho[r] = 0;
    if (h < hg.V) {
        const EoSite c = eo_coords(hg, h, 1);
        cx<R> acc[NR][12];
        eo_hop_all<true, R, S, G, NR>(hg, e.godd, e.geven, field_rhs<S>(e.y, Vs, r0), h, c, acc);
        const R tw = (R)(-a.twist), k2 = (R)(-a.kappa * a.kappa);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (!act[r]) continue;
            const double alpha = a.scal[r0 + r].alpha;
            cx<R> tc[12], q[12], rv[12], pv[12];
            load_spinor<S, R>(field_rhs<S>(a.t, Vs, r0 + r), Vs, h, tc);
#pragma unroll
            for (int k = 0; k < 12; k++) q[k] = tc[k];
            mul_diag(q, tw);
#pragma unroll
            for (int k = 0; k < 12; k++) q[k] = q[k] + k2 * acc[r][k];
            void* rp = field_rhs<S>(a.r, Vs, r0 + r);
            load_spinor_cp<S, R, TM_CP_K2>(rp, Vs, h, rv);
            const R al = (R)alpha;
#pragma unroll
            for (int k = 0; k < 12; k++) rv[k] = rv[k] - al * q[k];
            round_storage<S, R>(rv);
            store_spinor_cp<S, R, TM_CP_K2>(rp, Vs, h, rv);
            prr[r] = spinor_norm2(rv);
            if (!XFREE) {
                load_spinor_cp<S, R, TM_CP_K2>(field_rhs<S>(a.p, Vs, r0 + r), Vs, h, pv);
                cx<RX> xv[12];
                void* xp = field_rhs<X>(a.x, Vs, r0 + r);
                load_spinor_cp<X, RX, TM_CP_K2>(xp, Vs, h, xv);
                const RX alx = (RX)alpha;
#pragma unroll
                for (int k = 0; k < 12; k++)
                    xv[k] = {xv[k].re + alx * (RX)pv[k].re, xv[k].im + alx * (RX)pv[k].im};
                store_spinor_cp<X, RX, TM_CP_K2>(xp, Vs, h, xv);
            }
            if (TRACK) {
                cx<R> rh[12];
                void* hp = field_rhs<S>(a.rho, Vs, r0 + r);
                load_spinor_cp<S, R, TM_CP_K2>(hp, Vs, h, rh);
#pragma unroll
                for (int k = 0; k < 12; k++) rh[k] = rh[k] - al * tc[k];
                round_storage<S, R>(rh);
                store_spinor_cp<S, R, TM_CP_K2>(hp, Vs, h, rh);
                prho[r] = spinor_norm2(rh);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < NR; r++) {
        double v = block_sum256(prr[r], sh);
        if (threadIdx.x == 0) a.partials[(size_t)(r0 + r) * nb + bm.sb] = v;
        if (TRACK) {
            double w = block_sum256(prho[r], sh);
            if (threadIdx.x == 0) a.partials2[(size_t)(r0 + r) * nb + bm.sb] = w;
        }
    }
}

// x += sum over iterations k0 <= k < min(k1, iterations done) of alpha_k p_k,
// p_k in slot k % ring of dirs (FP32 x, directions of storage S); the first
// pass (k0 = 0) writes x = the sum (x is not initialised before).  The
// result goes to out as XO (the last pass may hand x over in FP16).
template <class S, class XO>
__global__ __launch_bounds__(256) void k_eo_xflush(CgArgs a, const void* dirs, size_t slot_bytes, int k0, int k1,
                                                   void* out) {
    const uint32_t h = blockIdx.x * 256u + threadIdx.x;
    const int r = blockIdx.y;
    if (h >= a.geo.V) return;
    const int kend = min(k1, (int)a.scal[r].iters);
    if (kend <= k0 && k0 > 0 && out == a.x) return;  // (nothing to add in place)
    const long Vs = a.geo.Vs;
    cx<float> xv[12];
    void* xp = field_rhs<SF32>(a.x, Vs, r);
    if (k0 > 0) {
        load_spinor_cp<SF32, float, kStream>(xp, Vs, h, xv);
    } else {
#pragma unroll
        for (int c = 0; c < 12; c++) xv[c] = {0.f, 0.f};
    }
    for (int k = k0; k < kend; k++) {
        const float al = (float)a.ahist[(size_t)r * a.ring + (k % a.ring)];
        const void* pk = field_rhs<S>((const char*)dirs + (size_t)(k % a.ring) * slot_bytes, Vs, r);
        cx<float> pv[12];
        load_spinor_cp<S, float, kStream>(pk, Vs, h, pv);
#pragma unroll
        for (int c = 0; c < 12; c++) xv[c] = {xv[c].re + al * pv[c].re, xv[c].im + al * pv[c].im};
    }
    store_spinor_cp<XO, float, kStream>(field_rhs<XO>(out, Vs, r), Vs, h, xv);
}

// Reliable update (gated, FP64): r64 = b64 - (D^dag t64 - kappa^2 H_oe^dag
// y64) with t64 = Mhat x64 and y64 = D^{-dag} H_eo^dag t64, r32 = r64, block
// partials of |r64|^2 and (a.eta64 = etahat set) of |etahat - t64|^2; NR
// sources per lane, a chunk runs if any of its sources has the flag; r is
// stored as S (the iteration's storage)
template <int NR, class S>
__global__ TM_STENCIL_R(NR, double) void k_eo_rel_resid(CgArgs a, EoCg e, const void* b64, const void* t64,
                                                       const void* y64) {
    __shared__ double sh[4];
    const int r0 = blockIdx.y * NR;
    bool flag[NR];
    bool any = false;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        flag[r] = a.scal[r0 + r].rflag != 0;
        any |= flag[r];
    }
    if (!any) return;
    const Geom& hg = a.geo;
    const long Vs = hg.Vs;
    const uint32_t nsb = (uint32_t)((hg.V + 255) / 256);
    double pr[NR], pt[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) pr[r] = pt[r] = 0;
    const double k2 = -a.kappa * a.kappa;
    for (uint32_t sb = blockIdx.x; sb < nsb; sb += gridDim.x) {
        const uint32_t h = eo_site(hg, sb, threadIdx.x);
        if (h >= hg.V) continue;
        const EoSite c = eo_coords(hg, h, 1);
        cx<double> acc[NR][12];
        eo_hop_all<true, double, SF64, GF64, NR>(hg, e.godd, e.geven, field_rhs<SF64>(y64, Vs, r0), h, c, acc);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (!flag[r]) continue;
            cx<double> tc[12], q[12], bv[12];
            load_spinor<SF64, double>(field_rhs<SF64>(t64, Vs, r0 + r), Vs, h, tc);
#pragma unroll
            for (int k = 0; k < 12; k++) q[k] = tc[k];
            mul_diag(q, -a.twist);
            load_spinor<SF64, double>(field_rhs<SF64>(b64, Vs, r0 + r), Vs, h, bv);
            cx<float> rf[12];
            const double isg = 1.0 / a.scal[r0 + r].sigma_next;  // (a power of two)
#pragma unroll
            for (int k = 0; k < 12; k++) {
                bv[k] = bv[k] - (q[k] + k2 * acc[r][k]);
                rf[k] = {(float)(isg * bv[k].re), (float)(isg * bv[k].im)};
            }
            store_spinor<S, float>(field_rhs<S>(a.r, Vs, r0 + r), Vs, h, rf);
            pr[r] += spinor_norm2(bv);
            if (a.eta64) {
                cx<double> ev[12];
                load_spinor<SF64, double>(field_rhs<SF64>(a.eta64, Vs, r0 + r), Vs, h, ev);
#pragma unroll
                for (int k = 0; k < 12; k++) ev[k] = ev[k] - tc[k];
                pt[r] += spinor_norm2(ev);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < NR; r++) {
        double v = block_sum256(pr[r], sh);
        if (threadIdx.x == 0) a.partials[(size_t)(r0 + r) * gridDim.x + blockIdx.x] = v;
        if (a.eta64) {
            double w = block_sum256(pt[r], sh);
            if (threadIdx.x == 0) a.partials2[(size_t)(r0 + r) * gridDim.x + blockIdx.x] = w;
        }
    }
}

// ---------------------------------------------------------------------------
// layout: full native planes <-> the two half layouts (np planes per field
// block, e.g. S::NV * nrhs for spinors, 12 or 36 for the links).  A block of
// many right-hand sides spans more than the 4 GiB that a 32-bit buffer
// offset reaches, so every plane gets its own 64-bit base.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_eo_split(Geom g, Geom hg, const void* in, int np, void* out_e, void* out_o) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= g.V) return;
    const Site c = site_coords(g, s);
    const int par = (c.x + c.y + c.z + c.t) & 1;
    const uint32_t h = s >> 1;  // (row * Lx + x) / 2 = row * Lx/2 + x/2 (Lx even)
    char* out = (char*)(par ? out_o : out_e);
    for (int k = blockIdx.y; k < np; k += gridDim.y) {
        const uint4 v = ld_plane<uint4>((const char*)in + (size_t)k * g.Vs * 16, g.Vs, 0, s);
        st_plane<uint4>(out + (size_t)k * hg.Vs * 16, hg.Vs, 0, h, v);
    }
}

__global__ __launch_bounds__(256) void k_eo_merge(Geom g, Geom hg, const void* in_e, const void* in_o, int np,
                                                  void* out) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= g.V) return;
    const Site c = site_coords(g, s);
    const int par = (c.x + c.y + c.z + c.t) & 1;
    const uint32_t h = s >> 1;
    const char* in = (const char*)(par ? in_o : in_e);
    for (int k = blockIdx.y; k < np; k += gridDim.y) {
        const uint4 v = ld_plane<uint4>(in + (size_t)k * hg.Vs * 16, hg.Vs, 0, h);
        st_plane<uint4>((char*)out + (size_t)k * g.Vs * 16, g.Vs, 0, s, v);
    }
}

// FP16 links of one parity from its FP64 links ([mu][9][Vs] double2 ->
// [mu][3][Vs] uint4 of (re, im) binary16 pairs, entry 8 then padding)
__global__ __launch_bounds__(256) void k_eo_links_h16(Geom hg, const void* g64, void* g16) {
    const uint32_t h = blockIdx.x * 256u + threadIdx.x;
    if (h >= hg.V) return;
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
        uint32_t w[12];
#pragma unroll
        for (int k = 0; k < 9; k++) {
            const double2 v = ld_plane<double2>(g64, hg.Vs, mu * 9 + k, h);
            w[k] = pack2_f16((float)v.x, (float)v.y);
        }
        w[9] = w[10] = w[11] = 0;
#pragma unroll
        for (int q = 0; q < 3; q++)
            st_plane<uint4>(g16, hg.Vs, mu * 3 + q, h, make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]));
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline uint32_t eo_blocks(const Geom& hg) { return (uint32_t)((hg.V + 255) / 256); }
constexpr uint32_t kEoGatedBlocks = 512;


template <typename R, class So, class G>
static void eo_src_nr(hipStream_t st, const EoArgs& a, int nr) {
    const uint32_t nb = eo_blocks(a.hg);
    if (nr >= 2 && a.nrhs % 2 == 0)
        hipLaunchKernelGGL((k_eo_src<R, So, G, 2>), dim3(nb * (unsigned)(a.nrhs / 2)), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_eo_src<R, So, G, 1>), dim3(nb * (unsigned)a.nrhs), dim3(256), 0, st, a);
}

// etahat into a.out in storage prec (FP64 arithmetic and links for P_F64,
// FP32 otherwise)
void launch_eo_src(hipStream_t st, const EoArgs& a, int prec, int nr) {
    switch (prec) {
    case P_F64: eo_src_nr<double, SF64, GF64>(st, a, nr); break;
    case P_F32: eo_src_nr<float, SF32, GF32>(st, a, nr); break;
    case P_F16: eo_src_nr<float, SF16, GF32>(st, a, nr); break;
    default: eo_src_nr<float, SBF16, GF32>(st, a, nr); break;
    }
}

// xprec: P_F64 (FP64 odd half and output) or P_F32
void launch_eo_rec_full(hipStream_t st, const EoArgs& a, int xprec, int nr, const Geom& g, void* full) {
    const uint32_t nb = eo_blocks(a.hg);
    if (xprec == P_F64) {
        if (nr >= 2)
            hipLaunchKernelGGL((k_eo_rec_full<double, SF64, GF64, 2>), dim3(nb * (unsigned)(a.nrhs / 2)), dim3(256), 0,
                               st, a, g, full);
        else
            hipLaunchKernelGGL((k_eo_rec_full<double, SF64, GF64, 1>), dim3(nb * (unsigned)a.nrhs), dim3(256), 0, st,
                               a, g, full);
        return;
    }
    switch (nr) {
    case 4:
        hipLaunchKernelGGL((k_eo_rec_full<float, SF32, GF32, 4>), dim3(nb * (unsigned)(a.nrhs / 4)), dim3(256), 0, st,
                           a, g, full);
        break;
    case 2:
        hipLaunchKernelGGL((k_eo_rec_full<float, SF32, GF32, 2>), dim3(nb * (unsigned)(a.nrhs / 2)), dim3(256), 0, st,
                           a, g, full);
        break;
    default:
        hipLaunchKernelGGL((k_eo_rec_full<float, SF32, GF32, 1>), dim3(nb * (unsigned)a.nrhs), dim3(256), 0, st, a, g,
                           full);
        break;
    }
}

void launch_eo_links_h16(hipStream_t st, const Geom& hg, const void* g64, void* g16) {
    hipLaunchKernelGGL(k_eo_links_h16, dim3(eo_blocks(hg)), dim3(256), 0, st, hg, g64, g16);
}
void launch_eo_split(hipStream_t st, const Geom& g, const Geom& hg, const void* in, int np, void* out_e,
                     void* out_o) {
    const unsigned gy = (unsigned)std::min(np, 64);
    hipLaunchKernelGGL(k_eo_split, dim3((unsigned)((g.V + 255) / 256), gy), dim3(256), 0, st, g, hg, in, np, out_e,
                       out_o);
}
void launch_eo_merge(hipStream_t st, const Geom& g, const Geom& hg, const void* in_e, const void* in_o, int np,
                     void* out) {
    const unsigned gy = (unsigned)std::min(np, 64);
    hipLaunchKernelGGL(k_eo_merge, dim3((unsigned)((g.V + 255) / 256), gy), dim3(256), 0, st, g, hg, in_e, in_o, np,
                       out);
}

void launch_eo_dinv(hipStream_t st, const Geom& hg, int prec, double twist, int nrhs, const void* in, void* out) {
    const dim3 grid(eo_blocks(hg), (unsigned)nrhs);
    switch (prec) {
    case P_F64: hipLaunchKernelGGL((k_eo_dinv<double, SF64>), grid, dim3(256), 0, st, hg, twist, nrhs, in, out); break;
    case P_F32: hipLaunchKernelGGL((k_eo_dinv<float, SF32>), grid, dim3(256), 0, st, hg, twist, nrhs, in, out); break;
    case P_F16: hipLaunchKernelGGL((k_eo_dinv<float, SF16>), grid, dim3(256), 0, st, hg, twist, nrhs, in, out); break;
    default: hipLaunchKernelGGL((k_eo_dinv<float, SBF16>), grid, dim3(256), 0, st, hg, twist, nrhs, in, out); break;
    }
}

template <bool DAG, bool PRE, bool POST, typename R, class Si, class So, class G>
static void eo_lin_nr(hipStream_t st, const EoArgs& a, int nr) {
    const uint32_t nb = eo_blocks(a.hg);
    if constexpr (sizeof(R) == 8) nr = std::min(nr, 2);
    if (a.gate != nullptr) {
        const unsigned gb = std::min(nb, kEoGatedBlocks);
        if (nr == 2)
            hipLaunchKernelGGL((k_eo_lin<DAG, PRE, POST, R, Si, So, G, 2>), dim3(gb * (unsigned)(a.nrhs / 2)),
                               dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_eo_lin<DAG, PRE, POST, R, Si, So, G, 1>), dim3(gb * (unsigned)a.nrhs), dim3(256),
                               0, st, a);
        return;
    }
    switch (nr) {
    case 4:
        hipLaunchKernelGGL((k_eo_lin<DAG, PRE, POST, R, Si, So, G, 4>), dim3(nb * (unsigned)(a.nrhs / 4)), dim3(256),
                           0, st, a);
        break;
    case 2:
        hipLaunchKernelGGL((k_eo_lin<DAG, PRE, POST, R, Si, So, G, 2>), dim3(nb * (unsigned)(a.nrhs / 2)), dim3(256),
                           0, st, a);
        break;
    default:
        hipLaunchKernelGGL((k_eo_lin<DAG, PRE, POST, R, Si, So, G, 1>), dim3(nb * (unsigned)a.nrhs), dim3(256), 0, st,
                           a);
        break;
    }
}

template <bool DAG, bool PRE, bool POST>
static void eo_lin_prec(hipStream_t st, const EoArgs& a, int prec, int nr) {
    switch (prec) {
    case P_F64: eo_lin_nr<DAG, PRE, POST, double, SF64, SF64, GF64>(st, a, nr); break;  // (at most 2)
    case P_F32: eo_lin_nr<DAG, PRE, POST, float, SF32, SF32, GF32>(st, a, nr); break;
    case P_F16: eo_lin_nr<DAG, PRE, POST, float, SF16, SF16, GH16>(st, a, nr); break;
    default: eo_lin_nr<DAG, PRE, POST, float, SBF16, SBF16, GF32>(st, a, nr); break;
    }
}

void launch_eo_lin(hipStream_t st, const EoArgs& a, int prec, int nr, int kind) {
    switch (kind) {
    case EO_Y: eo_lin_prec<false, false, true>(st, a, prec, nr); break;
    case EO_Y_DAG: eo_lin_prec<true, false, true>(st, a, prec, nr); break;
    case EO_T: eo_lin_prec<false, true, false>(st, a, prec, nr); break;
    case EO_T_DAG: eo_lin_prec<true, true, false>(st, a, prec, nr); break;
    case EO_SRC: eo_lin_prec<false, false, false>(st, a, prec, nr); break;
    default: eo_lin_prec<false, false, true>(st, a, prec, nr); break;  // EO_REC
    }
}

// reconstruction with an FP32 odd half (FP32 output); FP64 runs through launch_eo_lin
void launch_eo_rec_f32(hipStream_t st, const EoArgs& a, int nr) {
    eo_lin_nr<false, false, true, float, SF32, SF32, GF32>(st, a, nr);
}

template <typename R, class S, class G>
static void eo_mp_typed(hipStream_t st, const CgArgs& a, const EoCg& e, int nr) {
    const uint32_t nb = eo_blocks(a.geo);
    if constexpr (sizeof(R) == 8) nr = 1;
    switch (nr) {
    case 4: hipLaunchKernelGGL((k_eo_mp<R, S, G, 4>), dim3(nb * (unsigned)(a.nrhs / 4)), dim3(256), 0, st, a, e); break;
    case 2: hipLaunchKernelGGL((k_eo_mp<R, S, G, 2>), dim3(nb * (unsigned)(a.nrhs / 2)), dim3(256), 0, st, a, e); break;
    default: hipLaunchKernelGGL((k_eo_mp<R, S, G, 1>), dim3(nb * (unsigned)a.nrhs), dim3(256), 0, st, a, e); break;
    }
}

template <typename R, class S, class G, class X, typename RX>
static void eo_upd_typed(hipStream_t st, const CgArgs& a, const EoCg& e, int nr, bool track) {
    const uint32_t nb = eo_blocks(a.geo);
    if (track) {
        hipLaunchKernelGGL((k_eo_upd<R, S, G, X, RX, 1, true>), dim3(nb * (unsigned)a.nrhs), dim3(256), 0, st, a, e);
        return;
    }
    if constexpr (sizeof(R) == 8) nr = 1;
    switch (nr) {
    case 4:
        hipLaunchKernelGGL((k_eo_upd<R, S, G, X, RX, 4, false>), dim3(nb * (unsigned)(a.nrhs / 4)), dim3(256), 0, st,
                           a, e);
        break;
    case 2:
        hipLaunchKernelGGL((k_eo_upd<R, S, G, X, RX, 2, false>), dim3(nb * (unsigned)(a.nrhs / 2)), dim3(256), 0, st,
                           a, e);
        break;
    default:
        hipLaunchKernelGGL((k_eo_upd<R, S, G, X, RX, 1, false>), dim3(nb * (unsigned)a.nrhs), dim3(256), 0, st, a, e);
        break;
    }
}

template <typename R, class S, class G>
static void eo_upd_xfree_typed(hipStream_t st, const CgArgs& a, const EoCg& e, int nr, bool track) {
    const uint32_t nb = eo_blocks(a.geo);
    if (track) {
        hipLaunchKernelGGL((k_eo_upd<R, S, G, SF32, float, 1, true, true>), dim3(nb * (unsigned)a.nrhs), dim3(256), 0,
                           st, a, e);
        return;
    }
    switch (nr) {
    case 4:
        hipLaunchKernelGGL((k_eo_upd<R, S, G, SF32, float, 4, false, true>), dim3(nb * (unsigned)(a.nrhs / 4)),
                           dim3(256), 0, st, a, e);
        break;
    case 2:
        hipLaunchKernelGGL((k_eo_upd<R, S, G, SF32, float, 2, false, true>), dim3(nb * (unsigned)(a.nrhs / 2)),
                           dim3(256), 0, st, a, e);
        break;
    default:
        hipLaunchKernelGGL((k_eo_upd<R, S, G, SF32, float, 1, false, true>), dim3(nb * (unsigned)a.nrhs), dim3(256),
                           0, st, a, e);
        break;
    }
}

void launch_eo_upd_xfree(hipStream_t st, const CgArgs& a, const EoCg& e, int prec, int nr, bool track) {
    switch (prec) {
    case P_F32: eo_upd_xfree_typed<float, SF32, GF32>(st, a, e, nr, track); break;
    case P_F16: eo_upd_xfree_typed<float, SF16, GH16>(st, a, e, nr, track); break;
    default: eo_upd_xfree_typed<float, SBF16, GF32>(st, a, e, nr, track); break;
    }
}

template <class XO>
static void eo_xflush_out(hipStream_t st, const CgArgs& a, int prec, const void* dirs, size_t slot_bytes, int k0,
                          int k1, void* out) {
    const dim3 grid(eo_blocks(a.geo), (unsigned)a.nrhs);
    switch (prec) {
    case P_F32:
        hipLaunchKernelGGL((k_eo_xflush<SF32, XO>), grid, dim3(256), 0, st, a, dirs, slot_bytes, k0, k1, out);
        break;
    case P_F16:
        hipLaunchKernelGGL((k_eo_xflush<SF16, XO>), grid, dim3(256), 0, st, a, dirs, slot_bytes, k0, k1, out);
        break;
    default:
        hipLaunchKernelGGL((k_eo_xflush<SBF16, XO>), grid, dim3(256), 0, st, a, dirs, slot_bytes, k0, k1, out);
        break;
    }
}

void launch_eo_xflush(hipStream_t st, const CgArgs& a, int prec, const void* dirs, size_t slot_bytes, int k0, int k1,
                      void* out, int out_prec) {
    if (out == nullptr) out = a.x;
    if (out_prec == P_F16)
        eo_xflush_out<SF16>(st, a, prec, dirs, slot_bytes, k0, k1, out);
    else
        eo_xflush_out<SF32>(st, a, prec, dirs, slot_bytes, k0, k1, out);
}

void launch_eo_mp(hipStream_t st, const CgArgs& a, const EoCg& e, int prec, int nr) {
    switch (prec) {
    case P_F64: eo_mp_typed<double, SF64, GF64>(st, a, e, 1); break;
    case P_F32: eo_mp_typed<float, SF32, GF32>(st, a, e, nr); break;
    case P_F16: eo_mp_typed<float, SF16, GH16>(st, a, e, nr); break;
    default: eo_mp_typed<float, SBF16, GF32>(st, a, e, nr); break;
    }
}

void launch_eo_upd(hipStream_t st, const CgArgs& a, const EoCg& e, int prec, int nr, bool track) {
    switch (prec) {
    case P_F64: eo_upd_typed<double, SF64, GF64, SF64, double>(st, a, e, 1, track); break;
    case P_F32: eo_upd_typed<float, SF32, GF32, SF32, float>(st, a, e, nr, track); break;
    case P_F16: eo_upd_typed<float, SF16, GH16, SF32, float>(st, a, e, nr, track); break;
    default: eo_upd_typed<float, SBF16, GF32, SF32, float>(st, a, e, nr, track); break;
    }
}

uint32_t eo_gated_blocks(const Geom& hg) { return std::min(eo_blocks(hg), kEoGatedBlocks); }

template <class S>
static void eo_rel_resid_typed(hipStream_t st, const CgArgs& a, const EoCg& e, const void* b64, const void* t64,
                               const void* y64, int nr) {
    const uint32_t nb = eo_gated_blocks(a.geo);
    if (nr == 2)
        hipLaunchKernelGGL((k_eo_rel_resid<2, S>), dim3(nb, (unsigned)(a.nrhs / 2)), dim3(256), 0, st, a, e, b64, t64,
                           y64);
    else
        hipLaunchKernelGGL((k_eo_rel_resid<1, S>), dim3(nb, (unsigned)a.nrhs), dim3(256), 0, st, a, e, b64, t64, y64);
}

void launch_eo_rel_resid(hipStream_t st, const CgArgs& a, const EoCg& e, const void* b64, const void* t64,
                         const void* y64, int nr, int prec) {
    switch (prec) {
    case P_F16: eo_rel_resid_typed<SF16>(st, a, e, b64, t64, y64, nr); break;
    case P_BF16: eo_rel_resid_typed<SBF16>(st, a, e, b64, t64, y64, nr); break;
    default: eo_rel_resid_typed<SF32>(st, a, e, b64, t64, y64, nr); break;
    }
}

}  // namespace tmq
