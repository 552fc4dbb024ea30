// Twisted-mass Wilson-Dirac operator and the fused CG kernels (gfx950).
//
// M = 1 - kappa H + 2 i kappa mu gamma_5 in the hopping normalisation, with
// H psi(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^dag
// psi(x-mu) and the adjoint H^dag obtained by swapping the two projectors.
// (Flavour identities of section 2.3 of the paper; the twisted mass bounds
// M^dag M from below, section 2.2.)
//
// One lane per lattice site and NR right-hand sides: every link is loaded
// once per lane and applied to NR spinors.  Spin projection to two-spinor
// halves (the chiral basis makes every projector a signed permutation), so a
// hop costs two SU(3) matrix-vector products.  Sites are dealt to blocks of
// 256 with an XCD-aware block order.
//
// The CG iteration on M^dag M is five launches per step:
//   K1  t = M p,                               block partials of |t|^2
//   R1  alpha = |r|^2/|t|^2                    (one block per right-hand side)
//   K2  q = M^dag t,  r -= alpha q,  x += alpha p,  block partials of |r|^2
//   R2  beta, stop test                        (one block per right-hand side)
//   K3  p = r + beta p
// with the scalars of every right-hand side kept on the device.  The
// reductions are separate launches because a last-block-finalises pattern
// needs a device-scope release per block, which on a multi-XCD part writes
// back the XCD's L2 and costs more than the stencil itself.

#include "tm_device.h"
#include "tm_kernels.h"
#include "tm_stencil.h"

namespace tmq {



// ---------------------------------------------------------------------------
// plain application: out = op(in), op 0 = M, 1 = M^dag, 3 = H
// gate (nullable): apply only to right-hand sides whose reliable flag is set
// ---------------------------------------------------------------------------
template <int OP, typename R, class Si, class So, class G, int NR>
__global__ TM_STENCIL_R(NR, R) void k_apply(Geom geo, const void* gauge, R kappa, R twist, int nrhs,
                                               const void* in, void* out, const CgScal* gate) {
    const BlockMap bm = stencil_block((uint32_t)(nrhs / NR));
    const int r0 = bm.ch * NR;
    if (gate != nullptr && !gate[r0].rflag) return;  // gated launches use NR = 1
    const void* in0 = field_rhs<Si>(in, geo.Vs, r0);
    // gated launches use a small grid that strides over the site blocks
    const uint32_t nsb_all = (uint32_t)((geo.V + 255) / 256);
    for (uint32_t sb = bm.sb; sb < nsb_all; sb += bm.nsb) {
        const uint32_t s = sb * 256u + threadIdx.x;
        if (s >= geo.V) continue;
        const Site c = site_coords(geo, s);
        cx<R> acc[NR][12];
        hop_all<OP == 1, R, Si, G, NR>(geo, gauge, in0, s, c, acc);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<R> o[12];
            if (OP == 3) {
#pragma unroll
                for (int k = 0; k < 12; k++) o[k] = acc[r][k];
            } else {
                cx<R> pc[12];
                load_spinor<Si, R>(field_rhs<Si>(in0, geo.Vs, r), geo.Vs, s, pc);
                diag_combine(pc, acc[r], kappa, OP == 0 ? twist : -twist, o);
            }
            store_spinor<So, R>(field_rhs<So>(out, geo.Vs, r0 + r), geo.Vs, s, o);
        }
    }
}

// ---------------------------------------------------------------------------
// CG kernels
// ---------------------------------------------------------------------------

// End of one CG step for one right-hand side (single thread).
__device__ inline void cg_finish_step(CgScal& q, double rrn, double rhon) {
    q.iters += 1;
    if (!(rrn == rrn) || !(q.alpha == q.alpha) || rrn > 1e300) {  // NaN or overflow: breakdown
        q.status = 3;
        q.active = 0;
        q.rflag = 0;
        return;
    }
    if (q.stop == 1 && !q.reliable) q.rho2 = rhon;
    if (q.reliable) {
        if (rrn > q.maxrr) q.maxrr = rrn;
        if (rrn * q.sigma * q.sigma <= q.tol2 * q.bb || rrn < q.delta2 * q.maxrr) {
            q.rflag = 1;  // the reliable-update kernels finish this step
            // the recomputed residual is stored at the source's scale
            const double s = (rrn > 0 && q.bb > 0) ? q.sigma * sqrt(rrn / q.bb) : q.sigma;
            q.sigma_next = (s > 0 && s < 1e300) ? exp2(rint(log2(s))) : q.sigma;
            return;
        }
        q.beta = rrn / q.rr;
        q.rr = rrn;
        if (q.maxit >= 0 && q.iters >= q.maxit) {
            q.status = 2;
            q.active = 0;
        }
        return;
    }
    q.beta = rrn / q.rr;
    q.rr = rrn;
    const double rel2 = (q.stop == 1) ? q.rho2 / q.ee : rrn / q.bb;
    if (rel2 <= q.tol2) {
        q.status = 1;
        q.active = 0;
    } else if (q.maxit >= 0 && q.iters >= q.maxit) {
        q.status = 2;
        q.active = 0;
    }
}

// K1: t = M p and alpha
template <typename R, class S, class G, int NR>
__global__ TM_STENCIL_R(NR, R) void k_cg_mp(CgArgs a) {
    __shared__ double sh[4];
    const BlockMap bm = stencil_block((uint32_t)(a.nrhs / NR));
    const uint32_t nb = bm.nsb;
    const uint32_t s = bm.sb * 256u + threadIdx.x;
    const int r0 = bm.ch * NR;
    const long Vs = a.geo.Vs;
    bool act[NR];
    bool any = false;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        act[r] = a.scal[r0 + r].active != 0;
        any |= act[r];
    }
    if (!any) return;  // uniform over all blocks of this rhs chunk
    double part[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) part[r] = 0;
    if (s < a.geo.V) {
        const Site c = site_coords(a.geo, s);
        const void* p0 = field_rhs<S>(a.p, Vs, r0);
        cx<R> acc[NR][12];
        hop_all<false, R, S, G, NR>(a.geo, a.gauge, p0, s, c, acc);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (!act[r]) continue;
            cx<R> pc[12], t[12];
            load_spinor<S, R>(field_rhs<S>(p0, Vs, r), Vs, s, pc);
            diag_combine(pc, acc[r], (R)a.kappa, (R)a.twist, t);
            round_storage<S, R>(t);
            store_spinor_cp<S, R, TM_CP_K1T>(field_rhs<S>(a.t, Vs, r0 + r), Vs, s, t);
            part[r] = spinor_norm2(t);
        }
    }
#pragma unroll
    for (int r = 0; r < NR; r++) {
        double v = block_sum256(part[r], sh);
        if (threadIdx.x == 0) a.partials[(size_t)(r0 + r) * nb + bm.sb] = v;
    }
}

// Block partials of one right-hand side in a fixed order (the stencil
// launch that wrote them has completed); valid in thread 0.
__device__ __forceinline__ double sum_block_partials(const double* p, uint32_t n, double* sh) {
    double v = 0;
    for (uint32_t i = threadIdx.x; i < n; i += 256) v += p[i];
    return block_sum256(v, sh);
}

// after K1, one block per right-hand side: alpha = |r|^2 / |t|^2
__global__ __launch_bounds__(256) void k_cg_alpha(CgArgs a, uint32_t nb) {
    __shared__ double sh[4];
    const int r = blockIdx.x;
    if (!a.scal[r].active) return;
    const double tt = sum_block_partials(a.partials + (size_t)r * nb, nb, sh);
    if (threadIdx.x == 0) {
        CgScal& q = a.scal[r];
        q.tt = tt;
        q.alpha = tt > 0 ? q.rr / tt : 0.0;
        if (a.ahist) a.ahist[(size_t)r * a.ring + (q.iters % a.ring)] = q.alpha;
    }
}

// after K2, one block per right-hand side: |r|^2 (and |rho|^2), beta and the
// stop test
template <bool TRACK>
__global__ __launch_bounds__(256) void k_cg_beta(CgArgs a, uint32_t nb) {
    __shared__ double sh[4];
    const int r = blockIdx.x;
    if (!a.scal[r].active) return;
    const double rrn = sum_block_partials(a.partials + (size_t)r * nb, nb, sh);
    const double rhon = TRACK ? sum_block_partials(a.partials2 + (size_t)r * nb, nb, sh) : 0.0;
    if (threadIdx.x == 0) cg_finish_step(a.scal[r], rrn, rhon);
}

// K2: q = M^dag t, r -= alpha q, x += alpha p (x of storage X), |r|^2,
// optionally rho -= alpha t (recursive true residual)
template <typename R, class S, class G, class X, typename RX, int NR, bool TRACK>
__global__ TM_STENCIL_R(NR, R) void k_cg_upd(CgArgs a) {
    __shared__ double sh[4];
    const BlockMap bm = stencil_block((uint32_t)(a.nrhs / NR));
    const uint32_t nb = bm.nsb;
    const uint32_t s = bm.sb * 256u + threadIdx.x;
    const int r0 = bm.ch * NR;
    const long Vs = a.geo.Vs;
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
    if (s < a.geo.V) {
        const Site c = site_coords(a.geo, s);
        const void* t0 = field_rhs<S>(a.t, Vs, r0);
        cx<R> acc[NR][12];
        hop_all<true, R, S, G, NR>(a.geo, a.gauge, t0, s, c, acc);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (!act[r]) continue;
            const double alpha = a.scal[r0 + r].alpha;
            cx<R> tc[12], q[12], rv[12], pv[12];
            load_spinor<S, R>(field_rhs<S>(t0, Vs, r), Vs, s, tc);
            diag_combine(tc, acc[r], (R)a.kappa, (R)(-a.twist), q);
            void* rp = field_rhs<S>(a.r, Vs, r0 + r);
            load_spinor_cp<S, R, TM_CP_K2>(rp, Vs, s, rv);
            const R al = (R)alpha;
#pragma unroll
            for (int k = 0; k < 12; k++) rv[k] = rv[k] - al * q[k];
            round_storage<S, R>(rv);
            store_spinor_cp<S, R, TM_CP_K2>(rp, Vs, s, rv);
            prr[r] = spinor_norm2(rv);
            load_spinor_cp<S, R, TM_CP_K2>(field_rhs<S>(a.p, Vs, r0 + r), Vs, s, pv);
            cx<RX> xv[12];
            void* xp = field_rhs<X>(a.x, Vs, r0 + r);
            load_spinor_cp<X, RX, TM_CP_K2>(xp, Vs, s, xv);
            const RX alx = (RX)alpha;
#pragma unroll
            for (int k = 0; k < 12; k++) xv[k] = {xv[k].re + alx * (RX)pv[k].re, xv[k].im + alx * (RX)pv[k].im};
            store_spinor_cp<X, RX, TM_CP_K2>(xp, Vs, s, xv);
            if (TRACK) {
                cx<R> rh[12];
                void* hp = field_rhs<S>(a.rho, Vs, r0 + r);
                load_spinor_cp<S, R, TM_CP_K2>(hp, Vs, s, rh);
#pragma unroll
                for (int k = 0; k < 12; k++) rh[k] = rh[k] - al * tc[k];
                round_storage<S, R>(rh);
                store_spinor_cp<S, R, TM_CP_K2>(hp, Vs, s, rh);
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

// K3: p = r + beta p (one lane per site and right-hand side)
template <typename R, class S>
__global__ __launch_bounds__(256) void k_cg_p(CgArgs a) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= a.geo.V) return;
    const CgScal& q = a.scal[r];
    if (!q.active) return;
    const R beta = (R)q.beta;
    cx<R> rv[12], pv[12];
    load_spinor_cp<S, R, TM_CP_K3>(field_rhs<S>(a.r, a.geo.Vs, r), a.geo.Vs, s, rv);
    void* pp = field_rhs<S>(a.p, a.geo.Vs, r);
    load_spinor_cp<S, R, TM_CP_K3>(pp, a.geo.Vs, s, pv);
#pragma unroll
    for (int k = 0; k < 12; k++) pv[k] = rv[k] + beta * pv[k];
    store_spinor<S, R>(a.pn ? field_rhs<S>(a.pn, a.geo.Vs, r) : pp, a.geo.Vs, s, pv);
}

// Initialisation: r holds b = M^dag eta.  p = r, x = 0, (rho = eta), block
// partials of |b|^2 and, if eta is given, of |eta|^2 (k_cg_init_fin
// finishes).
template <typename R, class S, class X, typename RX, bool TRACK>
__global__ __launch_bounds__(256) void k_cg_init(CgArgs a, const void* eta) {
    __shared__ double sh[4];
    const uint32_t nb = gridDim.x;
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    const int r = blockIdx.y;
    const long Vs = a.geo.Vs;
    double pb = 0, pe = 0;
    if (s < a.geo.V) {
        cx<R> rv[12], ev[12];
        load_spinor<S, R>(field_rhs<S>(a.r, Vs, r), Vs, s, rv);
        store_spinor<S, R>(field_rhs<S>(a.p, Vs, r), Vs, s, rv);
        if (a.x) {  // (a solve that forms x from kept directions passes none)
            cx<RX> z[12];
#pragma unroll
            for (int k = 0; k < 12; k++) z[k] = {(RX)0, (RX)0};
            store_spinor<X, RX>(field_rhs<X>(a.x, Vs, r), Vs, s, z);
        }
        pb = spinor_norm2(rv);
        if (eta) {  // (none when |eta|^2 is known and nothing is tracked)
            load_spinor<S, R>(field_rhs<S>(eta, Vs, r), Vs, s, ev);
            pe = spinor_norm2(ev);
            if (TRACK) store_spinor<S, R>(field_rhs<S>(a.rho, Vs, r), Vs, s, ev);
        }
    }
    double v = block_sum256(pb, sh);
    if (threadIdx.x == 0) a.partials[(size_t)r * nb + blockIdx.x] = v;
    double w = block_sum256(pe, sh);
    if (threadIdx.x == 0) a.partials2[(size_t)r * nb + blockIdx.x] = w;
}

// Per-source state at the start of CG given |b|^2 and |eta|^2.
__device__ inline void cg_start(CgScal& q, double bb, double ee) {
    q.bb = q.rr = q.maxrr = bb;
    q.ee = q.rho2 = ee;
    q.sigma = q.sigma_next = 1.0;
    q.iters = 0;
    q.rflag = 0;
    q.n_reliable = 0;
    q.alpha = q.beta = 0;
    if (bb <= 0 || 1.0 <= q.tol2) {
        q.status = 1;
    } else if (q.maxit == 0) {
        q.status = 2;
    } else {
        q.status = 0;
    }
    q.active = q.status == 0;
}

// one block per right-hand side; with_ee = 0: |eta|^2 = ee_z4 (12 per site
// of a Z4 source on the whole lattice)
__global__ __launch_bounds__(256) void k_cg_init_fin(CgArgs a, uint32_t nb, int with_ee, double ee_z4) {
    __shared__ double sh[4];
    const int r = blockIdx.x;
    const double bb = sum_block_partials(a.partials + (size_t)r * nb, nb, sh);
    const double ee = with_ee ? sum_block_partials(a.partials2 + (size_t)r * nb, nb, sh) : ee_z4;
    if (threadIdx.x == 0) cg_start(a.scal[r], bb, ee);
}

// ---------------------------------------------------------------------------
// reliable updates (FP32 iterations, FP64 solution and true residual)
// ---------------------------------------------------------------------------

// init: r = b64, p = r (stored as S), x32 = 0, x64 = 0, block partials of
// |b64|^2
template <class S>
__global__ __launch_bounds__(256) void k_rel_init(CgArgs a, const void* b64, void* x64) {
    __shared__ double sh[4];
    const uint32_t nb = gridDim.x;
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    const int r = blockIdx.y;
    const long Vs = a.geo.Vs;
    double pb = 0;
    if (s < a.geo.V) {
        cx<double> bv[12], z[12];
        load_spinor<SF64, double>(field_rhs<SF64>(b64, Vs, r), Vs, s, bv);
        pb = spinor_norm2(bv);
        cx<float> rf[12], zf[12];
#pragma unroll
        for (int k = 0; k < 12; k++) {
            rf[k] = {(float)bv[k].re, (float)bv[k].im};
            zf[k] = {0.f, 0.f};
            z[k] = {0.0, 0.0};
        }
        store_spinor<S, float>(field_rhs<S>(a.r, Vs, r), Vs, s, rf);
        store_spinor<S, float>(field_rhs<S>(a.p, Vs, r), Vs, s, rf);
        store_spinor<SF32, float>(field_rhs<SF32>(a.x, Vs, r), Vs, s, zf);
        store_spinor<SF64, double>(field_rhs<SF64>(x64, Vs, r), Vs, s, z);
    }
    double v = block_sum256(pb, sh);
    if (threadIdx.x == 0) a.partials[(size_t)r * nb + blockIdx.x] = v;
}

// The kernels below run every iteration but act only on sources whose
// reliable flag is set, which is rare; they use a small grid that strides
// over the site blocks, so that an idle launch costs little.
constexpr uint32_t kGatedBlocks = 512;

// x64 += x32, x32 = 0 (where the reliable flag is set, or always if force)
__global__ __launch_bounds__(256) void k_rel_flush(CgArgs a, void* x64, int force) {
    const int r = blockIdx.y;
    if (!force && !a.scal[r].rflag) return;
    const long Vs = a.geo.Vs;
    const uint32_t nsb = (uint32_t)((a.geo.V + 255) / 256);
    void* xdp = field_rhs<SF64>(x64, Vs, r);
    void* xsp = field_rhs<SF32>(a.x, Vs, r);
    const double sg = a.scal[r].sigma;
    for (uint32_t sb = blockIdx.x; sb < nsb; sb += gridDim.x) {
        const uint32_t s = sb * 256u + threadIdx.x;
        if (s >= a.geo.V) continue;
        cx<double> xd[12], xs[12];
        cx<float> z[12];
        load_spinor<SF64, double>(xdp, Vs, s, xd);
        load_spinor<SF32, double>(xsp, Vs, s, xs);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            xd[k] = xd[k] + sg * xs[k];
            z[k] = {0.f, 0.f};
        }
        store_spinor<SF64, double>(xdp, Vs, s, xd);
        store_spinor<SF32, float>(xsp, Vs, s, z);
    }
}

// r64 = b64 - M^dag t64 (t64 = M x64), r32 = r64, block partials of |r64|^2
// and, when the solve stops on the true residual (a.eta64 set), of
// |eta - t64|^2 (grid: kGatedBlocks x nrhs, striding over site blocks)
__global__ TM_STENCIL_R(1, double) void k_rel_resid(CgArgs a, const void* gauge64, const void* b64, const void* t64) {
    __shared__ double sh[4];
    const int r = blockIdx.y;
    if (!a.scal[r].rflag) return;
    const long Vs = a.geo.Vs;
    const uint32_t nsb = (uint32_t)((a.geo.V + 255) / 256);
    const void* t0 = field_rhs<SF64>(t64, Vs, r);
    double pr = 0, pt = 0;
    for (uint32_t sb = blockIdx.x; sb < nsb; sb += gridDim.x) {
        const uint32_t s = sb * 256u + threadIdx.x;
        if (s >= a.geo.V) continue;
        const Site c = site_coords(a.geo, s);
        cx<double> acc[1][12];
        hop_all<true, double, SF64, GF64, 1>(a.geo, gauge64, t0, s, c, acc);
        cx<double> tc[12], q[12], bv[12];
        load_spinor<SF64, double>(t0, Vs, s, tc);
        diag_combine(tc, acc[0], a.kappa, -a.twist, q);
        load_spinor<SF64, double>(field_rhs<SF64>(b64, Vs, r), Vs, s, bv);
        cx<float> rf[12];
        const double isg = 1.0 / a.scal[r].sigma_next;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            bv[k] = bv[k] - q[k];
            rf[k] = {(float)(isg * bv[k].re), (float)(isg * bv[k].im)};
        }
        store_spinor<SF32, float>(field_rhs<SF32>(a.r, Vs, r), Vs, s, rf);
        pr += spinor_norm2(bv);
        if (a.eta64) {
            cx<double> ev[12];
            load_spinor<SF64, double>(field_rhs<SF64>(a.eta64, Vs, r), Vs, s, ev);
#pragma unroll
            for (int k = 0; k < 12; k++) ev[k] = ev[k] - tc[k];
            pt += spinor_norm2(ev);
        }
    }
    double v = block_sum256(pr, sh);
    if (threadIdx.x == 0) a.partials[(size_t)r * gridDim.x + blockIdx.x] = v;
    if (a.eta64) {
        double w = block_sum256(pt, sh);
        if (threadIdx.x == 0) a.partials2[(size_t)r * gridDim.x + blockIdx.x] = w;
    }
}

// one block per right-hand side with the reliable flag set: restart the
// recursion from the recomputed residual, stop test on it (or on the FP64
// true residual |eta - M x| when the solve stops on that)
__global__ __launch_bounds__(256) void k_rel_fin(CgArgs a, uint32_t nb) {
    __shared__ double sh[4];
    const int r = blockIdx.x;
    if (!a.scal[r].rflag) return;
    const double rrn = sum_block_partials(a.partials + (size_t)r * nb, nb, sh);
    const double rho2 = a.eta64 ? sum_block_partials(a.partials2 + (size_t)r * nb, nb, sh) : 0.0;
    if (threadIdx.x == 0) {
        CgScal& q = a.scal[r];
        // rrn is the true |r|^2; the next p = r + beta p in the new scale
        // takes the old p times sigma / sigma_next
        const double so = q.sigma, sn = q.sigma_next;
        q.beta = rrn / (q.rr * so * so) * (so / sn);
        q.rr = rrn / (sn * sn);
        q.maxrr = q.rr;
        q.sigma = sn;
        q.rflag = 0;
        q.n_reliable += 1;
        if (q.stop == 1) q.rho2 = rho2;
        if (q.stop == 1 ? rho2 <= q.tol2 * q.ee : rrn <= q.tol2 * q.bb) {
            q.status = 1;
            q.active = 0;
        } else if (q.maxit >= 0 && q.iters >= q.maxit) {
            q.status = 2;
            q.active = 0;
        }
    }
}

// FP64 true residual |eta - M x| / |eta| with eta regenerated from the hash:
// block partials of |eta - M x|^2 and |eta|^2 (k_true_resid_fin finishes)
template <class X, typename RXin>
__global__ TM_STENCIL_R(1, double) void k_true_resid(CgArgs a, const void* gauge64, uint64_t seed_mixed,
                                                    const uint64_t* ids) {
    __shared__ double sh[4];
    const BlockMap bm = stencil_block((uint32_t)a.nrhs);
    const uint32_t nb = bm.nsb;
    const uint32_t s = bm.sb * 256u + threadIdx.x;
    const int r = bm.ch;
    const long Vs = a.geo.Vs;
    double pr = 0, pe = 0;
    if (s < a.geo.V) {
        const Site c = site_coords(a.geo, s);
        const void* x0 = field_rhs<X>(a.x, Vs, r);
        cx<double> acc[1][12];
        hop_all<false, double, X, GF64, 1>(a.geo, gauge64, x0, s, c, acc);
        cx<double> xc[12], mx[12];
        load_spinor<X, double>(x0, Vs, s, xc);
        diag_combine(xc, acc[0], a.kappa, a.twist, mx);
        const uint64_t h = noise_bits(seed_mixed, ids[r], (uint64_t)a.geo.V, (uint64_t)s);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            cx<double> e = z4_value<double>((uint32_t)(h >> (2 * k)) & 3u);
            cx<double> d = e - mx[k];
            pr += norm2(d);
            pe += norm2(e);
        }
    }
    double v = block_sum256(pr, sh);
    if (threadIdx.x == 0) a.partials[(size_t)r * nb + bm.sb] = v;
    double w = block_sum256(pe, sh);
    if (threadIdx.x == 0) a.partials2[(size_t)r * nb + bm.sb] = w;
}

__global__ __launch_bounds__(256) void k_true_resid_fin(CgArgs a, uint32_t nb) {
    __shared__ double sh[4];
    const int r = blockIdx.x;
    const double rr = sum_block_partials(a.partials + (size_t)r * nb, nb, sh);
    const double ee = sum_block_partials(a.partials2 + (size_t)r * nb, nb, sh);
    if (threadIdx.x == 0) a.scal[r].resid_true = sqrt(rr / ee);
}

// per-right-hand-side solver settings
__global__ void k_scal_init(CgScal* sc, int n, double tol2, int maxit, int stop, int reliable, double delta2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    CgScal q = {};
    q.tol2 = tol2;
    q.maxit = maxit;
    q.stop = stop;
    q.reliable = reliable;
    q.delta2 = delta2;
    q.resid_true = -1.0;
    sc[i] = q;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
// 1-D grid of site blocks x right-hand-side chunks (see stencil_block)
static inline dim3 stencil_grid(const Geom& g, int nch) {
    return dim3((unsigned)(((g.V + 255) / 256) * nch), 1, 1);
}

static inline uint32_t site_blocks(const Geom& g) { return (uint32_t)((g.V + 255) / 256); }
static inline uint32_t gated_blocks(const Geom& g) { return std::min(site_blocks(g), kGatedBlocks); }

static inline dim3 site_grid(const Geom& g, int ychunks) {
    return dim3((unsigned)((g.V + 255) / 256), (unsigned)ychunks, 1);
}

template <int OP, typename R, class Si, class So, class G>
static void apply_nr(hipStream_t st, const Geom& g, const void* gauge, double kappa, double twist, int nrhs,
                     const void* in, void* out, int nr, const CgScal* gate) {
    if (gate != nullptr) {
        hipLaunchKernelGGL((k_apply<OP, R, Si, So, G, 1>), dim3(gated_blocks(g) * (unsigned)nrhs), dim3(256), 0, st, g,
                           gauge, (R)kappa, (R)twist, nrhs, in, out, gate);
        return;
    }
    if constexpr (sizeof(R) == 8) {
        hipLaunchKernelGGL((k_apply<OP, R, Si, So, G, 1>), stencil_grid(g, nrhs), dim3(256), 0, st, g, gauge, (R)kappa,
                           (R)twist, nrhs, in, out, gate);
        return;
    }
    switch (nr) {
    case 4:
        hipLaunchKernelGGL((k_apply<OP, R, Si, So, G, 4>), stencil_grid(g, nrhs / 4), dim3(256), 0, st, g, gauge, (R)kappa,
                           (R)twist, nrhs, in, out, gate);
        break;
    case 2:
        hipLaunchKernelGGL((k_apply<OP, R, Si, So, G, 2>), stencil_grid(g, nrhs / 2), dim3(256), 0, st, g, gauge, (R)kappa,
                           (R)twist, nrhs, in, out, gate);
        break;
    default:
        hipLaunchKernelGGL((k_apply<OP, R, Si, So, G, 1>), stencil_grid(g, nrhs), dim3(256), 0, st, g, gauge, (R)kappa,
                           (R)twist, nrhs, in, out, gate);
        break;
    }
}

template <int OP>
static void apply_prec(hipStream_t st, const Geom& g, int prec, const void* gauge, double kappa, double twist,
                       int nrhs, const void* in, void* out, int nr, const CgScal* gate) {
    switch (prec) {
    case P_F64:
        apply_nr<OP, double, SF64, SF64, GF64>(st, g, gauge, kappa, twist, nrhs, in, out, 1, gate);
        break;
    case P_F32:
        apply_nr<OP, float, SF32, SF32, GF32>(st, g, gauge, kappa, twist, nrhs, in, out, nr, gate);
        break;
    case P_F16:
        apply_nr<OP, float, SF16, SF16, GF32>(st, g, gauge, kappa, twist, nrhs, in, out, nr, gate);
        break;
    default:
        apply_nr<OP, float, SBF16, SBF16, GF32>(st, g, gauge, kappa, twist, nrhs, in, out, nr, gate);
        break;
    }
}

void launch_apply(hipStream_t st, const Geom& g, int prec, const void* gauge, double kappa, double twist, int op,
                  int nrhs, const void* in, void* out, int nr, const CgScal* gate) {
    if (op == 0)
        apply_prec<0>(st, g, prec, gauge, kappa, twist, nrhs, in, out, nr, gate);
    else if (op == 1)
        apply_prec<1>(st, g, prec, gauge, kappa, twist, nrhs, in, out, nr, gate);
    else
        apply_prec<3>(st, g, prec, gauge, kappa, twist, nrhs, in, out, nr, gate);
}

template <typename R, class S, class G>
static void cg_mp_typed(hipStream_t st, const CgArgs& a, int nr) {
    const Geom& g = a.geo;
    if constexpr (sizeof(R) == 8) {
        hipLaunchKernelGGL((k_cg_mp<R, S, G, 1>), stencil_grid(g, a.nrhs), dim3(256), 0, st, a);
        return;
    }
    switch (nr) {
    case 4:
        hipLaunchKernelGGL((k_cg_mp<R, S, G, 4>), stencil_grid(g, a.nrhs / 4), dim3(256), 0, st, a);
        break;
    case 2:
        hipLaunchKernelGGL((k_cg_mp<R, S, G, 2>), stencil_grid(g, a.nrhs / 2), dim3(256), 0, st, a);
        break;
    default:
        hipLaunchKernelGGL((k_cg_mp<R, S, G, 1>), stencil_grid(g, a.nrhs), dim3(256), 0, st, a);
        break;
    }
}

template <typename R, class S, class G, class X, typename RX>
static void cg_upd_typed(hipStream_t st, const CgArgs& a, int nr, bool track) {
    const Geom& g = a.geo;
    if (track) {
        hipLaunchKernelGGL((k_cg_upd<R, S, G, X, RX, 1, true>), stencil_grid(g, a.nrhs), dim3(256), 0, st, a);
    } else if constexpr (sizeof(R) == 8) {
        hipLaunchKernelGGL((k_cg_upd<R, S, G, X, RX, 1, false>), stencil_grid(g, a.nrhs), dim3(256), 0, st, a);
    } else {
        switch (nr) {
        case 4:
            hipLaunchKernelGGL((k_cg_upd<R, S, G, X, RX, 4, false>), stencil_grid(g, a.nrhs / 4), dim3(256), 0, st, a);
            break;
        case 2:
            hipLaunchKernelGGL((k_cg_upd<R, S, G, X, RX, 2, false>), stencil_grid(g, a.nrhs / 2), dim3(256), 0, st, a);
            break;
        default:
            hipLaunchKernelGGL((k_cg_upd<R, S, G, X, RX, 1, false>), stencil_grid(g, a.nrhs), dim3(256), 0, st, a);
            break;
        }
    }
}

template <typename R, class S>
static void cg_p_typed(hipStream_t st, const CgArgs& a) {
    hipLaunchKernelGGL((k_cg_p<R, S>), site_grid(a.geo, a.nrhs), dim3(256), 0, st, a);
}

void launch_cg_mp(hipStream_t st, const CgArgs& a, int prec, int nr) {
    switch (prec) {
    case P_F64: cg_mp_typed<double, SF64, GF64>(st, a, 1); break;
    case P_F32: cg_mp_typed<float, SF32, GF32>(st, a, nr); break;
    case P_F16: cg_mp_typed<float, SF16, GF32>(st, a, nr); break;
    default: cg_mp_typed<float, SBF16, GF32>(st, a, nr); break;
    }
}

void launch_cg_upd(hipStream_t st, const CgArgs& a, int prec, int nr, bool track) {
    switch (prec) {
    case P_F64: cg_upd_typed<double, SF64, GF64, SF64, double>(st, a, 1, track); break;
    case P_F32: cg_upd_typed<float, SF32, GF32, SF32, float>(st, a, nr, track); break;
    case P_F16: cg_upd_typed<float, SF16, GF32, SF32, float>(st, a, nr, track); break;
    default: cg_upd_typed<float, SBF16, GF32, SF32, float>(st, a, nr, track); break;
    }
}

void launch_cg_alpha(hipStream_t st, const CgArgs& a) {
    hipLaunchKernelGGL(k_cg_alpha, dim3((unsigned)a.nrhs), dim3(256), 0, st, a, a.npart);
}

void launch_cg_beta(hipStream_t st, const CgArgs& a, bool track) {
    const uint32_t nb = a.npart;
    if (track)
        hipLaunchKernelGGL(k_cg_beta<true>, dim3((unsigned)a.nrhs), dim3(256), 0, st, a, nb);
    else
        hipLaunchKernelGGL(k_cg_beta<false>, dim3((unsigned)a.nrhs), dim3(256), 0, st, a, nb);
}

void launch_cg_p(hipStream_t st, const CgArgs& a, int prec) {
    switch (prec) {
    case P_F64: cg_p_typed<double, SF64>(st, a); break;
    case P_F32: cg_p_typed<float, SF32>(st, a); break;
    case P_F16: cg_p_typed<float, SF16>(st, a); break;
    default: cg_p_typed<float, SBF16>(st, a); break;
    }
}

void launch_cg_init(hipStream_t st, const CgArgs& a, int prec, bool track, const void* eta, double ee_z4) {
    dim3 grid = site_grid(a.geo, a.nrhs);
    if (!track && ee_z4 > 0) eta = nullptr;  // |eta|^2 given, no rho
    switch (prec) {
    case P_F64:
        if (track)
            hipLaunchKernelGGL((k_cg_init<double, SF64, SF64, double, true>), grid, dim3(256), 0, st, a, eta);
        else
            hipLaunchKernelGGL((k_cg_init<double, SF64, SF64, double, false>), grid, dim3(256), 0, st, a, eta);
        break;
    case P_F32:
        if (track)
            hipLaunchKernelGGL((k_cg_init<float, SF32, SF32, float, true>), grid, dim3(256), 0, st, a, eta);
        else
            hipLaunchKernelGGL((k_cg_init<float, SF32, SF32, float, false>), grid, dim3(256), 0, st, a, eta);
        break;
    case P_F16:
        if (track)
            hipLaunchKernelGGL((k_cg_init<float, SF16, SF32, float, true>), grid, dim3(256), 0, st, a, eta);
        else
            hipLaunchKernelGGL((k_cg_init<float, SF16, SF32, float, false>), grid, dim3(256), 0, st, a, eta);
        break;
    default:
        if (track)
            hipLaunchKernelGGL((k_cg_init<float, SBF16, SF32, float, true>), grid, dim3(256), 0, st, a, eta);
        else
            hipLaunchKernelGGL((k_cg_init<float, SBF16, SF32, float, false>), grid, dim3(256), 0, st, a, eta);
        break;
    }
    hipLaunchKernelGGL(k_cg_init_fin, dim3((unsigned)a.nrhs), dim3(256), 0, st, a, site_blocks(a.geo),
                       ee_z4 > 0 ? 0 : 1, ee_z4);
}

void launch_scal_init(hipStream_t st, CgScal* sc, int n, double tol2, int maxit, int stop, int reliable,
                      double delta2) {
    hipLaunchKernelGGL(k_scal_init, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, sc, n, tol2, maxit, stop, reliable,
                       delta2);
}

void launch_rel_init(hipStream_t st, const CgArgs& a, const void* b64, void* x64, double ee_z4, int prec) {
    const dim3 grid = site_grid(a.geo, a.nrhs);
    switch (prec) {
    case P_F16: hipLaunchKernelGGL(k_rel_init<SF16>, grid, dim3(256), 0, st, a, b64, x64); break;
    case P_BF16: hipLaunchKernelGGL(k_rel_init<SBF16>, grid, dim3(256), 0, st, a, b64, x64); break;
    default: hipLaunchKernelGGL(k_rel_init<SF32>, grid, dim3(256), 0, st, a, b64, x64); break;
    }
    hipLaunchKernelGGL(k_cg_init_fin, dim3((unsigned)a.nrhs), dim3(256), 0, st, a, site_blocks(a.geo), 0,
                       ee_z4 > 0 ? ee_z4 : 12.0 * (double)a.geo.V);
}
void launch_rel_fin(hipStream_t st, const CgArgs& a, uint32_t nb) {
    hipLaunchKernelGGL(k_rel_fin, dim3((unsigned)a.nrhs), dim3(256), 0, st, a, nb);
}
void launch_rel_flush(hipStream_t st, const CgArgs& a, void* x64, int force) {
    hipLaunchKernelGGL(k_rel_flush, dim3(gated_blocks(a.geo), (unsigned)a.nrhs), dim3(256), 0, st, a, x64, force);
}
void launch_rel_resid(hipStream_t st, const CgArgs& a, const void* gauge64, const void* b64, const void* t64) {
    const uint32_t nb = gated_blocks(a.geo);
    hipLaunchKernelGGL(k_rel_resid, dim3(nb, (unsigned)a.nrhs), dim3(256), 0, st, a, gauge64, b64, t64);
    hipLaunchKernelGGL(k_rel_fin, dim3((unsigned)a.nrhs), dim3(256), 0, st, a, nb);
}

void launch_true_resid(hipStream_t st, const CgArgs& a, int xprec, const void* gauge64, uint64_t seed_mixed,
                       const uint64_t* ids) {
    dim3 grid = stencil_grid(a.geo, a.nrhs);
    if (xprec == P_F64)
        hipLaunchKernelGGL((k_true_resid<SF64, double>), grid, dim3(256), 0, st, a, gauge64, seed_mixed, ids);
    else
        hipLaunchKernelGGL((k_true_resid<SF32, float>), grid, dim3(256), 0, st, a, gauge64, seed_mixed, ids);
    hipLaunchKernelGGL(k_true_resid_fin, dim3((unsigned)a.nrhs), dim3(256), 0, st, a, site_blocks(a.geo));
}

}  // namespace tmq
