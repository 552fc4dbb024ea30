// Time-marching variants of the CG stencil kernels K1 and K2 (gfx950).
//
// A lane owns one site of the spatial volume (x, y, z) and walks a segment
// of `tseg` time slices.  The time-direction hops reuse what the lane
// already holds: the forward hop out of slice t and the backward hop into
// slice t+1 use the same link U_4(x, t), and the backward hop into t+1 is
// computed from the spinor of slice t and carried to the next step.  Per
// site a lane loads the next slice's spinor, the six spatial neighbours and
// seven links (a lane per site loads nine spinors and eight links), and the
// time neighbours never come back through the caches.
//
// The diagonal term enters at the start of a step, scaled by -1/kappa, so
// that the current spinor is not kept across the step:
//   out = p - kappa acc + i tw g5 p = -kappa (acc - (p + i tw g5 p) / kappa).
//
// Blocks: 256 consecutive spatial sites (a tile) x one time segment x one
// chunk of NR right-hand sides; chunks of a tile are consecutive after the
// XCD remap.  Each block writes one partial per right-hand side.

#include "tm_kernels.h"
#include "tm_stencil.h"

namespace tmq {

// Occupancy targets (waves per SIMD): the marching lane keeps the next
// slice's spinors and the carried hops besides the accumulators.
template <int NR, int RB>
struct MarchOcc {
    static constexpr int waves = (RB == 8 || NR > 1) ? 2 : 4;
};
#define TM_MARCH_R(NR, R) \
    __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(::tmq::MarchOcc<NR, (int)sizeof(R)>::waves)))

struct MarchMap {
    uint32_t ch, tile, seg, ntile;
};
__device__ __forceinline__ MarchMap march_block(uint32_t nch, uint32_t ntile) {
    const uint32_t L = xcd_block(blockIdx.x, gridDim.x);
    MarchMap m;
    m.ch = L % nch;
    const uint32_t rest = L / nch;
    m.tile = rest % ntile;
    m.seg = rest / ntile;
    m.ntile = ntile;
    return m;
}

// backward time hop into the slice after `cur`: U_4^dag (1 + SF g4) cur
template <bool DAG, typename R>
__device__ __forceinline__ void t_carry(const cx<R> U[3][3], const cx<R> cur[12], bool flip, cx<R> g[6]) {
    constexpr int SF = DAG ? -1 : 1;
    cx<R> h[6];
    proj<3, -SF>(cur, h);
    if (flip) negate6(h);
    su3_dag_mul(U, h, g);
}

// forward time hop: acc += U_4 (1 - SF g4) nxt
template <bool DAG, typename R>
__device__ __forceinline__ void t_fwd(const cx<R> U[3][3], const cx<R> nxt[12], bool flip, cx<R> acc[12]) {
    constexpr int SF = DAG ? -1 : 1;
    cx<R> h[6], g[6];
    proj<3, SF>(nxt, h);
    if (flip) negate6(h);
    su3_mul(U, h, g);
    recon<3, SF>(g, acc);
}

// acc = recon(carry) - (p + i tw g5 p) / kappa
template <bool DAG, typename R>
__device__ __forceinline__ void step_init(const cx<R> carry[6], const cx<R> p[12], R rkappa, R tw, cx<R> acc[12]) {
    constexpr int SF = DAG ? -1 : 1;
#pragma unroll
    for (int k = 0; k < 6; k++) acc[k] = {-rkappa * (p[k].re - tw * p[k].im), -rkappa * (p[k].im + tw * p[k].re)};
#pragma unroll
    for (int k = 6; k < 12; k++) acc[k] = {-rkappa * (p[k].re + tw * p[k].im), -rkappa * (p[k].im - tw * p[k].re)};
    recon<3, -SF>(carry, acc);
}

// One pass over a block's sites and time segment: the stencil of op (M, or
// M^dag if DAG) applied to field `in` for NR right-hand sides; `site(t, s,
// out[NR][12])` consumes the result at site s (time slice t).
template <bool DAG, typename R, class S, class G, int NR, class F>
__device__ __forceinline__ void march(const Geom& g, const void* gauge, const void* in, double kappa, double twist,
                                      uint32_t s3, uint32_t V3, int t0, int t1, F&& site) {
    const long Vs = g.Vs;
    const int Lt = g.L[3];
    const R rk = (R)(1.0 / kappa), mk = (R)(-kappa);
    const R tw = (R)(DAG ? -twist : twist);
    Site c = site_coords(g, s3);
    cx<R> carry[NR][6], cur[NR][12];
    {
        const int tp = (t0 == 0) ? Lt - 1 : t0 - 1;
        const uint32_t sp = s3 + V3 * (uint32_t)tp;
        const bool flip = (tp == Lt - 1) && (g.t_bc < 0);
        cx<R> U[3][3];
        load_link<G, R>(gauge, Vs, 3, sp, U);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<R> q[12];
            load_spinor<S, R>(field_rhs<S>(in, Vs, r), Vs, sp, q);
            t_carry<DAG, R>(U, q, flip, carry[r]);
            load_spinor<S, R>(field_rhs<S>(in, Vs, r), Vs, s3 + V3 * (uint32_t)t0, cur[r]);
        }
    }
    for (int t = t0; t < t1; t++) {
        const uint32_t s = s3 + V3 * (uint32_t)t;
        c.t = t;
        const bool flip = (t == Lt - 1) && (g.t_bc < 0);
        const uint32_t sn = (t == Lt - 1) ? s3 : s + V3;
        cx<R> acc[NR][12];
        {
            cx<R> U[3][3];
            load_link<G, R>(gauge, Vs, 3, s, U);
#pragma unroll
            for (int r = 0; r < NR; r++) {
                step_init<DAG, R>(carry[r], cur[r], rk, tw, acc[r]);
                t_carry<DAG, R>(U, cur[r], flip, carry[r]);
                load_spinor<S, R>(field_rhs<S>(in, Vs, r), Vs, sn, cur[r]);  // next slice
                t_fwd<DAG, R>(U, cur[r], flip, acc[r]);
            }
        }
        pin_acc<R, NR>(acc);
        TM_MEM_FENCE();
        hop_mu<0, DAG, R, S, G, NR>(g, gauge, in, s, c, acc);
        pin_acc<R, NR>(acc);
        TM_MEM_FENCE();
        hop_mu<1, DAG, R, S, G, NR>(g, gauge, in, s, c, acc);
        pin_acc<R, NR>(acc);
        TM_MEM_FENCE();
        hop_mu<2, DAG, R, S, G, NR>(g, gauge, in, s, c, acc);
#pragma unroll
        for (int r = 0; r < NR; r++)
#pragma unroll
            for (int k = 0; k < 12; k++) acc[r][k] = {mk * acc[r][k].re, mk * acc[r][k].im};
        site(t, s, acc);
    }
}

// K1: t = M p, block partials of |t|^2
template <typename R, class S, class G, int NR>
__global__ TM_MARCH_R(NR, R) void k_tm_mp(CgArgs a) {
    __shared__ double sh[4];
    const Geom& g = a.geo;
    const int Lt = g.L[3];
    const uint32_t V3 = (uint32_t)(g.V / Lt);
    const MarchMap m = march_block((uint32_t)(a.nrhs / NR), (V3 + 255) / 256);
    const int r0 = m.ch * NR;
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
    const uint32_t s3 = m.tile * 256u + threadIdx.x;
    const int t0 = (int)m.seg * a.tseg;
    const int t1 = min(t0 + a.tseg, Lt);
    if (s3 < V3) {
        const long Vs = g.Vs;
        march<false, R, S, G, NR>(g, a.gauge, field_rhs<S>(a.p, Vs, r0), a.kappa, a.twist, s3, V3, t0, t1,
                                  [&](int, uint32_t s, cx<R> (&out)[NR][12]) {
#pragma unroll
                                      for (int r = 0; r < NR; r++) {
                                          if (!act[r]) continue;
                                          round_storage<S, R>(out[r]);
                                          store_spinor_cp<S, R, TM_CP_K1T>(field_rhs<S>(a.t, Vs, r0 + r), Vs, s,
                                                                           out[r]);
                                          part[r] += spinor_norm2(out[r]);
                                      }
                                  });
    }
    const uint32_t blk = m.tile + m.ntile * m.seg;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        double v = block_sum256(part[r], sh);
        if (threadIdx.x == 0) a.partials[(size_t)(r0 + r) * a.npart + blk] = v;
    }
}

// K2: q = M^dag t, r -= alpha q, x += alpha p (x of storage X), block
// partials of |r|^2, optionally rho -= alpha t and its norm
template <typename R, class S, class G, class X, typename RX, int NR, bool TRACK>
__global__ TM_MARCH_R(NR, R) void k_tm_upd(CgArgs a) {
    __shared__ double sh[4];
    const Geom& g = a.geo;
    const int Lt = g.L[3];
    const uint32_t V3 = (uint32_t)(g.V / Lt);
    const MarchMap m = march_block((uint32_t)(a.nrhs / NR), (V3 + 255) / 256);
    const int r0 = m.ch * NR;
    bool act[NR];
    bool any = false;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        act[r] = a.scal[r0 + r].active != 0;
        any |= act[r];
    }
    if (!any) return;
    double prr[NR], prho[NR];
    R al[NR];
    RX alx[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) {
        prr[r] = prho[r] = 0;
        const double alpha = a.scal[r0 + r].alpha;
        al[r] = (R)alpha;
        alx[r] = (RX)alpha;
    }
    const uint32_t s3 = m.tile * 256u + threadIdx.x;
    const int t0 = (int)m.seg * a.tseg;
    const int t1 = min(t0 + a.tseg, Lt);
    if (s3 < V3) {
        const long Vs = g.Vs;
        march<true, R, S, G, NR>(
            g, a.gauge, field_rhs<S>(a.t, Vs, r0), a.kappa, a.twist, s3, V3, t0, t1,
            [&](int, uint32_t s, cx<R> (&q)[NR][12]) {
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    if (!act[r]) continue;
                    cx<R> rv[12];
                    void* rp = field_rhs<S>(a.r, Vs, r0 + r);
                    load_spinor_cp<S, R, TM_CP_K2>(rp, Vs, s, rv);
#pragma unroll
                    for (int k = 0; k < 12; k++) rv[k] = rv[k] - al[r] * q[r][k];
                    round_storage<S, R>(rv);
                    store_spinor_cp<S, R, TM_CP_K2>(rp, Vs, s, rv);
                    prr[r] += spinor_norm2(rv);
                    cx<R> pv[12];
                    load_spinor_cp<S, R, TM_CP_K2>(field_rhs<S>(a.p, Vs, r0 + r), Vs, s, pv);
                    cx<RX> xv[12];
                    void* xp = field_rhs<X>(a.x, Vs, r0 + r);
                    load_spinor_cp<X, RX, TM_CP_K2>(xp, Vs, s, xv);
#pragma unroll
                    for (int k = 0; k < 12; k++)
                        xv[k] = {xv[k].re + alx[r] * (RX)pv[k].re, xv[k].im + alx[r] * (RX)pv[k].im};
                    store_spinor_cp<X, RX, TM_CP_K2>(xp, Vs, s, xv);
                    if (TRACK) {
                        cx<R> tc[12], rh[12];
                        load_spinor<S, R>(field_rhs<S>(a.t, Vs, r0 + r), Vs, s, tc);
                        void* hp = field_rhs<S>(a.rho, Vs, r0 + r);
                        load_spinor_cp<S, R, TM_CP_K2>(hp, Vs, s, rh);
#pragma unroll
                        for (int k = 0; k < 12; k++) rh[k] = rh[k] - al[r] * tc[k];
                        round_storage<S, R>(rh);
                        store_spinor_cp<S, R, TM_CP_K2>(hp, Vs, s, rh);
                        prho[r] += spinor_norm2(rh);
                    }
                }
            });
    }
    const uint32_t blk = m.tile + m.ntile * m.seg;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        double v = block_sum256(prr[r], sh);
        if (threadIdx.x == 0) a.partials[(size_t)(r0 + r) * a.npart + blk] = v;
        if (TRACK) {
            double w = block_sum256(prho[r], sh);
            if (threadIdx.x == 0) a.partials2[(size_t)(r0 + r) * a.npart + blk] = w;
        }
    }
}

// Flexible CG with the marching stencils (p and t stored as S, the other
// fields FP32, complex alpha): F1 t = M p with block partials of |t|^2 (of
// t as stored); F2 q = M^dag t (kept for the direction update), x += alpha
// p, r -= alpha q, block partials of |r|^2.
template <int NR, class S>
__global__ TM_MARCH_R(NR, float) void k_fcg_tm_mp(FcgArgs a, int tseg, uint32_t npart) {
    __shared__ double sh[4];
    const Geom& g = a.geo;
    const int Lt = g.L[3];
    const uint32_t V3 = (uint32_t)(g.V / Lt);
    const MarchMap m = march_block((uint32_t)(a.nrhs / NR), (V3 + 255) / 256);
    const int r0 = m.ch * NR;
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
    const uint32_t s3 = m.tile * 256u + threadIdx.x;
    const int t0 = (int)m.seg * tseg;
    const int t1 = min(t0 + tseg, Lt);
    if (s3 < V3) {
        const long Vs = g.Vs;
        march<false, float, S, GF32, NR>(g, a.gauge, field_rhs<S>(a.p, Vs, r0), a.kappa, a.twist, s3, V3, t0, t1,
                                         [&](int, uint32_t s, cx<float> (&out)[NR][12]) {
#pragma unroll
                                             for (int r = 0; r < NR; r++) {
                                                 if (!act[r]) continue;
                                                 round_storage<S, float>(out[r]);
                                                 store_spinor<S, float>(field_rhs<S>(a.t, Vs, r0 + r), Vs, s, out[r]);
                                                 part[r] += spinor_norm2(out[r]);
                                             }
                                         });
    }
    const uint32_t blk = m.tile + m.ntile * m.seg;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        double v = block_sum256(part[r], sh);
        if (threadIdx.x == 0) a.partials[(size_t)(r0 + r) * npart + blk] = v;
    }
}

template <int NR, class S>
__global__ TM_MARCH_R(NR, float) void k_fcg_tm_upd(FcgArgs a, int tseg, uint32_t npart) {
    __shared__ double sh[4];
    const Geom& g = a.geo;
    const int Lt = g.L[3];
    const uint32_t V3 = (uint32_t)(g.V / Lt);
    const MarchMap m = march_block((uint32_t)(a.nrhs / NR), (V3 + 255) / 256);
    const int r0 = m.ch * NR;
    bool act[NR];
    bool any = false;
    cx<float> al[NR];
    double prr[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) {
        act[r] = a.scal[r0 + r].active != 0;
        any |= act[r];
        al[r] = {(float)a.scal[r0 + r].alpha_re, (float)a.scal[r0 + r].alpha_im};
        prr[r] = 0;
    }
    if (!any) return;
    const uint32_t s3 = m.tile * 256u + threadIdx.x;
    const int t0 = (int)m.seg * tseg;
    const int t1 = min(t0 + tseg, Lt);
    if (s3 < V3) {
        const long Vs = g.Vs;
        march<true, float, S, GF32, NR>(
            g, a.gauge, field_rhs<S>(a.t, Vs, r0), a.kappa, a.twist, s3, V3, t0, t1,
            [&](int, uint32_t s, cx<float> (&q)[NR][12]) {
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    if (!act[r]) continue;
                    store_spinor<SF32, float>(field_rhs<SF32>(a.q, Vs, r0 + r), Vs, s, q[r]);
                    void* rp = field_rhs<SF32>(a.r, Vs, r0 + r);
                    cx<float> rv[12];
                    load_spinor_cp<SF32, float, TM_CP_K2>(rp, Vs, s, rv);
#pragma unroll
                    for (int k = 0; k < 12; k++) rv[k] = rv[k] - al[r] * q[r][k];
                    store_spinor_cp<SF32, float, TM_CP_K2>(rp, Vs, s, rv);
                    prr[r] += spinor_norm2(rv);
                    void* xp = field_rhs<SF32>(a.x, Vs, r0 + r);
                    cx<float> pv[12], xv[12];
                    load_spinor_cp<S, float, TM_CP_K2>(field_rhs<S>(a.p, Vs, r0 + r), Vs, s, pv);
                    load_spinor_cp<SF32, float, TM_CP_K2>(xp, Vs, s, xv);
#pragma unroll
                    for (int k = 0; k < 12; k++) xv[k] = xv[k] + al[r] * pv[k];
                    store_spinor_cp<SF32, float, TM_CP_K2>(xp, Vs, s, xv);
                }
            });
    }
    const uint32_t blk = m.tile + m.ntile * m.seg;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        double v = block_sum256(prr[r], sh);
        if (threadIdx.x == 0) a.partials[(size_t)(r0 + r) * npart + blk] = v;
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
uint32_t march_partials(const Geom& g, int tseg) {
    const uint32_t V3 = (uint32_t)(g.V / g.L[3]);
    return ((V3 + 255) / 256) * (uint32_t)((g.L[3] + tseg - 1) / tseg);
}

template <typename R, class S, class G>
static void tm_mp_typed(hipStream_t st, const CgArgs& a, int nr) {
    const unsigned nb = march_partials(a.geo, a.tseg);
    if constexpr (sizeof(R) == 8) {
        hipLaunchKernelGGL((k_tm_mp<R, S, G, 1>), dim3(nb * a.nrhs), dim3(256), 0, st, a);
    } else {
        if (nr == 2)
            hipLaunchKernelGGL((k_tm_mp<R, S, G, 2>), dim3(nb * (a.nrhs / 2)), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_tm_mp<R, S, G, 1>), dim3(nb * a.nrhs), dim3(256), 0, st, a);
    }
}

template <typename R, class S, class G, class X, typename RX>
static void tm_upd_typed(hipStream_t st, const CgArgs& a, int nr, bool track) {
    const unsigned nb = march_partials(a.geo, a.tseg);
    if (track) {
        hipLaunchKernelGGL((k_tm_upd<R, S, G, X, RX, 1, true>), dim3(nb * a.nrhs), dim3(256), 0, st, a);
        return;
    }
    if constexpr (sizeof(R) == 8) {
        hipLaunchKernelGGL((k_tm_upd<R, S, G, X, RX, 1, false>), dim3(nb * a.nrhs), dim3(256), 0, st, a);
    } else {
        if (nr == 2)
            hipLaunchKernelGGL((k_tm_upd<R, S, G, X, RX, 2, false>), dim3(nb * (a.nrhs / 2)), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_tm_upd<R, S, G, X, RX, 1, false>), dim3(nb * a.nrhs), dim3(256), 0, st, a);
    }
}

template <class S>
static void fcg_tm_typed(hipStream_t st, const FcgArgs& a, int nr, int tseg, bool upd) {
    const uint32_t np = march_partials(a.geo, tseg);
    const dim3 gr(np * (unsigned)(nr == 2 ? a.nrhs / 2 : a.nrhs));
    if (upd) {
        if (nr == 2)
            hipLaunchKernelGGL((k_fcg_tm_upd<2, S>), gr, dim3(256), 0, st, a, tseg, np);
        else
            hipLaunchKernelGGL((k_fcg_tm_upd<1, S>), gr, dim3(256), 0, st, a, tseg, np);
        launch_fcg_upd_fin(st, a, np);
    } else {
        if (nr == 2)
            hipLaunchKernelGGL((k_fcg_tm_mp<2, S>), gr, dim3(256), 0, st, a, tseg, np);
        else
            hipLaunchKernelGGL((k_fcg_tm_mp<1, S>), gr, dim3(256), 0, st, a, tseg, np);
        launch_fcg_mp_fin(st, a, np);
    }
}
static void fcg_tm(hipStream_t st, const FcgArgs& a, int nr, int tseg, bool upd) {
    if (a.prec == P_F16)
        fcg_tm_typed<SF16>(st, a, nr, tseg, upd);
    else if (a.prec == P_BF16)
        fcg_tm_typed<SBF16>(st, a, nr, tseg, upd);
    else
        fcg_tm_typed<SF32>(st, a, nr, tseg, upd);
}
void launch_fcg_tm_mp(hipStream_t st, const FcgArgs& a, int nr, int tseg) { fcg_tm(st, a, nr, tseg, false); }
void launch_fcg_tm_upd(hipStream_t st, const FcgArgs& a, int nr, int tseg) { fcg_tm(st, a, nr, tseg, true); }

void launch_tm_mp(hipStream_t st, const CgArgs& a, int prec, int nr) {
    switch (prec) {
    case P_F64: tm_mp_typed<double, SF64, GF64>(st, a, 1); break;
    case P_F32: tm_mp_typed<float, SF32, GF32>(st, a, nr); break;
    case P_F16: tm_mp_typed<float, SF16, GF32>(st, a, nr); break;
    default: tm_mp_typed<float, SBF16, GF32>(st, a, nr); break;
    }
}

void launch_tm_upd(hipStream_t st, const CgArgs& a, int prec, int nr, bool track) {
    switch (prec) {
    case P_F64: tm_upd_typed<double, SF64, GF64, SF64, double>(st, a, 1, track); break;
    case P_F32: tm_upd_typed<float, SF32, GF32, SF32, float>(st, a, nr, track); break;
    case P_F16: tm_upd_typed<float, SF16, GF32, SF32, float>(st, a, nr, track); break;
    default: tm_upd_typed<float, SBF16, GF32, SF32, float>(st, a, nr, track); break;
    }
}

}  // namespace tmq
