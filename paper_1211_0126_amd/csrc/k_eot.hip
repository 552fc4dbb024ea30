// Even-odd half-hops with the links of a site tile shared by every
// right-hand side of the launch (gfx950, FP32 links, FP32 arithmetic,
// FP32/FP16/BF16 spinor storage).
//
// Every link enters a half-hop exactly once (each joins one even and one odd
// site), so a launch that applies the hop to n right-hand sides in chunks of
// NR per lane reads the link field n/NR times unless the chunks share it.
// Here a block owns a tile of 64 half-sites and all n right-hand sides: its
// four waves first stage the tile's 8 x 64 links (forward links of the tile's
// sites from the output parity's copy, backward links from the input
// parity's copy at the neighbours; 24 KiB) in LDS, then each wave takes the
// NR-chunks w, w + 4, ... and reads the links from LDS; the neighbour indices
// of a lane are computed once for all chunks.  Reductions are per wave and
// chunk (each wave owns its right-hand sides), one partial per tile.
//
// Kernels (the even-odd CG of k_eo.hip; same arithmetic, another traversal):
//   k_eot_y    y = D^{-1} H_eo p  (DAG: D^{-dag} H_eo^dag t)
//   k_eot_mp   t = D p - kappa^2 H_oe y, |t|^2
//   k_eot_upd  q = D^dag t - kappa^2 H_oe^dag y, r -= alpha q, x += alpha p, |r|^2
//   k_eot_src  etahat = eta_o + kappa H_oe D^{-1} eta_e, with eta from the hash
//   k_eot_rec  the whole solution in the full native layout: the even half
//              D^{-1} (eta_e + kappa H_eo x_o) and the odd half copied

#include <algorithm>

#include "tm_device.h"
#include "tm_eo.h"
#include "tm_kernels.h"
#include "tm_stencil.h"

namespace tmq {

constexpr int kEoTile = 64;   // half-sites per block (one per lane)
constexpr int kEoWaves = 4;   // waves per block
constexpr int kEoLinkF4 = 24; // float4 per site in LDS: 8 links x 3

template <int NR>
struct EotOcc {
    static constexpr int waves = NR == 1 ? 4 : (NR == 2 ? 3 : 2);
};
#define TM_EOT(NR) __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(::tmq::EotOcc<NR>::waves)))

// the tile's links into LDS: slot l < 4 forward link U_l(x) of the tile's
// site, slot 4 + l backward link U_l(x - l) at the neighbour; L[(3 l + j) *
// 64 + site] is row-plane j of slot l
__device__ __forceinline__ void eot_stage(const Geom& hg, const void* gout, const void* gin, int pout, uint32_t h0,
                                          float4* L) {
    const long Vs = hg.Vs;
    for (int i = threadIdx.x; i < kEoLinkF4 * kEoTile; i += 256) {
        const int site = i & (kEoTile - 1);
        const int pj = i >> 6;
        const int l = pj / 3, j = pj - 3 * l;
        const uint32_t h = h0 + (uint32_t)site;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (h < hg.V) {
            if (l < 4) {
                v = ld_plane<float4>(gout, Vs, l * 3 + j, h);
            } else {
                const EoSite c = eo_coords(hg, h, pout);
                v = ld_plane<float4>(gin, Vs, (l - 4) * 3 + j, eo_nb(hg, h, c, l - 4, false));
            }
        }
        L[pj * kEoTile + site] = v;
    }
    __syncthreads();
}

__device__ __forceinline__ void eot_link(const float4* L, int slot, int lane, cx<float> U[3][3]) {
    link_from_rows(L[(3 * slot + 0) * kEoTile + lane], L[(3 * slot + 1) * kEoTile + lane],
                   L[(3 * slot + 2) * kEoTile + lane], U);
}

// a lane's neighbours: half index of neighbour k (k < 4 forward in
// direction k, else backward in direction k - 4) and the time-boundary flips
struct EotNb {
    uint32_t y[8];
    bool ff, fb;
};
__device__ __forceinline__ EotNb eot_neighbours(const Geom& hg, uint32_t h, const EoSite& c) {
    EotNb n;
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
        n.y[mu] = eo_nb(hg, h, c, mu, true);
        n.y[4 + mu] = eo_nb(hg, h, c, mu, false);
    }
    n.ff = (c.t + 1 == hg.L[3]) && (hg.t_bc < 0);
    n.fb = (c.t == 0) && (hg.t_bc < 0);
    return n;
}

// both hops in direction MU for NR right-hand sides; in(r, k, p) yields the
// input spinor of right-hand side r at neighbour k
template <int MU, bool DAG, int NR, class In>
__device__ __forceinline__ void eot_hop_mu(const float4* L, int lane, const EotNb& n, In&& in,
                                           cx<float> (&acc)[NR][12]) {
    constexpr int SF = DAG ? -1 : 1;
    {
        cx<float> U[3][3];
        eot_link(L, MU, lane, U);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<float> p[12], hh[6], g[6];
            in(r, MU, p);
            proj<MU, SF>(p, hh);
            if (MU == 3 && n.ff) negate6(hh);
            su3_mul(U, hh, g);
            recon<MU, SF>(g, acc[r]);
        }
    }
    {
        cx<float> U[3][3];
        eot_link(L, 4 + MU, lane, U);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<float> p[12], hh[6], g[6];
            in(r, 4 + MU, p);
            proj<MU, -SF>(p, hh);
            if (MU == 3 && n.fb) negate6(hh);
            su3_dag_mul(U, hh, g);
            recon<MU, -SF>(g, acc[r]);
        }
    }
}

template <bool DAG, int NR, class In>
__device__ __forceinline__ void eot_hop_all(const float4* L, int lane, const EotNb& n, In&& in,
                                            cx<float> (&acc)[NR][12]) {
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int k = 0; k < 12; k++) acc[r][k] = {0.f, 0.f};
    eot_hop_mu<0, DAG, NR>(L, lane, n, in, acc);
    pin_acc<float, NR>(acc);
    TM_MEM_FENCE();
    eot_hop_mu<1, DAG, NR>(L, lane, n, in, acc);
    pin_acc<float, NR>(acc);
    TM_MEM_FENCE();
    eot_hop_mu<2, DAG, NR>(L, lane, n, in, acc);
    pin_acc<float, NR>(acc);
    TM_MEM_FENCE();
    eot_hop_mu<3, DAG, NR>(L, lane, n, in, acc);
}

struct EotTile {
    uint32_t tile, h;
    int lane, wave;
    bool valid;
};
__device__ __forceinline__ EotTile eot_tile(const Geom& hg) {
    EotTile t;
    t.tile = xcd_block(blockIdx.x, gridDim.x);
    t.lane = threadIdx.x & 63;
    t.wave = threadIdx.x >> 6;
    t.h = t.tile * kEoTile + (uint32_t)t.lane;
    t.valid = t.h < hg.V;
    return t;
}

// chunk ch is skipped when none of its right-hand sides is active
template <int NR>
__device__ __forceinline__ bool eot_chunk_active(const CgScal* sc, int r0, bool (&act)[NR]) {
    bool any = false;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        act[r] = sc == nullptr || sc[r0 + r].active != 0;
        any |= act[r];
    }
    return any;
}

// ---------------------------------------------------------------------------
// y = D^{-1} H in (DAG: D^{-dag} H^dag in); output parity a.pout
// ---------------------------------------------------------------------------
template <bool DAG, class S, int NR>
__global__ TM_EOT(NR) void k_eot_y(EoArgs a, const CgScal* sc) {
    __shared__ float4 L[kEoLinkF4 * kEoTile];
    const Geom& hg = a.hg;
    const EotTile T = eot_tile(hg);
    eot_stage(hg, a.gout, a.gin, a.pout, T.tile * kEoTile, L);
    const long Vs = hg.Vs;
    EotNb n = {};
    if (T.valid) n = eot_neighbours(hg, T.h, eo_coords(hg, T.h, a.pout));
    const float tw = (float)(DAG ? -a.twist : a.twist);
    const float inv = (float)(1.0 / (1.0 + a.twist * a.twist));
    const int nch = a.nrhs / NR;
    for (int ch = T.wave; ch < nch; ch += kEoWaves) {
        const int r0 = ch * NR;
        bool act[NR];
        if (!eot_chunk_active<NR>(sc, r0, act) || !T.valid) continue;
        cx<float> acc[NR][12];
        auto in = [&](int r, int k, cx<float> p[12]) {
            load_spinor<S, float>(field_rhs<S>(a.in, Vs, r0 + r), Vs, n.y[k], p);
        };
        eot_hop_all<DAG, NR>(L, T.lane, n, in, acc);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (!act[r]) continue;
            mul_diag_inv(acc[r], tw, inv);
            store_spinor<S, float>(field_rhs<S>(a.out, Vs, r0 + r), Vs, T.h, acc[r]);
        }
    }
}

// ---------------------------------------------------------------------------
// K1b: out = D c - kappa^2 H_oe y with c = a.p and out = a.t, partials of
// |out|^2 (one per tile); DAG: D^dag c - kappa^2 H_oe^dag y (with c = etahat
// and out = r this is b = Mhat^dag etahat of the CG start)
// ---------------------------------------------------------------------------
template <bool DAG, class S, int NR>
__global__ TM_EOT(NR) void k_eot_mp(CgArgs a, EoCg e, const void* cin, void* cout) {
    __shared__ float4 L[kEoLinkF4 * kEoTile];
    const Geom& hg = a.geo;
    const EotTile T = eot_tile(hg);
    eot_stage(hg, e.godd, e.geven, 1, T.tile * kEoTile, L);
    const long Vs = hg.Vs;
    EotNb n = {};
    if (T.valid) n = eot_neighbours(hg, T.h, eo_coords(hg, T.h, 1));
    const float tw = (float)(DAG ? -a.twist : a.twist), k2 = (float)(-a.kappa * a.kappa);
    const int nch = a.nrhs / NR;
    for (int ch = T.wave; ch < nch; ch += kEoWaves) {
        const int r0 = ch * NR;
        bool act[NR];
        if (!eot_chunk_active<NR>(a.scal, r0, act)) continue;
        double part[NR];
#pragma unroll
        for (int r = 0; r < NR; r++) part[r] = 0;
        if (T.valid) {
            cx<float> acc[NR][12];
            auto in = [&](int r, int k, cx<float> p[12]) {
                load_spinor<S, float>(field_rhs<S>(e.y, Vs, r0 + r), Vs, n.y[k], p);
            };
            eot_hop_all<DAG, NR>(L, T.lane, n, in, acc);
#pragma unroll
            for (int r = 0; r < NR; r++) {
                if (!act[r]) continue;
                cx<float> t[12];
                load_spinor<S, float>(field_rhs<S>(cin, Vs, r0 + r), Vs, T.h, t);
                mul_diag(t, tw);
#pragma unroll
                for (int k = 0; k < 12; k++) t[k] = t[k] + k2 * acc[r][k];
                round_storage<S, float>(t);
                store_spinor_cp<S, float, TM_CP_K1T>(field_rhs<S>(cout, Vs, r0 + r), Vs, T.h, t);
                part[r] = spinor_norm2(t);
            }
        }
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const double v = wave_sum(part[r]);
            if (T.lane == 0 && act[r]) a.partials[(size_t)(r0 + r) * a.npart + T.tile] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// K2b: q = D^dag t - kappa^2 H_oe^dag y, r -= alpha q, x += alpha p, |r|^2;
// TRACK: rho -= alpha t and |rho|^2
// ---------------------------------------------------------------------------
template <class S, class X, int NR, bool TRACK>
__global__ TM_EOT(NR) void k_eot_upd(CgArgs a, EoCg e) {
    __shared__ float4 L[kEoLinkF4 * kEoTile];
    const Geom& hg = a.geo;
    const EotTile T = eot_tile(hg);
    eot_stage(hg, e.godd, e.geven, 1, T.tile * kEoTile, L);
    const long Vs = hg.Vs;
    EotNb n = {};
    if (T.valid) n = eot_neighbours(hg, T.h, eo_coords(hg, T.h, 1));
    const float tw = (float)(-a.twist), k2 = (float)(-a.kappa * a.kappa);
    const int nch = a.nrhs / NR;
    for (int ch = T.wave; ch < nch; ch += kEoWaves) {
        const int r0 = ch * NR;
        bool act[NR];
        if (!eot_chunk_active<NR>(a.scal, r0, act)) continue;
        double prr[NR], prho[NR];
#pragma unroll
        for (int r = 0; r < NR; r++) prr[r] = prho[r] = 0;
        if (T.valid) {
            cx<float> acc[NR][12];
            auto in = [&](int r, int k, cx<float> p[12]) {
                load_spinor<S, float>(field_rhs<S>(e.y, Vs, r0 + r), Vs, n.y[k], p);
            };
            eot_hop_all<true, NR>(L, T.lane, n, in, acc);
#pragma unroll
            for (int r = 0; r < NR; r++) {
                if (!act[r]) continue;
                const double alpha = a.scal[r0 + r].alpha;
                const float al = (float)alpha;
                cx<float> tc[12], q[12], rv[12], pv[12];
                load_spinor<S, float>(field_rhs<S>(a.t, Vs, r0 + r), Vs, T.h, tc);
#pragma unroll
                for (int k = 0; k < 12; k++) q[k] = tc[k];
                mul_diag(q, tw);
#pragma unroll
                for (int k = 0; k < 12; k++) q[k] = q[k] + k2 * acc[r][k];
                void* rp = field_rhs<S>(a.r, Vs, r0 + r);
                load_spinor_cp<S, float, TM_CP_K2>(rp, Vs, T.h, rv);
#pragma unroll
                for (int k = 0; k < 12; k++) rv[k] = rv[k] - al * q[k];
                round_storage<S, float>(rv);
                store_spinor_cp<S, float, TM_CP_K2>(rp, Vs, T.h, rv);
                prr[r] = spinor_norm2(rv);
                load_spinor_cp<S, float, TM_CP_K2>(field_rhs<S>(a.p, Vs, r0 + r), Vs, T.h, pv);
                cx<float> xv[12];
                void* xp = field_rhs<X>(a.x, Vs, r0 + r);
                load_spinor_cp<X, float, TM_CP_K2>(xp, Vs, T.h, xv);
#pragma unroll
                for (int k = 0; k < 12; k++) xv[k] = {xv[k].re + al * pv[k].re, xv[k].im + al * pv[k].im};
                store_spinor_cp<X, float, TM_CP_K2>(xp, Vs, T.h, xv);
                if (TRACK) {
                    cx<float> rh[12];
                    void* hp = field_rhs<S>(a.rho, Vs, r0 + r);
                    load_spinor_cp<S, float, TM_CP_K2>(hp, Vs, T.h, rh);
#pragma unroll
                    for (int k = 0; k < 12; k++) rh[k] = rh[k] - al * tc[k];
                    round_storage<S, float>(rh);
                    store_spinor_cp<S, float, TM_CP_K2>(hp, Vs, T.h, rh);
                    prho[r] = spinor_norm2(rh);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const double v = wave_sum(prr[r]);
            if (T.lane == 0 && act[r]) a.partials[(size_t)(r0 + r) * a.npart + T.tile] = v;
            if (TRACK) {
                const double w = wave_sum(prho[r]);
                if (T.lane == 0 && act[r]) a.partials2[(size_t)(r0 + r) * a.npart + T.tile] = w;
            }
        }
    }
}

// full-lattice index of the neighbour k of a site (k < 4 forward in
// direction k, else backward in direction k - 4)
__device__ __forceinline__ uint32_t full_nb(const Geom& hg, const EoSite& c, int k) {
    int x = c.x, y = c.y, z = c.z, t = c.t;
    const int mu = k & 3;
    const int d = k < 4 ? 1 : -1;
    if (mu == 0) x = (x + d + hg.L[0]) % hg.L[0];
    if (mu == 1) y = (y + d + hg.L[1]) % hg.L[1];
    if (mu == 2) z = (z + d + hg.L[2]) % hg.L[2];
    if (mu == 3) t = (t + d + hg.L[3]) % hg.L[3];
    return (uint32_t)(x + hg.L[0] * (y + hg.L[1] * (z + hg.L[2] * t)));
}

// ---------------------------------------------------------------------------
// source: etahat = eta_o + kappa H_oe D^{-1} eta_e with eta from the hash
// (the odd output sites and their even neighbours); no input field
// ---------------------------------------------------------------------------
template <class S, int NR>
__global__ TM_EOT(NR) void k_eot_src(EoArgs a) {
    __shared__ float4 L[kEoLinkF4 * kEoTile];
    const Geom& hg = a.hg;
    const EotTile T = eot_tile(hg);
    eot_stage(hg, a.gout, a.gin, 1, T.tile * kEoTile, L);
    const long Vs = hg.Vs;
    const uint64_t Vf = (uint64_t)(2 * hg.V);
    EoSite c = {};
    EotNb n = {};
    uint32_t sf[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (T.valid) {
        c = eo_coords(hg, T.h, 1);
        n = eot_neighbours(hg, T.h, c);
#pragma unroll
        for (int k = 0; k < 8; k++) sf[k] = full_nb(hg, c, k);
    }
    const float tw = (float)a.twist;
    const float inv = (float)(1.0 / (1.0 + a.twist * a.twist));
    const float kap = (float)a.kappa;
    const int nch = a.nrhs / NR;
    for (int ch = T.wave; ch < nch; ch += kEoWaves) {
        const int r0 = ch * NR;
        if (!T.valid) continue;
        cx<float> acc[NR][12];
        auto in = [&](int r, int k, cx<float> p[12]) {
            noise_at<float>(a.seed_mixed, a.ids[r0 + r], Vf, sf[k], p);
            mul_diag_inv(p, tw, inv);
        };
        eot_hop_all<false, NR>(L, T.lane, n, in, acc);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<float> o[12];
            noise_at<float>(a.seed_mixed, a.ids[r0 + r], Vf, eo_full_site(T.h, c), o);
#pragma unroll
            for (int k = 0; k < 12; k++) o[k] = o[k] + kap * acc[r][k];
            store_spinor<S, float>(field_rhs<S>(a.out, Vs, r0 + r), Vs, T.h, o);
        }
    }
}

// ---------------------------------------------------------------------------
// the whole solution, full native layout of X (stride g.Vs): even site of
// tile lane h gets D^{-1} (eta_e + kappa H_eo x_o), the odd site with the same
// half index gets x_o(h)
// ---------------------------------------------------------------------------
template <class X, int NR>
__global__ TM_EOT(NR) void k_eot_rec(EoArgs a, Geom g, void* full) {
    __shared__ float4 L[kEoLinkF4 * kEoTile];
    const Geom& hg = a.hg;
    const EotTile T = eot_tile(hg);
    eot_stage(hg, a.gout, a.gin, 0, T.tile * kEoTile, L);
    const long Vs = hg.Vs;
    const uint64_t Vf = (uint64_t)(2 * hg.V);
    EoSite c = {};
    EotNb n = {};
    uint32_t se = 0, so = 0;
    if (T.valid) {
        c = eo_coords(hg, T.h, 0);
        n = eot_neighbours(hg, T.h, c);
        se = eo_full_site(T.h, c);
        so = se - (uint32_t)c.x + (uint32_t)(c.x ^ 1);  // the odd site of the same half index
    }
    const float tw = (float)a.twist;
    const float inv = (float)(1.0 / (1.0 + a.twist * a.twist));
    const float kap = (float)a.kappa;
    const int nch = a.nrhs / NR;
    for (int ch = T.wave; ch < nch; ch += kEoWaves) {
        const int r0 = ch * NR;
        if (!T.valid) continue;
        cx<float> acc[NR][12];
        auto in = [&](int r, int k, cx<float> p[12]) {
            load_spinor<X, float>(field_rhs<X>(a.in, Vs, r0 + r), Vs, n.y[k], p);
        };
        eot_hop_all<false, NR>(L, T.lane, n, in, acc);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<float> o[12];
            noise_at<float>(a.seed_mixed, a.ids[r0 + r], Vf, se, o);
#pragma unroll
            for (int k = 0; k < 12; k++) o[k] = o[k] + kap * acc[r][k];
            mul_diag_inv(o, tw, inv);
            cx<float> xo[12];
            load_spinor<X, float>(field_rhs<X>(a.in, Vs, r0 + r), Vs, T.h, xo);
            void* f = field_rhs<X>(full, g.Vs, r0 + r);
            if (c.x & 1)
                store_site_pair<X, float>(f, g.Vs, so, xo, se, o);
            else
                store_site_pair<X, float>(f, g.Vs, se, o, so, xo);
        }
    }
}

// ---------------------------------------------------------------------------
// host launchers (grid: one block of 256 threads per tile of 64 half-sites)
// ---------------------------------------------------------------------------
uint32_t eot_tiles(const Geom& hg) { return (uint32_t)((hg.V + kEoTile - 1) / kEoTile); }

template <bool DAG, class S>
static void eot_y_s(hipStream_t st, const EoArgs& a, int nr, const CgScal* sc) {
    const dim3 grid(eot_tiles(a.hg));
    if (nr == 4)
        hipLaunchKernelGGL((k_eot_y<DAG, S, 4>), grid, dim3(256), 0, st, a, sc);
    else if (nr == 2)
        hipLaunchKernelGGL((k_eot_y<DAG, S, 2>), grid, dim3(256), 0, st, a, sc);
    else
        hipLaunchKernelGGL((k_eot_y<DAG, S, 1>), grid, dim3(256), 0, st, a, sc);
}

void launch_eot_y(hipStream_t st, const EoArgs& a, int prec, int nr, bool dag, const CgScal* sc) {
    switch (prec) {
    case P_F32: dag ? eot_y_s<true, SF32>(st, a, nr, sc) : eot_y_s<false, SF32>(st, a, nr, sc); break;
    case P_F16: dag ? eot_y_s<true, SF16>(st, a, nr, sc) : eot_y_s<false, SF16>(st, a, nr, sc); break;
    default: dag ? eot_y_s<true, SBF16>(st, a, nr, sc) : eot_y_s<false, SBF16>(st, a, nr, sc); break;
    }
}

template <bool DAG, class S>
static void eot_mp_s(hipStream_t st, const CgArgs& a, const EoCg& e, int nr, const void* cin, void* cout) {
    const dim3 grid(eot_tiles(a.geo));
    if (nr == 4)
        hipLaunchKernelGGL((k_eot_mp<DAG, S, 4>), grid, dim3(256), 0, st, a, e, cin, cout);
    else if (nr == 2)
        hipLaunchKernelGGL((k_eot_mp<DAG, S, 2>), grid, dim3(256), 0, st, a, e, cin, cout);
    else
        hipLaunchKernelGGL((k_eot_mp<DAG, S, 1>), grid, dim3(256), 0, st, a, e, cin, cout);
}

void launch_eot_mp(hipStream_t st, const CgArgs& a, const EoCg& e, int prec, int nr, bool dag, const void* cin,
                   void* cout) {
    switch (prec) {
    case P_F32: dag ? eot_mp_s<true, SF32>(st, a, e, nr, cin, cout) : eot_mp_s<false, SF32>(st, a, e, nr, cin, cout); break;
    case P_F16: dag ? eot_mp_s<true, SF16>(st, a, e, nr, cin, cout) : eot_mp_s<false, SF16>(st, a, e, nr, cin, cout); break;
    default: dag ? eot_mp_s<true, SBF16>(st, a, e, nr, cin, cout) : eot_mp_s<false, SBF16>(st, a, e, nr, cin, cout); break;
    }
}

template <class S>
static void eot_upd_s(hipStream_t st, const CgArgs& a, const EoCg& e, int nr, bool track) {
    const dim3 grid(eot_tiles(a.geo));
    if (track) {
        hipLaunchKernelGGL((k_eot_upd<S, SF32, 1, true>), grid, dim3(256), 0, st, a, e);
        return;
    }
    if (nr == 4)
        hipLaunchKernelGGL((k_eot_upd<S, SF32, 4, false>), grid, dim3(256), 0, st, a, e);
    else if (nr == 2)
        hipLaunchKernelGGL((k_eot_upd<S, SF32, 2, false>), grid, dim3(256), 0, st, a, e);
    else
        hipLaunchKernelGGL((k_eot_upd<S, SF32, 1, false>), grid, dim3(256), 0, st, a, e);
}

void launch_eot_upd(hipStream_t st, const CgArgs& a, const EoCg& e, int prec, int nr, bool track) {
    switch (prec) {
    case P_F32: eot_upd_s<SF32>(st, a, e, nr, track); break;
    case P_F16: eot_upd_s<SF16>(st, a, e, nr, track); break;
    default: eot_upd_s<SBF16>(st, a, e, nr, track); break;
    }
}

template <class S>
static void eot_src_s(hipStream_t st, const EoArgs& a, int nr) {
    const dim3 grid(eot_tiles(a.hg));
    if (nr == 4)
        hipLaunchKernelGGL((k_eot_src<S, 4>), grid, dim3(256), 0, st, a);
    else if (nr == 2)
        hipLaunchKernelGGL((k_eot_src<S, 2>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_eot_src<S, 1>), grid, dim3(256), 0, st, a);
}

void launch_eot_src(hipStream_t st, const EoArgs& a, int prec, int nr) {
    switch (prec) {
    case P_F32: eot_src_s<SF32>(st, a, nr); break;
    case P_F16: eot_src_s<SF16>(st, a, nr); break;
    default: eot_src_s<SBF16>(st, a, nr); break;
    }
}

void launch_eot_rec(hipStream_t st, const EoArgs& a, int nr, const Geom& g, void* full) {
    const dim3 grid(eot_tiles(a.hg));
    if (nr == 4)
        hipLaunchKernelGGL((k_eot_rec<SF32, 4>), grid, dim3(256), 0, st, a, g, full);
    else if (nr == 2)
        hipLaunchKernelGGL((k_eot_rec<SF32, 2>), grid, dim3(256), 0, st, a, g, full);
    else
        hipLaunchKernelGGL((k_eot_rec<SF32, 1>), grid, dim3(256), 0, st, a, g, full);
}

}  // namespace tmq
