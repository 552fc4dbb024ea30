// Gauge-covariant parallel-transport layers of the learned preconditioner
// (gfx950): forward/adjoint application and the weight gradient.
//
// A layer maps cin spinor fields phi_b to cout fields
//     psi_a(x) = sum_b sum_p W[p][a][b] (T_p phi_b)(x),
// p over nine paths (identity, U_mu(x) phi(x+mu), U_mu(x-mu)^dag phi(x-mu),
// with the time-boundary sign), W[p][a][b] a complex 4x4 spin matrix,
// identity on colour.  Both kernels below follow the same three steps:
//   1. gather: every (site, path, channel) transport is computed once with
//      the FP32 links and written as bfloat16 into an LDS tile A whose rows
//      are (colour, site) and columns (path, channel, spin, re/im);
//   2. mix: the dense channel/spin mixing is a real GEMM A(rows x K) B(K x 16)
//      on the matrix cores (v_mfma_f32_16x16x16_bf16, FP32 accumulation),
//      B the real form of the complex weights, K = 72 cin padded to 16;
//   3. the FP32 result is staged in LDS and written as spinor planes.
// The adjoint layer is the same kernel with weights W'[p*][b][a] = W[p][a][b]^dag
// (p* the reversed path), prepared on the host.
// The weight gradient dW = sum_{x,c} g (T_p phi)^dag is the GEMM
// G^T (16 x rows) A (rows x K) per block of PT_TS sites, FP32 block partials
// reduced in a fixed order.

#include "tm_device.h"
#include "tm_kernels.h"

namespace tmq {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// weight gradient: 32 sites per block (a 28 KB bfloat16 A tile)
constexpr int PT_TS = 32;             // sites per block
constexpr int PT_ROWS = 3 * PT_TS;    // (colour, site) rows
constexpr int PT_NT = PT_ROWS / 16;   // 16-row MFMA tiles, dealt to the 4 waves
constexpr int PT_KMAX = 144;          // 72 * cin for cin <= 2
constexpr int PT_KP = PT_KMAX + 4;    // LDS row stride (bf16), padded against bank conflicts
constexpr int PT_GP = 16 + 4;         // LDS row stride of the gradient tile

__device__ __forceinline__ uint16_t to_bf16(float f) { return (uint16_t)f32_to_bf16(f); }

// Transport of channel b of `in` along path p, at site s (12 complex, FP32).
template <class Si>
__device__ __forceinline__ void transport_site(const Geom& geo, const void* gauge, const void* in, int b, int p,
                                               uint32_t s, cx<float> v[12]) {
    const void* f = field_rhs<Si>(in, geo.Vs, b);
    if (p == 0) {
        load_spinor<Si, float>(f, geo.Vs, s, v);
        return;
    }
    const int mu = (p - 1) >> 1;
    const bool fwd = (p & 1) != 0;
    const Site c = site_coords(geo, s);
    uint32_t y;
    bool flip;
    switch (mu) {
    case 0: y = fwd ? nb_fwd(geo, s, c, 0) : nb_bwd(geo, s, c, 0); flip = false; break;
    case 1: y = fwd ? nb_fwd(geo, s, c, 1) : nb_bwd(geo, s, c, 1); flip = false; break;
    case 2: y = fwd ? nb_fwd(geo, s, c, 2) : nb_bwd(geo, s, c, 2); flip = false; break;
    default:
        y = fwd ? nb_fwd(geo, s, c, 3) : nb_bwd(geo, s, c, 3);
        flip = geo.t_bc < 0 && (fwd ? (c.t + 1 == geo.L[3]) : (c.t == 0));
        break;
    }
    cx<float> U[3][3], psi[12];
    load_link<GF32, float>(gauge, geo.Vs, mu, fwd ? s : y, U);
    load_spinor<Si, float>(f, geo.Vs, y, psi);
    const float sg = flip ? -1.f : 1.f;
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int i = 0; i < 3; i++) {
            cx<float> t = {0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 3; k++) t = t + (fwd ? U[i][k] * psi[3 * a + k] : cmulc(U[k][i], psi[3 * a + k]));
            v[3 * a + i] = sg * t;
        }
}

// Fill the gradient's A tile: rows (colour c, site i) = c*PT_TS + i, columns
// k = ((p*cin + b)*4 + spin)*2 + re/im, zero-padded to kpad.
template <class Si>
__device__ __forceinline__ void gather_tile(const PtArgs& a, uint32_t site0, uint16_t* As, int kpad) {
    const Geom& geo = a.geo;
    const int nitems = PT_TS * 9 * a.cin;
    for (int item = threadIdx.x; item < nitems; item += 256) {
        const int i = item % PT_TS;
        const int rest = item / PT_TS;
        const int p = rest % 9;
        const int b = rest / 9;
        const uint32_t s = site0 + i;
        cx<float> v[12];
        if (s < geo.V) {
            transport_site<Si>(geo, a.gauge, a.in, b, p, s, v);
        } else {
#pragma unroll
            for (int k = 0; k < 12; k++) v[k] = {0.f, 0.f};
        }
        const int kb = (p * a.cin + b) * 8;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            uint16_t* row = As + (c * PT_TS + i) * PT_KP + kb;
#pragma unroll
            for (int si = 0; si < 4; si++) {
                row[2 * si] = to_bf16(v[3 * si + c].re);
                row[2 * si + 1] = to_bf16(v[3 * si + c].im);
            }
        }
    }
    const int k0 = 72 * a.cin;
    const int kw = kpad - k0;
    if (kw > 0) {
        for (int item = threadIdx.x; item < PT_ROWS * kw; item += 256) {
            const int r = item / kw, k = k0 + item % kw;
            As[r * PT_KP + k] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// Layer application.  A block owns 64 consecutive sites and loops over the
// right-hand sides; it runs nine waves, wave p handling path p with one lane
// per site.  The wave's effective link (sign and adjoint folded in) is loaded
// once and kept in registers for all right-hand sides, and the input planes
// of the next right-hand side are loaded while the current one is
// transported, mixed and stored.  Per right-hand side:
//   gather: the lane's CIN transports, packed to bfloat16, one 16-byte LDS
//           store per colour into the tile (rows (colour, site), columns
//           (path, channel, spin, re/im), row stride kpad + 8 bfloat16 so the
//           16-byte stores and the 8-byte MFMA operand reads are conflict-free);
//   mix:    the twelve 16-row MFMA tiles dealt to the waves, the FP32 result
//           staged in its own LDS array;
//   store:  one (channel, plane) of 16-byte elements per wave and pass.
// The barriers wait for LDS traffic only, so the prefetched global loads
// stay in flight across them.
// ---------------------------------------------------------------------------
constexpr int LY_TS = 64;
constexpr int LY_ROWS = 3 * LY_TS;
constexpr int LY_THREADS = 9 * 64;
constexpr int LY_OS = 20;  // staging row stride (floats): conflict-free MFMA result writes

template <int CIN>
struct LyShape {
    static constexpr int KP = (72 * CIN + 15) / 16 * 16;  // 80 or 144
    static constexpr int KS = KP + 8;                      // LDS row stride (bfloat16)
};

// LDS-only workgroup barrier: outstanding global loads are not waited for.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// raw storage planes of one spinor
template <class S>
struct RawSpinor {
    typename S::V v[S::NV];
};
template <class S>
__device__ __forceinline__ void raw_load(const void* base, long Vs, uint32_t s, RawSpinor<S>& q) {
#pragma unroll
    for (int k = 0; k < S::NV; k++) q.v[k] = ld_plane<typename S::V>(base, Vs, k, s);
}
// the spinor as twelve bfloat16 (re, im) pairs, the order of the half planes
__device__ __forceinline__ void raw_pairs(const RawSpinor<SF32>& q, uint32_t p[12]) {
#pragma unroll
    for (int k = 0; k < 6; k++) {
        p[2 * k] = pack2_bf16(q.v[k].x, q.v[k].y);
        p[2 * k + 1] = pack2_bf16(q.v[k].z, q.v[k].w);
    }
}
__device__ __forceinline__ void raw_pairs(const RawSpinor<SBF16>& q, uint32_t p[12]) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
        p[4 * k] = q.v[k].x;
        p[4 * k + 1] = q.v[k].y;
        p[4 * k + 2] = q.v[k].z;
        p[4 * k + 3] = q.v[k].w;
    }
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
// acc + a.lo b.lo + a.hi b.hi, bfloat16 pairs, FP32 accumulation (v_dot2_f32_bf16)
__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float acc) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, a), __builtin_bit_cast(bf16x2, b), acc, false);
}

template <int P, class Si, class So, int CIN, int COUT>
__device__ __forceinline__ void ly_run(const PtArgs& a, uint32_t nrhs, uint32_t site0, int lane, uint16_t* As,
                                       float* Os) {
    constexpr int KP = LyShape<CIN>::KP, KS = LyShape<CIN>::KS;
    constexpr int MU = (P - 1) >> 1;
    constexpr bool FWD = (P & 1) != 0;
    constexpr int NT = LY_ROWS / 16;  // MFMA row tiles
    constexpr int NP = So::NV;        // output planes per field
    constexpr int CPP = 12 / NP;      // complex components per output plane
    const Geom& geo = a.geo;
    const long Vs = geo.Vs;
    const uint32_t s = site0 + lane;
    const bool valid = s < geo.V;

    // effective link L = sign * U_mu(x), or sign * U_mu(x-mu)^dag, as bfloat16
    // pairs: (Re t, Im t) += (psi . LA, psi . LB) with LA = (Re L, -Im L),
    // LB = (Im L, Re L) for psi = (Re psi, Im psi); zero past the lattice
    uint32_t LA[3][3], LB[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) LA[i][k] = LB[i][k] = 0u;
    uint32_t y = s;
    if (P > 0 && valid) {
        const Site c = site_coords(geo, s);
        y = FWD ? nb_fwd(geo, s, c, MU) : nb_bwd(geo, s, c, MU);
        cx<float> U[3][3];
        load_link<GF32, float>(a.gauge, Vs, MU, FWD ? s : y, U);
        const bool flip = MU == 3 && geo.t_bc < 0 && (FWD ? (c.t + 1 == geo.L[3]) : (c.t == 0));
        const float sg = flip ? -1.f : 1.f;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const cx<float> m = FWD ? cx<float>{sg * U[i][k].re, sg * U[i][k].im}
                                        : cx<float>{sg * U[k][i].re, -sg * U[k][i].im};
                LA[i][k] = pack2_bf16(m.re, -m.im);
                LB[i][k] = pack2_bf16(m.im, m.re);
            }
    }
    // input planes of the current right-hand side; those of the next one are
    // loaded into the same registers once the current ones are unpacked
    // (lanes past the lattice keep zeros)
    RawSpinor<Si> nxt[CIN];
#pragma unroll
    for (int b = 0; b < CIN; b++)
#pragma unroll
        for (int k = 0; k < Si::NV; k++) nxt[b].v[k] = typename Si::V{};
    if (valid) {
#pragma unroll
        for (int b = 0; b < CIN; b++) raw_load(field_rhs<Si>(a.in, Vs, b), Vs, y, nxt[b]);
    }

    for (uint32_t r = 0; r < nrhs; r++) {
        // gather
#pragma unroll
        for (int b = 0; b < CIN; b++) {
            uint32_t psi[12];
            raw_pairs(nxt[b], psi);
            if (valid && r + 1 < nrhs) raw_load(field_rhs<Si>(a.in, Vs, (int)((r + 1) * CIN + b)), Vs, y, nxt[b]);
#pragma unroll
            for (int c = 0; c < 3; c++) {
                uint32_t q[4];
#pragma unroll
                for (int sp = 0; sp < 4; sp++) {
                    if (P == 0) {
                        q[sp] = psi[3 * sp + c];
                    } else {
                        float tr = 0.f, ti = 0.f;
#pragma unroll
                        for (int k = 0; k < 3; k++) {
                            tr = dot2(psi[3 * sp + k], LA[c][k], tr);
                            ti = dot2(psi[3 * sp + k], LB[c][k], ti);
                        }
                        q[sp] = pack2_bf16(tr, ti);
                    }
                }
                *(uint4*)(As + (c * LY_TS + lane) * KS + (P * CIN + b) * 8) = make_uint4(q[0], q[1], q[2], q[3]);
            }
        }
        if (KP > 72 * CIN && P == 0 && r == 0) {
#pragma unroll
            for (int c = 0; c < 3; c++) *(uint4*)(As + (c * LY_TS + lane) * KS + 72 * CIN) = make_uint4(0, 0, 0, 0);
        }
        lds_barrier();

        // mix
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const int tt = P + 9 * j;
            if (tt >= NT) continue;
            v4f acc = (v4f){0.f, 0.f, 0.f, 0.f};
            const int row = tt * 16 + (lane & 15);
#pragma unroll
            for (int ks = 0; ks < KP / 16; ks++) {
                const v4s af = *(const v4s*)(As + row * KS + ks * 16 + 4 * (lane >> 4));
                const v4s bf = ((const v4s*)a.wfrag)[ks * 64 + lane];
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af, bf, acc, 0, 0, 0);
            }
#pragma unroll
            for (int e = 0; e < 4; e++) Os[(tt * 16 + 4 * (lane >> 4) + e) * LY_OS + (lane & 15)] = acc[e];
        }
        lds_barrier();

        // store
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const int u = P + 9 * j;
            if (u >= COUT * NP || !valid) continue;
            const int ch = u / NP, k = u - ch * NP;
            float val[2 * CPP];
#pragma unroll
            for (int q = 0; q < CPP; q++) {
                const int comp = k * CPP + q, sp = comp / 3, col = comp - 3 * sp;
                const float* src = Os + (col * LY_TS + lane) * LY_OS + (ch * 4 + sp) * 2;
                val[2 * q] = src[0];
                val[2 * q + 1] = src[1];
            }
            void* dst = field_rhs<So>(a.out, Vs, (int)(r * COUT + ch));
            if constexpr (NP == 6) {
                st_plane(dst, Vs, k, s, make_float4(val[0], val[1], val[2], val[3]));
            } else {
                st_plane(dst, Vs, k, s,
                         make_uint4(pack2_bf16(val[0], val[1]), pack2_bf16(val[2], val[3]),
                                    pack2_bf16(val[4], val[5]), pack2_bf16(val[6], val[7])));
            }
        }
    }
}

// Two blocks (18 waves) per compute unit need at most 96 registers per lane,
// which the bfloat16-input kernels meet without spilling; the FP32-input
// two-channel kernels (training activations) run one block per unit.
template <class Si, int CIN>
constexpr int ly_min_waves() { return (std::is_same<Si, SF32>::value && CIN == 2) ? 1 : 5; }

template <class Si, class So, int CIN, int COUT>
__global__ __launch_bounds__(LY_THREADS, (ly_min_waves<Si, CIN>())) void k_pt_layer(PtArgs a, uint32_t nrhs) {
    constexpr int KS = LyShape<CIN>::KS;
    __shared__ __attribute__((aligned(16))) uint16_t As[LY_ROWS * KS];
    __shared__ __attribute__((aligned(16))) float Os[LY_ROWS * LY_OS];
    const uint32_t site0 = xcd_block(blockIdx.x, gridDim.x) * LY_TS;
    const int lane = threadIdx.x & 63;
    switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
    case 0: ly_run<0, Si, So, CIN, COUT>(a, nrhs, site0, lane, As, Os); break;
    case 1: ly_run<1, Si, So, CIN, COUT>(a, nrhs, site0, lane, As, Os); break;
    case 2: ly_run<2, Si, So, CIN, COUT>(a, nrhs, site0, lane, As, Os); break;
    case 3: ly_run<3, Si, So, CIN, COUT>(a, nrhs, site0, lane, As, Os); break;
    case 4: ly_run<4, Si, So, CIN, COUT>(a, nrhs, site0, lane, As, Os); break;
    case 5: ly_run<5, Si, So, CIN, COUT>(a, nrhs, site0, lane, As, Os); break;
    case 6: ly_run<6, Si, So, CIN, COUT>(a, nrhs, site0, lane, As, Os); break;
    case 7: ly_run<7, Si, So, CIN, COUT>(a, nrhs, site0, lane, As, Os); break;
    default: ly_run<8, Si, So, CIN, COUT>(a, nrhs, site0, lane, As, Os); break;
    }
}

// Weight gradient of one layer for one right-hand side: block partials of
// C[m][k] = sum_rows G[row][m] A[row][k], m = (out channel, spin, re/im).
template <class Si, class Sg>
__global__ __launch_bounds__(256) void k_pt_wgrad(PtArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t As[PT_ROWS * PT_KP];
    __shared__ __attribute__((aligned(16))) uint16_t Gs[PT_ROWS * PT_GP];
    const uint32_t blk = blockIdx.x;
    const uint32_t site0 = blk * PT_TS;
    const int kpad = a.kpad;
    gather_tile<Si>(a, site0, As, kpad);
    for (int item = threadIdx.x; item < PT_TS * 2; item += 256) {
        const int i = item % PT_TS, ch = item / PT_TS;
        const uint32_t s = site0 + i;
        cx<float> g[12];
        if (ch < a.cout && s < a.geo.V) {
            load_spinor<Sg, float>(field_rhs<Sg>(a.g, a.geo.Vs, ch), a.geo.Vs, s, g);
        } else {
#pragma unroll
            for (int k = 0; k < 12; k++) g[k] = {0.f, 0.f};
        }
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
            for (int so = 0; so < 4; so++) {
                Gs[(c * PT_TS + i) * PT_GP + (ch * 4 + so) * 2] = to_bf16(g[3 * so + c].re);
                Gs[(c * PT_TS + i) * PT_GP + (ch * 4 + so) * 2 + 1] = to_bf16(g[3 * so + c].im);
            }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nct = kpad / 16;
    for (int ct = w; ct < nct; ct += 4) {
        v4f acc = (v4f){0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < PT_ROWS / 16; ks++) {
            v4s af, bf;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int row = ks * 16 + 4 * (lane >> 4) + j;
                af[j] = (short)Gs[row * PT_GP + (lane & 15)];
                bf[j] = (short)As[row * PT_KP + ct * 16 + (lane & 15)];
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af, bf, acc, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; j++)
            a.partials[((size_t)blk * 16 + 4 * (lane >> 4) + j) * kpad + ct * 16 + (lane & 15)] = acc[j];
    }
}

// grad[m][k] += scale * sum over blocks of partials (fixed order), FP64
__global__ void k_pt_wgrad_reduce(const float* partials, int nblocks, int kpad, const double* scale, double* grad) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 16 * kpad) return;
    double s = 0;
    for (int b = 0; b < nblocks; b++) s += (double)partials[(size_t)b * 16 * kpad + e];
    grad[e] += (*scale) * s;
}

// Output error of a training pair: g = y - e (FP32 field), |y - e|^2 and
// |e|^2, and (last block) the pair's loss share and gradient scale
// 1 / (|e|^2 npairs); loss accumulates into scal[2].
template <class Se>
__global__ __launch_bounds__(256) void k_pt_loss(Geom geo, const void* y, const void* e, void* g, double* partials,
                                                 unsigned int* counter, double* scal, int npairs) {
    __shared__ double sh[4];
    __shared__ int sflag;
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    double pd = 0, pe = 0;
    if (s < geo.V) {
        cx<float> yv[12], ev[12], gv[12];
        load_spinor<SF32, float>(y, geo.Vs, s, yv);
        load_spinor<Se, float>(e, geo.Vs, s, ev);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            gv[k] = yv[k] - ev[k];
            pd += (double)gv[k].re * gv[k].re + (double)gv[k].im * gv[k].im;
            pe += (double)ev[k].re * ev[k].re + (double)ev[k].im * ev[k].im;
        }
        store_spinor<SF32, float>(g, geo.Vs, s, gv);
    }
    const uint32_t nb = gridDim.x;
    double v = block_sum256(pd, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = v;
    double u = block_sum256(pe, sh);
    if (threadIdx.x == 0) partials[nb + blockIdx.x] = u;
    if (take_last_ticket(counter, nb, &sflag)) {
        double d2 = sum_partials(partials, nb, sh);
        double e2 = sum_partials(partials + nb, nb, sh);
        if (threadIdx.x == 0) {
            scal[0] = 1.0 / (e2 * npairs);      // gradient scale of this pair
            scal[1] = d2 / e2;                   // this pair's relative error
            scal[2] += d2 / e2 / npairs;         // running loss
            *counter = 0;
        }
    }
}

template <class Si, class So>
static void launch_pt_layer_t(hipStream_t st, const PtArgs& a, int nrhs) {
    const dim3 grid((unsigned)((a.geo.V + LY_TS - 1) / LY_TS)), blk(LY_THREADS);
    const uint32_t n = (uint32_t)nrhs;
    if (a.cin == 1 && a.cout == 1) hipLaunchKernelGGL((k_pt_layer<Si, So, 1, 1>), grid, blk, 0, st, a, n);
    else if (a.cin == 1) hipLaunchKernelGGL((k_pt_layer<Si, So, 1, 2>), grid, blk, 0, st, a, n);
    else if (a.cout == 1) hipLaunchKernelGGL((k_pt_layer<Si, So, 2, 1>), grid, blk, 0, st, a, n);
    else hipLaunchKernelGGL((k_pt_layer<Si, So, 2, 2>), grid, blk, 0, st, a, n);
}

void launch_pt_layer(hipStream_t st, const PtArgs& a, int in_prec, int out_prec, int nrhs) {
    const bool ib = in_prec == P_BF16, ob = out_prec == P_BF16;
    if (ib && ob) launch_pt_layer_t<SBF16, SBF16>(st, a, nrhs);
    else if (ib) launch_pt_layer_t<SBF16, SF32>(st, a, nrhs);
    else if (ob) launch_pt_layer_t<SF32, SBF16>(st, a, nrhs);
    else launch_pt_layer_t<SF32, SF32>(st, a, nrhs);
}

void launch_pt_wgrad(hipStream_t st, const PtArgs& a, int in_prec, const double* scale, double* grad) {
    const int nb = (int)((a.geo.V + PT_TS - 1) / PT_TS);
    if (in_prec == P_BF16)
        hipLaunchKernelGGL((k_pt_wgrad<SBF16, SF32>), dim3(nb), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_pt_wgrad<SF32, SF32>), dim3(nb), dim3(256), 0, st, a);
    const int n = 16 * a.kpad;
    hipLaunchKernelGGL(k_pt_wgrad_reduce, dim3((n + 255) / 256), dim3(256), 0, st, a.partials, nb, a.kpad, scale, grad);
}

void launch_pt_loss(hipStream_t st, const Geom& g, const void* y, const void* e, int e_prec, void* gout,
                    double* partials, unsigned int* counter, double* scal, int npairs) {
    dim3 grid((unsigned)((g.V + 255) / 256));
    if (e_prec == P_BF16)
        hipLaunchKernelGGL((k_pt_loss<SBF16>), grid, dim3(256), 0, st, g, y, e, gout, partials, counter, scal, npairs);
    else
        hipLaunchKernelGGL((k_pt_loss<SF32>), grid, dim3(256), 0, st, g, y, e, gout, partials, counter, scal, npairs);
}

int pt_blocks(const Geom& g) { return (int)((g.V + PT_TS - 1) / PT_TS); }

// Training pair from an iterate x_k: r = eta - M x_k, e = x* - x_k (FP64
// arithmetic, stored as bfloat16); eta regenerated from the hash.
__global__ __launch_bounds__(256) void k_make_pair(Geom geo, uint64_t seed_mixed, const uint64_t* id, const void* xk,
                                                   const void* xstar, const void* mxk, void* r_out, void* e_out) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= geo.V) return;
    cx<double> x[12], xs[12], mx[12];
    load_spinor<SF64, double>(xk, geo.Vs, s, x);
    load_spinor<SF64, double>(xstar, geo.Vs, s, xs);
    load_spinor<SF64, double>(mxk, geo.Vs, s, mx);
    const uint64_t h = noise_bits(seed_mixed, *id, (uint64_t)geo.V, (uint64_t)s);
    cx<float> r[12], e[12];
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const cx<double> eta = z4_value<double>((uint32_t)(h >> (2 * k)) & 3u);
        const cx<double> rv = eta - mx[k], ev = xs[k] - x[k];
        r[k] = {(float)rv.re, (float)rv.im};
        e[k] = {(float)ev.re, (float)ev.im};
    }
    store_spinor<SBF16, float>(r_out, geo.Vs, s, r);
    store_spinor<SBF16, float>(e_out, geo.Vs, s, e);
}

void launch_make_pair(hipStream_t st, const Geom& g, uint64_t seed_mixed, const uint64_t* id, const void* xk,
                      const void* xstar, const void* mxk, void* r_out, void* e_out) {
    hipLaunchKernelGGL(k_make_pair, dim3((unsigned)((g.V + 255) / 256)), dim3(256), 0, st, g, seed_mixed, id, xk, xstar,
                       mxk, r_out, e_out);
}

}  // namespace tmq
