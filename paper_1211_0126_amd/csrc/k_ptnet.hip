// Gauge-covariant parallel-transport layers of the learned preconditioner
// (gfx950): forward/adjoint application and the weight gradient.
//
// A layer maps cin spinor fields phi_b to cout fields
//     psi_a(x) = sum_b sum_p W[p][a][b] (T_p phi_b)(x),
// p over nine paths (identity, U_mu(x) phi(x+mu), U_mu(x-mu)^dag phi(x-mu),
// with the time-boundary sign), W[p][a][b] a complex 4x4 spin matrix,
// identity on colour.  The channel/spin mixing is a real GEMM over
// K = 72 cin (path, channel, spin, re/im; padded to 16) on the matrix cores
// (v_mfma_f32_16x16x16_bf16, FP32 accumulation) with the real form of the
// complex weights:
//   * layer application (k_pt_layer): the sites are the GEMM's N side and the
//     transports are computed in registers straight into its B operand (see
//     the comment at the kernel);
//   * weight gradient (k_pt_wgrad): dW = sum_{x,c} g (T_p phi)^dag as the GEMM
//     G^T (16 x rows) A (rows x K) per block of PT_TS sites, A the transports
//     gathered into an LDS tile with rows (colour, site), FP32 block partials
//     reduced in a fixed order.
// The adjoint layer is the same kernel with weights W'[p*][b][a] = W[p][a][b]^dag
// (p* the reversed path), prepared on the host.

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
// Layer application.  Every wave is independent: it owns 16 consecutive
// sites and loops over the right-hand sides.  The mixing is computed with the
// sites on the N side of the matrix cores,
//     D[out][site] += Wt[out][k] T[k][site]   (v_mfma_f32_16x16x16_bf16),
// one product per colour, so the transports T go from registers straight into
// the B operand: lane l = 16 g + i holds, for site i, the four k = 4g..4g+3 of
// the current k-step, i.e. one (path, channel) and the spin pair 2(g&1),
// 2(g&1)+1.  Each lane therefore transports a half spinor per k-step (18
// complex multiply-adds as bfloat16 dot2 with FP32 accumulation); the link
// comes from a bfloat16-pair copy of the gauge field.  The D layout gives
// lane l the output channel g>>1 and the same spin pair, which it writes as
// its half of the output spinor.  No LDS and no barriers.
// K-steps: for two input channels step ks is path ks (lane channel g>>1); for
// one channel step ks covers paths 2ks and 2ks+1 (lane path 2ks + (g>>1)),
// the tenth "path" being zero padding.
// ---------------------------------------------------------------------------
constexpr int LY_TS = 64;         // sites per block: four waves of 16
constexpr int LY_THREADS = 256;

__device__ __forceinline__ uint4 ldv128(const void* base, uint32_t voff) {
    return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rsrc_of(base), voff, 0, 0));
}
__device__ __forceinline__ uint2 ldv64(const void* base, uint32_t voff) {
    return __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(rsrc_of(base), voff, 0, 0));
}
__device__ __forceinline__ uint32_t ldv32(const void* base, uint32_t voff) {
    return __builtin_amdgcn_raw_buffer_load_b32(rsrc_of(base), voff, 0, 0);
}
// (see st_plane for the wait states after a 128-bit store)
__device__ __forceinline__ void stv128(void* base, uint32_t voff, uint4 val) {
    using V4 = unsigned int __attribute__((ext_vector_type(4)));
    const V4 v = __builtin_bit_cast(V4, val);
    __builtin_amdgcn_raw_buffer_store_b128(v, rsrc_of(base), voff, 0, 0);
    asm volatile("s_nop 4" ::"v"(v) : "memory");
}
__device__ __forceinline__ void stv64(void* base, uint32_t voff, uint2 val) {
    using V2 = unsigned int __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, val), rsrc_of(base), voff, 0, 0);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
// acc + a.lo b.lo + a.hi b.hi, bfloat16 pairs, FP32 accumulation (v_dot2_f32_bf16)
__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float acc) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, a), __builtin_bit_cast(bf16x2, b), acc, false);
}
// a.lo b.lo + a.hi b.hi: the three-operand form with a zero accumulator (the
// builtin would first move a zero into a register for the two-operand form)
__device__ __forceinline__ float dot2_0(uint32_t a, uint32_t b) {
    float d;
    asm("v_dot2_f32_bf16 %0, %1, %2, 0" : "=v"(d) : "v"(a), "v"(b));
    return d;
}

// Hidden activations of the network (internal to the layers): bfloat16 pairs
// in three 16-byte planes arranged so that each half spinor is one plane and
// one half plane: plane 0 = components 0-3, plane 1 = 6-9, plane 2 = 4, 5 |
// 10, 11.
struct SBH {
    using V = uint4;
    static constexpr int NV = 3;
};
__device__ __forceinline__ uint32_t swap16(uint32_t x) { return __builtin_amdgcn_alignbit(x, x, 16); }

// The lane's half spinor (components 6h .. 6h+5, spins 2h and 2h+1) of
// channel b at site y, as bfloat16 (re, im) pairs.
__device__ __forceinline__ void half_spinor(const void* f, uint32_t PB, int b, uint32_t y, int h, uint32_t q[6],
                                            SBF16) {
    // planes of 4 components: h = 0 -> plane 0 + low half of plane 1; h = 1 -> high half of plane 1 + plane 2
    const uint32_t base = (y << 4) + (uint32_t)b * 3u * PB;
    const uint4 full = ldv128(f, base + (h ? 2u * PB : 0u));
    const uint2 half = ldv64(f, base + PB + (h ? 8u : 0u));
    q[0] = h ? half.x : full.x;
    q[1] = h ? half.y : full.y;
    q[2] = h ? full.x : full.z;
    q[3] = h ? full.y : full.w;
    q[4] = h ? full.z : half.x;
    q[5] = h ? full.w : half.y;
}
__device__ __forceinline__ void half_spinor(const void* f, uint32_t PB, int b, uint32_t y, int h, uint32_t q[6],
                                            SBH) {
    const uint32_t base = (y << 4) + (uint32_t)b * 3u * PB;
    const uint4 full = ldv128(f, base + (uint32_t)h * PB);
    const uint2 half = ldv64(f, base + 2u * PB + (uint32_t)h * 8u);
    q[0] = full.x;
    q[1] = full.y;
    q[2] = full.z;
    q[3] = full.w;
    q[4] = half.x;
    q[5] = half.y;
}
__device__ __forceinline__ void half_spinor(const void* f, uint32_t PB, int b, uint32_t y, int h, uint32_t q[6],
                                            SF32) {
    // planes of 2 components: planes 3h, 3h+1, 3h+2
    const uint32_t base = (y << 4) + (uint32_t)b * 6u * PB + (uint32_t)h * 3u * PB;
#pragma unroll
    for (int j = 0; j < 3; j++) {
        const float4 v = __builtin_bit_cast(float4, ldv128(f, base + (uint32_t)j * PB));
        q[2 * j] = pack2_bf16(v.x, v.y);
        q[2 * j + 1] = pack2_bf16(v.z, v.w);
    }
}

// Per-lane description of the (path, channel) of one k-step.
struct LyPath {
    uint32_t y;      // neighbour site
    uint32_t lsite;  // site of the link
    uint32_t lplane; // byte offset of the link's first plane
    uint32_t flip;   // 0x80008000 where the time-boundary sign applies
    bool fwd, ident, pad;
};

template <int P>
__device__ __forceinline__ LyPath ly_path(const uint32_t ys[9], uint32_t s, uint32_t flip_f, uint32_t flip_b,
                                          uint32_t PB) {
    LyPath d;
    d.pad = P >= 9;
    d.ident = P == 0;
    d.y = (P >= 1 && P <= 8) ? ys[P] : s;
    d.fwd = (P & 1) != 0;
    const int mu = (P >= 1 && P <= 8) ? (P - 1) >> 1 : 0;  // identity and padding read direction 0's link
    d.lsite = d.fwd || P == 0 ? s : d.y;
    d.lplane = (uint32_t)(mu * 3) * PB;
    d.flip = (P == 7) ? flip_f : (P == 8) ? flip_b : 0u;
    return d;
}
__device__ __forceinline__ LyPath ly_select(bool hi, const LyPath& a, const LyPath& b) {
    LyPath d;
    d.y = hi ? b.y : a.y;
    d.lsite = hi ? b.lsite : a.lsite;
    d.lplane = hi ? b.lplane : a.lplane;
    d.flip = hi ? b.flip : a.flip;
    d.fwd = hi ? b.fwd : a.fwd;
    d.ident = hi ? b.ident : a.ident;
    d.pad = hi ? b.pad : a.pad;
    return d;
}

// The link of a k-step, oriented and as bfloat16 pairs: m[c][k] = U[c][k]
// (forward) or U[k][c] (backward, to be used with the conjugating operand
// signs below).
__device__ __forceinline__ void ly_link(const PtArgs& a, uint32_t PB, const LyPath& d, uint32_t m[9]) {
    const uint32_t lb = (d.lsite << 4) + d.lplane;
    const uint4 u0 = ldv128(a.gaugebf, lb);
    const uint4 u1 = ldv128(a.gaugebf, lb + PB);
    const uint32_t u8 = ldv32(a.gaugebf, lb + 2u * PB);
    const uint32_t u[9] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w, u8};
#pragma unroll
    for (int c = 0; c < 3; c++)
#pragma unroll
        for (int k = 0; k < 3; k++) m[3 * c + k] = d.fwd ? u[3 * c + k] : u[3 * k + c];
}

// B operand of one k-step and one right-hand side for the three colours: the
// lane's two spins of the transported (or, for the identity path, the plain)
// half spinor.
//   forward:  Re t = (Re, -Im) psi . U,   Im t = (Im, Re) psi . U
//   backward: Re t = psi . U^T,           Im t = (Im, -Re) psi . U^T
template <class Si>
__device__ __forceinline__ void ly_operand(const void* in, uint32_t PB, int h, int b, const LyPath& d,
                                           const uint32_t m[9], uint32_t B[3][2]) {
    uint32_t q[6];
    half_spinor(in, PB, b, d.y, h, q, Si{});
    const uint32_t s1 = d.fwd ? 0x80000000u : 0u, s2 = d.fwd ? 0u : 0x80000000u;
    uint32_t a1[6], a2[6];
#pragma unroll
    for (int j = 0; j < 6; j++) {
        a1[j] = q[j] ^ s1;
        a2[j] = swap16(q[j]) ^ s2;
    }
#pragma unroll
    for (int c = 0; c < 3; c++)
#pragma unroll
        for (int t = 0; t < 2; t++) {
            float tr = dot2_0(a1[3 * t], m[3 * c]), ti = dot2_0(a2[3 * t], m[3 * c]);
            tr = dot2(a1[3 * t + 1], m[3 * c + 1], tr);
            ti = dot2(a2[3 * t + 1], m[3 * c + 1], ti);
            tr = dot2(a1[3 * t + 2], m[3 * c + 2], tr);
            ti = dot2(a2[3 * t + 2], m[3 * c + 2], ti);
            const uint32_t tv = pack2_bf16(tr, ti) ^ d.flip;
            B[c][t] = d.pad ? 0u : d.ident ? q[3 * t + c] : tv;
        }
}

// Right-hand sides are processed in chunks of LY_RC: each k-step's link is
// loaded once and applied to all of the chunk's right-hand sides, whose MFMA
// accumulators stay live.  A block handles TM_LY_CHUNKS_RC right-hand sides of
// its tile, and the grid runs chunk-major, so the lattice is swept once per
// group of right-hand sides and the time neighbours of a sweep stay in cache.
// (Measured on 24^3 x 48 with 8 right-hand sides: chunks of 2 and 2 per block
// are 5-15% faster than 1, 4 or all right-hand sides per block.)
#ifndef TM_LY_RC
#define TM_LY_RC 2
#endif
constexpr int LY_RC = TM_LY_RC;
#ifndef TM_LY_CHUNKS_RC
#define TM_LY_CHUNKS_RC 2
#endif

template <class Si, class So, int CIN, int COUT>
__global__ __launch_bounds__(LY_THREADS) void k_pt_layer(PtArgs a, uint32_t nrhs) {
    constexpr int NKS = (9 * CIN + 1) / 2;  // k-steps of 16
    const Geom& geo = a.geo;
    const long Vs = geo.Vs;
    const uint32_t PB = (uint32_t)Vs * 16u;  // plane bytes
    const int lane = threadIdx.x & 63, g = lane >> 4, h = g & 1;
    // blocks: (right-hand-side chunk, site tile), chunk slowest
    const uint32_t ntile = (geo.V + LY_TS - 1) / LY_TS;
    const uint32_t L = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t chunk = L / ntile, tile = L - chunk * ntile;
    const uint32_t r_beg = chunk * (uint32_t)TM_LY_CHUNKS_RC;
    const uint32_t r_end = r_beg + (uint32_t)TM_LY_CHUNKS_RC < nrhs ? r_beg + (uint32_t)TM_LY_CHUNKS_RC : nrhs;
    if (a.gate) {  // flexible CG: nothing to do for converged or fallen-back right-hand sides
        bool any = false;
        for (uint32_t r = r_beg; r < r_end; r++) any |= a.gate[r].active != 0 && a.gate[r].fell == 0;
        if (!any) return;
    }
    const uint32_t s0 = tile * LY_TS + (threadIdx.x >> 6) * 16 + (lane & 15);
    const bool valid = s0 < geo.V;
    const uint32_t s = valid ? s0 : 0u;  // lanes past the lattice compute site 0 and store nothing

    uint32_t ys[9];
    uint32_t flip_f = 0, flip_b = 0;
    {
        const Site c = site_coords(geo, s);
        ys[0] = s;
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            ys[1 + 2 * mu] = nb_fwd(geo, s, c, mu);
            ys[2 + 2 * mu] = nb_bwd(geo, s, c, mu);
        }
        if (geo.t_bc < 0) {
            flip_f = (c.t + 1 == geo.L[3]) ? 0x80008000u : 0u;
            flip_b = (c.t == 0) ? 0x80008000u : 0u;
        }
    }
    v4s wf[NKS];
#pragma unroll
    for (int ks = 0; ks < NKS; ks++) wf[ks] = ((const v4s*)a.wfrag)[ks * 64 + lane];

    for (uint32_t r0 = r_beg; r0 < r_end; r0 += LY_RC) {
        const uint32_t nrhs_left = r_end;
        const uint32_t nr = nrhs_left - r0 < (uint32_t)LY_RC ? nrhs_left - r0 : (uint32_t)LY_RC;
        v4f D[LY_RC][3];
#pragma unroll
        for (int j = 0; j < LY_RC; j++)
#pragma unroll
            for (int c = 0; c < 3; c++) D[j][c] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < NKS; ks++) {
            LyPath d;
            int b;
            if constexpr (CIN == 2) {
                d = ks == 0 ? ly_path<0>(ys, s, flip_f, flip_b, PB)
                  : ks == 1 ? ly_path<1>(ys, s, flip_f, flip_b, PB)
                  : ks == 2 ? ly_path<2>(ys, s, flip_f, flip_b, PB)
                  : ks == 3 ? ly_path<3>(ys, s, flip_f, flip_b, PB)
                  : ks == 4 ? ly_path<4>(ys, s, flip_f, flip_b, PB)
                  : ks == 5 ? ly_path<5>(ys, s, flip_f, flip_b, PB)
                  : ks == 6 ? ly_path<6>(ys, s, flip_f, flip_b, PB)
                  : ks == 7 ? ly_path<7>(ys, s, flip_f, flip_b, PB)
                            : ly_path<8>(ys, s, flip_f, flip_b, PB);
                b = g >> 1;
            } else {
                const bool hi = (g >> 1) != 0;
                d = ks == 0 ? ly_select(hi, ly_path<0>(ys, s, flip_f, flip_b, PB), ly_path<1>(ys, s, flip_f, flip_b, PB))
                  : ks == 1 ? ly_select(hi, ly_path<2>(ys, s, flip_f, flip_b, PB), ly_path<3>(ys, s, flip_f, flip_b, PB))
                  : ks == 2 ? ly_select(hi, ly_path<4>(ys, s, flip_f, flip_b, PB), ly_path<5>(ys, s, flip_f, flip_b, PB))
                  : ks == 3 ? ly_select(hi, ly_path<6>(ys, s, flip_f, flip_b, PB), ly_path<7>(ys, s, flip_f, flip_b, PB))
                            : ly_select(hi, ly_path<8>(ys, s, flip_f, flip_b, PB), ly_path<9>(ys, s, flip_f, flip_b, PB));
                b = 0;
            }
            uint32_t m[9];
            ly_link(a, PB, d, m);
#pragma unroll
            for (int j = 0; j < LY_RC; j++) {
                if ((uint32_t)j >= nr) break;
                uint32_t B[3][2];
                ly_operand<Si>(field_rhs<Si>(a.in, Vs, (int)((r0 + j) * CIN)), PB, h, b, d, m, B);
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const v4s bo = __builtin_bit_cast(v4s, make_uint2(B[c][0], B[c][1]));
                    D[j][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wf[ks], bo, D[j][c], 0, 0, 0);
                }
            }
        }
        // lane holds channel g>>1, spins 2h and 2h+1: component 6h + 3t + c is
        // (D[c][2t], D[c][2t + 1])
        const int ch = g >> 1;
        if (!valid || ch >= COUT) continue;
#pragma unroll
        for (int j = 0; j < LY_RC; j++) {
            if ((uint32_t)j >= nr) break;
            void* out = field_rhs<So>(a.out, Vs, (int)((r0 + j) * COUT));
            float o[12];
#pragma unroll
            for (int t = 0; t < 2; t++)
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    o[2 * (3 * t + c)] = D[j][c][2 * t];
                    o[2 * (3 * t + c) + 1] = D[j][c][2 * t + 1];
                }
            if constexpr (std::is_same<So, SBH>::value) {
                uint32_t w[6];
#pragma unroll
                for (int q = 0; q < 6; q++) w[q] = pack2_bf16(o[2 * q], o[2 * q + 1]);
                const uint32_t base = (s << 4) + (uint32_t)ch * 3u * PB;
                stv128(out, base + (uint32_t)h * PB, make_uint4(w[0], w[1], w[2], w[3]));
                stv64(out, base + 2u * PB + (uint32_t)h * 8u, make_uint2(w[4], w[5]));
            } else if constexpr (std::is_same<So, SF32>::value) {
                const uint32_t base = (s << 4) + (uint32_t)ch * 6u * PB + (uint32_t)h * 3u * PB;
#pragma unroll
                for (int q = 0; q < 3; q++)
                    stv128(out, base + (uint32_t)q * PB,
                           make_uint4(__float_as_uint(o[4 * q]), __float_as_uint(o[4 * q + 1]),
                                      __float_as_uint(o[4 * q + 2]), __float_as_uint(o[4 * q + 3])));
            } else {
                static_assert(std::is_same<So, SF32>::value || std::is_same<So, SBH>::value, "FP32 or SBH output");
            }
        }
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

// grad[m][k] += scale * sum over blocks of partials, FP64, in two coalesced
// stages with a fixed order: chunk sums of WG_CH block partials, then the sum
// of the chunk sums.
constexpr int WG_CH = 256;
__global__ __launch_bounds__(256) void k_pt_wgrad_sum1(const float* partials, int nblocks, int ne, double* part2) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    const int b0 = blockIdx.y * WG_CH, b1 = min(b0 + WG_CH, nblocks);
    double s = 0;
    for (int b = b0; b < b1; b++) s += (double)partials[(size_t)b * ne + e];
    part2[(size_t)blockIdx.y * ne + e] = s;
}
__global__ __launch_bounds__(256) void k_pt_wgrad_sum2(const double* part2, int nchunk, int ne, const double* scale,
                                                       double* grad) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    double s = 0;
    for (int c = 0; c < nchunk; c++) s += part2[(size_t)c * ne + e];
    grad[e] += (*scale) * s;
}

// Output error of a training pair: g = y - e (FP32 field), block partials of
// |y - e|^2 and |e|^2; k_pt_loss_fin turns them into the pair's loss share
// and gradient scale.
template <class Se>
__global__ __launch_bounds__(256) void k_pt_loss(Geom geo, const void* y, const void* e, void* g, double* partials) {
    __shared__ double sh[4];
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
}

// one block: the pair's gradient scale 1 / (|e|^2 npairs) into scal[0], its
// relative error into scal[1], and its loss share added to scal[2]
__global__ __launch_bounds__(256) void k_pt_loss_fin(const double* partials, uint32_t nb, double* scal, int npairs) {
    __shared__ double sh[4];
    double d = 0, e = 0;
    for (uint32_t i = threadIdx.x; i < nb; i += 256) {
        d += partials[i];
        e += partials[nb + i];
    }
    const double d2 = block_sum256(d, sh);
    const double e2 = block_sum256(e, sh);
    if (threadIdx.x == 0) {
        scal[0] = 1.0 / (e2 * npairs);
        scal[1] = d2 / e2;
        scal[2] += d2 / e2 / npairs;
    }
}

template <class Si, class So>
static void launch_pt_layer_t(hipStream_t st, const PtArgs& a, int nrhs) {
    const unsigned nchunk = (unsigned)((nrhs + TM_LY_CHUNKS_RC - 1) / TM_LY_CHUNKS_RC);
    const dim3 grid((unsigned)((a.geo.V + LY_TS - 1) / LY_TS) * nchunk), blk(LY_THREADS);
    const uint32_t n = (uint32_t)nrhs;
    if (a.cin == 1 && a.cout == 1) hipLaunchKernelGGL((k_pt_layer<Si, So, 1, 1>), grid, blk, 0, st, a, n);
    else if (a.cin == 1) hipLaunchKernelGGL((k_pt_layer<Si, So, 1, 2>), grid, blk, 0, st, a, n);
    else if (a.cout == 1) hipLaunchKernelGGL((k_pt_layer<Si, So, 2, 1>), grid, blk, 0, st, a, n);
    else hipLaunchKernelGGL((k_pt_layer<Si, So, 2, 2>), grid, blk, 0, st, a, n);
}

void launch_pt_layer(hipStream_t st, const PtArgs& a, int in_prec, int out_prec, int nrhs) {
    const bool ob = out_prec == P_BH;
    if (in_prec == P_BH) {
        if (ob) launch_pt_layer_t<SBH, SBH>(st, a, nrhs);
        else launch_pt_layer_t<SBH, SF32>(st, a, nrhs);
    } else if (in_prec == P_BF16) {
        if (ob) launch_pt_layer_t<SBF16, SBH>(st, a, nrhs);
        else launch_pt_layer_t<SBF16, SF32>(st, a, nrhs);
    } else {
        if (ob) launch_pt_layer_t<SF32, SBH>(st, a, nrhs);
        else launch_pt_layer_t<SF32, SF32>(st, a, nrhs);
    }
}

void launch_pt_wgrad(hipStream_t st, const PtArgs& a, int in_prec, const double* scale, double* grad) {
    const int nb = (int)((a.geo.V + PT_TS - 1) / PT_TS);
    if (in_prec == P_BF16)
        hipLaunchKernelGGL((k_pt_wgrad<SBF16, SF32>), dim3(nb), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_pt_wgrad<SF32, SF32>), dim3(nb), dim3(256), 0, st, a);
    const int ne = 16 * a.kpad, nchunk = (nb + WG_CH - 1) / WG_CH;
    hipLaunchKernelGGL(k_pt_wgrad_sum1, dim3((ne + 255) / 256, nchunk), dim3(256), 0, st, a.partials, nb, ne, a.partials2);
    hipLaunchKernelGGL(k_pt_wgrad_sum2, dim3((ne + 255) / 256), dim3(256), 0, st, a.partials2, nchunk, ne, scale, grad);
}

void launch_pt_loss(hipStream_t st, const Geom& g, const void* y, const void* e, int e_prec, void* gout,
                    double* partials, double* scal, int npairs) {
    const unsigned nb = (unsigned)((g.V + 255) / 256);
    if (e_prec == P_BF16)
        hipLaunchKernelGGL((k_pt_loss<SBF16>), dim3(nb), dim3(256), 0, st, g, y, e, gout, partials);
    else
        hipLaunchKernelGGL((k_pt_loss<SF32>), dim3(nb), dim3(256), 0, st, g, y, e, gout, partials);
    hipLaunchKernelGGL(k_pt_loss_fin, dim3(1), dim3(256), 0, st, partials, nb, scal, npairs);
}

int pt_blocks(const Geom& g) { return (int)((g.V + PT_TS - 1) / PT_TS); }
int pt_chunks(const Geom& g) { return (pt_blocks(g) + WG_CH - 1) / WG_CH; }

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
