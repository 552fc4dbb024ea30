// Loop contraction and the TSM combination (gfx950).
//
// For one source the loop is (section 2.3 of the paper, for all insertion
// times as in section 3)
//   L_n(t, p) = f sum_{x in t} exp(-i p.x) Tr[X_n S(x)],
//   S_{ba}(x) = sum_c u_{bc}(x) conj(v_{ac}(x)),
// in one of three forms:
//   est 0 (standard):     u = s, v = eta, X_n = Gamma_n, f = 1,
//                         eta regenerated from the noise hash;
//   est 1 (Eq. 5):        u = v = s, X_n = g5 Gamma_n, f = -2i (2 kappa mu);
//   est 2 (Eq. 6):        u = D s, v = s, X_n = g5 Gamma_n g5, f = 2,
//                         D s = (1 - kappa H) s from the FP64 stencil.
// The one-end forms estimate Tr[X (M_u^{-1} -+ M_d^{-1})] with M_d the
// operator at -mu.  est 3 gives the one-derivative loops of
// psibar Gamma_n Dsym_mu psi, Dsym = (Dfwd - Dbwd)/2, one set per direction:
//   S_{ba}(x) = (1/4) sum_c [f_{bc}(x) conj(eta_{ac}(x)) - s_{bc}(x) conj(g_{ac}(x))],
//   f = U_mu(x) s(x+mu) - U_mu(x-mu)^dag s(x-mu), g the same of eta,
// with the time-boundary factor on hops across t (k_contract_d).  The
// Fourier sum is separable,
// so it is done one axis at a time over the distinct per-axis momentum
// components (3 each for the 27 momenta with |n_i| <= 1):
//   A: per (x, z, t) row, sum over y with the y phases   (reads s once)
//   B: sum over x with the x phases
//   C: sum over z with the z phases and the Gamma traces (each Gamma_n is
//      a phase-signed permutation: 4 terms)
// The sums are in FP64, except stage A of the standard loop of an FP32
// solution: its products with the noise are exact in FP32 and its y sums
// (Ly terms) are taken in FP32, about 1e-7 relative, far below the FP32
// solution's own rounding.  Every sum runs in a fixed order (bitwise
// reproducible).

#include <type_traits>

#include "tm_device.h"
#include "tm_kernels.h"

namespace tmq {

// Plane `plane` of site s where the plane may differ between the lanes of a
// wave (the spin half h of a lane): its offset goes into the per-lane
// offset of the buffer load, not the scalar one (plane * Vs * 16 < 2^32, as
// tm_create bounds Vs).
template <typename T>
__device__ __forceinline__ T ld_plane_lane(const void* base, long Vs, int plane, uint32_t s) {
    const uint32_t off = (s << 4) + (uint32_t)plane * (uint32_t)Vs * 16u;
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(rsrc_of(base), off, 0u, 0));
}

// load the six components of spin rows 2h, 2h+1
template <class S>
__device__ __forceinline__ void load_half_spinor(const void* base, long Vs, uint32_t s, int h, cx<double> p[6]);

template <>
__device__ __forceinline__ void load_half_spinor<SF64>(const void* base, long Vs, uint32_t s, int h, cx<double> p[6]) {
#pragma unroll
    for (int k = 0; k < 6; k++) {
        double2 v = ld_plane_lane<double2>(base, Vs, 6 * h + k, s);
        p[k] = {v.x, v.y};
    }
}
template <>
__device__ __forceinline__ void load_half_spinor<SF32>(const void* base, long Vs, uint32_t s, int h, cx<double> p[6]) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
        float4 v = ld_plane_lane<float4>(base, Vs, 3 * h + k, s);
        p[2 * k] = {(double)v.x, (double)v.y};
        p[2 * k + 1] = {(double)v.z, (double)v.w};
    }
}

// the six components of spin rows 2h, 2h+1 in arithmetic A (FP32 only from
// an FP32 field)
template <class S, typename A>
__device__ __forceinline__ void load_half_spinor_as(const void* base, long Vs, uint32_t s, int h, cx<A> p[6]) {
    if constexpr (std::is_same<A, double>::value) {
        load_half_spinor<S>(base, Vs, s, h, p);
    } else if constexpr (std::is_same<S, SF16>::value) {
        // components 6h .. 6h + 5 of the planes of four packed pairs
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const uint4 v = ld_plane_lane<uint4>(base, Vs, (6 * h) / 4 + k, s);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int c = 4 * ((6 * h) / 4 + k) + j - 6 * h;
                if (c >= 0 && c < 6) p[c] = {f16_to_f32(w[j] & 0xFFFFu), f16_to_f32(w[j] >> 16)};
            }
        }
    } else {
        static_assert(std::is_same<S, SF32>::value, "FP32 sums read FP32 or FP16 solutions");
#pragma unroll
        for (int k = 0; k < 3; k++) {
            float4 v = ld_plane_lane<float4>(base, Vs, 3 * h + k, s);
            p[2 * k] = {v.x, v.y};
            p[2 * k + 1] = {v.z, v.w};
        }
    }
}

// The same from a base address that differs between the lanes of a wave
// (the two half fields of the even-odd solver): plain global loads with
// per-lane 64-bit addresses, since a buffer descriptor must be uniform.
template <class S, typename A>
__device__ __forceinline__ void load_half_spinor_lane(const void* base, long Vs, uint32_t s, int h, cx<A> p[6]) {
    static_assert(std::is_same<A, float>::value, "FP32 sums");
    const uint4* q = (const uint4*)base + s;
    if constexpr (std::is_same<S, SF16>::value) {
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const int pl = (6 * h) / 4 + k;
            const uint4 v = q[(size_t)pl * Vs];
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int c = 4 * pl + j - 6 * h;
                if (c >= 0 && c < 6) p[c] = {f16_to_f32(w[j] & 0xFFFFu), f16_to_f32(w[j] >> 16)};
            }
        }
    } else {
        static_assert(std::is_same<S, SF32>::value, "FP32 or FP16 halves");
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const float4 v = __builtin_bit_cast(float4, q[(size_t)(3 * h + k) * Vs]);
            p[2 * k] = {v.x, v.y};
            p[2 * k + 1] = {v.z, v.w};
        }
    }
}

// conj(i^k) p for a Z4 noise component i^k: a permutation and signs
template <typename A>
__device__ __forceinline__ cx<A> z4_conj_times(uint32_t k, cx<A> p) {
    const A re = (k & 1u) ? p.im : p.re;
    const A im = (k & 1u) ? p.re : p.im;
    // k = 0: (re, im); 1: (im, -re); 2: (-re, -im); 3: (-im, re)
    const A sr = (k == 2u || k == 3u) ? (A)-1 : (A)1;
    const A si = (k == 1u || k == 2u) ? (A)-1 : (A)1;
    return {sr * re, si * im};
}

// With HALVES (standard loop of an FP32 or FP16 solution only): a.sol and
// a.sol_e hold the odd and even half of each solution in the half layout of
// a.hgeo.
template <class S, int E, bool HALVES = false>
__global__ __launch_bounds__(256) void k_contract_a(ContractArgs a) {
    const Geom& g = a.geo;
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    const long nrow = (long)Lx * Lz * Lt;
    const long tid = (long)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (tid >= 2 * nrow) return;
    const int h = tid >= nrow ? 1 : 0;
    const long q = tid - h * nrow;
    const int x = (int)(q % Lx);
    const long q2 = q / Lx;
    const int z = (int)(q2 % Lz);
    const int t = (int)(q2 / Lz);
    const int npy = a.npy;
    static_assert(!HALVES || (E == 0 && (std::is_same<S, SF32>::value || std::is_same<S, SF16>::value)),
                  "halves: standard loop, FP32 or FP16");
    const void* sol = field_rhs<S>(a.sol, HALVES ? a.hgeo.Vs : g.Vs, r);
    const void* sol_e = HALVES ? field_rhs<S>(a.sol_e, a.hgeo.Vs, r) : nullptr;
    const uint64_t id = a.ids[r];
    // the y sums of the standard loop of an FP32 solution in FP32
    using A = typename std::conditional<E == 0 && (std::is_same<S, SF32>::value || std::is_same<S, SF16>::value),
                                        float, double>::type;
    cx<A> acc[3][8];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int e = 0; e < 8; e++) acc[i][e] = {(A)0, (A)0};
    // four sites of the row in flight per lane
#pragma unroll 4
    for (int y = 0; y < Ly; y++) {
        const uint32_t s = x + Lx * (y + Ly * (z + Lz * t));
        cx<A> S8[8];
        if constexpr (E == 0) {
            cx<A> p[6];
            if constexpr (HALVES) {
                const uint32_t hs = s >> 1;  // x/2 + (Lx/2)(y + Ly(z + Lz t)): Lx is even
                load_half_spinor_lane<S, A>(((x + y + z + t) & 1) ? sol : sol_e, a.hgeo.Vs, hs, h, p);
            } else {
                load_half_spinor_as<S, A>(sol, g.Vs, s, h, p);
            }
            const uint64_t bits = noise_bits(a.seed_mixed, id, (uint64_t)g.V, (uint64_t)s);
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int al = 0; al < 4; al++) {
                    cx<A> v = {(A)0, (A)0};
#pragma unroll
                    for (int c = 0; c < 3; c++)
                        v = v + z4_conj_times((uint32_t)(bits >> (2 * (3 * al + c))) & 3u, p[3 * b + c]);
                    S8[4 * b + al] = v;
                }
        } else {
            // v = s (all four spin rows); u = rows 2h, 2h+1 of s or of D s
            cx<double> q[12], u[6];
            load_half_spinor<S>(sol, g.Vs, s, 0, q);
            load_half_spinor<S>(sol, g.Vs, s, 1, q + 6);
            if constexpr (E == 1) {
#pragma unroll
                for (int k = 0; k < 6; k++) u[k] = h ? q[6 + k] : q[k];
            } else {
                load_half_spinor<S>(field_rhs<S>(a.dsol, g.Vs, r), g.Vs, s, h, u);  // (D s in s's precision)
            }
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int al = 0; al < 4; al++) {
                    cx<double> v = {0.0, 0.0};
#pragma unroll
                    for (int c = 0; c < 3; c++) v = v + cmulc(q[3 * al + c], u[3 * b + c]);
                    S8[4 * b + al] = v;
                }
        }
        // fully unrolled with predicates: a runtime bound on i would index
        // acc dynamically and move it to scratch memory
#pragma unroll
        for (int i = 0; i < 3; i++) {
            if (i < npy) {
                const double2 ph = a.phy[i * Ly + y];
                const cx<A> w = {(A)ph.x, (A)ph.y};
#pragma unroll
                for (int e = 0; e < 8; e++) acc[i][e] = acc[i][e] + w * S8[e];
            }
        }
    }
    // A[r][t][z][iy][x][entry]: a lane writes its eight entries in one run,
    // and stage B reads the 16 entries of an x as one run
#pragma unroll
    for (int i = 0; i < 3; i++) {
        if (i < npy) {
            double2* o = a.A + (((((size_t)r * Lt + t) * Lz + z) * npy + i) * Lx + x) * 16 + 8 * h;
#pragma unroll
            for (int e = 0; e < 8; e++) o[e] = make_double2((double)acc[i][e].re, (double)acc[i][e].im);
        }
    }
}

// U psi (fwd) or U^dag psi (!fwd) of one colour vector, times ph
template <typename A>
__device__ __forceinline__ void su3_apply_d(const cx<A> U[3][3], bool fwd, A ph, const cx<A> v[3], cx<A> o[3]) {
#pragma unroll
    for (int i = 0; i < 3; i++) {
        cx<A> acc = {(A)0, (A)0};
#pragma unroll
        for (int k = 0; k < 3; k++) acc = acc + (fwd ? U[i][k] * v[k] : cmulc(U[k][i], v[k]));
        o[i] = ph * acc;
    }
}

// One-derivative loops, stage A: one lane per (x, z, t) row, spin half h
// and direction mu (grid z); the A slice of (source r, direction mu) is
// r * 4 + mu.  The source-side transport is moved onto the solution,
//   sum_c conj((U eta')_{ac}) s_{bc} = sum_k conj(eta'_{ak}) (U^dag s)_{bk},
// so every product with the noise is a Z4 permutation:
//   4 S_{ba} = sum_k [ f_{bk} conj(eta_{ak}(x))
//                      - ph+ (U_mu(x)^dag s(x))_{bk} conj(eta_{ak}(x+mu))
//                      + ph- (U_mu(x-mu) s(x))_{bk} conj(eta_{ak}(x-mu)) ],
//   f = ph+ U_mu(x) s(x+mu) - ph- U_mu(x-mu)^dag s(x-mu).
// An FP32 solution takes FP32 links and FP32 arithmetic (its y sums too,
// about 1e-6 relative); an FP64 one FP64 throughout.
template <class S>
__global__ __launch_bounds__(256) void k_contract_d(ContractArgs a) {
    using A = typename std::conditional<std::is_same<S, SF64>::value, double, float>::type;
    using GL = typename std::conditional<std::is_same<S, SF64>::value, GF64, GF32>::type;
    const void* gl = std::is_same<S, SF64>::value ? a.gauge64 : a.gauge32;
    const Geom& g = a.geo;
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    const long nrow = (long)Lx * Lz * Lt;
    // the source is the fastest grid index: the blocks of all sources on
    // the same rows run together and share the links through L2
    const long tid = (long)blockIdx.y * 256 + threadIdx.x;
    const int r = blockIdx.x;
    const int mu = blockIdx.z;
    if (tid >= 2 * nrow) return;
    const int h = tid >= nrow ? 1 : 0;
    const long q = tid - h * nrow;
    const int x = (int)(q % Lx);
    const long q2 = q / Lx;
    const int z = (int)(q2 % Lz);
    const int t = (int)(q2 / Lz);
    const int npy = a.npy;
    const void* sol = field_rhs<S>(a.sol, g.Vs, r);
    const uint64_t id = a.ids[r];
    const uint64_t V = (uint64_t)g.V;
    cx<A> acc[3][8];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int e = 0; e < 8; e++) acc[i][e] = {(A)0, (A)0};
    for (int y = 0; y < Ly; y++) {
        // neighbour coordinates by selects (a coordinate array indexed by mu
        // would live in scratch memory)
        const uint32_t s0 = x + Lx * (y + Ly * (z + Lz * t));
        const int cmu = mu == 0 ? x : (mu == 1 ? y : (mu == 2 ? z : t));
        const int Lmu = mu == 0 ? Lx : (mu == 1 ? Ly : (mu == 2 ? Lz : Lt));
        const bool wrap_p = cmu + 1 == Lmu, wrap_m = cmu == 0;
        const int up = wrap_p ? 0 : cmu + 1, dn = wrap_m ? Lmu - 1 : cmu - 1;
        const uint32_t sp = (mu == 0 ? up : x) + Lx * ((mu == 1 ? up : y) + Ly * ((mu == 2 ? up : z) + Lz * (mu == 3 ? up : t)));
        const uint32_t sm = (mu == 0 ? dn : x) + Lx * ((mu == 1 ? dn : y) + Ly * ((mu == 2 ? dn : z) + Lz * (mu == 3 ? dn : t)));
        const A php = (mu == 3 && wrap_p) ? (A)g.t_bc : (A)1;
        const A phm = (mu == 3 && wrap_m) ? (A)g.t_bc : (A)1;
        cx<A> S8[8];
#pragma unroll
        for (int e = 0; e < 8; e++) S8[e] = {(A)0, (A)0};
        cx<A> p0[6];
        load_half_spinor_as<S, A>(sol, g.Vs, s0, h, p0);
        // S8[4b + al] += sgn sum_k conj(eta_{al k}) v[3b + k] for the noise
        // bits nb: each Z4 code becomes the unit (c, d) = conj(i^k) once and
        // serves both spin rows as two FP64 products
        auto add_z4 = [&](uint64_t nb, const cx<A> v[6], A sgn) {
#pragma unroll
            for (int al = 0; al < 4; al++)
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    const uint32_t code = (uint32_t)(nb >> (2 * (3 * al + k))) & 3u;
                    // conj(i^code): 1, -i, -1, i
                    const A c = code == 0u ? sgn : (code == 2u ? -sgn : (A)0);
                    const A d = code == 1u ? -sgn : (code == 3u ? sgn : (A)0);
#pragma unroll
                    for (int b = 0; b < 2; b++) {
                        const cx<A> x0 = v[3 * b + k];
                        S8[4 * b + al] = {S8[4 * b + al].re + (c * x0.re - d * x0.im),
                                          S8[4 * b + al].im + (c * x0.im + d * x0.re)};
                    }
                }
        };
        const uint64_t b0 = noise_bits(a.seed_mixed, id, V, (uint64_t)s0);
        {
            // forward hop through U_mu(x): +ph+ (U s(x+mu)) conj(eta(x)) and
            // -ph+ (U^dag s(x)) conj(eta(x+mu))
            cx<A> U[3][3], p[6], v[6];
            load_link<GL, A>(gl, g.Vs, mu, s0, U);
            load_half_spinor_as<S, A>(sol, g.Vs, sp, h, p);
            su3_apply_d(U, true, php, p, v);
            su3_apply_d(U, true, php, p + 3, v + 3);
            add_z4(b0, v, (A)1);
            su3_apply_d(U, false, php, p0, v);
            su3_apply_d(U, false, php, p0 + 3, v + 3);
            add_z4(noise_bits(a.seed_mixed, id, V, (uint64_t)sp), v, (A)-1);
        }
        {
            // backward hop through U_mu(x - mu): -ph- (U^dag s(x-mu)) conj(eta(x))
            // and +ph- (U s(x)) conj(eta(x-mu))
            cx<A> U[3][3], p[6], v[6];
            load_link<GL, A>(gl, g.Vs, mu, sm, U);
            load_half_spinor_as<S, A>(sol, g.Vs, sm, h, p);
            su3_apply_d(U, false, phm, p, v);
            su3_apply_d(U, false, phm, p + 3, v + 3);
            add_z4(b0, v, (A)-1);
            su3_apply_d(U, true, phm, p0, v);
            su3_apply_d(U, true, phm, p0 + 3, v + 3);
            add_z4(noise_bits(a.seed_mixed, id, V, (uint64_t)sm), v, (A)1);
        }
#pragma unroll
        for (int i = 0; i < 3; i++) {
            if (i < npy) {
                const double2 ph = a.phy[i * Ly + y];
                const cx<A> w = {(A)(0.25 * ph.x), (A)(0.25 * ph.y)};
#pragma unroll
                for (int e = 0; e < 8; e++) acc[i][e] = acc[i][e] + w * S8[e];
            }
        }
    }
    const int rs = r * 4 + mu;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        if (i < npy) {
            double2* o = a.A + (((((size_t)rs * Lt + t) * Lz + z) * npy + i) * Lx + x) * 16 + 8 * h;
#pragma unroll
            for (int e = 0; e < 8; e++) o[e] = make_double2((double)acc[i][e].re, (double)acc[i][e].im);
        }
    }
}

__global__ __launch_bounds__(256) void k_contract_b(ContractArgs a) {
    const Geom& g = a.geo;
    const int Lx = g.L[0], Lz = g.L[2], Lt = g.L[3];
    const int npy = a.npy, npx = a.npx;
    const long n = 16L * npy * Lz * Lt;
    const long tid = (long)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (tid >= n) return;
    const int e = (int)(tid % 16);
    long q = tid / 16;
    const int iy = (int)(q % npy);
    q /= npy;
    const int z = (int)(q % Lz);
    const int t = (int)(q / Lz);
    cx<double> acc[3];
#pragma unroll
    for (int i = 0; i < 3; i++) acc[i] = {0.0, 0.0};
    // the 16 lanes of one (iy, z, t) read the 16 entries of an x together
    const double2* in = a.A + ((((size_t)r * Lt + t) * Lz + z) * npy + iy) * Lx * 16 + e;
    for (int x = 0; x < Lx; x++) {
        const double2 v = in[(size_t)x * 16];
        const cx<double> vv = {v.x, v.y};
#pragma unroll
        for (int i = 0; i < 3; i++) {
            if (i < npx) {
                const double2 ph = a.phx[i * Lx + x];
                acc[i] = acc[i] + cx<double>{ph.x, ph.y} * vv;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 3; i++)
        if (i < npx)
            a.B[(((((size_t)r * Lt + t) * Lz + z) * npx + i) * npy + iy) * 16 + e] =
                make_double2(acc[i].re, acc[i].im);
}

__global__ __launch_bounds__(256) void k_contract_c(ContractArgs a) {
    const Geom& g = a.geo;
    const int Lz = g.L[2], Lt = g.L[3];
    const int npx = a.npx, npy = a.npy;
    const long n = 16L * a.n_mom * Lt;
    const long tid = (long)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (tid >= n) return;
    const int gn = (int)(tid % 16);
    long q = tid / 16;
    const int m = (int)(q % a.n_mom);
    const int t = (int)(q / a.n_mom);
    const int ix = a.mom_idx[3 * m], iy = a.mom_idx[3 * m + 1], iz = a.mom_idx[3 * m + 2];
    cx<double> acc = {0.0, 0.0};
    for (int z = 0; z < Lz; z++) {
        const double2* bz = a.B + (((((size_t)r * Lt + t) * Lz + z) * npx + ix) * npy + iy) * 16;
        cx<double> tr = {0.0, 0.0};
#pragma unroll
        for (int al = 0; al < 4; al++) {
            const int be = a.gam_col[gn * 4 + al];
            const double2 v = bz[be * 4 + al];
            const cx<double> ph = z4_value<double>((uint32_t)a.gam_ph[gn * 4 + al]);
            tr = tr + ph * cx<double>{v.x, v.y};
        }
        const double2 pz = a.phz[iz * Lz + z];
        acc = acc + cx<double>{pz.x, pz.y} * tr;
    }
    acc = cx<double>{a.coef.x, a.coef.y} * acc;
    // slice r of the scratch is direction r % nmu of source r / nmu
    double2* o = a.out + (size_t)a.out_slot[r / a.nmu] * a.out_stride + (size_t)(r % a.nmu) * 16 * a.n_mom * Lt;
    o[((size_t)gn * a.n_mom + m) * Lt + t] = make_double2(acc.re, acc.im);
}

void launch_contract(hipStream_t st, const ContractArgs& a0, int xprec) {
    const Geom& g = a0.geo;
    const long nrow = 2L * g.L[0] * g.L[2] * g.L[3];
    dim3 ga((unsigned)((nrow + 255) / 256), (unsigned)a0.nrhs);
    // stages B and C see one slice per (source, direction)
    ContractArgs a = a0;
    a.nrhs = a0.nrhs * a0.nmu;
    if (a0.est == 3) {
        dim3 gd(ga.y, ga.x, 4);
        if (xprec == P_F64)
            hipLaunchKernelGGL((k_contract_d<SF64>), gd, dim3(256), 0, st, a0);
        else
            hipLaunchKernelGGL((k_contract_d<SF32>), gd, dim3(256), 0, st, a0);
    }
    auto run_a = [&](auto est) {
        constexpr int E = decltype(est)::value;
        if (xprec == P_F64)
            hipLaunchKernelGGL((k_contract_a<SF64, E>), ga, dim3(256), 0, st, a0);
        else
            hipLaunchKernelGGL((k_contract_a<SF32, E>), ga, dim3(256), 0, st, a0);
    };
    if (a.est == 1)
        run_a(std::integral_constant<int, 1>{});
    else if (a.est == 2)
        run_a(std::integral_constant<int, 2>{});
    else if (a.est == 0 && a0.sol_e != nullptr && xprec == P_F16)
        hipLaunchKernelGGL((k_contract_a<SF16, 0, true>), ga, dim3(256), 0, st, a0);
    else if (a.est == 0 && a0.sol_e != nullptr)
        hipLaunchKernelGGL((k_contract_a<SF32, 0, true>), ga, dim3(256), 0, st, a0);
    else if (a.est == 0)
        run_a(std::integral_constant<int, 0>{});
    const long nb = 16L * a.npy * g.L[2] * g.L[3];
    hipLaunchKernelGGL(k_contract_b, dim3((unsigned)((nb + 255) / 256), (unsigned)a.nrhs), dim3(256), 0, st, a);
    const long nc = 16L * a.n_mom * g.L[3];
    hipLaunchKernelGGL(k_contract_c, dim3((unsigned)((nc + 255) / 256), (unsigned)a.nrhs), dim3(256), 0, st, a);
}

// ---------------------------------------------------------------------------
// Projection onto all L^3 momenta (the paper's FFT step) in three passes.
// The Gamma traces are linear, so they are taken at each site, before the
// Fourier transform: T_n(x) = sum_a Gamma_n[a][col] S_{col a}(x) with the
// site matrix S_{ba} = sum_c s_{bc} conj(eta_{ac}) (eta regenerated from the
// hash), and the 16 T_n are transformed along x, y and z by DFTs of length L
// (phases exp(-2 pi i m / L) from a table; radix-2 passes in LDS for powers
// of two, direct sums otherwise):
//   X: traces of a few x lines and their x transform, written as
//      [r][t][z][y][kx][16];
//   Y: the y transform in place of that layout (k_dft_axis);
//   Z: the z transform of T consecutive time slices of one (kx, ky) column,
//      written straight into loops[slot][n][m][t], m = kx + Lx (ky + Ly kz).
// HBM traffic per source: the solution once, three writes and two reads of
// 16 complex per site.
// ---------------------------------------------------------------------------

// LDS tiles [L][W] of W lines (W a power of two >= 16): entry (j, w) at
// j * W + lds_pos(w), the low four bits of w swizzled with the next four so
// that lanes walking either of them hit distinct banks
__device__ __forceinline__ int lds_pos(int w) { return (w & ~15) | ((w ^ (w >> 4)) & 15); }

__device__ __forceinline__ int ilog2(int L) {
    int lg = 0;
    while ((1 << lg) < L) lg++;
    return lg;
}

// In-place radix-2 DFT (decimation in time) along the slow index of a tile
// [L][W] (L and W powers of two) whose rows were stored bit-reversed; ph[m] =
// exp(-2 pi i m / L) (in LDS).
__device__ void lds_dft_pow2(double2* tile, int W, int L, const double2* ph) {
    const int lgW = ilog2(W), lgL = ilog2(L);
    for (int lgl = 1; lgl <= lgL; lgl++) {
        const int half = 1 << (lgl - 1);
        for (int b = threadIdx.x; b < (L >> 1) << lgW; b += blockDim.x) {
            const int c = b & (W - 1), qb = b >> lgW;
            const int j = qb & (half - 1);
            const int i0 = ((qb >> (lgl - 1)) << lgl) + j, i1 = i0 + half;
            const double2 w = ph[j << (lgL - lgl)];
            double2* pu = tile + i0 * W + lds_pos(c);
            double2* pv = tile + i1 * W + lds_pos(c);
            const double2 u = *pu, v = *pv;
            const cx<double> wv = cx<double>{w.x, w.y} * cx<double>{v.x, v.y};
            *pu = make_double2(u.x + wv.re, u.y + wv.im);
            *pv = make_double2(u.x - wv.re, u.y - wv.im);
        }
        __syncthreads();
    }
}

// output k of line c: the transformed tile entry (power of two), else the
// direct sum over the untransformed tile
__device__ __forceinline__ double2 lds_dft_out(const double2* tile, int W, int L, bool pow2, const double2* ph,
                                               int k, int c) {
    const int lc = lds_pos(c);
    if (pow2) return tile[k * W + lc];
    cx<double> acc = {0.0, 0.0};
    int m = 0;
    for (int j = 0; j < L; j++) {
        const double2 v = tile[j * W + lc];
        const double2 w = ph[m];
        acc = acc + cx<double>{w.x, w.y} * cx<double>{v.x, v.y};
        m += k;
        if (m >= L) m -= L;
    }
    return make_double2(acc.re, acc.im);
}

// row of element j in a tile of L rows: bit-reversed for the radix-2 passes
__device__ __forceinline__ int dft_row(int j, bool pow2, int lg) {
    return pow2 && lg > 0 ? (int)(__brev((unsigned)j) >> (32 - lg)) : j;
}

// Gamma_n = g1^b0 g2^b1 g3^b2 g4^b3 of the Euclidean chiral basis as the
// column and phase i^k of each row's one nonzero, built at compile time from
// the four gammas (each a phase-signed permutation, so a product's row a has
// column colB(colA(a)) and phase phA(a) + phB(colA(a)))
struct GammaTable {
    int col[16][4];
    int ph[16][4];
};
constexpr GammaTable gamma_table() {
    // gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = [[0, 1], [1, 0]]
    constexpr int gc[4][4] = {{3, 2, 1, 0}, {3, 2, 1, 0}, {2, 3, 0, 1}, {2, 3, 0, 1}};
    constexpr int gp[4][4] = {{3, 3, 1, 1}, {2, 0, 0, 2}, {3, 1, 1, 3}, {0, 0, 0, 0}};
    GammaTable t{};
    for (int n = 0; n < 16; n++) {
        for (int a = 0; a < 4; a++) {
            t.col[n][a] = a;
            t.ph[n][a] = 0;
        }
        for (int mu = 0; mu < 4; mu++)
            if ((n >> mu) & 1)
                for (int a = 0; a < 4; a++) {
                    const int k = t.col[n][a];
                    t.col[n][a] = gc[mu][k];
                    t.ph[n][a] = (t.ph[n][a] + gp[mu][k]) & 3;
                }
    }
    return t;
}

// i^k p: a permutation and signs
__device__ __forceinline__ cx<double> z4_times(int k, cx<double> p) {
    const double re = (k & 1) ? -p.im : p.re;
    const double im = (k & 1) ? p.re : p.im;
    return (k & 2) ? cx<double>{-re, -im} : cx<double>{re, im};
}

// X pass: block (r, t, z, y0 .. y0 + NL - 1); its sites' 16 Gamma traces
// into the tile [x][NL * 16] (line 16 l + n), the x transform, rows written
// line by line
template <class S>
__global__ __launch_bounds__(256) void k_allmom_x(ContractArgs a, double2* out, const double2* tw, int NL) {
    extern __shared__ double2 lds[];
    const Geom& g = a.geo;
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2];
    const int W = 16 * NL;
    double2* tile = lds;
    double2* ph = lds + Lx * W;
    for (int i = threadIdx.x; i < Lx; i += blockDim.x) ph[i] = tw[i];
    const int r = blockIdx.y;
    const int nyb = Ly / NL;
    const long plane = (long)blockIdx.x / nyb;  // t * Lz + z
    const int y0 = (int)(blockIdx.x % nyb) * NL;
    const bool pow2 = (Lx & (Lx - 1)) == 0;
    const int lg = ilog2(Lx);
    const void* sol = field_rhs<S>(a.sol, g.Vs, r);
    const uint64_t id = a.ids[r];
    for (int i = threadIdx.x; i < Lx * NL; i += blockDim.x) {
        const int x = pow2 ? (i & (Lx - 1)) : i % Lx, l = pow2 ? (i >> lg) : i / Lx;
        const uint32_t s = (uint32_t)(x + (long)Lx * (y0 + l + (long)Ly * plane));
        cx<double> p[12];
        load_half_spinor<S>(sol, g.Vs, s, 0, p);
        load_half_spinor<S>(sol, g.Vs, s, 1, p + 6);
        const uint64_t bits = noise_bits(a.seed_mixed, id, (uint64_t)g.V, (uint64_t)s);
        cx<double> Sm[16];
#pragma unroll
        for (int b = 0; b < 4; b++)
#pragma unroll
            for (int al = 0; al < 4; al++) {
                cx<double> v = {0.0, 0.0};
#pragma unroll
                for (int c = 0; c < 3; c++)
                    v = v + z4_conj_times((uint32_t)(bits >> (2 * (3 * al + c))) & 3u, p[3 * b + c]);
                Sm[4 * b + al] = v;
            }
        // the basis is fixed at compile time: each trace is a sum of four
        // entries of S with signs and swaps
        constexpr GammaTable G = gamma_table();
        double2* o = tile + dft_row(x, pow2, lg) * W;
#pragma unroll
        for (int n = 0; n < 16; n++) {
            cx<double> tr = {0.0, 0.0};
#pragma unroll
            for (int al = 0; al < 4; al++) tr = tr + z4_times(G.ph[n][al], Sm[4 * G.col[n][al] + al]);
            o[lds_pos(16 * l + n)] = make_double2(tr.re, tr.im);
        }
    }
    __syncthreads();
    if (pow2) lds_dft_pow2(tile, W, Lx, ph);
    double2* ob = out + (((size_t)r * g.L[3] * Lz + plane) * Ly + y0) * Lx * 16;
    for (int o = threadIdx.x; o < Lx * W; o += blockDim.x) {
        const int n = o & 15, rest = o >> 4;
        const int kx = pow2 ? (rest & (Lx - 1)) : rest % Lx, l = pow2 ? (rest >> lg) : rest / Lx;
        ob[((size_t)l * Lx + kx) * 16 + n] = lds_dft_out(tile, W, Lx, pow2, ph, kx, 16 * l + n);
    }
}

// out[.., k, ..] = sum_j in[.., j, ..] tw[(k j) mod L] along one axis of
// length L <= kDftMaxL whose elements are `stride` double2 apart (stride a
// multiple of 16).  A block takes one line group of 16 consecutive inner
// elements: it stages the L x 16 tile in LDS (each element read once from
// memory); power-of-two lengths are transformed in place by radix-2 passes,
// other lengths by direct sums, each lane forming outputs (k, c) from LDS.
// in may equal out (each block reads its lines before writing them).
constexpr int kDftMaxL = 128;  // 32 KB of LDS at the largest L
__global__ __launch_bounds__(256) void k_dft_axis(const double2* in, double2* out, int L, long stride,
                                                  const double2* tw) {
    extern __shared__ double2 lds[];  // L * 16 tile entries, then L phases
    double2* tile = lds;
    double2* ph = lds + L * 16;
    const long nchunk = stride / 16;
    const long outer = (long)blockIdx.x / nchunk;
    const long base = outer * L * stride + ((long)blockIdx.x % nchunk) * 16;
    const bool pow2 = (L & (L - 1)) == 0;
    const int lg = ilog2(L);
    for (int idx = threadIdx.x; idx < L * 16; idx += 256) {
        const int jj = idx >> 4;
        tile[dft_row(jj, pow2, lg) * 16 + (idx & 15)] = in[base + (long)jj * stride + (idx & 15)];
    }
    for (int idx = threadIdx.x; idx < L; idx += 256) ph[idx] = tw[idx];
    __syncthreads();
    if (pow2) lds_dft_pow2(tile, 16, L, ph);
    for (int o = threadIdx.x; o < L * 16; o += 256)
        out[base + (long)(o >> 4) * stride + (o & 15)] = lds_dft_out(tile, 16, L, pow2, ph, o >> 4, o & 15);
}

// Z pass: block (r, channel half, t0 .. t0 + T - 1, ky, kx) of the
// [r][t][z][ky][kx][16] spectrum; the z transform of its T * 8 lines (line
// 8 tt + c), written with t fastest into loops[slot][n][m][t] (runs of T
// consecutive t)
__global__ __launch_bounds__(256) void k_allmom_z(ContractArgs a, const double2* in, const double2* tw, int T) {
    extern __shared__ double2 lds[];
    const Geom& g = a.geo;
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    const long V3 = (long)Lx * Ly * Lz;
    const int W = std::max(16, 8 * T);  // lines, padded to the swizzle's group of 16
    double2* tile = lds;
    double2* ph = lds + Lz * W;
    const int r = blockIdx.y;
    const long XY = (long)Lx * Ly;
    const long col = blockIdx.x % XY;  // kx + Lx ky
    const int t0 = (int)((blockIdx.x / XY) % (Lt / T)) * T;
    const int c0 = (int)(blockIdx.x / (XY * (Lt / T))) * 8;
    const bool pow2 = (Lz & (Lz - 1)) == 0;
    const int lg = ilog2(Lz), lgT = ilog2(T);
    for (int i = threadIdx.x; i < Lz; i += blockDim.x) ph[i] = tw[i];
    const double2* ib = in + ((size_t)r * Lt * Lz * XY + col) * 16 + c0;
    for (int i = threadIdx.x; i < Lz * 8 * T; i += blockDim.x) {
        const int c = i & 7, rest = i >> 3;
        const int tt = rest & (T - 1), z = rest >> lgT;
        tile[dft_row(z, pow2, lg) * W + lds_pos(8 * tt + c)] = ib[(((size_t)(t0 + tt) * Lz + z) * XY) * 16 + c];
    }
    __syncthreads();
    if (pow2) lds_dft_pow2(tile, W, Lz, ph);
    double2* ob = a.out + (size_t)a.out_slot[r] * a.out_stride + col * Lt + t0;
    for (int o = threadIdx.x; o < Lz * 8 * T; o += blockDim.x) {
        const int tt = o & (T - 1), rest = o >> lgT;
        const int c = rest & 7, kz = rest >> 3;
        ob[(size_t)(c0 + c) * V3 * Lt + (size_t)kz * XY * Lt + tt] =
            lds_dft_out(tile, W, Lz, pow2, ph, kz, 8 * tt + c);
    }
}

// largest power of two <= cap dividing n with a tile of L rows x w k lines
// within 32 KB of LDS (several blocks per CU)
static int pick_lines(int n, int L, int w, int cap) {
    int k = 1;
    while (k * 2 <= cap && n % (k * 2) == 0 && (size_t)L * w * (k * 2) * sizeof(double2) <= (32u << 10)) k *= 2;
    return k;
}

void launch_contract_all_momenta(hipStream_t st, const ContractArgs& a, int xprec, double2* buf0, double2* buf1,
                                 const double2* tw) {
    const Geom& g = a.geo;
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    const int NL = pick_lines(Ly, Lx, 16, 8);
    const unsigned lds_x = (unsigned)(sizeof(double2) * (Lx * 16 * NL + Lx));
    const dim3 gx((unsigned)((long)Lt * Lz * (Ly / NL)), (unsigned)a.nrhs);
    // one thread per site of the block's lines (at least a wave, at most 256)
    const unsigned bx = (unsigned)std::min(256, std::max(64, (Lx * NL + 63) / 64 * 64));
    if (xprec == P_F64)
        hipLaunchKernelGGL(k_allmom_x<SF64>, gx, dim3(bx), lds_x, st, a, buf0, tw, NL);
    else
        hipLaunchKernelGGL(k_allmom_x<SF32>, gx, dim3(bx), lds_x, st, a, buf0, tw, NL);
    // y transform in place: one block per (r, t, z, kx) line group
    hipLaunchKernelGGL(k_dft_axis, dim3((unsigned)((long)a.nrhs * g.V / Ly)), dim3(256),
                       (unsigned)(sizeof(double2) * 17 * Ly), st, (const double2*)buf0, buf0, Ly, 16L * Lx, tw + Lx);
    // half the channels per block, T = 8 consecutive time slices: 128-byte
    // runs of the output
    const int T = pick_lines(Lt, Lz, 8, 8);
    const unsigned lds_z = (unsigned)(sizeof(double2) * (Lz * std::max(16, 8 * T) + Lz));
    hipLaunchKernelGGL(k_allmom_z, dim3((unsigned)((long)Lx * Ly * (Lt / T) * 2), (unsigned)a.nrhs), dim3(256),
                       lds_z, st, a, (const double2*)buf0, tw + Lx + Ly, T);
    (void)buf1;
}

// TSM combination of Eq. 4 from the per-source loops ps[j][slot][k]
// (slot 0 LP, 1 HP), k over nl = 16 * n_mom * Lt elements.  Two passes in
// source order: means, then the spread.  out/err: [3][nl] (C, B, T).
__global__ __launch_bounds__(256) void k_tsm_final(const double2* ps, long nl, int n_hp, int n_lp, double2* out,
                                                   double2* err) {
    const long k = (long)blockIdx.x * 256 + threadIdx.x;
    if (k >= nl) return;
    double cr = 0, ci = 0, br = 0, bi = 0;
    for (int j = 0; j < n_hp; j++) {
        double2 lp = ps[((size_t)j * 2 + 0) * nl + k], hp = ps[((size_t)j * 2 + 1) * nl + k];
        cr += hp.x - lp.x;
        ci += hp.y - lp.y;
    }
    for (int j = n_hp; j < n_hp + n_lp; j++) {
        double2 lp = ps[((size_t)j * 2 + 0) * nl + k];
        br += lp.x;
        bi += lp.y;
    }
    if (n_hp > 0) {
        cr /= n_hp;
        ci /= n_hp;
    }
    if (n_lp > 0) {
        br /= n_lp;
        bi /= n_lp;
    }
    double vcr = 0, vci = 0, vbr = 0, vbi = 0;
    if (n_hp > 1) {
        for (int j = 0; j < n_hp; j++) {
            double2 lp = ps[((size_t)j * 2 + 0) * nl + k], hp = ps[((size_t)j * 2 + 1) * nl + k];
            double dr = (hp.x - lp.x) - cr, di = (hp.y - lp.y) - ci;
            vcr += dr * dr;
            vci += di * di;
        }
        vcr /= (double)(n_hp - 1) * n_hp;
        vci /= (double)(n_hp - 1) * n_hp;
    }
    if (n_lp > 1) {
        for (int j = n_hp; j < n_hp + n_lp; j++) {
            double2 lp = ps[((size_t)j * 2 + 0) * nl + k];
            double dr = lp.x - br, di = lp.y - bi;
            vbr += dr * dr;
            vbi += di * di;
        }
        vbr /= (double)(n_lp - 1) * n_lp;
        vbi /= (double)(n_lp - 1) * n_lp;
    }
    out[k] = make_double2(cr, ci);
    out[nl + k] = make_double2(br, bi);
    out[2 * nl + k] = make_double2(cr + br, ci + bi);
    err[k] = make_double2(sqrt(vcr), sqrt(vci));
    err[nl + k] = make_double2(sqrt(vbr), sqrt(vbi));
    err[2 * nl + k] = make_double2(sqrt(vcr + vbr), sqrt(vci + vbi));
}

void launch_tsm_final(hipStream_t st, const double* ps, long nl, int n_hp, int n_lp, double* out, double* err) {
    hipLaunchKernelGGL(k_tsm_final, dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, st, (const double2*)ps, nl, n_hp,
                       n_lp, (double2*)out, (double2*)err);
}

}  // namespace tmq
