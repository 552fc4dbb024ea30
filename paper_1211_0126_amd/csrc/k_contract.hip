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
// All sums are in FP64 and in a fixed order (bitwise reproducible).

#include <type_traits>

#include "tm_device.h"
#include "tm_kernels.h"

namespace tmq {

// load the six components of spin rows 2h, 2h+1
template <class S>
__device__ __forceinline__ void load_half_spinor(const void* base, long Vs, uint32_t s, int h, cx<double> p[6]);

template <>
__device__ __forceinline__ void load_half_spinor<SF64>(const void* base, long Vs, uint32_t s, int h, cx<double> p[6]) {
#pragma unroll
    for (int k = 0; k < 6; k++) {
        double2 v = ld_plane<double2>(base, Vs, 6 * h + k, s);
        p[k] = {v.x, v.y};
    }
}
template <>
__device__ __forceinline__ void load_half_spinor<SF32>(const void* base, long Vs, uint32_t s, int h, cx<double> p[6]) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
        float4 v = ld_plane<float4>(base, Vs, 3 * h + k, s);
        p[2 * k] = {(double)v.x, (double)v.y};
        p[2 * k + 1] = {(double)v.z, (double)v.w};
    }
}

// conj(i^k) p for a Z4 noise component i^k: a permutation and signs
__device__ __forceinline__ cx<double> z4_conj_times(uint32_t k, cx<double> p) {
    const double re = (k & 1u) ? p.im : p.re;
    const double im = (k & 1u) ? p.re : p.im;
    // k = 0: (re, im); 1: (im, -re); 2: (-re, -im); 3: (-im, re)
    const double sr = (k == 2u || k == 3u) ? -1.0 : 1.0;
    const double si = (k == 1u || k == 2u) ? -1.0 : 1.0;
    return {sr * re, si * im};
}

template <class S, int E>
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
    const void* sol = field_rhs<S>(a.sol, g.Vs, r);
    const uint64_t id = a.ids[r];
    cx<double> acc[3][8];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int e = 0; e < 8; e++) acc[i][e] = {0.0, 0.0};
    for (int y = 0; y < Ly; y++) {
        const uint32_t s = x + Lx * (y + Ly * (z + Lz * t));
        cx<double> S8[8];
        if constexpr (E == 0) {
            cx<double> p[6];
            load_half_spinor<S>(sol, g.Vs, s, h, p);
            const uint64_t bits = noise_bits(a.seed_mixed, id, (uint64_t)g.V, (uint64_t)s);
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int al = 0; al < 4; al++) {
                    cx<double> v = {0.0, 0.0};
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
                load_half_spinor<SF64>(field_rhs<SF64>(a.dsol, g.Vs, r), g.Vs, s, h, u);
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
                const cx<double> w = {ph.x, ph.y};
#pragma unroll
                for (int e = 0; e < 8; e++) acc[i][e] = acc[i][e] + w * S8[e];
            }
        }
    }
    // A[r][t][z][iy][entry][x]: lanes of consecutive x write consecutive
    // elements
#pragma unroll
    for (int i = 0; i < 3; i++) {
        if (i < npy) {
            double2* o = a.A + ((((((size_t)r * Lt + t) * Lz + z) * npy + i) * 16 + 8 * h) * Lx + x);
#pragma unroll
            for (int e = 0; e < 8; e++) o[(size_t)e * Lx] = make_double2(acc[i][e].re, acc[i][e].im);
        }
    }
}

// U psi (fwd) or U^dag psi (!fwd) of one colour vector, times ph
__device__ __forceinline__ void su3_apply_d(const cx<double> U[3][3], bool fwd, double ph, const cx<double> v[3],
                                            cx<double> o[3]) {
#pragma unroll
    for (int i = 0; i < 3; i++) {
        cx<double> acc = {0.0, 0.0};
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
template <class S>
__global__ __launch_bounds__(256) void k_contract_d(ContractArgs a) {
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
    cx<double> acc[3][8];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int e = 0; e < 8; e++) acc[i][e] = {0.0, 0.0};
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
        const double php = (mu == 3 && wrap_p) ? (double)g.t_bc : 1.0;
        const double phm = (mu == 3 && wrap_m) ? (double)g.t_bc : 1.0;
        cx<double> S8[8];
#pragma unroll
        for (int e = 0; e < 8; e++) S8[e] = {0.0, 0.0};
        cx<double> p0[6];
        load_half_spinor<S>(sol, g.Vs, s0, h, p0);
        // S8[4b + al] += sgn sum_k conj(eta_{al k}) v[3b + k] for the noise
        // bits nb: each Z4 code becomes the unit (c, d) = conj(i^k) once and
        // serves both spin rows as two FP64 products
        auto add_z4 = [&](uint64_t nb, const cx<double> v[6], double sgn) {
#pragma unroll
            for (int al = 0; al < 4; al++)
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    const uint32_t code = (uint32_t)(nb >> (2 * (3 * al + k))) & 3u;
                    // conj(i^code): 1, -i, -1, i
                    const double c = code == 0u ? sgn : (code == 2u ? -sgn : 0.0);
                    const double d = code == 1u ? -sgn : (code == 3u ? sgn : 0.0);
#pragma unroll
                    for (int b = 0; b < 2; b++) {
                        const cx<double> x0 = v[3 * b + k];
                        S8[4 * b + al] = {S8[4 * b + al].re + (c * x0.re - d * x0.im),
                                          S8[4 * b + al].im + (c * x0.im + d * x0.re)};
                    }
                }
        };
        const uint64_t b0 = noise_bits(a.seed_mixed, id, V, (uint64_t)s0);
        {
            // forward hop through U_mu(x): +ph+ (U s(x+mu)) conj(eta(x)) and
            // -ph+ (U^dag s(x)) conj(eta(x+mu))
            cx<double> U[3][3], p[6], v[6];
            load_link<GF64, double>(a.gauge64, g.Vs, mu, s0, U);
            load_half_spinor<S>(sol, g.Vs, sp, h, p);
            su3_apply_d(U, true, php, p, v);
            su3_apply_d(U, true, php, p + 3, v + 3);
            add_z4(b0, v, 1.0);
            su3_apply_d(U, false, php, p0, v);
            su3_apply_d(U, false, php, p0 + 3, v + 3);
            add_z4(noise_bits(a.seed_mixed, id, V, (uint64_t)sp), v, -1.0);
        }
        {
            // backward hop through U_mu(x - mu): -ph- (U^dag s(x-mu)) conj(eta(x))
            // and +ph- (U s(x)) conj(eta(x-mu))
            cx<double> U[3][3], p[6], v[6];
            load_link<GF64, double>(a.gauge64, g.Vs, mu, sm, U);
            load_half_spinor<S>(sol, g.Vs, sm, h, p);
            su3_apply_d(U, false, phm, p, v);
            su3_apply_d(U, false, phm, p + 3, v + 3);
            add_z4(b0, v, -1.0);
            su3_apply_d(U, true, phm, p0, v);
            su3_apply_d(U, true, phm, p0 + 3, v + 3);
            add_z4(noise_bits(a.seed_mixed, id, V, (uint64_t)sm), v, 1.0);
        }
#pragma unroll
        for (int i = 0; i < 3; i++) {
            if (i < npy) {
                const double2 ph = a.phy[i * Ly + y];
                const cx<double> w = {0.25 * ph.x, 0.25 * ph.y};
#pragma unroll
                for (int e = 0; e < 8; e++) acc[i][e] = acc[i][e] + w * S8[e];
            }
        }
    }
    const int rs = r * 4 + mu;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        if (i < npy) {
            double2* o = a.A + ((((((size_t)rs * Lt + t) * Lz + z) * npy + i) * 16 + 8 * h) * Lx + x);
#pragma unroll
            for (int e = 0; e < 8; e++) o[(size_t)e * Lx] = make_double2(acc[i][e].re, acc[i][e].im);
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
    const double2* in = a.A + (((((size_t)r * Lt + t) * Lz + z) * npy + iy) * 16 + e) * Lx;
    for (int x = 0; x < Lx; x++) {
        const double2 v = in[x];
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
    else if (a.est == 0)
        run_a(std::integral_constant<int, 0>{});
    const long nb = 16L * a.npy * g.L[2] * g.L[3];
    hipLaunchKernelGGL(k_contract_b, dim3((unsigned)((nb + 255) / 256), (unsigned)a.nrhs), dim3(256), 0, st, a);
    const long nc = 16L * a.n_mom * g.L[3];
    hipLaunchKernelGGL(k_contract_c, dim3((unsigned)((nc + 255) / 256), (unsigned)a.nrhs), dim3(256), 0, st, a);
}

// ---------------------------------------------------------------------------
// Projection onto all L^3 momenta (the paper's FFT step): the site matrices
// S_{ba}(x) = sum_c s_{bc}(x) conj(eta_{ac}(x)) of the standard loop are
// written out, transformed along x, y and z by direct DFTs of length L
// (phases from a table exp(-2 pi i m / L)), then traced with each Gamma_n.
// Layout of the site and spectrum buffers: [r][t][z][y][x][16], entry
// 4 b + a.
// ---------------------------------------------------------------------------
template <class S>
__global__ __launch_bounds__(256) void k_site_matrix(ContractArgs a, double2* out) {
    const Geom& g = a.geo;
    const long tid = (long)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (tid >= 2 * g.V) return;
    const int h = tid >= g.V ? 1 : 0;
    const uint32_t s = (uint32_t)(tid - h * g.V);
    cx<double> p[6];
    load_half_spinor<S>(field_rhs<S>(a.sol, g.Vs, r), g.Vs, s, h, p);
    const uint64_t bits = noise_bits(a.seed_mixed, a.ids[r], (uint64_t)g.V, (uint64_t)s);
    double2* o = out + ((size_t)r * g.V + s) * 16 + 8 * h;
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
        for (int al = 0; al < 4; al++) {
            cx<double> v = {0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 3; c++)
                v = v + z4_conj_times((uint32_t)(bits >> (2 * (3 * al + c))) & 3u, p[3 * b + c]);
            o[4 * b + al] = make_double2(v.re, v.im);
        }
}

// out[.., k, ..] = sum_j in[.., j, ..] tw[(k j) mod L] along one axis of
// length L <= kDftMaxL whose elements are `stride` double2 apart (stride a
// multiple of 16).  A block takes one line group of 16 consecutive inner
// elements: it stages the L x 16 tile and the phases in LDS (each element
// read once from memory); power-of-two lengths are transformed in place by
// radix-2 passes, other lengths by direct sums, each lane forming outputs
// (k, c) from LDS.
constexpr int kDftMaxL = 128;  // 34 KB of LDS at the largest L
__global__ __launch_bounds__(256) void k_dft_axis(const double2* in, double2* out, int L, long stride,
                                                  const double2* tw) {
    extern __shared__ double2 lds[];  // L * 16 tile entries, then L phases
    double2* tile = lds;
    double2* ph = lds + L * 16;
    const long nchunk = stride / 16;
    const long outer = (long)blockIdx.x / nchunk;
    const long base = outer * L * stride + ((long)blockIdx.x % nchunk) * 16;
    const int n = L * 16;
    const bool pow2 = (L & (L - 1)) == 0;
    int lg = 0;
    while ((1 << lg) < L) lg++;
    for (int idx = threadIdx.x; idx < n; idx += 256) {
        const int jj = idx >> 4;
        // power-of-two lengths: stored in bit-reversed order for the radix-2 passes
        const int at = pow2 ? (int)(__brev((unsigned)jj) >> (32 - lg)) : jj;
        tile[(lg == 0 ? jj : at) * 16 + (idx & 15)] = in[base + (long)jj * stride + (idx & 15)];
    }
    for (int idx = threadIdx.x; idx < L; idx += 256) ph[idx] = tw[idx];
    __syncthreads();
    if (pow2) {
        // iterative radix-2 decimation in time: log2 L passes of L/2 x 16
        // butterflies, twiddle exp(-2 pi i pos / len) = ph[pos * L / len]
        for (int len = 2; len <= L; len <<= 1) {
            const int half = len >> 1, step = L / len;
            for (int b = threadIdx.x; b < (L >> 1) * 16; b += 256) {
                const int c = b & 15, qb = b >> 4;
                const int i0 = (qb / half) * len + qb % half, i1 = i0 + half;
                const double2 w = ph[(qb % half) * step];
                const double2 u = tile[i0 * 16 + c], v = tile[i1 * 16 + c];
                const cx<double> wv = cx<double>{w.x, w.y} * cx<double>{v.x, v.y};
                tile[i0 * 16 + c] = make_double2(u.x + wv.re, u.y + wv.im);
                tile[i1 * 16 + c] = make_double2(u.x - wv.re, u.y - wv.im);
            }
            __syncthreads();
        }
        for (int o = threadIdx.x; o < n; o += 256) out[base + (long)(o >> 4) * stride + (o & 15)] = tile[o];
        return;
    }
    for (int o = threadIdx.x; o < n; o += 256) {
        const int k = o >> 4, c = o & 15;
        cx<double> acc = {0.0, 0.0};
        int m = 0;
        for (int jj = 0; jj < L; jj++) {
            const double2 v = tile[jj * 16 + c];
            const double2 w = ph[m];
            acc = acc + cx<double>{w.x, w.y} * cx<double>{v.x, v.y};
            m += k;
            if (m >= L) m -= L;
        }
        out[base + (long)k * stride + c] = make_double2(acc.re, acc.im);
    }
}

// loops[r][n][m][t] = sum_a Gamma_n[a][col] S~_{col a}(t, m), m = kx + Lx (ky + Ly kz):
// one lane per (m, t) with t fastest reads its 16 spectrum entries (one
// contiguous 256-byte block) and writes all 16 Gamma traces, so each write
// instruction of a wave covers consecutive t
__global__ __launch_bounds__(256) void k_trace_all(ContractArgs a, const double2* spec, double2* out) {
    const Geom& g = a.geo;
    const long V3 = (long)g.L[0] * g.L[1] * g.L[2];
    const int Lt = g.L[3];
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= V3 * Lt) return;
    const int t = (int)(i % Lt);
    const long m = i / Lt;
    const double2* e = spec + (((size_t)r * Lt + t) * V3 + m) * 16;
    double2* o = out + (size_t)a.out_slot[r] * a.out_stride + m * Lt + t;
#pragma unroll
    for (int gn = 0; gn < 16; gn++) {
        cx<double> tr = {0.0, 0.0};
#pragma unroll
        for (int al = 0; al < 4; al++) {
            // the lane's 256-byte block stays in the caches across the 16 traces
            const double2 v = e[a.gam_col[gn * 4 + al] * 4 + al];
            tr = tr + z4_value<double>((uint32_t)a.gam_ph[gn * 4 + al]) * cx<double>{v.x, v.y};
        }
        o[(size_t)gn * V3 * Lt] = make_double2(tr.re, tr.im);
    }
}

void launch_contract_all_momenta(hipStream_t st, const ContractArgs& a, int xprec, double2* buf0, double2* buf1,
                                 const double2* tw) {
    const Geom& g = a.geo;
    const long nsite = 2L * g.V;
    dim3 gs((unsigned)((nsite + 255) / 256), (unsigned)a.nrhs);
    if (xprec == P_F64)
        hipLaunchKernelGGL(k_site_matrix<SF64>, gs, dim3(256), 0, st, a, buf0);
    else
        hipLaunchKernelGGL(k_site_matrix<SF32>, gs, dim3(256), 0, st, a, buf0);
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2];
    // one block per line group of 16 inner elements: nrhs * V / L blocks per
    // axis; phase tables back to back: x, y, z
    auto blocks = [&](int L) { return dim3((unsigned)((long)a.nrhs * g.V / L)); };
    auto lds = [](int L) { return (unsigned)(sizeof(double2) * 17 * L); };
    hipLaunchKernelGGL(k_dft_axis, blocks(Lx), dim3(256), lds(Lx), st, (const double2*)buf0, buf1, Lx, 16L, tw);
    hipLaunchKernelGGL(k_dft_axis, blocks(Ly), dim3(256), lds(Ly), st, (const double2*)buf1, buf0, Ly, 16L * Lx,
                       tw + Lx);
    hipLaunchKernelGGL(k_dft_axis, blocks(Lz), dim3(256), lds(Lz), st, (const double2*)buf0, buf1, Lz,
                       16L * Lx * Ly, tw + Lx + Ly);
    const long n_el = (long)Lx * Ly * Lz * g.L[3];
    hipLaunchKernelGGL(k_trace_all, dim3((unsigned)((n_el + 255) / 256), (unsigned)a.nrhs), dim3(256), 0, st, a,
                       (const double2*)buf1, a.out);
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
