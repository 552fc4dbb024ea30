// Layout conversion and Z4 noise kernels (gfx950).
//
// Canonical layouts (the ABI's): spinors [rhs][site][12] complex, gauge
// complex128 [site][mu][3][3].  Native layouts: component planes of 16-byte
// vectors with a padded site stride Vs, so that a wave's 64 lanes read
// 1 KiB of contiguous memory per plane.

#include <type_traits>

#include "tm_device.h"
#include "tm_kernels.h"

namespace tmq {

// Canonical <-> native for spinors of one precision: a permutation of E-byte
// complex numbers (E = 16, 8, 4 for F64, F32, F16/BF16), C = 16/E of them per
// 16-byte native vector.
template <int E, bool TO_NATIVE>
__global__ __launch_bounds__(256) void k_permute_spinor(Geom geo, int nrhs, const void* in, void* out) {
    constexpr int C = 16 / E;
    constexpr int NV = 12 / C;
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= geo.V) return;
    using U = typename std::conditional<E == 16, uint4, typename std::conditional<E == 8, uint2, uint32_t>::type>::type;
    const size_t canon_base = ((size_t)r * geo.V + s) * 12;
    const size_t nat_base = (size_t)r * NV * geo.Vs;
    if (TO_NATIVE) {
        const U* cin = (const U*)in + canon_base;
        U* nout = (U*)out;
#pragma unroll
        for (int k = 0; k < NV; k++)
#pragma unroll
            for (int j = 0; j < C; j++) nout[(nat_base + k * geo.Vs + s) * C + j] = cin[k * C + j];
    } else {
        const U* nin = (const U*)in;
        U* cout_ = (U*)out + canon_base;
#pragma unroll
        for (int k = 0; k < NV; k++)
#pragma unroll
            for (int j = 0; j < C; j++) cout_[k * C + j] = nin[(nat_base + k * geo.Vs + s) * C + j];
    }
}

void launch_field_convert(hipStream_t st, const Geom& g, int prec, int nrhs, bool to_native, const void* in,
                          void* out) {
    dim3 grid((unsigned)((g.V + 255) / 256), (unsigned)nrhs);
    switch (prec) {
    case P_F64:
        if (to_native)
            hipLaunchKernelGGL((k_permute_spinor<16, true>), grid, dim3(256), 0, st, g, nrhs, in, out);
        else
            hipLaunchKernelGGL((k_permute_spinor<16, false>), grid, dim3(256), 0, st, g, nrhs, in, out);
        break;
    case P_F32:
        if (to_native)
            hipLaunchKernelGGL((k_permute_spinor<8, true>), grid, dim3(256), 0, st, g, nrhs, in, out);
        else
            hipLaunchKernelGGL((k_permute_spinor<8, false>), grid, dim3(256), 0, st, g, nrhs, in, out);
        break;
    default:
        if (to_native)
            hipLaunchKernelGGL((k_permute_spinor<4, true>), grid, dim3(256), 0, st, g, nrhs, in, out);
        else
            hipLaunchKernelGGL((k_permute_spinor<4, false>), grid, dim3(256), 0, st, g, nrhs, in, out);
        break;
    }
}

// native (F64 or F32 storage) -> canonical complex128
template <class S>
__global__ __launch_bounds__(256) void k_native_to_c128(Geom geo, int nrhs, const void* in, double* out) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= geo.V) return;
    cx<double> p[12];
    load_spinor<S, double>(field_rhs<S>(in, geo.Vs, r), geo.Vs, s, p);
    double2* o = (double2*)out + ((size_t)r * geo.V + s) * 12;
#pragma unroll
    for (int k = 0; k < 12; k++) o[k] = make_double2(p[k].re, p[k].im);
}

void launch_native_to_c128(hipStream_t st, const Geom& g, int prec, int nrhs, const void* in, double* out) {
    dim3 grid((unsigned)((g.V + 255) / 256), (unsigned)nrhs);
    if (prec == P_F64)
        hipLaunchKernelGGL((k_native_to_c128<SF64>), grid, dim3(256), 0, st, g, nrhs, in, out);
    else
        hipLaunchKernelGGL((k_native_to_c128<SF32>), grid, dim3(256), 0, st, g, nrhs, in, out);
}

// Solutions (native, F64 or F32 storage, rhs 0..nrhs-1) -> right-hand sides
// r0.. of the caller's field: canonical [rhs][site][12] complex of out_prec
// (complex128, complex64, or (re, im) pairs of binary16 / bfloat16 as the
// native half planes hold them), or native planes of out_prec
template <class S, typename R>
__global__ __launch_bounds__(256) void k_sol_out(Geom geo, const void* in, void* out, int out_prec, int native,
                                                 int r0) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= geo.V) return;
    cx<R> p[12];
    load_spinor<S, R>(field_rhs<S>(in, geo.Vs, r), geo.Vs, s, p);
    if (native) {
        if (out_prec == P_F64) {
            cx<double> q[12];
#pragma unroll
            for (int k = 0; k < 12; k++) q[k] = {(double)p[k].re, (double)p[k].im};
            store_spinor<SF64, double>(field_rhs<SF64>(out, geo.Vs, r0 + r), geo.Vs, s, q);
        } else {
            cx<float> q[12];
#pragma unroll
            for (int k = 0; k < 12; k++) q[k] = {(float)p[k].re, (float)p[k].im};
            if (out_prec == P_F32)
                store_spinor<SF32, float>(field_rhs<SF32>(out, geo.Vs, r0 + r), geo.Vs, s, q);
            else if (out_prec == P_F16)
                store_spinor<SF16, float>(field_rhs<SF16>(out, geo.Vs, r0 + r), geo.Vs, s, q);
            else
                store_spinor<SBF16, float>(field_rhs<SBF16>(out, geo.Vs, r0 + r), geo.Vs, s, q);
        }
        return;
    }
    const size_t base = ((size_t)(r0 + r) * geo.V + s) * 12;
    if (out_prec == P_F64) {
        double2* o = (double2*)out + base;
#pragma unroll
        for (int k = 0; k < 12; k++) o[k] = make_double2((double)p[k].re, (double)p[k].im);
    } else if (out_prec == P_F32) {
        float2* o = (float2*)out + base;
#pragma unroll
        for (int k = 0; k < 12; k++) o[k] = make_float2((float)p[k].re, (float)p[k].im);
    } else {
        uint32_t* o = (uint32_t*)out + base;
        const bool bf = out_prec == P_BF16;
#pragma unroll
        for (int k = 0; k < 12; k++)
            o[k] = bf ? pack2_bf16((float)p[k].re, (float)p[k].im) : pack2_f16((float)p[k].re, (float)p[k].im);
    }
}

void launch_sol_out(hipStream_t st, const Geom& g, int prec, int nrhs, const void* in, void* out, int out_prec,
                    bool native, int r0) {
    dim3 grid((unsigned)((g.V + 255) / 256), (unsigned)nrhs);
    if (prec == P_F64)
        hipLaunchKernelGGL((k_sol_out<SF64, double>), grid, dim3(256), 0, st, g, in, out, out_prec, native ? 1 : 0,
                           r0);
    else
        hipLaunchKernelGGL((k_sol_out<SF32, float>), grid, dim3(256), 0, st, g, in, out, out_prec, native ? 1 : 0,
                           r0);
}

// canonical complex128 -> native storage S (values rounded to S)
template <class S, typename R>
__global__ __launch_bounds__(256) void k_c128_to_native(Geom geo, int nrhs, const double* in, void* out) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= geo.V) return;
    const double2* c = (const double2*)in + ((size_t)r * geo.V + s) * 12;
    cx<R> p[12];
#pragma unroll
    for (int k = 0; k < 12; k++) p[k] = {(R)c[k].x, (R)c[k].y};
    store_spinor<S, R>(field_rhs<S>(out, geo.Vs, r), geo.Vs, s, p);
}

void launch_c128_to_native(hipStream_t st, const Geom& g, int prec, int nrhs, const double* in, void* out) {
    dim3 grid((unsigned)((g.V + 255) / 256), (unsigned)nrhs);
    switch (prec) {
    case P_F64: hipLaunchKernelGGL((k_c128_to_native<SF64, double>), grid, dim3(256), 0, st, g, nrhs, in, out); break;
    case P_F32: hipLaunchKernelGGL((k_c128_to_native<SF32, float>), grid, dim3(256), 0, st, g, nrhs, in, out); break;
    case P_F16: hipLaunchKernelGGL((k_c128_to_native<SF16, float>), grid, dim3(256), 0, st, g, nrhs, in, out); break;
    default: hipLaunchKernelGGL((k_c128_to_native<SBF16, float>), grid, dim3(256), 0, st, g, nrhs, in, out); break;
    }
}

// canonical complex128 (device) -> native F64 (full links) and F32 (rows 0, 1)
__global__ __launch_bounds__(256) void k_gauge_convert(Geom geo, const double2* canon, double2* g64, float4* g32,
                                                       uint4* gbf) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    const int mu = blockIdx.y;
    if (s >= geo.V) return;
    const double2* u = canon + ((size_t)s * 4 + mu) * 9;
    const size_t Vs = geo.Vs;
#pragma unroll
    for (int k = 0; k < 9; k++) g64[((size_t)mu * 9 + k) * Vs + s] = u[k];
#pragma unroll
    for (int k = 0; k < 3; k++)
        g32[((size_t)mu * 3 + k) * Vs + s] =
            make_float4((float)u[2 * k].x, (float)u[2 * k].y, (float)u[2 * k + 1].x, (float)u[2 * k + 1].y);
    // bfloat16 pairs: entries 0-3, 4-7 and 8 (the rest of the last plane zero)
    uint32_t w[12];
#pragma unroll
    for (int k = 0; k < 12; k++) w[k] = k < 9 ? pack2_bf16((float)u[k].x, (float)u[k].y) : 0u;
#pragma unroll
    for (int k = 0; k < 3; k++)
        gbf[((size_t)mu * 3 + k) * Vs + s] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
}

void launch_gauge_convert(hipStream_t st, const Geom& g, const double* canon, void* g64, void* g32, void* gbf) {
    dim3 grid((unsigned)((g.V + 255) / 256), 4);
    hipLaunchKernelGGL(k_gauge_convert, grid, dim3(256), 0, st, g, (const double2*)canon, (double2*)g64, (float4*)g32,
                       (uint4*)gbf);
}

// Z4 sources (Eq. 1) in native storage S, one per id
template <class S, typename R>
__global__ __launch_bounds__(256) void k_noise_native(Geom geo, uint64_t seed_mixed, const uint64_t* ids, void* out) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= geo.V) return;
    const uint64_t h = noise_bits(seed_mixed, ids[r], (uint64_t)geo.V, (uint64_t)s);
    cx<R> e[12];
#pragma unroll
    for (int k = 0; k < 12; k++) e[k] = z4_value<R>((uint32_t)(h >> (2 * k)) & 3u);
    store_spinor<S, R>(field_rhs<S>(out, geo.Vs, r), geo.Vs, s, e);
}

void launch_noise_native(hipStream_t st, const Geom& g, int prec, uint64_t seed_mixed, const uint64_t* ids, int nrhs,
                         void* out) {
    dim3 grid((unsigned)((g.V + 255) / 256), (unsigned)nrhs);
    switch (prec) {
    case P_F64: hipLaunchKernelGGL((k_noise_native<SF64, double>), grid, dim3(256), 0, st, g, seed_mixed, ids, out); break;
    case P_F32: hipLaunchKernelGGL((k_noise_native<SF32, float>), grid, dim3(256), 0, st, g, seed_mixed, ids, out); break;
    case P_F16: hipLaunchKernelGGL((k_noise_native<SF16, float>), grid, dim3(256), 0, st, g, seed_mixed, ids, out); break;
    default: hipLaunchKernelGGL((k_noise_native<SBF16, float>), grid, dim3(256), 0, st, g, seed_mixed, ids, out); break;
    }
}

// Z4 sources as canonical complex128 [nrhs][V][12]
__global__ __launch_bounds__(256) void k_noise_c128(Geom geo, uint64_t seed_mixed, const uint64_t* ids, double2* out) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= geo.V) return;
    const uint64_t h = noise_bits(seed_mixed, ids[r], (uint64_t)geo.V, (uint64_t)s);
    double2* o = out + ((size_t)r * geo.V + s) * 12;
#pragma unroll
    for (int k = 0; k < 12; k++) {
        cx<double> e = z4_value<double>((uint32_t)(h >> (2 * k)) & 3u);
        o[k] = make_double2(e.re, e.im);
    }
}

void launch_noise_c128(hipStream_t st, const Geom& g, uint64_t seed_mixed, const uint64_t* ids, int nrhs, double* out) {
    dim3 grid((unsigned)((g.V + 255) / 256), (unsigned)nrhs);
    hipLaunchKernelGGL(k_noise_c128, grid, dim3(256), 0, st, g, seed_mixed, ids, (double2*)out);
}

}  // namespace tmq
