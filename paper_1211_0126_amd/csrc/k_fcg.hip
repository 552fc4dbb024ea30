// Flexible CG on M^dag M with the network preconditioner z = N(N^dag(r))
// (Notay 2000; Golub & Ye 1999), FP64 complex scalars.  The stencil inputs
// p and t are stored in a.prec (FP32, FP16 or BF16: the search direction
// and M p as the stored values, so q = M^dag M p and the updates of x and r
// use the same rounded p); q, r, x and z are FP32.
//   F1  t = M p, |t|^2                         -> alpha = <z,r> / |t|^2
//   F2  q = M^dag t (kept), x += alpha p, r -= alpha q, |r|^2 -> stop tests,
//       stagnation test (|r| not below its value five steps earlier)
//   net z = N(N^dag(r))                        (transport layers)
//   F3  <z,q>, <z,r>                           -> beta = -alpha <z,q> / <z,r>_old
//       (Polak-Ribiere, since r_new - r_old = -alpha q), or fallback
//   F4  p = z + beta p   | p = r + beta p (plain CG after fallback) | p = r (restart)
// A source falls back to plain CG (directions restarted from its current
// iterate) when Re<z,r> <= 0, a scalar is not finite, or it stagnates.

#include "tm_kernels.h"
#include "tm_stencil.h"

namespace tmq {

// out = M in (DAG: M^dag in), single right-hand side stored as S, FP32
// arithmetic
template <bool DAG, class S>
__device__ __forceinline__ void fop(const Geom& geo, const void* gauge, float kappa, float tw, const void* in,
                                    uint32_t s, cx<float> out[12]) {
    const Site c = site_coords(geo, s);
    cx<float> acc[1][12], p[12];
    hop_all<DAG, float, S, GF32, 1>(geo, gauge, in, s, c, acc);
    load_spinor<S, float>(in, geo.Vs, s, p);
    diag_combine(p, acc[0], kappa, DAG ? -tw : tw, out);
}

__device__ __forceinline__ bool finite_d(double v) { return v == v && v < 1e300 && v > -1e300; }

// F1: t = M p, alpha = <z,r> / |t|^2 (|t|^2 of t as stored)
template <class S>
__global__ TM_STENCIL(1) void k_fcg_mp(FcgArgs a) {
    __shared__ double sh[4];
    const uint32_t nb = gridDim.x, b = xcd_block(blockIdx.x, nb);
    const uint32_t s = b * 256u + threadIdx.x;
    const int r = blockIdx.y;
    if (!a.scal[r].active) return;
    const long Vs = a.geo.Vs;
    double part = 0;
    if (s < a.geo.V) {
        cx<float> t[12];
        fop<false, S>(a.geo, a.gauge, (float)a.kappa, (float)a.twist, field_rhs<S>(a.p, Vs, r), s, t);
        round_storage<S, float>(t);
        store_spinor<S, float>(field_rhs<S>(a.t, Vs, r), Vs, s, t);
#pragma unroll
        for (int k = 0; k < 12; k++) part += (double)t[k].re * t[k].re + (double)t[k].im * t[k].im;
    }
    double v = block_sum256(part, sh);
    if (threadIdx.x == 0) a.partials[(size_t)r * nb + blockIdx.x] = v;
}

// Block partials of one source in a fixed order; valid in thread 0.
__device__ __forceinline__ double fsum(const double* p, uint32_t n, double* sh) {
    double v = 0;
    for (uint32_t i = threadIdx.x; i < n; i += 256) v += p[i];
    return block_sum256(v, sh);
}

// after F1, one block per source: alpha = <z,r> / |t|^2
__global__ __launch_bounds__(256) void k_fcg_mp_fin(FcgArgs a, uint32_t nb) {
    __shared__ double sh[4];
    const int r = blockIdx.x;
    if (!a.scal[r].active) return;
    const double tt = fsum(a.partials + (size_t)r * nb, nb, sh);
    if (threadIdx.x == 0) {
        FcgScal& q = a.scal[r];
        q.tt = tt;
        q.alpha_re = tt > 0 ? q.zr_re / tt : 0.0;
        q.alpha_im = tt > 0 ? q.zr_im / tt : 0.0;
    }
}

// F2: q = M^dag t, x += alpha p, r -= alpha q, |r|^2, stop and stagnation tests
template <class S>
__global__ TM_STENCIL(1) void k_fcg_upd(FcgArgs a) {
    __shared__ double sh[4];
    const uint32_t nb = gridDim.x, b = xcd_block(blockIdx.x, nb);
    const uint32_t s = b * 256u + threadIdx.x;
    const int r = blockIdx.y;
    if (!a.scal[r].active) return;
    const long Vs = a.geo.Vs;
    double part = 0;
    if (s < a.geo.V) {
        const float ar = (float)a.scal[r].alpha_re, ai = (float)a.scal[r].alpha_im;
        cx<float> q[12], rv[12], pv[12], xv[12];
        fop<true, S>(a.geo, a.gauge, (float)a.kappa, (float)a.twist, field_rhs<S>(a.t, Vs, r), s, q);
        store_spinor<SF32, float>(field_rhs<SF32>(a.q, Vs, r), Vs, s, q);
        void* rp = field_rhs<SF32>(a.r, Vs, r);
        void* xp = field_rhs<SF32>(a.x, Vs, r);
        load_spinor<SF32, float>(rp, Vs, s, rv);
        load_spinor<S, float>(field_rhs<S>(a.p, Vs, r), Vs, s, pv);
        load_spinor<SF32, float>(xp, Vs, s, xv);
        const cx<float> al = {ar, ai};
#pragma unroll
        for (int k = 0; k < 12; k++) {
            xv[k] = xv[k] + al * pv[k];
            rv[k] = rv[k] - al * q[k];
            part += (double)rv[k].re * rv[k].re + (double)rv[k].im * rv[k].im;
        }
        store_spinor<SF32, float>(rp, Vs, s, rv);
        store_spinor<SF32, float>(xp, Vs, s, xv);
    }
    double v = block_sum256(part, sh);
    if (threadIdx.x == 0) a.partials[(size_t)r * nb + blockIdx.x] = v;
}

// after F2, one block per source: stop and stagnation tests
__global__ __launch_bounds__(256) void k_fcg_upd_fin(FcgArgs a, uint32_t nb) {
    __shared__ double sh[4];
    const int r = blockIdx.x;
    if (!a.scal[r].active) return;
    {
        double rrn = fsum(a.partials + (size_t)r * nb, nb, sh);
        if (threadIdx.x == 0) {
            FcgScal& q = a.scal[r];
            q.iters += 1;
            q.rr_prev = q.rr;
            q.rr = rrn;
            const int slot = q.iters % 5;
            q.stagnant = (q.iters >= 5 && !(rrn < q.hist[slot])) ? 1 : 0;
            q.hist[slot] = rrn;
            if (!finite_d(rrn) || !finite_d(q.alpha_re) || !finite_d(q.alpha_im)) {
                q.status = 3;
                q.active = 0;
            } else if (rrn <= q.tol2 * q.bb) {
                q.status = 1;
                q.active = 0;
            } else if (q.maxit >= 0 && q.iters >= q.maxit) {
                q.status = 2;
                q.active = 0;
            }
        }
    }
}

// F3 (and the initial step, init = 1): <z,q>, <z,r>; choose the direction mode
__global__ __launch_bounds__(256) void k_fcg_dot(FcgArgs a, int init) {
    __shared__ double sh[4];
    const uint32_t nb = gridDim.x;
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    const int r = blockIdx.y;
    if (!a.scal[r].active) return;
    const long Vs = a.geo.Vs;
    double zq_re = 0, zq_im = 0, zr_re = 0, zr_im = 0;
    if (s < a.geo.V) {
        cx<float> z[12], q[12], rv[12];
        load_spinor<SF32, float>(field_rhs<SF32>(a.z, Vs, r), Vs, s, z);
        load_spinor<SF32, float>(field_rhs<SF32>(a.r, Vs, r), Vs, s, rv);
        if (!init) load_spinor<SF32, float>(field_rhs<SF32>(a.q, Vs, r), Vs, s, q);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            zr_re += (double)z[k].re * rv[k].re + (double)z[k].im * rv[k].im;
            zr_im += (double)z[k].re * rv[k].im - (double)z[k].im * rv[k].re;
            if (!init) {
                zq_re += (double)z[k].re * q[k].re + (double)z[k].im * q[k].im;
                zq_im += (double)z[k].re * q[k].im - (double)z[k].im * q[k].re;
            }
        }
    }
    double* P = a.partials + (size_t)r * nb * 4;
    double v0 = block_sum256(zr_re, sh);
    double v1 = block_sum256(zr_im, sh);
    double v2 = block_sum256(zq_re, sh);
    double v3 = block_sum256(zq_im, sh);
    if (threadIdx.x == 0) {
        P[blockIdx.x] = v0;
        P[nb + blockIdx.x] = v1;
        P[2 * nb + blockIdx.x] = v2;
        P[3 * nb + blockIdx.x] = v3;
    }
}

// after F3, one block per source: beta and the direction mode, or fallback
__global__ __launch_bounds__(256) void k_fcg_dot_fin(FcgArgs a, uint32_t nb, int init) {
    __shared__ double sh[4];
    const int r = blockIdx.x;
    if (!a.scal[r].active) return;
    const double* P = a.partials + (size_t)r * nb * 4;
    {
        double zrr = fsum(P, nb, sh);
        double zri = fsum(P + nb, nb, sh);
        double zqr = fsum(P + 2 * nb, nb, sh);
        double zqi = fsum(P + 3 * nb, nb, sh);
        if (threadIdx.x == 0) {
            FcgScal& q = a.scal[r];
            const bool bad = !(zrr > 0) || !finite_d(zrr) || !finite_d(zri) || !finite_d(zqr) || !finite_d(zqi);
            if (init) {
                if (q.fell || bad) {
                    q.fell = 1;
                    q.mode = 2;  // p = r
                    q.zr_re = q.rr;
                    q.zr_im = 0;
                } else {
                    q.mode = 3;  // p = z
                    q.zr_re = zrr;
                    q.zr_im = zri;
                }
            } else if (q.fell) {
                // plain CG: beta = |r_new|^2 / |r_old|^2
                q.mode = 1;
                q.beta_re = q.rr / q.zr_re;
                q.beta_im = 0;
                q.zr_re = q.rr;
                q.zr_im = 0;
            } else if (q.stagnant || bad) {
                q.fell = 1;
                q.mode = 2;  // restart: p = r
                q.zr_re = q.rr;
                q.zr_im = 0;
            } else {
                // beta = -alpha <z,q> / zr_old
                const double nr = -(q.alpha_re * zqr - q.alpha_im * zqi);
                const double ni = -(q.alpha_re * zqi + q.alpha_im * zqr);
                const double den = q.zr_re * q.zr_re + q.zr_im * q.zr_im;
                q.beta_re = (nr * q.zr_re + ni * q.zr_im) / den;
                q.beta_im = (ni * q.zr_re - nr * q.zr_im) / den;
                q.mode = 0;
                q.zr_re = zrr;
                q.zr_im = zri;
            }
        }
    }
}

// F4: p = z + beta p (mode 0), r + beta p (1), r (2), z (3); p stored as S
template <class S>
__global__ __launch_bounds__(256) void k_fcg_p(FcgArgs a) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= a.geo.V) return;
    const FcgScal& q = a.scal[r];
    if (!q.active) return;
    const long Vs = a.geo.Vs;
    cx<float> src[12], pv[12];
    load_spinor<SF32, float>(field_rhs<SF32>((q.mode == 0 || q.mode == 3) ? a.z : a.r, Vs, r), Vs, s, src);
    void* pp = field_rhs<S>(a.p, Vs, r);
    if (q.mode <= 1) {
        const cx<float> be = {(float)q.beta_re, (float)q.beta_im};
        load_spinor<S, float>(pp, Vs, s, pv);
#pragma unroll
        for (int k = 0; k < 12; k++) pv[k] = src[k] + be * pv[k];
        store_spinor<S, float>(pp, Vs, s, pv);
    } else {
        store_spinor<S, float>(pp, Vs, s, src);
    }
}

// init: x = 0, |b|^2 (r holds b = M^dag eta), scalars
__global__ __launch_bounds__(256) void k_fcg_init(FcgArgs a) {
    __shared__ double sh[4];
    const uint32_t nb = gridDim.x;
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    const int r = blockIdx.y;
    const long Vs = a.geo.Vs;
    double part = 0;
    if (s < a.geo.V) {
        cx<float> rv[12], z[12];
        load_spinor<SF32, float>(field_rhs<SF32>(a.r, Vs, r), Vs, s, rv);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            part += (double)rv[k].re * rv[k].re + (double)rv[k].im * rv[k].im;
            z[k] = {0.f, 0.f};
        }
        store_spinor<SF32, float>(field_rhs<SF32>(a.x, Vs, r), Vs, s, z);
    }
    double v = block_sum256(part, sh);
    if (threadIdx.x == 0) a.partials[(size_t)r * nb + blockIdx.x] = v;
}

__global__ __launch_bounds__(256) void k_fcg_init_fin(FcgArgs a, uint32_t nb, double tol2, int maxit, int fell) {
    __shared__ double sh[4];
    const int r = blockIdx.x;
    {
        double bb = fsum(a.partials + (size_t)r * nb, nb, sh);
        if (threadIdx.x == 0) {
            FcgScal q = {};
            q.bb = q.rr = q.rr_prev = bb;
            for (int k = 0; k < 5; k++) q.hist[k] = bb;
            q.tol2 = tol2;
            q.maxit = maxit;
            q.fell = fell;
            q.resid_true = -1.0;
            q.status = (bb <= 0 || 1.0 <= tol2) ? 1 : (maxit == 0 ? 2 : 0);
            q.active = q.status == 0;
            a.scal[r] = q;
        }
    }
}

static inline dim3 fgrid(const Geom& g, int n) { return dim3((unsigned)((g.V + 255) / 256), (unsigned)n); }

static inline uint32_t fblocks(const Geom& g) { return (uint32_t)((g.V + 255) / 256); }

// each partial-writing kernel is followed by its one-block-per-source
// finaliser (no device-scope release per block; see the CG kernels)
void launch_fcg_init(hipStream_t st, const FcgArgs& a, double tol2, int maxit, int fell) {
    hipLaunchKernelGGL(k_fcg_init, fgrid(a.geo, a.nrhs), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_fcg_init_fin, dim3((unsigned)a.nrhs), dim3(256), 0, st, a, fblocks(a.geo), tol2, maxit, fell);
}
void launch_fcg_mp(hipStream_t st, const FcgArgs& a) {
    const dim3 gr = fgrid(a.geo, a.nrhs);
    if (a.prec == P_F16)
        hipLaunchKernelGGL(k_fcg_mp<SF16>, gr, dim3(256), 0, st, a);
    else if (a.prec == P_BF16)
        hipLaunchKernelGGL(k_fcg_mp<SBF16>, gr, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_fcg_mp<SF32>, gr, dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_fcg_mp_fin, dim3((unsigned)a.nrhs), dim3(256), 0, st, a, fblocks(a.geo));
}
void launch_fcg_upd(hipStream_t st, const FcgArgs& a) {
    const dim3 gr = fgrid(a.geo, a.nrhs);
    if (a.prec == P_F16)
        hipLaunchKernelGGL(k_fcg_upd<SF16>, gr, dim3(256), 0, st, a);
    else if (a.prec == P_BF16)
        hipLaunchKernelGGL(k_fcg_upd<SBF16>, gr, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_fcg_upd<SF32>, gr, dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_fcg_upd_fin, dim3((unsigned)a.nrhs), dim3(256), 0, st, a, fblocks(a.geo));
}
void launch_fcg_mp_fin(hipStream_t st, const FcgArgs& a, uint32_t nb) {
    hipLaunchKernelGGL(k_fcg_mp_fin, dim3((unsigned)a.nrhs), dim3(256), 0, st, a, nb);
}
void launch_fcg_upd_fin(hipStream_t st, const FcgArgs& a, uint32_t nb) {
    hipLaunchKernelGGL(k_fcg_upd_fin, dim3((unsigned)a.nrhs), dim3(256), 0, st, a, nb);
}
void launch_fcg_dot(hipStream_t st, const FcgArgs& a, int init) {
    hipLaunchKernelGGL(k_fcg_dot, fgrid(a.geo, a.nrhs), dim3(256), 0, st, a, init);
    hipLaunchKernelGGL(k_fcg_dot_fin, dim3((unsigned)a.nrhs), dim3(256), 0, st, a, fblocks(a.geo), init);
}
void launch_fcg_p(hipStream_t st, const FcgArgs& a) {
    const dim3 gr = fgrid(a.geo, a.nrhs);
    if (a.prec == P_F16)
        hipLaunchKernelGGL(k_fcg_p<SF16>, gr, dim3(256), 0, st, a);
    else if (a.prec == P_BF16)
        hipLaunchKernelGGL(k_fcg_p<SBF16>, gr, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_fcg_p<SF32>, gr, dim3(256), 0, st, a);
}

}  // namespace tmq
