// Learned preconditioner: network state, application, loss gradient,
// training (pair harvesting + Adam) and the flexible-CG solve.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <random>
#include <vector>

#include "tm_ctx.h"
#include "tm_learn.h"

using cplx = std::complex<double>;

struct NetState {
    int nl = 0;
    int widths[TM_NET_MAX_LAYERS + 1] = {0};
    std::vector<cplx> W;
    std::vector<size_t> off;              // complex offset of each layer
    std::vector<short*> frag_fwd, frag_adj;  // in the context's fragment pool
    std::vector<int> kpad_fwd, kpad_adj;
};

namespace tmq {

static int kpad_of(int cin) { return (72 * cin + 15) / 16 * 16; }

static uint16_t host_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

static int adj_path(int p) { return p == 0 ? 0 : ((p & 1) ? p + 1 : p - 1); }

// Real B matrix (K x 16) of a layer in the MFMA fragment order
// frag[ks][lane][j] = B[16 ks + 4 (lane / 16) + j][lane % 16].  The adjoint
// layer (cout -> cin) has weights W'[p*][b][a] = W[p][a][b]^dag.
static std::vector<uint16_t> layer_fragments(const cplx* W, int cin, int cout, bool adjoint, int* kpad_out) {
    const int ci = adjoint ? cout : cin, co = adjoint ? cin : cout;
    const int K = 72 * ci, kpad = kpad_of(ci);
    std::vector<float> B((size_t)kpad * 16, 0.f);
    for (int pe = 0; pe < 9; pe++)
        for (int ae = 0; ae < co; ae++)
            for (int be = 0; be < ci; be++)
                for (int so = 0; so < 4; so++)
                    for (int si = 0; si < 4; si++) {
                        cplx w;
                        if (!adjoint) {
                            w = W[((((size_t)pe * cout + ae) * cin + be) * 4 + so) * 4 + si];
                        } else {
                            // effective W'[pe][ae = b][be = a][so][si] = conj(W[p][a][b][si][so])
                            const int p = adj_path(pe);
                            w = std::conj(W[((((size_t)p * cout + be) * cin + ae) * 4 + si) * 4 + so]);
                        }
                        const int k = ((pe * ci + be) * 4 + si) * 2;
                        const int n = (ae * 4 + so) * 2;
                        B[(size_t)k * 16 + n] = (float)w.real();
                        B[(size_t)(k + 1) * 16 + n] = (float)-w.imag();
                        B[(size_t)k * 16 + n + 1] = (float)w.imag();
                        B[(size_t)(k + 1) * 16 + n + 1] = (float)w.real();
                    }
    (void)K;
    std::vector<uint16_t> frag((size_t)(kpad / 16) * 64 * 4);
    for (int ks = 0; ks < kpad / 16; ks++)
        for (int lane = 0; lane < 64; lane++)
            for (int j = 0; j < 4; j++)
                frag[((size_t)ks * 64 + lane) * 4 + j] = host_bf16(B[(size_t)(16 * ks + 4 * (lane / 16) + j) * 16 + lane % 16]);
    *kpad_out = kpad;
    return frag;
}

static bool shape_ok(const tm_net_shape* s) {
    if (!s || s->n_layers < 1 || s->n_layers > TM_NET_MAX_LAYERS) return false;
    if (s->widths[0] != 1 || s->widths[s->n_layers] != 1) return false;
    for (int l = 0; l <= s->n_layers; l++)
        if (s->widths[l] < 1 || s->widths[l] > 2) return false;
    return true;
}

static size_t weight_count(const tm_net_shape* s) {
    size_t n = 0;
    for (int l = 0; l < s->n_layers; l++) n += (size_t)9 * s->widths[l] * s->widths[l + 1] * 16;
    return n;
}

// (Re)build the device fragments from ctx->net->W.
static tm_status upload_fragments(tm_ctx* ctx) {
    NetState* ns = ctx->net;
    for (int l = 0; l < ns->nl; l++) {
        int kf, ka;
        auto ff = layer_fragments(ns->W.data() + ns->off[l], ns->widths[l], ns->widths[l + 1], false, &kf);
        auto fa = layer_fragments(ns->W.data() + ns->off[l], ns->widths[l], ns->widths[l + 1], true, &ka);
        if (ff.size() * 2 > kNetFragBytes || fa.size() * 2 > kNetFragBytes || l >= TM_NET_MAX_LAYERS)
            return set_error(ctx, TM_ENOTSUP, "network layer larger than its fragment slot");
        if ((int)ns->frag_fwd.size() <= l) {
            short* a = (short*)((char*)ctx->net_frag_pool + (size_t)(2 * l) * kNetFragBytes);
            short* b = (short*)((char*)ctx->net_frag_pool + (size_t)(2 * l + 1) * kNetFragBytes);
            ns->frag_fwd.push_back(a);
            ns->frag_adj.push_back(b);
            ns->kpad_fwd.push_back(kf);
            ns->kpad_adj.push_back(ka);
        }
        TM_HIP(hipMemcpyAsync(ns->frag_fwd[l], ff.data(), ff.size() * 2, hipMemcpyHostToDevice, ctx->stream));
        TM_HIP(hipMemcpyAsync(ns->frag_adj[l], fa.data(), fa.size() * 2, hipMemcpyHostToDevice, ctx->stream));
        TM_HIP(hipStreamSynchronize(ctx->stream));  // host vectors go out of scope
    }
    return TM_OK;
}

static tm_status install(tm_ctx* ctx, const tm_net_shape* shape, const cplx* W) {
    if (!shape_ok(shape)) return set_error(ctx, TM_ENOTSUP, "network widths must be 1 at both ends and 1..2 inside");
    delete ctx->net;
    ctx->net = new NetState();
    NetState* ns = ctx->net;
    ns->nl = shape->n_layers;
    for (int l = 0; l <= ns->nl; l++) ns->widths[l] = shape->widths[l];
    size_t n = 0;
    for (int l = 0; l < ns->nl; l++) {
        ns->off.push_back(n);
        n += (size_t)9 * ns->widths[l] * ns->widths[l + 1] * 16;
    }
    ns->W.assign(W, W + n);
    return upload_fragments(ctx);
}

// one layer: in (cin fields per rhs, storage in_prec) -> out (cout fields per
// rhs, storage out_prec: FP32 or bfloat16)
static void layer_launch(tm_ctx* ctx, int l, bool adjoint, const void* in, int in_prec, void* out, int nrhs,
                         int out_prec = P_F32, const FcgScal* gate = nullptr) {
    NetState* ns = ctx->net;
    PtArgs a;
    std::memset(&a, 0, sizeof(a));
    a.geo = ctx->geo;
    a.gauge = ctx->gauge32;
    a.gaugebf = ctx->gaugebf;
    a.cin = adjoint ? ns->widths[l + 1] : ns->widths[l];
    a.cout = adjoint ? ns->widths[l] : ns->widths[l + 1];
    a.kpad = adjoint ? ns->kpad_adj[l] : ns->kpad_fwd[l];
    a.in = in;
    a.out = out;
    a.wfrag = adjoint ? ns->frag_adj[l] : ns->frag_fwd[l];
    a.gate = gate;
    launch_pt_layer(ctx->stream, a, in_prec, out_prec, nrhs);
}

// out = N(in) or N^dag(in); single fields, nrhs of them.  The hidden
// activations are stored as bfloat16 (the precision the mixing GEMM reads
// them in) in the layers' half-split plane order (P_BH); out is written in
// out_prec (FP32 or P_BH).
tm_status net_apply(tm_ctx* ctx, bool adjoint, int nrhs, const void* in, int in_prec, void* out, int out_prec,
                    const FcgScal* gate, int cap) {
    NetState* ns = ctx->net;
    tm_status s = TM_OK;
    const size_t fb = field_bytes(ctx->geo, P_BH, 2 * std::max(nrhs, cap));
    void* A = ws_get(ctx, "net_a", fb, &s);
    void* B = ws_get(ctx, "net_b", fb, &s);
    if (s != TM_OK) return s;
    const void* cur = in;
    int cur_prec = in_prec;
    for (int i = 0; i < ns->nl; i++) {
        const int l = adjoint ? ns->nl - 1 - i : i;
        const bool last = i == ns->nl - 1;
        void* dst = last ? out : ((i % 2 == 0) ? A : B);
        const int dst_prec = last ? out_prec : P_BH;
        prof_begin(ctx, TM_KC_OTHER);
        layer_launch(ctx, l, adjoint, cur, cur_prec, dst, nrhs, dst_prec, gate);
        prof_end(ctx, TM_KC_OTHER, 0.0);
        cur = dst;
        cur_prec = dst_prec;
    }
    TM_HIP(hipGetLastError());
    return TM_OK;
}

// z = N(N^dag(r)), r and z FP32, the middle field bfloat16 (P_BH); right-hand sides
// that gate marks converged or fallen back are skipped (z keeps its values)
tm_status net_precondition(tm_ctx* ctx, int nrhs, const void* r, void* z, const FcgScal* gate, int cap) {
    tm_status s = TM_OK;
    void* tmp = ws_get(ctx, "net_mid", field_bytes(ctx->geo, P_BH, std::max(nrhs, cap)), &s);
    if (s != TM_OK) return s;
    if ((s = net_apply(ctx, true, nrhs, r, P_F32, tmp, P_BH, gate, cap)) != TM_OK) return s;
    return net_apply(ctx, false, nrhs, tmp, P_BH, z, P_F32, gate, cap);
}

bool net_installed(const tm_ctx* ctx) { return ctx->net != nullptr; }
void net_release(tm_ctx* ctx) {
    delete ctx->net;
    ctx->net = nullptr;
}

// Loss and accumulated gradient of a list of pairs (native fields, r in
// r_prec, e in e_prec), into per-layer device gradients [16][kpad] double.
// scal[2] accumulates the loss.  grads must be zeroed by the caller.
// mode 0: error loss |N(r) - e|^2 / |e|^2; mode 1: residual loss
// |M N(r) - r|^2 / |r|^2 (e unused), whose gradient with respect to N(r) is
// M^dag (M N(r) - r).
static tm_status loss_grad_pairs(tm_ctx* ctx, int npairs, const void* r, int r_prec, const void* e, int e_prec,
                                 size_t pair_stride_r, size_t pair_stride_e, std::vector<double*>& grads,
                                 double* scal, int mode = 0) {
    NetState* ns = ctx->net;
    const Geom& g = ctx->geo;
    tm_status s = TM_OK;
    const size_t f2 = field_bytes(g, P_F32, 2);
    std::vector<void*> act(ns->nl + 1);
    for (int l = 1; l <= ns->nl; l++) act[l] = ws_get(ctx, "lg_act" + std::to_string(l), f2, &s);
    void* g0 = ws_get(ctx, "lg_g0", f2, &s);
    void* g1 = ws_get(ctx, "lg_g1", f2, &s);
    const int nb = pt_blocks(g);
    float* partials = (float*)ws_get(ctx, "lg_partials", sizeof(float) * (size_t)nb * 16 * 144, &s);
    double* partials2 = (double*)ws_get(ctx, "lg_partials2", sizeof(double) * (size_t)pt_chunks(g) * 16 * 144, &s);
    double* lpart = (double*)ws_get(ctx, "lg_lpart", sizeof(double) * 2 * ((g.V + 255) / 256), &s);
    void* mw = mode == 1 ? ws_get(ctx, "lg_mw", f2, &s) : nullptr;
    void* gd = mode == 1 ? ws_get(ctx, "lg_gd", f2, &s) : nullptr;
    if (s != TM_OK) return s;
    for (int i = 0; i < npairs; i++) {
        const void* ri = (const char*)r + i * pair_stride_r;
        const void* ei = (const char*)e + i * pair_stride_e;
        // forward, keeping activations
        const void* cur = ri;
        int cur_prec = r_prec;
        for (int l = 0; l < ns->nl; l++) {
            layer_launch(ctx, l, false, cur, cur_prec, act[l + 1], 1);
            cur = act[l + 1];
            cur_prec = P_F32;
        }
        if (mode == 1) {
            launch_apply(ctx->stream, g, P_F32, ctx->gauge32, ctx->lat.kappa, ctx->twist, 0, 1, act[ns->nl], mw, 1,
                         nullptr);
            launch_pt_loss(ctx->stream, g, mw, ri, r_prec, gd, lpart, scal, npairs);
            launch_apply(ctx->stream, g, P_F32, ctx->gauge32, ctx->lat.kappa, ctx->twist, 1, 1, gd, g0, 1, nullptr);
        } else {
            launch_pt_loss(ctx->stream, g, act[ns->nl], ei, e_prec, g0, lpart, scal, npairs);
        }
        // backward
        void* gcur = g0;
        void* gnext = g1;
        for (int l = ns->nl - 1; l >= 0; l--) {
            PtArgs a;
            std::memset(&a, 0, sizeof(a));
            a.geo = g;
            a.gauge = ctx->gauge32;
            a.cin = ns->widths[l];
            a.cout = ns->widths[l + 1];
            a.kpad = ns->kpad_fwd[l];
            a.in = l == 0 ? ri : act[l];
            a.g = gcur;
            a.partials = partials;
            a.partials2 = partials2;
            launch_pt_wgrad(ctx->stream, a, l == 0 ? r_prec : P_F32, scal, grads[l]);
            if (l > 0) {
                layer_launch(ctx, l, true, gcur, P_F32, gnext, 1);
                std::swap(gcur, gnext);
            }
        }
        TM_HIP(hipGetLastError());
    }
    return TM_OK;
}

// complex Wirtinger gradient of a layer from its real [16][kpad] sums
static void layer_grad_to_complex(const double* C, int cin, int cout, int kpad, cplx* G) {
    for (int p = 0; p < 9; p++)
        for (int a = 0; a < cout; a++)
            for (int b = 0; b < cin; b++)
                for (int so = 0; so < 4; so++)
                    for (int si = 0; si < 4; si++) {
                        const int m = (a * 4 + so) * 2;
                        const int k = ((p * cin + b) * 4 + si) * 2;
                        const double rr = C[(size_t)m * kpad + k], ii = C[(size_t)(m + 1) * kpad + k + 1];
                        const double ir = C[(size_t)(m + 1) * kpad + k], ri = C[(size_t)m * kpad + k + 1];
                        G[((((size_t)p * cout + a) * cin + b) * 4 + so) * 4 + si] = cplx(rr + ii, ir - ri);
                    }
}

static tm_status alloc_grads(tm_ctx* ctx, std::vector<double*>& grads) {
    NetState* ns = ctx->net;
    tm_status s = TM_OK;
    grads.resize(ns->nl);
    for (int l = 0; l < ns->nl; l++) {
        grads[l] = (double*)ws_get(ctx, "lg_grad" + std::to_string(l), sizeof(double) * 16 * ns->kpad_fwd[l], &s);
        if (s != TM_OK) return s;
        TM_HIP(hipMemsetAsync(grads[l], 0, sizeof(double) * 16 * ns->kpad_fwd[l], ctx->stream));
    }
    return TM_OK;
}

static tm_status read_grads(tm_ctx* ctx, std::vector<double*>& grads, std::vector<cplx>& G) {
    NetState* ns = ctx->net;
    G.assign(ns->W.size(), cplx(0, 0));
    for (int l = 0; l < ns->nl; l++) {
        std::vector<double> C((size_t)16 * ns->kpad_fwd[l]);
        TM_COPY(C.data(), grads[l], sizeof(double) * C.size(), hipMemcpyDeviceToHost);
        layer_grad_to_complex(C.data(), ns->widths[l], ns->widths[l + 1], ns->kpad_fwd[l], G.data() + ns->off[l]);
    }
    return TM_OK;
}

// ---- workspace bounds (the buffers the paths above carve) ----

// the loss-gradient buffers of loss_grad_pairs and the per-layer gradients,
// for the largest network (TM_NET_MAX_LAYERS layers of width 2)
static size_t ws_loss_buffers(const Geom& g) {
    const size_t f2 = align256(field_bytes(g, P_F32, 2));
    size_t b = (size_t)(TM_NET_MAX_LAYERS + 4) * f2;  // activations, g0, g1, mw, gd
    b += align256(sizeof(float) * (size_t)pt_blocks(g) * 16 * 144);
    b += align256(sizeof(double) * (size_t)pt_chunks(g) * 16 * 144);
    b += align256(sizeof(double) * 2 * (size_t)((g.V + 255) / 256));
    b += (size_t)TM_NET_MAX_LAYERS * align256(sizeof(double) * 16 * kpad_of(2));
    return b;
}

size_t ws_net_apply(const Geom& g, int nrhs) { return 2 * align256(field_bytes(g, P_BH, 2 * nrhs)); }

size_t ws_loss_grad(const Geom& g, int npairs) {
    return 2 * align256(field_bytes(g, P_F32, 1) * npairs) + align256(sizeof(double) * 4) + ws_loss_buffers(g);
}

size_t ws_train(const Geom& g, const Geom& hg, bool eo_ok, int npairs, int nsrc) {
    const size_t f64 = align256(field_bytes(g, P_F64, 1));
    size_t b = 2 * align256(field_bytes(g, P_BF16, 1) * npairs) + align256(sizeof(uint64_t) * nsrc) + f64;
    // the FP64 history solve: six fields, its scalars, the two partial arrays
    b += 6 * f64 + align256(sizeof(CgScal) * kMaxBlock) +
         2 * align256(sizeof(double) * partials_per_rhs(g, hg, eo_ok) * kMaxBlock);
    return b + align256(sizeof(double) * 4) + ws_loss_buffers(g);
}

}  // namespace tmq

using namespace tmq;

extern "C" {

size_t tm_precond_weight_count(const tm_net_shape* shape) { return shape_ok(shape) ? weight_count(shape) : 0; }

tm_status tm_precond_set(tm_ctx* ctx, const tm_net_shape* shape, const double* weights_host) {
    if (!ctx || !shape || !weights_host) return set_error(ctx, TM_EINVAL, "tm_precond_set: null argument");
    if (ctx->sticky) return set_error(ctx, TM_EDEVICE, "context has a sticky device error");
    return install(ctx, shape, (const cplx*)weights_host);
}

tm_status tm_precond_get(tm_ctx* ctx, tm_net_shape* shape_out, double* weights_host) {
    if (!ctx || !shape_out) return set_error(ctx, TM_EINVAL, "tm_precond_get: null argument");
    if (!ctx->net) return set_error(ctx, TM_ESTATE, "no network installed");
    std::memset(shape_out, 0, sizeof(*shape_out));
    shape_out->n_layers = ctx->net->nl;
    for (int l = 0; l <= ctx->net->nl; l++) shape_out->widths[l] = ctx->net->widths[l];
    if (weights_host) std::memcpy(weights_host, ctx->net->W.data(), sizeof(cplx) * ctx->net->W.size());
    return TM_OK;
}

tm_status tm_precond_apply(tm_ctx* ctx, int32_t adjoint, int32_t nrhs, const double* in_dev, double* out_dev) {
    if (!ctx || !in_dev || !out_dev || nrhs < 1 || nrhs > 65535)
        return set_error(ctx, TM_EINVAL, "tm_precond_apply: bad argument");
    if (ctx->sticky) return set_error(ctx, TM_EDEVICE, "context has a sticky device error");
    WsScope scope(ctx);
    if (!ctx->gauge_loaded || !ctx->net) return set_error(ctx, TM_ESTATE, "tm_precond_apply: gauge or network missing");
    tm_status s = TM_OK;
    const size_t fb = field_bytes(ctx->geo, P_F32, nrhs);
    void* a = ws_get(ctx, "pa_in", fb, &s);
    void* b = ws_get(ctx, "pa_out", fb, &s);
    if (s != TM_OK) return s;
    launch_c128_to_native(ctx->stream, ctx->geo, P_F32, nrhs, in_dev, a);
    if ((s = net_apply(ctx, adjoint != 0, nrhs, a, P_F32, b, P_F32, nullptr)) != TM_OK) return s;
    launch_native_to_c128(ctx->stream, ctx->geo, P_F32, nrhs, b, out_dev);
    TM_HIP(hipGetLastError());
    return TM_OK;
}

tm_status tm_precond_loss_grad(tm_ctx* ctx, int32_t npairs, const double* r_dev, const double* e_dev,
                               double* loss_host, double* grad_host) {
    if (!ctx || npairs < 1 || !r_dev || !e_dev || !loss_host || !grad_host)
        return set_error(ctx, TM_EINVAL, "tm_precond_loss_grad: bad argument");
    if (ctx->sticky) return set_error(ctx, TM_EDEVICE, "context has a sticky device error");
    WsScope scope(ctx);
    if (!ctx->gauge_loaded || !ctx->net) return set_error(ctx, TM_ESTATE, "gauge or network missing");
    const Geom& g = ctx->geo;
    tm_status s = TM_OK;
    const size_t f1 = field_bytes(g, P_F32, 1);
    void* r = ws_get(ctx, "plg_r", f1 * npairs, &s);
    void* e = ws_get(ctx, "plg_e", f1 * npairs, &s);
    double* scal = (double*)ws_get(ctx, "plg_scal", sizeof(double) * 4, &s);
    if (s != TM_OK) return s;
    launch_c128_to_native(ctx->stream, g, P_F32, npairs, r_dev, r);
    launch_c128_to_native(ctx->stream, g, P_F32, npairs, e_dev, e);
    TM_HIP(hipMemsetAsync(scal, 0, sizeof(double) * 4, ctx->stream));
    std::vector<double*> grads;
    if ((s = alloc_grads(ctx, grads)) != TM_OK) return s;
    if ((s = loss_grad_pairs(ctx, npairs, r, P_F32, e, P_F32, f1, f1, grads, scal)) != TM_OK) return s;
    double sc[4];
    TM_COPY(sc, scal, sizeof(sc), hipMemcpyDeviceToHost);
    *loss_host = sc[2];
    std::vector<cplx> G;
    if ((s = read_grads(ctx, grads, G)) != TM_OK) return s;
    std::memcpy(grad_host, G.data(), sizeof(cplx) * G.size());
    return TM_OK;
}

// Euclidean chiral gammas (gamma_k = [[0, -i s_k], [i s_k, 0]], gamma_4 =
// [[0, 1], [1, 0]], gamma_5 = diag(1, 1, -1, -1)), g[mu][row][col] with
// mu = 0..3 for gamma_1..gamma_4 and mu = 4 for gamma_5.
static void chiral_gammas(cplx g[5][4][4]) {
    const cplx I(0, 1);
    for (int m = 0; m < 5; m++)
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) g[m][a][b] = 0;
    const cplx sig[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
    for (int k = 0; k < 3; k++)
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                g[k][a][2 + b] = -I * sig[k][a][b];
                g[k][2 + a][b] = I * sig[k][a][b];
            }
    for (int a = 0; a < 2; a++) {
        g[3][a][2 + a] = 1;
        g[3][2 + a][a] = 1;
    }
    for (int a = 0; a < 4; a++) g[4][a][a] = a < 2 ? 1 : -1;
}

// Layer l of the third-order Neumann series of M^{-1}: with A = 1 - M (path
// 0: -2 i kappa mu g5; path +mu: kappa (1 - g_mu); path -mu: kappa (1 + g_mu))
//   layer 0 (1 -> 2): c0 = psi,  c1 = psi + A psi
//   layer 1 (2 -> 2): c0 = c0,   c1 = c0 + A c1
//   layer 2 (2 -> 1): out = c0 + A c1
// so out = psi + A psi + A^2 psi + A^3 psi.  W is added to (layout
// [p][cout][cin][4][4]).
static void neumann_layer(const tm_ctx* ctx, int l, int cin, int cout, cplx* W) {
    cplx g[5][4][4];
    chiral_gammas(g);
    const double kappa = ctx->lat.kappa, tw = ctx->twist;  // tw = 2 kappa mu
    auto at = [&](int p, int a, int b) { return W + (((size_t)p * cout + a) * cin + b) * 16; };
    auto add_identity = [&](cplx* w) {
        for (int i = 0; i < 4; i++) w[i * 4 + i] += 1.0;
    };
    auto add_a = [&](int a, int b) {  // A from channel b into channel a
        cplx* w0 = at(0, a, b);
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) w0[i * 4 + j] += cplx(0, -tw) * g[4][i][j];
        for (int m = 0; m < 4; m++) {
            cplx* wf = at(1 + 2 * m, a, b);
            cplx* wb = at(2 + 2 * m, a, b);
            for (int i = 0; i < 4; i++)
                for (int j = 0; j < 4; j++) {
                    const cplx d = i == j ? 1.0 : 0.0;
                    wf[i * 4 + j] += kappa * (d - g[m][i][j]);
                    wb[i * 4 + j] += kappa * (d + g[m][i][j]);
                }
        }
    };
    if (l == 0) {  // 1 -> 2
        add_identity(at(0, 0, 0));
        add_identity(at(0, 1, 0));
        add_a(1, 0);
    } else if (l == 1) {  // 2 -> 2
        add_identity(at(0, 0, 0));
        add_identity(at(0, 1, 0));
        add_a(1, 1);
    } else {  // 2 -> 1
        add_identity(at(0, 0, 0));
        add_a(0, 1);
    }
}

tm_status tm_precond_train(tm_ctx* ctx, const tm_train_params* P, tm_train_stats* stats) {
    using clk = std::chrono::steady_clock;
    if (!ctx || !P) return set_error(ctx, TM_EINVAL, "tm_precond_train: null argument");
    if (ctx->sticky) return set_error(ctx, TM_EDEVICE, "context has a sticky device error");
    WsScope scope(ctx);
    if (!ctx->gauge_loaded) return set_error(ctx, TM_ESTATE, "tm_precond_train: no gauge field loaded");
    const bool init_only = P->n_pairs == 0 && P->epochs == 0;
    if ((!init_only && (P->n_sources < 1 || P->n_pairs < 1 || P->epochs < 0 || P->batch < 1 || !(P->lr > 0) ||
                        !(P->hp_tol > 0))) ||
        P->init_mode < 0 || P->init_mode > 1 || P->loss_mode < 0 || P->loss_mode > 1)
        return set_error(ctx, TM_EINVAL, "tm_precond_train: bad parameters");
    const Geom& g = ctx->geo;
    tm_status s = TM_OK;
    // initial network (init_mode) plus noise; a network already installed
    // is trained from where it is, unless only the initial one is asked for
    if (!ctx->net || init_only) {
        tm_net_shape sh;
        std::memset(&sh, 0, sizeof(sh));
        sh.n_layers = 3;
        sh.widths[0] = 1;
        sh.widths[1] = 2;
        sh.widths[2] = 2;
        sh.widths[3] = 1;
        std::vector<cplx> W(weight_count(&sh), cplx(0, 0));
        std::mt19937_64 rng(P->init_seed);
        std::normal_distribution<double> nd(0.0, 1.0);
        size_t off = 0;
        for (int l = 0; l < sh.n_layers; l++) {
            const int cin = sh.widths[l], cout = sh.widths[l + 1];
            for (size_t k = 0; k < (size_t)9 * cin * cout * 16; k++)
                W[off + k] = P->init_scale * cplx(nd(rng), nd(rng));
            if (P->init_mode == 0) {
                for (int si = 0; si < 4; si++) W[off + (size_t)si * 4 + si] += 1.0;  // p = 0, a = 0, b = 0
            } else {
                neumann_layer(ctx, l, cin, cout, W.data() + off);
            }
            off += (size_t)9 * cin * cout * 16;
        }
        if ((s = install(ctx, &sh, W.data())) != TM_OK) return s;
    }
    if (init_only) {
        if (stats) std::memset(stats, 0, sizeof(*stats));
        return TM_OK;
    }
    NetState* ns = ctx->net;
    auto t0 = clk::now();

    // ---- harvest pairs ----
    const size_t fbf = field_bytes(g, P_BF16, 1);
    const int npairs_max = P->n_pairs;
    void* R = ws_get(ctx, "tr_r", fbf * npairs_max, &s);
    void* E = ws_get(ctx, "tr_e", fbf * npairs_max, &s);
    uint64_t* ids = (uint64_t*)ws_get(ctx, "tr_ids", sizeof(uint64_t) * P->n_sources, &s);
    void* xstar = ws_get(ctx, "tr_xstar", field_bytes(g, P_F64, 1), &s);
    if (s != TM_OK) return s;
    std::vector<uint64_t> idh(P->n_sources);
    for (int j = 0; j < P->n_sources; j++) idh[j] = (uint64_t)j;
    TM_COPY(ids, idh.data(), sizeof(uint64_t) * P->n_sources, hipMemcpyHostToDevice);
    const uint64_t sm = seed_mix(P->seed);
    const int per_src = (npairs_max + P->n_sources - 1) / P->n_sources;
    int npairs = 0;
    for (int j = 0; j < P->n_sources && npairs < npairs_max; j++) {
        // pass 1: converged solution and residual history
        std::vector<double> hist;
        if ((s = solve_f64_history(ctx, sm, ids + j, P->hp_tol, -1, &hist, xstar, nullptr)) != TM_OK) return s;
        int kmax = 0;
        while (kmax < (int)hist.size() && std::sqrt(hist[kmax]) > P->min_rel_err) kmax++;
        kmax = std::max(kmax, 1);
        const int take = std::min(per_src, npairs_max - npairs);
        std::vector<int> ks;
        for (int i = 0; i < take; i++) ks.push_back((int)((long)i * kmax / take));
        ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
        // pass 2: replay the same iteration and cut pairs at the chosen steps
        PairSink sink{R, E, fbf, npairs, ks, xstar, sm, ids + j};
        if ((s = solve_f64_history(ctx, sm, ids + j, P->hp_tol, ks.back(), nullptr, nullptr, &sink)) != TM_OK)
            return s;
        npairs = sink.next;
    }
    TM_HIP(hipStreamSynchronize(ctx->stream));
    auto t1 = clk::now();

    // ---- Adam ----
    const size_t nw = ns->W.size();
    std::vector<double> m(2 * nw, 0.0), v(2 * nw, 0.0);
    double* scal = (double*)ws_get(ctx, "tr_scal", sizeof(double) * 4, &s);
    if (s != TM_OK) return s;
    std::vector<int> order(npairs);
    for (int i = 0; i < npairs; i++) order[i] = i;
    std::mt19937_64 rng(P->init_seed ^ 0x5DEECE66DULL);
    const double b1 = 0.9, b2 = 0.999, eps = 1e-12;
    int step = 0;
    double first = 0, last = 0;
    const int bsz = std::min(P->batch, std::max(npairs, 1));
    for (int ep = 0; ep < P->epochs; ep++) {
        std::shuffle(order.begin(), order.end(), rng);
        double ep_loss = 0;
        int nsteps = 0;
        for (int b0 = 0; b0 + bsz <= npairs; b0 += bsz) {
            std::vector<double*> grads;
            if ((s = alloc_grads(ctx, grads)) != TM_OK) return s;
            TM_HIP(hipMemsetAsync(scal, 0, sizeof(double) * 4, ctx->stream));
            for (int i = 0; i < bsz; i++) {
                const int pi = order[b0 + i];
                if ((s = loss_grad_pairs(ctx, 1, (const char*)R + pi * fbf, P_BF16, (const char*)E + pi * fbf, P_BF16,
                                         fbf, fbf, grads, scal, P->loss_mode)) != TM_OK)
                    return s;
            }
            double sc[4];
            TM_COPY(sc, scal, sizeof(sc), hipMemcpyDeviceToHost);
            ep_loss += sc[2] / bsz;
            nsteps++;
            std::vector<cplx> G;
            if ((s = read_grads(ctx, grads, G)) != TM_OK) return s;
            step++;
            const double c1 = 1 - std::pow(b1, step), c2 = 1 - std::pow(b2, step);
            for (size_t k = 0; k < nw; k++) {
                // gradient of the mean loss with respect to Re W and Im W
                const double gr = 2 * G[k].real() / bsz, gi = 2 * G[k].imag() / bsz;
                m[2 * k] = b1 * m[2 * k] + (1 - b1) * gr;
                m[2 * k + 1] = b1 * m[2 * k + 1] + (1 - b1) * gi;
                v[2 * k] = b2 * v[2 * k] + (1 - b2) * gr * gr;
                v[2 * k + 1] = b2 * v[2 * k + 1] + (1 - b2) * gi * gi;
                const double dr = P->lr * (m[2 * k] / c1) / (std::sqrt(v[2 * k] / c2) + eps);
                const double di = P->lr * (m[2 * k + 1] / c1) / (std::sqrt(v[2 * k + 1] / c2) + eps);
                ns->W[k] -= cplx(dr, di);
            }
            if ((s = upload_fragments(ctx)) != TM_OK) return s;
        }
        if (nsteps) ep_loss /= nsteps;
        if (ep == 0) first = ep_loss;
        last = ep_loss;
    }
    auto t2 = clk::now();
    if (stats) {
        stats->loss_first = first;
        stats->loss_last = last;
        stats->ms_generate = std::chrono::duration<double, std::milli>(t1 - t0).count();
        stats->ms_train = std::chrono::duration<double, std::milli>(t2 - t1).count();
        stats->pairs = npairs;
        stats->steps = step;
    }
    return TM_OK;
}

}  // extern "C"
