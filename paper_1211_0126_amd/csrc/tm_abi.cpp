// C ABI: lifecycle, gauge load, operator application, noise, instrumentation.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <array>
#include <complex>
#include <mutex>
#include <vector>

#include "tm_ctx.h"
#include "tm_learn.h"

namespace tmq {

// Scratch of tm_dslash_noalloc, for callers that cannot allocate device
// memory (code under graph capture, serving loops): a file-scope device
// array of kScratchBytes, one copy on every GPU the library runs on, held
// until the process ends.  Host code never passes the array's name to a
// kernel or a copy: it uses the per-device address that tm_create obtains
// with hipGetSymbolAddress (the name is only a host-side stand-in).
constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// with device dev current: look up (once per device) the address of scratch
static hipError_t scratch_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
    return hipSuccess;
}

static void* scratch_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

// error text of the last failed tm_create on this thread (tm_last_error(NULL))
static thread_local std::string g_create_error = "no error";

tm_status set_error(tm_ctx* ctx, tm_status code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return code;
}

tm_status dev_error(tm_ctx* ctx, hipError_t e, const char* what) {
    if (ctx) {
        ctx->sticky = 1;
        ctx->err = std::string("HIP error ") + hipGetErrorString(e) + " in " + what;
    }
    return TM_EDEVICE;
}

static uint64_t digest_mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9E3779B97F4A7C15ULL + (h << 6) + (h >> 2);
    return seed_mix(h);
}

void* ws_get(tm_ctx* ctx, const std::string& name, size_t bytes, tm_status* st) {
    auto it = ctx->ws.find(name);
    if (it != ctx->ws.end() && it->second.bytes >= bytes) return ctx->arena.base + it->second.off;
    auto& A = ctx->arena;
    const size_t need = align256(bytes > 0 ? bytes : 1);
    size_t off = A.sp;
    // a name that grows in place when it is the last buffer carved
    if (it != ctx->ws.end() && it->second.off + align256(it->second.bytes) == A.sp) off = it->second.off;
    if (off + need > A.top) {
        *st = set_error(ctx, TM_ENOMEM,
                        "workspace too small: " + name + " needs " + std::to_string(need) + " bytes at offset " +
                            std::to_string(off) + " with " + std::to_string(A.bytes - A.top) +
                            " bytes persistent in a workspace of " + std::to_string(A.bytes) +
                            " (size it with tm_workspace_bytes)");
        return nullptr;
    }
    A.sp = off + need;
    A.peak_sp = std::max(A.peak_sp, A.sp);
    ctx->ws[name] = {off, need};
    uint64_t h = ctx->ws_digest;
    for (char c : name) h = digest_mix(h, (uint64_t)(unsigned char)c);
    ctx->ws_digest = digest_mix(h, off ^ (need << 1));
    return A.base + off;
}

void* ws_persist(tm_ctx* ctx, size_t bytes, const char* what, tm_status* st) {
    auto& A = ctx->arena;
    const size_t need = align256(bytes > 0 ? bytes : 1);
    if (A.top < need || A.top - need < A.sp) {
        *st = set_error(ctx, TM_ENOMEM,
                        std::string("workspace too small: ") + what + " needs " + std::to_string(need) +
                            " persistent bytes; " + std::to_string(A.top - A.sp) + " of " + std::to_string(A.bytes) +
                            " are free (size it with tm_workspace_bytes)");
        return nullptr;
    }
    A.top -= need;
    return A.base + A.top;
}

size_t field_bytes(const Geom& g, int prec, int nrhs) {
    const int nv = prec == P_F64 ? 12 : (prec == P_F32 ? 6 : 3);
    return (size_t)nrhs * nv * 16 * (size_t)g.Vs;
}

// splitmix64 output mix (Steele, Lea & Flood 2014), host side
uint64_t seed_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

tm_status copy_sync(tm_ctx* ctx, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
    hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return dev_error(ctx, e, "copy");
    return TM_OK;
}

void prof_begin(tm_ctx* ctx, int kc, int tag) {
    if (!ctx->prof) return;
    while (ctx->ev_used + 2 > ctx->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
            ctx->prof = false;
            return;
        }
        ctx->ev_pool.push_back(e);
    }
    hipEvent_t a = ctx->ev_pool[ctx->ev_used++];
    hipEvent_t b = ctx->ev_pool[ctx->ev_used++];
    (void)hipEventRecord(a, ctx->stream);
    ctx->recs.push_back({kc, tag, a, b, 0.0});
}

void prof_end(tm_ctx* ctx, int kc, double bytes) {
    if (!ctx->prof || ctx->recs.empty()) return;
    auto& r = ctx->recs.back();
    (void)kc;
    r.bytes = bytes;
    (void)hipEventRecord(r.b, ctx->stream);
}

// Gamma_n = g1^b0 g2^b1 g3^b2 g4^b3 of the Euclidean chiral basis
// (gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = [[0, 1], [1, 0]]),
// as the column and phase i^k of the one nonzero entry of each row.  Table
// e = 0 holds Gamma_n, e = 1 g5 Gamma_n and e = 2 g5 Gamma_n g5 (the
// matrices of the standard loop and of the two one-end loops of Eqs. 5 and
// 6), g5 = Gamma_15; each is again a phase-signed permutation.
static void gamma_tables(int col[3][16][4], int ph[3][16][4]) {
    using C = std::complex<double>;
    using M4 = std::array<std::array<C, 4>, 4>;
    const C I(0, 1);
    auto mul = [](const M4& a, const M4& b) {
        M4 t{};
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++)
                for (int k = 0; k < 4; k++) t[i][j] += a[i][k] * b[k][j];
        return t;
    };
    M4 g[4] = {};
    // gamma_1
    g[0][0][3] = -I; g[0][1][2] = -I; g[0][2][1] = I; g[0][3][0] = I;
    // gamma_2
    g[1][0][3] = -1.0; g[1][1][2] = 1.0; g[1][2][1] = 1.0; g[1][3][0] = -1.0;
    // gamma_3
    g[2][0][2] = -I; g[2][1][3] = I; g[2][2][0] = I; g[2][3][1] = -I;
    // gamma_4
    g[3][0][2] = 1.0; g[3][1][3] = 1.0; g[3][2][0] = 1.0; g[3][3][1] = 1.0;
    M4 G[16];
    for (int n = 0; n < 16; n++) {
        M4 m{};
        for (int i = 0; i < 4; i++) m[i][i] = 1.0;
        for (int mu = 0; mu < 4; mu++)
            if ((n >> mu) & 1) m = mul(m, g[mu]);
        G[n] = m;
    }
    for (int e = 0; e < 3; e++)
        for (int n = 0; n < 16; n++) {
            M4 m = G[n];
            if (e >= 1) m = mul(G[15], m);
            if (e == 2) m = mul(m, G[15]);
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) {
                    if (std::abs(m[a][b]) < 0.5) continue;
                    col[e][n][a] = b;
                    const C v = m[a][b];
                    ph[e][n][a] = v.real() > 0.5 ? 0 : (v.imag() > 0.5 ? 1 : (v.real() < -0.5 ? 2 : 3));
                }
        }
}

// ---------------------------------------------------------------------------
// operator application shared by tm_dslash and tm_dslash_noalloc
// ---------------------------------------------------------------------------
static tm_status dslash_check(tm_ctx* ctx, int32_t op, int32_t prec, int32_t nrhs, int32_t layout, const void* in_dev,
                              void* out_dev, const char* who) {
    if (!ctx) return TM_EINVAL;
    if (ctx->sticky) return set_error(ctx, TM_EDEVICE, "context has a sticky device error");
    if (!ctx->gauge_loaded) return set_error(ctx, TM_ESTATE, std::string(who) + ": no gauge field loaded");
    if (op < 0 || op > 3 || prec < 0 || prec > 3 || nrhs < 1 || nrhs > 65535 || !in_dev || !out_dev ||
        in_dev == out_dev || (layout != TM_LAYOUT_CANONICAL && layout != TM_LAYOUT_NATIVE))
        return set_error(ctx, TM_EINVAL, std::string(who) + ": bad argument");
    return TM_OK;
}


// scratch of one application: native staging of a canonical input and output,
// and the intermediate M in of M^dag M
static size_t dslash_scratch_bytes(const Geom& g, int op, int prec, int nrhs, int layout) {
    const size_t fb = align256(field_bytes(g, prec, nrhs));
    return (layout == TM_LAYOUT_CANONICAL ? 2 * fb : 0) + (op == TM_OP_MDAGM ? fb : 0);
}

// stage_in / stage_out: native buffers for a canonical layout (else unused);
// tmp: the intermediate field of M^dag M (else unused)
static tm_status dslash_run(tm_ctx* ctx, int op, int prec, int nrhs, int layout, const void* in_dev, void* out_dev,
                            void* stage_in, void* stage_out, void* tmp, bool prof) {
    const Geom& g = ctx->geo;
    const void* gauge = prec == TM_PREC_F64 ? ctx->gauge64 : ctx->gauge32;
    const int nr = (prec == TM_PREC_F64) ? 1 : (nrhs % 4 == 0 ? 4 : (nrhs % 2 == 0 ? 2 : 1));
    const void* in = in_dev;
    void* out = out_dev;
    if (layout == TM_LAYOUT_CANONICAL) {
        launch_field_convert(ctx->stream, g, prec, nrhs, true, in_dev, stage_in);
        in = stage_in;
        out = stage_out;
    }
    const double bs = prec == TM_PREC_F64 ? 8 : (prec == TM_PREC_F32 ? 4 : 2);
    const double gb = prec == TM_PREC_F64 ? 4 * 18 * 8 : 4 * 12 * 4;
    const double bytes_one = (double)g.V * (nrhs * 48.0 * bs + gb);
    auto apply = [&](int o, const void* src, void* dst) {
        if (prof) prof_begin(ctx, TM_KC_APPLY);
        launch_apply(ctx->stream, g, prec, gauge, ctx->lat.kappa, ctx->twist, o, nrhs, src, dst, nr, nullptr);
        if (prof) prof_end(ctx, TM_KC_APPLY, bytes_one);
    };
    if (op == TM_OP_MDAGM) {
        apply(TM_OP_M, in, tmp);
        apply(TM_OP_MDAG, tmp, out);
    } else {
        apply(op, in, out);
    }
    if (layout == TM_LAYOUT_CANONICAL) launch_field_convert(ctx->stream, g, prec, nrhs, false, out, out_dev);
    TM_HIP(hipGetLastError());
    return TM_OK;
}

bool geom_setup(const tm_lattice* lat, Geom* gp, Geom* hp, bool* eo_ok, std::string* why) {
    long V = 1;
    for (int d = 0; d < 4; d++) {
        if (lat->dims[d] < 2 || lat->dims[d] > 4096) {
            *why = "every extent must be in 2..4096";
            return false;
        }
        V *= lat->dims[d];
    }
    if (V >= (1L << 26)) {
        *why = "lattice too large";
        return false;
    }
    if (lat->t_bc != 1 && lat->t_bc != -1) {
        *why = "t_bc must be +1 or -1";
        return false;
    }
    Geom& g = *gp;
    g.brick = 0;
    for (int d = 0; d < 4; d++) g.L[d] = lat->dims[d];
    g.t_bc = lat->t_bc;
    g.V = V;
    // Plane stride: a multiple of 256 sites, made an odd multiple so that the
    // byte distance between planes (16 * Vs) is an odd multiple of 4 KiB.  A
    // power-of-two distance (every even lattice with 2^k sites) puts the same
    // site of all planes, and of all right-hand sides, on the same memory
    // channel.
    g.Vs = (V + 255) / 256 * 256;
#ifndef TM_POW2_PLANES
    if ((g.Vs / 256) % 2 == 0) g.Vs += 256;
#endif
    // Buffer instructions address a field's planes with 32-bit byte offsets
    // from one base; the most planes behind one base are the FP64 links'
    // 4 x 9, so 36 planes of 16 Vs bytes must stay below 4 GiB.
    if (g.Vs * 16 * 36 > 0xFFFFFFFFL) {
        *why = "lattice too large: 576 * (volume padded to 256) must stay below 2^32 bytes";
        return false;
    }
    for (int d = 0; d < 3; d++) {
        uint64_t dd = (uint64_t)g.L[d];
        uint64_t m = ((1ULL << 32) + dd - 1) / dd;
        // exactness of floor(n * m / 2^32) = n / d for every n < V
        uint64_t e = m * dd - (1ULL << 32);
        if ((uint64_t)V * e >= (1ULL << 32)) {
            *why = "no exact 32-bit division for these extents";
            return false;
        }
        g.m[d] = (uint32_t)m;
    }
    // even-odd half geometry: planes of V/2 sites with their own stride, and
    // division by Lx/2 for the half index (exact for every n < V/2)
    *eo_ok = (g.L[0] % 2 == 0) && (g.L[1] % 2 == 0) && (g.L[2] % 2 == 0) && (g.L[3] % 2 == 0);
    Geom& h = *hp;
    h = g;
    if (*eo_ok) {
        h.V = V / 2;
        h.Vs = (h.V + 255) / 256 * 256;
        if ((h.Vs / 256) % 2 == 0) h.Vs += 256;
        const uint64_t dd = (uint64_t)(g.L[0] / 2);
        const uint64_t m = ((1ULL << 32) + dd - 1) / dd;
        const uint64_t e = m * dd - (1ULL << 32);
        if (dd == 1)
            h.m[0] = 0;  // Lx = 2: the half index is the row
        else if ((uint64_t)h.V * e >= (1ULL << 32))
            *eo_ok = false;
        else
            h.m[0] = (uint32_t)m;
    }
#ifndef TM_EO_NATURAL
    // brick order of the half-lattice site blocks: a wave is 64 / (Lx/2)
    // whole rows, a block four z planes of them
    if (*eo_ok) {
        const int Lxh = g.L[0] / 2;
        if (64 % Lxh == 0 && g.L[1] % (64 / Lxh) == 0 && g.L[2] % 4 == 0) h.brick = (uint32_t)(64 / Lxh);
    }
#endif
    return true;
}

size_t partials_per_rhs(const Geom& g, const Geom& hg, bool eo_ok) {
    size_t n = (size_t)((g.V + 255) / 256);
    // time-marching kernels: a partial per 256 sites of a time slice and per
    // segment (at most one segment per slice)
    n = std::max(n, (size_t)((g.V / g.L[3] + 255) / 256) * (size_t)g.L[3]);
    if (eo_ok) n = std::max(n, (size_t)eot_tiles(hg));
    return n;
}

static size_t create_bytes() { return align256(sizeof(int) * 384) + align256(kNetFragPoolBytes); }

size_t ws_persistent(const Geom& g, const Geom& hg, bool eo_ok) {
    // the links: FP64, FP32 and bfloat16 copies, and the parity-split FP32,
    // FP64 and binary16 copies of the even-odd solver
    size_t b = align256((size_t)4 * 9 * 16 * g.Vs) + 2 * align256((size_t)4 * 3 * 16 * g.Vs);
    if (eo_ok) b += 2 * (2 * align256((size_t)4 * 3 * 16 * hg.Vs) + align256((size_t)4 * 9 * 16 * hg.Vs));
    return create_bytes() + b;
}

size_t ws_abi_scratch(const Geom& g, int field_rhs, int tune_rhs) {
    size_t b = align256((size_t)g.V * 4 * 9 * 16);                                   // gauge upload
    b = std::max(b, 3 * align256(field_bytes(g, P_F64, field_rhs)));                  // canonical M^dag M
    b = std::max(b, align256(sizeof(uint64_t) * 65535));                              // noise ids
    b = std::max(b, 2 * align256(field_bytes(g, P_F64, tune_rhs)) + align256(sizeof(uint64_t) * tune_rhs));
    return b;
}

}  // namespace tmq

using namespace tmq;

extern "C" {

int32_t tm_abi_version(void) { return TM_ABI_VERSION; }

tm_status tm_create(const tm_lattice* lat, void* dev_ws, size_t ws_bytes, void* hip_stream, tm_ctx** out) {
    if (!lat || !out) return TM_EINVAL;
    *out = nullptr;
    Geom g, h;
    bool eo_ok = false;
    std::string why;
    if (!geom_setup(lat, &g, &h, &eo_ok, &why)) {
        g_create_error = "tm_create: " + why;
        return TM_EINVAL;
    }
    if (!std::isfinite(lat->kappa) || !std::isfinite(lat->mu)) {
        g_create_error = "tm_create: kappa and mu must be finite";
        return TM_EINVAL;
    }
    if (dev_ws && ((uintptr_t)dev_ws % 256 != 0)) {
        g_create_error = "tm_create: the workspace must be 256-byte aligned";
        return TM_EINVAL;
    }
    ws_bytes = ws_bytes / 256 * 256;
    if (ws_bytes < create_bytes()) {
        g_create_error = "tm_create: a workspace of " + std::to_string(ws_bytes) + " bytes is below the " +
                         std::to_string(create_bytes()) + " the context itself holds (size it with tm_workspace_bytes)";
        return TM_ENOMEM;
    }
    tm_ctx* ctx = new tm_ctx();
    ctx->lat = *lat;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->geo = g;
    ctx->hgeo = h;
    ctx->eo_ok = eo_ok;
    ctx->twist = 2.0 * lat->kappa * lat->mu;
    auto fail = [&](tm_status code, const std::string& msg) {
        g_create_error = "tm_create: " + msg;
        (void)hipGetLastError();
        if (ctx->arena.owned && ctx->arena.base) (void)hipFree(ctx->arena.base);
        if (ctx->scal_host) (void)hipHostFree(ctx->scal_host);
        delete ctx;
        return code;
    };
    hipError_t e = hipGetDevice(&ctx->device);
    if (e != hipSuccess) return fail(TM_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    e = scratch_setup(ctx->device);
    if (e != hipSuccess) return fail(TM_EDEVICE, std::string("address of the device scratch: ") + hipGetErrorString(e));
    // the workspace: the caller's, or (null dev_ws) one allocation made here
    // and released by tm_destroy; zeroed once
    ctx->arena.bytes = ws_bytes;
    ctx->arena.top = ws_bytes;
    if (dev_ws) {
        ctx->arena.base = (char*)dev_ws;
    } else {
        e = hipMalloc((void**)&ctx->arena.base, ws_bytes);
        if (e != hipSuccess) return fail(TM_ENOMEM, "allocation of " + std::to_string(ws_bytes) + " bytes failed");
        ctx->arena.owned = true;
    }
    e = hipMemsetAsync(ctx->arena.base, 0, ws_bytes, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(TM_EDEVICE, std::string("clearing the workspace: ") + hipGetErrorString(e));
    // pinned host mirror of the per-source CG scalars
    e = hipHostMalloc((void**)&ctx->scal_host, sizeof(CgScal) * kScalHostEntries);
    if (e != hipSuccess) return fail(TM_EDEVICE, std::string("pinned host buffer: ") + hipGetErrorString(e));
    ctx->scal_host_n = kScalHostEntries;
    int col[3][16][4], ph[3][16][4];
    gamma_tables(col, ph);
    int tab[384];  // per table e: [16][4] columns, then [16][4] phases
    for (int t = 0; t < 3; t++) {
        std::memcpy(tab + 128 * t, col[t], sizeof(col[t]));
        std::memcpy(tab + 128 * t + 64, ph[t], sizeof(ph[t]));
    }
    tm_status st = TM_OK;
    ctx->gam_dev = (int*)ws_persist(ctx, sizeof(tab), "insertion tables", &st);
    ctx->net_frag_pool = (short*)ws_persist(ctx, kNetFragPoolBytes, "network fragments", &st);
    if (st != TM_OK) return fail(st, ctx->err);
    e = hipMemcpyAsync(ctx->gam_dev, tab, sizeof(tab), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(TM_EDEVICE, std::string("device set-up: ") + hipGetErrorString(e));
    *out = ctx;
    return TM_OK;
}

tm_status tm_destroy(tm_ctx* ctx) {
    if (!ctx) return TM_EINVAL;
    (void)hipStreamSynchronize(ctx->stream);
    net_release(ctx);
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
    if (ctx->scal_host) (void)hipHostFree(ctx->scal_host);
    if (ctx->arena.owned && ctx->arena.base) (void)hipFree(ctx->arena.base);
    delete ctx;
    return TM_OK;
}

tm_status tm_workspace_usage(const tm_ctx* ctx, size_t* persistent, size_t* peak_scratch, size_t* total) {
    if (!ctx) return TM_EINVAL;
    if (persistent) *persistent = ctx->arena.bytes - ctx->arena.top;
    if (peak_scratch) *peak_scratch = ctx->arena.peak_sp;
    if (total) *total = ctx->arena.bytes;
    return TM_OK;
}

const char* tm_last_error(const tm_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

tm_status tm_gauge_load(tm_ctx* ctx, const double* links_host) {
    if (!ctx || !links_host) return set_error(ctx, TM_EINVAL, "null argument");
    if (ctx->sticky) return set_error(ctx, TM_EDEVICE, "context has a sticky device error");
    WsScope scope(ctx);
    const Geom& g = ctx->geo;
    const Geom& h = ctx->hgeo;
    tm_status st = TM_OK;
    // the link copies: carved from the top at the first load, kept after
    if (!ctx->gauge64) {
        ctx->gauge64 = ws_persist(ctx, (size_t)4 * 9 * 16 * g.Vs, "FP64 links", &st);
        ctx->gauge32 = ws_persist(ctx, (size_t)4 * 3 * 16 * g.Vs, "FP32 links", &st);
        ctx->gaugebf = ws_persist(ctx, (size_t)4 * 3 * 16 * g.Vs, "bfloat16 links", &st);
        for (int q = 0; q < 2 && ctx->eo_ok; q++) {
            ctx->gauge32eo[q] = ws_persist(ctx, (size_t)4 * 3 * 16 * h.Vs, "FP32 parity links", &st);
            ctx->gauge64eo[q] = ws_persist(ctx, (size_t)4 * 9 * 16 * h.Vs, "FP64 parity links", &st);
            ctx->gauge16eo[q] = ws_persist(ctx, (size_t)4 * 3 * 16 * h.Vs, "binary16 parity links", &st);
        }
        if (st != TM_OK) {
            ctx->gauge64 = ctx->gauge32 = ctx->gaugebf = nullptr;
            return st;
        }
    }
    const size_t canon_bytes = (size_t)g.V * 4 * 9 * 16;
    void* tmp = ws_get(ctx, "gauge_upload", canon_bytes, &st);
    if (!tmp) return st;
    hipError_t e = hipMemcpyAsync(tmp, links_host, canon_bytes, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) {
        launch_gauge_convert(ctx->stream, g, (const double*)tmp, ctx->gauge64, ctx->gauge32, ctx->gaugebf);
        e = hipGetLastError();
    }
    if (e == hipSuccess && ctx->eo_ok) {
        launch_eo_split(ctx->stream, g, h, ctx->gauge32, 12, ctx->gauge32eo[0], ctx->gauge32eo[1]);
        launch_eo_split(ctx->stream, g, h, ctx->gauge64, 36, ctx->gauge64eo[0], ctx->gauge64eo[1]);
        for (int q = 0; q < 2; q++) launch_eo_links_h16(ctx->stream, h, ctx->gauge64eo[q], ctx->gauge16eo[q]);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return dev_error(ctx, e, "gauge load");
    ctx->gauge_loaded = true;
    return TM_OK;
}

size_t tm_field_bytes(const tm_ctx* ctx, int32_t prec, int32_t nrhs, int32_t layout) {
    if (!ctx || prec < 0 || prec > 3 || nrhs < 0) return 0;
    if (layout == TM_LAYOUT_NATIVE) return field_bytes(ctx->geo, prec, nrhs);
    const size_t e = prec == TM_PREC_F64 ? 16 : (prec == TM_PREC_F32 ? 8 : 4);
    return (size_t)nrhs * ctx->geo.V * 12 * e;
}

tm_status tm_field_convert(tm_ctx* ctx, int32_t prec, int32_t nrhs, int32_t to_native, const void* in_dev,
                           void* out_dev) {
    if (!ctx) return TM_EINVAL;
    if (ctx->sticky) return set_error(ctx, TM_EDEVICE, "context has a sticky device error");
    if (prec < 0 || prec > 3 || nrhs < 1 || nrhs > 65535 || !in_dev || !out_dev || in_dev == out_dev)
        return set_error(ctx, TM_EINVAL, "tm_field_convert: bad argument");
    launch_field_convert(ctx->stream, ctx->geo, prec, nrhs, to_native != 0, in_dev, out_dev);
    TM_HIP(hipGetLastError());
    return TM_OK;
}

tm_status tm_dslash(tm_ctx* ctx, int32_t op, int32_t prec, int32_t nrhs, int32_t layout, const void* in_dev,
                    void* out_dev) {
    tm_status st = dslash_check(ctx, op, prec, nrhs, layout, in_dev, out_dev, "tm_dslash");
    if (st != TM_OK) return st;
    WsScope scope(ctx);
    const size_t fb = field_bytes(ctx->geo, prec, nrhs);
    void *a = nullptr, *b = nullptr, *tmp = nullptr;
    if (layout == TM_LAYOUT_CANONICAL) {
        a = ws_get(ctx, "dslash_in", fb, &st);
        if (!a) return st;
        b = ws_get(ctx, "dslash_out", fb, &st);
        if (!b) return st;
    }
    if (op == TM_OP_MDAGM) {
        tmp = ws_get(ctx, "dslash_tmp", fb, &st);
        if (!tmp) return st;
    }
    return dslash_run(ctx, op, prec, nrhs, layout, in_dev, out_dev, a, b, tmp, true);
}

tm_status tm_dslash_noalloc(tm_ctx* ctx, int32_t op, int32_t prec, int32_t nrhs, int32_t layout, const void* in_dev,
                            void* out_dev) {
    tm_status st = dslash_check(ctx, op, prec, nrhs, layout, in_dev, out_dev, "tm_dslash_noalloc");
    if (st != TM_OK) return st;
    const size_t need = dslash_scratch_bytes(ctx->geo, op, prec, nrhs, layout);
    if (need > kScratchBytes)
        return set_error(ctx, TM_EINVAL, "tm_dslash_noalloc: this call needs " + std::to_string(need) +
                                             " bytes of scratch; the maximum is " + std::to_string(kScratchBytes) +
                                             " (use tm_dslash)");
    char* base = (char*)scratch_ptr(ctx->device);
    if (!base) return set_error(ctx, TM_ESTATE, "tm_dslash_noalloc: no scratch address for this device");
    const size_t fb = align256(field_bytes(ctx->geo, prec, nrhs));
    void *a = nullptr, *b = nullptr, *tmp = nullptr;
    size_t off = 0;
    if (layout == TM_LAYOUT_CANONICAL) {
        a = base;
        b = base + fb;
        off = 2 * fb;
    }
    if (op == TM_OP_MDAGM) tmp = base + off;
    return dslash_run(ctx, op, prec, nrhs, layout, in_dev, out_dev, a, b, tmp, false);
}

tm_status tm_noise_z4(tm_ctx* ctx, uint64_t seed, int32_t nsrc, const uint64_t* ids_host, double* out_dev) {
    if (!ctx) return TM_EINVAL;
    if (ctx->sticky) return set_error(ctx, TM_EDEVICE, "context has a sticky device error");
    WsScope scope(ctx);
    if (nsrc < 1 || nsrc > 65535 || !ids_host || !out_dev) return set_error(ctx, TM_EINVAL, "tm_noise_z4: bad argument");
    tm_status st = TM_OK;
    uint64_t* ids = (uint64_t*)ws_get(ctx, "noise_ids", sizeof(uint64_t) * nsrc, &st);
    if (!ids) return st;
    TM_HIP(hipMemcpyAsync(ids, ids_host, sizeof(uint64_t) * nsrc, hipMemcpyHostToDevice, ctx->stream));
    launch_noise_c128(ctx->stream, ctx->geo, seed_mix(seed), ids, nsrc, out_dev);
    TM_HIP(hipGetLastError());
    TM_HIP(hipStreamSynchronize(ctx->stream));  // ids_host may be released on return
    return TM_OK;
}

tm_status tm_set_graphs(tm_ctx* ctx, int32_t on, int64_t* replays) {
    if (!ctx) return TM_EINVAL;
    if (on >= 0) ctx->use_graphs = on != 0;
    if (replays) *replays = ctx->graph_launches;
    return TM_OK;
}

tm_status tm_set_march(tm_ctx* ctx, int32_t prec, int32_t tseg) {
    if (!ctx || prec < 0 || prec > 3 || tseg < 0 || tseg > 65535)
        return ctx ? set_error(ctx, TM_EINVAL, "tm_set_march: bad argument") : TM_EINVAL;
    ctx->march[prec] = tseg;
    return TM_OK;
}

tm_status tm_set_eo_tiles(tm_ctx* ctx, int32_t prec, int32_t on) {
    if (!ctx || prec < 0 || prec > 3 || on < 0 || on > 1)
        return ctx ? set_error(ctx, TM_EINVAL, "tm_set_eo_tiles: bad argument") : TM_EINVAL;
    ctx->eo_tiles[prec] = prec == TM_PREC_F64 ? 0 : on;
    return TM_OK;
}

tm_status tm_set_lane_rhs(tm_ctx* ctx, int32_t prec, int32_t nr) {
    if (!ctx || prec < 0 || prec > 3 || !(nr == 0 || nr == 1 || nr == 2 || nr == 4))
        return set_error(ctx, TM_EINVAL, "tm_set_lane_rhs: bad argument");
    ctx->lane_rhs[prec] = prec == TM_PREC_F64 ? (nr ? 1 : 0) : nr;
    return TM_OK;
}

tm_status tm_autotune(tm_ctx* ctx, int32_t prec, int32_t nrhs, int32_t* best_nr, double* ms_host) {
    if (!ctx || prec < 0 || prec > 3 || nrhs < 1 || nrhs > 32 || !best_nr)
        return set_error(ctx, TM_EINVAL, "tm_autotune: bad argument");
    if (ctx->sticky) return set_error(ctx, TM_EDEVICE, "context has a sticky device error");
    WsScope scope(ctx);
    if (!ctx->gauge_loaded) return set_error(ctx, TM_ESTATE, "tm_autotune: no gauge field loaded");
    const Geom& g = ctx->geo;
    tm_status s = TM_OK;
    const size_t fb = field_bytes(g, prec, nrhs);
    void* in = ws_get(ctx, "tune_in", fb, &s);
    void* out = ws_get(ctx, "tune_out", fb, &s);
    uint64_t* ids = (uint64_t*)ws_get(ctx, "tune_ids", sizeof(uint64_t) * nrhs, &s);
    if (s != TM_OK) return s;
    std::vector<uint64_t> idh(nrhs);
    for (int i = 0; i < nrhs; i++) idh[i] = (uint64_t)i;
    if ((s = copy_sync(ctx, ids, idh.data(), sizeof(uint64_t) * nrhs, hipMemcpyHostToDevice)) != TM_OK) return s;
    launch_noise_native(ctx->stream, g, prec, seed_mix(12345), ids, nrhs, in);
    const void* gauge = prec == TM_PREC_F64 ? ctx->gauge64 : ctx->gauge32;
    hipEvent_t e0, e1;
    TM_HIP(hipEventCreate(&e0));
    TM_HIP(hipEventCreate(&e1));
    const int cand[3] = {1, 2, 4};
    double best = 1e300;
    int bnr = 1;
    for (int c = 0; c < 3; c++) {
        const int nr = cand[c];
        if (ms_host) ms_host[c] = -1.0;
        if (nrhs % nr != 0 || (prec == TM_PREC_F64 && nr != 1)) continue;
        for (int w = 0; w < 2; w++)
            launch_apply(ctx->stream, g, prec, gauge, ctx->lat.kappa, ctx->twist, 0, nrhs, in, out, nr, nullptr);
        const int reps = 10;
        (void)hipEventRecord(e0, ctx->stream);
        for (int i = 0; i < reps; i++)
            launch_apply(ctx->stream, g, prec, gauge, ctx->lat.kappa, ctx->twist, 0, nrhs, in, out, nr, nullptr);
        (void)hipEventRecord(e1, ctx->stream);
        hipError_t e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return dev_error(ctx, e, "tm_autotune timing");
        }
        const double per = ms / reps;
        if (ms_host) ms_host[c] = per;
        if (per < best) {
            best = per;
            bnr = nr;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->lane_rhs[prec] = bnr;
    *best_nr = bnr;
    return TM_OK;
}

tm_status tm_profile_enable(tm_ctx* ctx, int32_t on) {
    if (!ctx) return TM_EINVAL;
    TM_HIP(hipStreamSynchronize(ctx->stream));
    ctx->prof = on != 0;
    ctx->recs.clear();
    ctx->ev_used = 0;
    ctx->prof_variants.clear();
    for (int k = 0; k < TM_KC_COUNT; k++) {
        ctx->prof_launches[k] = 0;
        ctx->prof_ms[k] = 0;
        ctx->prof_bytes[k] = 0;
    }
    return TM_OK;
}

// fold the recorded launches into the per-class and per-variant sums
static tm_status prof_drain(tm_ctx* ctx) {
    TM_HIP(hipStreamSynchronize(ctx->stream));
    for (auto& r : ctx->recs) {
        float t = 0;
        TM_HIP(hipEventElapsedTime(&t, r.a, r.b));
        ctx->prof_launches[r.kc] += 1;
        ctx->prof_ms[r.kc] += t;
        ctx->prof_bytes[r.kc] += r.bytes;
        auto& v = ctx->prof_variants[{r.kc, r.tag}];
        v.launches += 1;
        v.ms += t;
        v.bytes += r.bytes;
    }
    ctx->recs.clear();
    ctx->ev_used = 0;
    return TM_OK;
}

tm_status tm_profile_entries(tm_ctx* ctx, tm_profile_entry* out, int32_t cap, int32_t* n) {
    if (!ctx || !out || !n || cap < 0) return ctx ? set_error(ctx, TM_EINVAL, "tm_profile_entries: bad arguments")
                                                  : TM_EINVAL;
    tm_status s = prof_drain(ctx);
    if (s != TM_OK) return s;
    int32_t k = 0;
    for (auto& kv : ctx->prof_variants) {
        if (k >= cap) break;
        const int tag = kv.first.second;
        tm_profile_entry& e = out[k++];
        e.kc = kv.first.first;
        e.prec = tag < 0 ? -1 : (tag & 15);
        e.lane_rhs = tag < 0 ? -1 : ((tag >> 4) & 15);
        e.solver = tag < 0 ? -1 : ((tag >> 8) & 15);
        e.tseg = tag < 0 ? -1 : ((tag >> 12) & 255);
        e.reliable = tag < 0 ? -1 : ((tag >> 20) & 1);
        e.launches = kv.second.launches;
        e.ms = kv.second.ms;
        e.bytes = kv.second.bytes;
    }
    *n = k;
    return TM_OK;
}

tm_status tm_profile_read(tm_ctx* ctx, int64_t* launches, double* ms, double* bytes) {
    if (!ctx) return TM_EINVAL;
    tm_status s = prof_drain(ctx);
    if (s != TM_OK) return s;
    for (int k = 0; k < TM_KC_COUNT; k++) {
        if (launches) launches[k] = ctx->prof_launches[k];
        if (ms) ms[k] = ctx->prof_ms[k];
        if (bytes) bytes[k] = ctx->prof_bytes[k];
    }
    return TM_OK;
}

}  // extern "C"
