// Host-side context of the library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/tmqcd.h"
#include "tm_kernels.h"
#include "tm_types.h"

struct tm_ctx {
    tm_lattice lat;
    tmq::Geom geo;
    hipStream_t stream = nullptr;
    int device = 0;
    double twist = 0;  // 2 kappa mu

    void* gauge64 = nullptr;  // double2 [4][9][Vs]
    void* gauge32 = nullptr;  // float4  [4][3][Vs]
    void* gaugebf = nullptr;  // uint4   [4][3][Vs]: bfloat16 (re, im) pairs of the 9 entries, for the network
    bool gauge_loaded = false;

    // even-odd form (every extent even): the half geometry (V = sites of one
    // parity, Vs their plane stride, m[0] divides by Lx/2) and the links split
    // by parity, each copy holding the forward links of its sites
    bool eo_ok = false;
    tmq::Geom hgeo;
    void* gauge32eo[2] = {nullptr, nullptr};  // float4  [4][3][Vhs] per parity
    void* gauge64eo[2] = {nullptr, nullptr};  // double2 [4][9][Vhs] per parity
    void* gauge16eo[2] = {nullptr, nullptr};  // uint4 [4][3][Vhs] per parity: binary16 pairs (FP16 storage hops)

    // The caller's device workspace.  Every device buffer of the context is
    // carved from it: buffers that live until tm_destroy (links, tables,
    // network fragments) from the top down, the scratch of one API call from
    // the bottom up, released when the next call begins.
    struct Arena {
        char* base = nullptr;
        size_t bytes = 0;
        bool owned = false;   // allocated by tm_create (null dev_ws)
        size_t top = 0;       // persistent buffers occupy [top, bytes)
        size_t sp = 0;        // scratch of the current call occupies [0, sp)
        size_t peak_sp = 0;   // largest sp since tm_create
        int depth = 0;        // nesting of API scopes (the outermost resets sp)
    } arena;
    struct Buf {
        size_t off = 0;
        size_t bytes = 0;
    };
    std::map<std::string, Buf> ws;  // named scratch of the current call
    // right-hand sides the buffers of a solve tag are sized for in this call
    // (at least the block being solved)
    std::map<std::string, int> ws_cap;
    // digest of the names and offsets of the current call's scratch (part of
    // the keys of captured graphs, which hold buffer addresses)
    uint64_t ws_digest = 0;

    tmq::CgScal* scal_host = nullptr;  // pinned mirror for stop checks
    int scal_host_n = 0;
    // device memory of the network weight fragments (TM_NET_MAX_LAYERS layers,
    // forward and adjoint), carved at tm_create
    short* net_frag_pool = nullptr;

    // insertion tables on the device (row a -> column, phase i^k): [3][2][16][4]
    // for Gamma_n, g5 Gamma_n, g5 Gamma_n g5
    int* gam_dev = nullptr;

    // learned preconditioner (weights and their bfloat16 fragments)
    struct NetState* net = nullptr;

    // right-hand sides per lane chosen by tm_autotune / tm_set_lane_rhs, per
    // storage precision (0: built-in default)
    int lane_rhs[4] = {0, 0, 0, 0};
    // time slices per lane of the time-marching CG stencils, per storage
    // precision (0: one lane per site)
    int march[4] = {0, 0, 0, 0};
    // even-odd CG half-hops per storage precision: 1 the tile kernels (links
    // staged in LDS and shared by all right-hand sides), 0 a lane per site
    int eo_tiles[4] = {0, 0, 0, 0};

    // captured CG chunks (replayed with hipGraphLaunch), keyed by buffers and
    // launch configuration; used on a non-null stream when profiling is off
    bool use_graphs = true;
    std::map<std::string, hipGraphExec_t> graphs;
    // CG iterations of the last block solved with given settings (the first
    // chunk of steps between host checks of the next such block)
    std::map<std::string, int> chunk_hint;
    int64_t graph_launches = 0;

    std::string err;
    int sticky = 0;

    // instrumentation
    bool prof = false;
    struct Rec {
        int kc;
        int tag;  // prof_tag() of the launch, -1 if none
        hipEvent_t a, b;
        double bytes;
    };
    struct Acc {
        int64_t launches = 0;
        double ms = 0, bytes = 0;
    };
    std::map<std::pair<int, int>, Acc> prof_variants;  // (kc, tag)
    std::vector<Rec> recs;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    int64_t prof_launches[TM_KC_COUNT] = {0};
    double prof_ms[TM_KC_COUNT] = {0};
    double prof_bytes[TM_KC_COUNT] = {0};
};

namespace tmq {

// most right-hand sides of one solve block
constexpr int kMaxBlock = 32;
// entries of the pinned host mirror of the CG scalars (two blocks of 32)
constexpr int kScalHostEntries = 64;
// device bytes of one layer's weight fragments in one direction, for widths
// up to 2 (144 padded K rows: 9 MFMA K-steps of 64 lanes x 4 bfloat16), and
// of the pool holding every layer in both directions
constexpr size_t kNetFragBytes = 9 * 64 * 4 * 2;
constexpr size_t kNetFragPoolBytes = (size_t)TM_NET_MAX_LAYERS * 2 * kNetFragBytes;

tm_status set_error(tm_ctx* ctx, tm_status code, const std::string& msg);
tm_status dev_error(tm_ctx* ctx, hipError_t e, const char* what);
// Named scratch of the current API call (sized for bytes; a name asked for
// again in the same call returns its buffer if it is large enough).  Null and
// *st = TM_ENOMEM if the workspace cannot hold it.
void* ws_get(tm_ctx* ctx, const std::string& name, size_t bytes, tm_status* st);
// A buffer that lives until tm_destroy, from the top of the workspace.
void* ws_persist(tm_ctx* ctx, size_t bytes, const char* what, tm_status* st);
// right-hand sides to size the buffers of a solve tag for in this call
inline int ws_rhs(const tm_ctx* ctx, const std::string& tag, int nrhs) {
    auto it = ctx->ws_cap.find(tag);
    return it == ctx->ws_cap.end() ? nrhs : (it->second > nrhs ? it->second : nrhs);
}
inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }
// reduction partials per right-hand side, the most any CG or FCG kernel
// writes (lane-per-site, time-marching and even-odd tile traversals)
size_t partials_per_rhs(const Geom& g, const Geom& hg, bool eo_ok);
// geometry of a lattice (plane strides, divisors) and of its even-odd half;
// false with the reason in *why for an unsupported lattice
bool geom_setup(const tm_lattice* lat, Geom* g, Geom* hg, bool* eo_ok, std::string* why);
// workspace bounds: the buffers kept until tm_destroy (tables, network
// fragments, links), and the scratch of the calls of the lifecycle and
// operator part (gauge upload, canonical tm_dslash with field_rhs
// right-hand sides, noise ids, tm_autotune with tune_rhs)
size_t ws_persistent(const Geom& g, const Geom& hg, bool eo_ok);
size_t ws_abi_scratch(const Geom& g, int field_rhs, int tune_rhs);
size_t field_bytes(const Geom& g, int prec, int nrhs);
uint64_t seed_mix(uint64_t seed);

// Copy on the context's stream and wait for it (and for all work queued
// before it).  A plain hipMemcpy runs on the null stream, which does not
// wait for a non-blocking stream such as the caller's.
tm_status copy_sync(tm_ctx* ctx, void* dst, const void* src, size_t bytes, hipMemcpyKind kind);
#define TM_COPY(dst, src, bytes, kind)                                          \
    do {                                                                        \
        const tm_status cs_ = ::tmq::copy_sync(ctx, (dst), (src), (bytes), (kind)); \
        if (cs_ != TM_OK) return cs_;                                           \
    } while (0)

// instrumentation around a launch of kernel class kc moving `bytes`
// tag: prof_tag(prec, lane_rhs, solver) of the launched kernel, -1 if none
void prof_begin(tm_ctx* ctx, int kc, int tag = -1);
inline int prof_tag(int prec, int lane_rhs, int solver, int tseg = 0, bool reliable = false) {
    return prec | (lane_rhs << 4) | (solver << 8) | (tseg << 12) | ((int)reliable << 20);
}
void prof_end(tm_ctx* ctx, int kc, double bytes);

}  // namespace tmq

// Scope of one API call: the outermost scope on a context starts a fresh
// scratch region (the previous call's scratch is dead: every use of it was
// enqueued on the context's stream before this call's work).
struct WsScope {
    tm_ctx* c;
    explicit WsScope(tm_ctx* ctx) : c(ctx) {
        if (c && c->arena.depth++ == 0) {
            c->arena.sp = 0;
            c->ws.clear();
            c->ws_cap.clear();
            c->ws_digest = 0;
        }
    }
    ~WsScope() {
        if (c) c->arena.depth--;
    }
    WsScope(const WsScope&) = delete;
    WsScope& operator=(const WsScope&) = delete;
};

#define TM_HIP(call)                                             \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return tmq::dev_error(ctx, e_, #call); \
    } while (0)
