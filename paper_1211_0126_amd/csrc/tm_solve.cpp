// Solver and TSM drivers: tsm_solve_batch, tsm_contract, tsm_loops.
//
// A block of right-hand sides is solved together: all vectors and all
// per-source scalars live on the device, every CG step is three kernel
// launches, and the host only polls the per-source stop flags once per
// chunk of steps.  Each source's arithmetic is independent of the others in
// its block (per-source scalars, masks and reductions in a fixed order), so
// the LP solution of a source does not depend on how the sources are
// batched: the HP-minus-LP correction of Eq. 4 sees one fixed LP map.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "tm_ctx.h"
#include "tm_learn.h"

namespace tmq {

static const int kIterCap = 20000;  // safety cap for max_iter = -1
// search directions kept by the even-odd CG without reliable updates
constexpr int kEoRing = 8;
// sources per launch of the FP32 solution reconstruction (a multiple of every
// right-hand-sides-per-lane setting)
constexpr int kRecSub = 8;

static tm_status check_solve_params(tm_ctx* ctx, const tsm_solve_params* p) {
    if (!p) return set_error(ctx, TM_EINVAL, "null solve parameters");
    if (p->prec < 0 || p->prec > 3) return set_error(ctx, TM_EINVAL, "solve: bad precision");
    if (p->solver != TM_SOLVER_CG && p->solver != TM_SOLVER_FCG_LEARNED && p->solver != TM_SOLVER_CG_EO)
        return set_error(ctx, TM_EINVAL, "solve: unknown solver");
    if (p->solver == TM_SOLVER_CG_EO && !ctx->eo_ok)
        return set_error(ctx, TM_ENOTSUP, "solve: the even-odd solver needs every lattice extent even");
    if (p->solver == TM_SOLVER_FCG_LEARNED) {
        if (p->prec == TM_PREC_F64 || p->reliable || p->stop != TM_STOP_NORMAL)
            return set_error(ctx, TM_ENOTSUP,
                             "solve: flexible CG stores its directions in FP32/FP16/BF16, stops on the normal "
                             "equations, has no reliable updates");
        if (!net_installed(ctx)) return set_error(ctx, TM_ESTATE, "solve: no network installed (tm_precond_set/train)");
    }
    if (!(p->tol >= 0) || !std::isfinite(p->tol)) return set_error(ctx, TM_EINVAL, "solve: bad tolerance");
    if (p->max_iter < -1) return set_error(ctx, TM_EINVAL, "solve: bad max_iter");
    if (p->stop != TM_STOP_NORMAL && p->stop != TM_STOP_TRUE) return set_error(ctx, TM_EINVAL, "solve: bad stop");
    if (p->reliable != 0 && p->reliable != 1) return set_error(ctx, TM_EINVAL, "solve: bad reliable flag");
    if (p->reliable) {
        // FP32 iterations; FP32, FP16 or BF16 storage on the even-odd solver
        if (p->prec == TM_PREC_F64 || (p->prec != TM_PREC_F32 && p->solver != TM_SOLVER_CG_EO))
            return set_error(ctx, TM_ENOTSUP,
                             "solve: reliable updates need FP32 iterations (FP32 storage, or FP32/FP16/BF16 on the "
                             "even-odd solver)");
        if (!(p->delta > 0 && p->delta < 1)) return set_error(ctx, TM_EINVAL, "solve: delta must be in (0, 1)");
    }
    if (p->rhs_block < 0 || p->rhs_block > kMaxBlock) return set_error(ctx, TM_EINVAL, "solve: rhs_block in 0..32");
    return TM_OK;
}

static int default_block(const tsm_solve_params* p) {
    if (p->rhs_block > 0) return p->rhs_block;
    if (p->prec == TM_PREC_F64) return 4;
    return p->reliable ? 8 : 16;
}

// right-hand sides per lane in the stencil kernels: the tuned choice when it
// divides the block, else the largest of 4, 2, 1 that does
static int lane_rhs(const tm_ctx* ctx, const tsm_solve_params* p, int block) {
    if (p->prec == TM_PREC_F64 || (p->stop == TM_STOP_TRUE && !p->reliable)) return 1;
    const int t = ctx->lane_rhs[p->prec];
    if (t > 0 && block % t == 0) return t;
    if (block % 4 == 0) return 4;
    if (block % 2 == 0) return 2;
    return 1;
}

// time slices per lane of the time-marching K1 / K2 (0: lane per site)
// autotuner candidates (right-hand sides per lane, time slices per lane)
constexpr int kTuneCandidates = 8;
constexpr int kTuneNr[kTuneCandidates] = {1, 2, 4, 1, 1, 1, 2, 2};
constexpr int kTuneTseg[kTuneCandidates] = {0, 0, 0, 4, 8, 16, 4, 8};

static int march_tseg(const tm_ctx* ctx, const tsm_solve_params* p, int nr) {
    const int t = ctx->march[p->prec];
    if (t <= 0 || nr > 2) return 0;
    return std::min(t, ctx->geo.L[3]);
}

// the pinned mirror (allocated by tm_create) holds a block's scalars
static tm_status ensure_scal_host(tm_ctx* ctx, int n) {
    if (ctx->scal_host_n >= n) return TM_OK;
    return set_error(ctx, TM_EINVAL, "block larger than the scalar mirror");
}

// CG steps between host checks.  The first chunk is the iteration count of
// the previous block solved with the same settings (one graph replay then
// covers a typical solve), else `dflt`; later chunks are shorter, so that few
// launches run past convergence (such launches return at once).  With
// per-launch profiling every step is checked, so that each timed launch has
// active right-hand sides and its bytes count only those.
static std::string chunk_key(const tsm_solve_params* p, const std::string& tag, int nrhs) {
    char k[160];
    std::snprintf(k, sizeof(k), "%s|%d|%d|%d|%d|%.6g|%d|%d", tag.c_str(), p->prec, p->solver, p->reliable, p->stop,
                  p->tol, p->max_iter, nrhs);
    return k;
}
static int first_chunk(const tm_ctx* ctx, const std::string& key, int dflt) {
    if (ctx->prof) return 1;
    auto it = ctx->chunk_hint.find(key);
    return it == ctx->chunk_hint.end() ? dflt : std::max(1, it->second);
}
static int later_chunk(const tm_ctx* ctx, int dflt) { return ctx->prof ? 1 : std::max(1, dflt / 4); }
static int active_count(const tm_ctx* ctx, int nrhs) {
    int n = 0;
    for (int r = 0; r < nrhs; r++) n += ctx->scal_host[r].active != 0;
    return n;
}
static void remember_chunk(tm_ctx* ctx, const std::string& key, int nrhs) {
    int m = 0;
    for (int r = 0; r < nrhs; r++) m = std::max(m, (int)ctx->scal_host[r].iters);
    if (m > 0) ctx->chunk_hint[key] = m;
}

// bytes of the CG kernels per launch (algorithmic: each field touched once,
// each link once per site)
struct CgBytes {
    double k1, k2, k3;
};
static CgBytes cg_bytes(const Geom& g, int prec, int nrhs, bool reliable_x64, bool track) {
    const double bs = prec == P_F64 ? 8 : (prec == P_F32 ? 4 : 2);
    const double bx = prec == P_F64 ? 8 : 4;
    const double gb = prec == P_F64 ? 4 * 18 * 8 : 4 * 12 * 4;
    (void)reliable_x64;
    CgBytes b;
    b.k1 = (double)g.V * (nrhs * 48.0 * bs + gb);
    b.k2 = (double)g.V * (nrhs * (24.0 * bs + 48.0 * bs + 24.0 * bs + 48.0 * bx + (track ? 48.0 * bs : 0.0)) + gb);
    b.k3 = (double)g.V * nrhs * 72.0 * bs;
    return b;
}

struct BlockResult {
    void* x;             // the native solutions, or with xe their odd halves
    int xprec;
    void* xe = nullptr;  // (halves only) the even halves, in xprec (FP32, or FP16 for FP16 solves)
};

// Flexible CG with the network preconditioner for a block of sources; the
// final state is written into ctx->scal_host in CgScal form.
static tm_status solve_block_fcg(tm_ctx* ctx, const tsm_solve_params* p, uint64_t seed_mixed,
                                 const uint64_t* ids_dev, int nrhs, int nr, const std::string& tag,
                                 BlockResult* res) {
    const Geom& g = ctx->geo;
    hipStream_t st = ctx->stream;
    tm_status s = TM_OK;
    const size_t fb = field_bytes(g, P_F32, ws_rhs(ctx, tag, nrhs));
    // the stencil inputs p and t in the storage precision
    const int prec = p->prec;
    const size_t fbs = field_bytes(g, prec, ws_rhs(ctx, tag, nrhs));
    const size_t npart = partials_per_rhs(g, ctx->hgeo, ctx->eo_ok);
    FcgArgs a;
    std::memset(&a, 0, sizeof(a));
    a.geo = g;
    a.gauge = ctx->gauge32;
    a.kappa = ctx->lat.kappa;
    a.twist = ctx->twist;
    a.nrhs = nrhs;
    a.prec = prec;
    a.p = ws_get(ctx, tag + "_fp", fbs, &s);
    a.t = ws_get(ctx, tag + "_ft", fbs, &s);
    a.q = ws_get(ctx, tag + "_fq", fb, &s);
    a.r = ws_get(ctx, tag + "_fr", fb, &s);
    a.x = ws_get(ctx, tag + "_fx", fb, &s);
    a.z = ws_get(ctx, tag + "_fz", fb, &s);
    void* eta = ws_get(ctx, tag + "_feta", fb, &s);
    a.scal = (FcgScal*)ws_get(ctx, tag + "_fscal", sizeof(FcgScal) * kMaxBlock, &s);
    a.partials = (double*)ws_get(ctx, "fpartials", sizeof(double) * npart * kMaxBlock * 4, &s);
    CgScal* tscal = (CgScal*)ws_get(ctx, tag + "_ftscal", sizeof(CgScal) * kMaxBlock, &s);
    double* part1 = (double*)ws_get(ctx, "partials", sizeof(double) * npart * kMaxBlock, &s);
    double* part2 = (double*)ws_get(ctx, "partials2", sizeof(double) * npart * kMaxBlock, &s);
    if (s != TM_OK) return s;
    if ((s = ensure_scal_host(ctx, nrhs)) != TM_OK) return s;

    prof_begin(ctx, TM_KC_OTHER);
    launch_noise_native(st, g, P_F32, seed_mixed, ids_dev, nrhs, eta);
    launch_apply(st, g, P_F32, ctx->gauge32, ctx->lat.kappa, ctx->twist, 1, nrhs, eta, a.r, 1, nullptr);
    launch_fcg_init(st, a, p->tol * p->tol, p->max_iter, 0);
    prof_end(ctx, TM_KC_OTHER, 0.0);
    if ((s = net_precondition(ctx, nrhs, a.r, a.z, nullptr, ws_rhs(ctx, tag, nrhs))) != TM_OK) return s;
    launch_fcg_dot(st, a, 1);
    launch_fcg_p(st, a);
    TM_HIP(hipGetLastError());
    const CgBytes by = cg_bytes(g, prec, nrhs, false, false);
    std::vector<FcgScal> fs(nrhs);
    int done = 0;
    // the stencil steps march in time when a segment length is set for FP32
    // (nr right-hand sides per lane, 1 or 2), else one lane per site
    const int tseg = march_tseg(ctx, p, nr);
    for (;;) {
        // iterations between host checks: the network skips finished
        // right-hand sides, so an iteration past convergence costs launches only
        int k = 2;
        if (p->max_iter >= 0) k = std::max(1, std::min(k, p->max_iter - done));
        for (int i = 0; i < k; i++) {
            prof_begin(ctx, TM_KC_DSLASH, prof_tag(prec, tseg > 0 ? nr : 1, TM_SOLVER_FCG_LEARNED, tseg));
            if (tseg > 0)
                launch_fcg_tm_mp(st, a, nr, tseg);
            else
                launch_fcg_mp(st, a);
            prof_end(ctx, TM_KC_DSLASH, by.k1);
            prof_begin(ctx, TM_KC_DSLASH_UPD, prof_tag(prec, tseg > 0 ? nr : 1, TM_SOLVER_FCG_LEARNED, tseg));
            if (tseg > 0)
                launch_fcg_tm_upd(st, a, nr, tseg);
            else
                launch_fcg_upd(st, a);
            prof_end(ctx, TM_KC_DSLASH_UPD, by.k2);
            if ((s = net_precondition(ctx, nrhs, a.r, a.z, a.scal, ws_rhs(ctx, tag, nrhs))) != TM_OK) return s;
            launch_fcg_dot(st, a, 0);
            prof_begin(ctx, TM_KC_BLAS, prof_tag(prec, 1, TM_SOLVER_FCG_LEARNED));
            launch_fcg_p(st, a);
            prof_end(ctx, TM_KC_BLAS, by.k3);
        }
        TM_HIP(hipGetLastError());
        done += k;
        TM_HIP(hipMemcpyAsync(fs.data(), a.scal, sizeof(FcgScal) * nrhs, hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
        bool any = false;
        for (int r = 0; r < nrhs; r++) any |= fs[r].active != 0;
        if (!any || done >= kIterCap) break;
    }
    res->x = a.x;
    res->xprec = P_F32;
    std::vector<CgScal> ts(nrhs);
    std::memset(ts.data(), 0, sizeof(CgScal) * nrhs);
    if (p->true_resid) {
        CgArgs at;
        std::memset(&at, 0, sizeof(at));
        at.geo = g;
        at.kappa = ctx->lat.kappa;
        at.twist = ctx->twist;
        at.x = a.x;
        at.scal = tscal;
        at.partials = part1;
        at.partials2 = part2;
        at.nrhs = nrhs;
        launch_true_resid(st, at, P_F32, ctx->gauge64, seed_mixed, ids_dev);
        TM_HIP(hipGetLastError());
        TM_HIP(hipMemcpyAsync(ts.data(), tscal, sizeof(CgScal) * nrhs, hipMemcpyDeviceToHost, st));
    }
    TM_HIP(hipStreamSynchronize(st));
    for (int r = 0; r < nrhs; r++) {
        CgScal q;
        std::memset(&q, 0, sizeof(q));
        q.iters = fs[r].iters;
        q.status = fs[r].status;
        q.rr = fs[r].rr;
        q.bb = fs[r].bb;
        q.resid_true = p->true_resid ? ts[r].resid_true : -1.0;
        q.fell_back = fs[r].fell;
        ctx->scal_host[r] = q;
    }
    return TM_OK;
}

tm_status solve_f64_history(tm_ctx* ctx, uint64_t seed_mixed, const uint64_t* id_dev, double tol, int maxit,
                            std::vector<double>* hist, void* xstar_out, PairSink* sink) {
    const Geom& g = ctx->geo;
    hipStream_t st = ctx->stream;
    tm_status s = TM_OK;
    const size_t nblk = (size_t)((g.V + 255) / 256);
    const size_t fb = field_bytes(g, P_F64, 1);
    CgArgs a;
    std::memset(&a, 0, sizeof(a));
    a.geo = g;
    a.gauge = ctx->gauge64;
    a.kappa = ctx->lat.kappa;
    a.twist = ctx->twist;
    a.nrhs = 1;
    a.npart = (uint32_t)nblk;
    a.p = ws_get(ctx, "h_p", fb, &s);
    a.t = ws_get(ctx, "h_t", fb, &s);
    a.r = ws_get(ctx, "h_r", fb, &s);
    a.x = ws_get(ctx, "h_x", fb, &s);
    void* eta = ws_get(ctx, "h_eta", fb, &s);
    void* mx = ws_get(ctx, "h_mx", fb, &s);
    a.scal = (CgScal*)ws_get(ctx, "h_scal", sizeof(CgScal) * kMaxBlock, &s);
    a.partials = (double*)ws_get(ctx, "partials", sizeof(double) * partials_per_rhs(g, ctx->hgeo, ctx->eo_ok) * kMaxBlock, &s);
    a.partials2 = (double*)ws_get(ctx, "partials2", sizeof(double) * partials_per_rhs(g, ctx->hgeo, ctx->eo_ok) * kMaxBlock, &s);
    if (s != TM_OK) return s;
    launch_scal_init(st, a.scal, 1, tol * tol, maxit, 0, 0, 0.0);
    launch_noise_native(st, g, P_F64, seed_mixed, id_dev, 1, eta);
    launch_apply(st, g, P_F64, ctx->gauge64, ctx->lat.kappa, ctx->twist, 1, 1, eta, a.r, 1, nullptr);
    launch_cg_init(st, a, P_F64, false, eta);
    TM_HIP(hipGetLastError());
    size_t cut = 0;
    auto maybe_cut = [&](int it) -> tm_status {
        if (!sink || cut >= sink->ks.size() || sink->ks[cut] != it) return TM_OK;
        launch_apply(st, g, P_F64, ctx->gauge64, ctx->lat.kappa, ctx->twist, 0, 1, a.x, mx, 1, nullptr);
        launch_make_pair(st, g, seed_mixed, id_dev, a.x, sink->xstar, mx, (char*)sink->R + sink->next * sink->fb,
                         (char*)sink->E + sink->next * sink->fb);
        TM_HIP(hipGetLastError());
        sink->next++;
        cut++;
        return TM_OK;
    };
    CgScal q;
    TM_HIP(hipMemcpyAsync(&q, a.scal, sizeof(CgScal), hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    if (hist) hist->push_back(q.rr / q.bb);
    if ((s = maybe_cut(0)) != TM_OK) return s;
    while (q.active && q.iters < kIterCap) {
        launch_cg_mp(st, a, P_F64, 1);
        launch_cg_alpha(st, a);
        launch_cg_upd(st, a, P_F64, 1, false);
        launch_cg_beta(st, a, false);
        launch_cg_p(st, a, P_F64);
        TM_HIP(hipGetLastError());
        TM_HIP(hipMemcpyAsync(&q, a.scal, sizeof(CgScal), hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
        if (hist) hist->push_back(q.rr / q.bb);
        if ((s = maybe_cut(q.iters)) != TM_OK) return s;
    }
    if (xstar_out) TM_HIP(hipMemcpyAsync(xstar_out, a.x, fb, hipMemcpyDeviceToDevice, st));
    TM_HIP(hipStreamSynchronize(st));
    return TM_OK;
}

// Bytes of the even-odd CG kernels per launch (algorithmic, per half site:
// each field touched once, every link once per half-hop)
struct EoBytes {
    double hop, mp, upd, p;
};
static EoBytes eo_bytes(const Geom& hg, int prec, int nrhs, bool track, bool xfree) {
    const double bs = prec == P_F64 ? 8 : (prec == P_F32 ? 4 : 2);
    const double bx = prec == P_F64 ? 8 : 4;
    const double gb = prec == P_F64 ? 8 * 18 * 8 : 8 * 12 * 4;  // the FP16 copy holds 9 of 12 words
    const double V = (double)hg.V;
    EoBytes b;
    b.hop = V * (nrhs * 48.0 * bs + gb);
    b.mp = V * (nrhs * 72.0 * bs + gb);
    // y, t, r read and r written; without the ring also p and x read, x written
    b.upd = V * (nrhs * (96.0 * bs + (xfree ? 0.0 : 24.0 * bs + 48.0 * bx) + (track ? 48.0 * bs : 0.0)) + gb);
    b.p = V * nrhs * 72.0 * bs;
    return b;
}

// CG on the normal equations of the even-odd Schur complement (solver
// TM_SOLVER_CG_EO): the odd-site source etahat = eta_o + kappa H_oe D^{-1}
// eta_e and b = Mhat^dag etahat, the CG chunks on half fields (four
// half-hops per iteration), then x_e = D^{-1} (eta_e + kappa H_eo x_o) and
// the full native solution in res.  Reliable updates recompute
// r = b - Mhat^dag Mhat x in FP64 on the half lattice.
// halves: the caller can take the solution as its two halves (the standard
// loop's contraction), FP32, or FP16 for an FP16 solve, which saves writing
// the full native field
static tm_status solve_block_eo(tm_ctx* ctx, const tsm_solve_params* p, uint64_t seed_mixed,
                                const uint64_t* ids_dev, int nrhs, int nr, const std::string& tag,
                                BlockResult* res, bool halves) {
    const Geom& g = ctx->geo;
    const Geom& hg = ctx->hgeo;
    hipStream_t st = ctx->stream;
    tm_status s = TM_OK;
    const int prec = p->prec;
    const bool rel = p->reliable != 0;
    const bool track = p->stop == TM_STOP_TRUE && !rel;
    const int xprec = prec == P_F64 ? P_F64 : P_F32;
    const size_t nblk_full = (size_t)((g.V + 255) / 256);
    const uint32_t nblk = (uint32_t)((hg.V + 255) / 256);
    const size_t fbh = field_bytes(hg, prec, nrhs);
    // buffers sized for the tag's capacity (at least nrhs)
    const int nc = ws_rhs(ctx, tag, nrhs);
    const size_t fbc = field_bytes(hg, prec, nc);
    const double kappa = ctx->lat.kappa, tw = ctx->twist;
    const double ee_z4 = 12.0 * (double)g.V;

    // FP32 arithmetic runs the tile kernels (links staged in LDS, shared by
    // the block's right-hand sides); FP64 the lane-per-site kernels
    const bool tiles = prec != P_F64 && ctx->eo_tiles[prec] != 0;
    CgArgs a;
    std::memset(&a, 0, sizeof(a));
    a.geo = hg;
    a.kappa = kappa;
    a.twist = tw;
    a.nrhs = nrhs;
    a.npart = tiles ? eot_tiles(hg) : nblk;
    // search directions in a ring (CgArgs::pn): without reliable updates, on
    // the lane-per-site kernels; x is formed from the step lengths every
    // kRing - 1 iterations and at the end
    const bool ringm = !rel && prec != P_F64 && !tiles;
    constexpr int kRing = kEoRing;
    void* dirs = nullptr;
    if (ringm) {
        dirs = ws_get(ctx, tag + "_eo_dirs", fbc * kRing, &s);
        a.ahist = (double*)ws_get(ctx, tag + "_eo_ahist", sizeof(double) * kMaxBlock * kRing, &s);
        a.ring = kRing;
        a.p = dirs;  // p_0, written by the CG start
    } else {
        a.p = ws_get(ctx, tag + "_eo_p", fbc, &s);
    }
    auto slot = [&](int k) { return (void*)((char*)dirs + (size_t)(k % kRing) * fbh); };
    a.t = ws_get(ctx, tag + "_eo_t", fbc, &s);
    a.r = ws_get(ctx, tag + "_eo_r", fbc, &s);
    a.x = ws_get(ctx, tag + "_eo_x", field_bytes(hg, xprec, nc), &s);
    void* y = ws_get(ctx, tag + "_eo_y", fbc, &s);
    a.scal = (CgScal*)ws_get(ctx, tag + "_scal", sizeof(CgScal) * kMaxBlock, &s);
    const size_t npart_max = partials_per_rhs(g, hg, ctx->eo_ok);
    a.partials = (double*)ws_get(ctx, "partials", sizeof(double) * npart_max * kMaxBlock, &s);
    a.partials2 = (double*)ws_get(ctx, "partials2", sizeof(double) * npart_max * kMaxBlock, &s);
    if (track) a.rho = ws_get(ctx, tag + "_eo_rho", fbc, &s);
    // the full solution handed to the contraction
    const int fprec = rel ? P_F64 : xprec;
    void* xfull = ws_get(ctx, tag + "_eo_xfull", field_bytes(g, fprec, nc), &s);
    // source preparation at the iteration precision (FP64 with reliable
    // updates); the tile kernels take the sources from the hash
    const int sp = rel ? P_F64 : prec;
    // FP64 half-hops: two sources per lane (the links are read once per pair)
    const int nr64 = nrhs % 2 == 0 ? 2 : 1;
    const int snr = sp == P_F64 ? nr64 : nr;
    void* eh = ws_get(ctx, tag + "_eo_eh", field_bytes(hg, sp, nc), &s);
    void *b64 = nullptr, *x64 = nullptr, *t64 = nullptr, *y64 = nullptr;
    if (rel) {
        b64 = ws_get(ctx, tag + "_eo_b64", field_bytes(hg, P_F64, nc), &s);
        x64 = ws_get(ctx, tag + "_eo_x64", field_bytes(hg, P_F64, nc), &s);
        t64 = ws_get(ctx, tag + "_eo_t64", field_bytes(hg, P_F64, nc), &s);
        y64 = ws_get(ctx, tag + "_eo_y64", field_bytes(hg, P_F64, nc), &s);
    }
    if (s != TM_OK) return s;
    if ((s = ensure_scal_host(ctx, nrhs)) != TM_OK) return s;

    const void* g32e = ctx->gauge32eo[0];
    const void* g32o = ctx->gauge32eo[1];
    const void* g64e = ctx->gauge64eo[0];
    const void* g64o = ctx->gauge64eo[1];
    // links of the iteration: FP64, FP32, or FP16 for the FP16-storage hops
    // of the lane-per-site kernels
    const bool h16 = prec == P_F16 && !tiles;
    const void* ge = prec == P_F64 ? g64e : (h16 ? ctx->gauge16eo[0] : g32e);
    const void* go = prec == P_F64 ? g64o : (h16 ? ctx->gauge16eo[1] : g32o);
    // half-hop arguments: output parity q, input field, output field
    auto lin = [&](int q, bool f64, const void* in, void* out, const void* b, double c, int n) {
        EoArgs e;
        std::memset(&e, 0, sizeof(e));
        e.hg = hg;
        e.gout = q == 0 ? (f64 ? g64e : ge) : (f64 ? g64o : go);
        e.gin = q == 0 ? (f64 ? g64o : go) : (f64 ? g64e : ge);
        e.pout = q;
        e.kappa = kappa;
        e.twist = tw;
        e.in = in;
        e.out = out;
        e.b = b;
        e.c = c;
        e.seed_mixed = seed_mixed;
        e.ids = ids_dev;
        e.nrhs = n;
        return e;
    };
    const double k2 = -kappa * kappa;

    launch_scal_init(st, a.scal, nrhs, p->tol * p->tol, p->max_iter, p->stop, rel ? 1 : 0,
                     rel ? p->delta * p->delta : 0.0);
    // sources: etahat = eta_o + kappa H_oe D^{-1} eta_e,
    // b = Mhat^dag etahat = D^dag etahat - kappa^2 H_oe^dag D^{-dag} H_eo^dag etahat
    prof_begin(ctx, TM_KC_OTHER);
    void* ys = rel ? y64 : y;
    if (tiles && !rel) {
        EoArgs es = lin(1, false, nullptr, eh, nullptr, kappa, nrhs);
        launch_eot_src(st, es, prec, nr);
        launch_eot_y(st, lin(0, false, eh, y, nullptr, 1.0, nrhs), prec, nr, true, nullptr);
        EoCg ei;
        ei.geven = g32e;
        ei.godd = g32o;
        ei.y = y;
        // r = b = D^dag etahat - kappa^2 H_oe^dag y (all sources active: no
        // scalars yet)
        CgArgs ai = a;
        ai.scal = nullptr;
        launch_eot_mp(st, ai, ei, prec, nr, true, eh, a.r);
        launch_cg_init(st, a, prec, track, eh, ee_z4);  // (the tile path updates x: no ring)
    } else {
        // etahat from the hash, then y = D^{-dag} H_eo^dag etahat and b
        EoArgs es = lin(1, sp == P_F64, nullptr, eh, nullptr, kappa, nrhs);
        if (sp != P_F64) {  // FP32 arithmetic with FP32 links
            es.gout = g32o;
            es.gin = g32e;
        }
        launch_eo_src(st, es, sp, snr);
        launch_eo_lin(st, lin(0, rel, eh, ys, nullptr, 1.0, nrhs), sp, snr, EO_Y_DAG);
        if (rel) {
            launch_eo_lin(st, lin(1, true, ys, b64, eh, k2, nrhs), P_F64, nr64, EO_T_DAG);
            if (p->stop == TM_STOP_TRUE) a.eta64 = eh;
            launch_rel_init(st, a, b64, x64, ee_z4, prec);
        } else {
            launch_eo_lin(st, lin(1, false, ys, a.r, eh, k2, nrhs), prec, snr, EO_T_DAG);
            CgArgs ai = a;
            if (ringm) ai.x = nullptr;  // x is written by the first pass over the kept directions
            launch_cg_init(st, ai, prec, track, eh, ee_z4);
        }
    }
    prof_end(ctx, TM_KC_OTHER, 0.0);
    TM_HIP(hipGetLastError());

    EoCg ec;
    ec.geven = ge;
    ec.godd = go;
    ec.y = y;
    EoCg ec64;
    ec64.geven = g64e;
    ec64.godd = g64o;
    ec64.y = y64;
    const CgArgs a0 = a;
    const int vtag = prof_tag(prec, prec == P_F64 ? 1 : nr, TM_SOLVER_CG_EO, 0, rel);
    const int dflt = rel ? 16 : 8;
    const std::string ckey = chunk_key(p, tag, nrhs);
    int chunk = first_chunk(ctx, ckey, dflt);
    int n_active = nrhs;
    if (ctx->prof) {
        TM_HIP(hipMemcpyAsync(ctx->scal_host, a.scal, sizeof(CgScal) * nrhs, hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
        n_active = active_count(ctx, nrhs);
    }
    int done = 0;
    int k0 = 0;  // ring: first iteration not yet added to x
    auto flush = [&](int k1) {
        if (k1 > k0) {
            prof_begin(ctx, TM_KC_OTHER);
            launch_eo_xflush(st, a, prec, dirs, fbh, k0, k1);
            prof_end(ctx, TM_KC_OTHER, 0.0);
        }
        k0 = k1;
    };
    for (;;) {
        int k = chunk;
        if (p->max_iter >= 0) k = std::max(1, std::min(chunk, p->max_iter - done));
        chunk = later_chunk(ctx, dflt);
        if (ringm) {
            if (done - k0 >= kRing - 1) flush(done);
            k = std::min(k, kRing - 1 - (done - k0));
        }
        const EoBytes by = eo_bytes(hg, prec, n_active, track, ringm);
        auto steps = [&](int n) {
            for (int i = 0; i < n; i++) {
                CgArgs a = a0;  // this iteration's direction slots
                if (ringm) {
                    a.p = slot(done + i);
                    a.pn = slot(done + i + 1);
                }
                EoArgs ey = lin(0, false, a.p, y, nullptr, 1.0, nrhs);
                ey.act = a.scal;
                prof_begin(ctx, TM_KC_EO_HOP, vtag);
                if (tiles)
                    launch_eot_y(st, ey, prec, nr, false, a.scal);
                else
                    launch_eo_lin(st, ey, prec, nr, EO_Y);
                prof_end(ctx, TM_KC_EO_HOP, by.hop);
                prof_begin(ctx, TM_KC_DSLASH, vtag);
                if (tiles)
                    launch_eot_mp(st, a, ec, prec, nr, false, a.p, a.t);
                else
                    launch_eo_mp(st, a, ec, prec, nr);
                prof_end(ctx, TM_KC_DSLASH, by.mp);
                prof_begin(ctx, TM_KC_OTHER);
                launch_cg_alpha(st, a);
                prof_end(ctx, TM_KC_OTHER, 0.0);
                EoArgs ey2 = lin(0, false, a.t, y, nullptr, 1.0, nrhs);
                ey2.act = a.scal;
                prof_begin(ctx, TM_KC_EO_HOP_DAG, vtag);
                if (tiles)
                    launch_eot_y(st, ey2, prec, nr, true, a.scal);
                else
                    launch_eo_lin(st, ey2, prec, nr, EO_Y_DAG);
                prof_end(ctx, TM_KC_EO_HOP_DAG, by.hop);
                const int utag = track ? prof_tag(prec, 1, TM_SOLVER_CG_EO, 0) : vtag;
                prof_begin(ctx, TM_KC_DSLASH_UPD, utag);
                if (tiles)
                    launch_eot_upd(st, a, ec, prec, track ? 1 : nr, track);
                else if (ringm)
                    launch_eo_upd_xfree(st, a, ec, prec, track ? 1 : nr, track);
                else
                    launch_eo_upd(st, a, ec, prec, track ? 1 : nr, track);
                prof_end(ctx, TM_KC_DSLASH_UPD, by.upd);
                prof_begin(ctx, TM_KC_OTHER);
                launch_cg_beta(st, a, track);
                prof_end(ctx, TM_KC_OTHER, 0.0);
                if (rel) {
                    // gated on the reliable flag: x64 += x, t64 = Mhat x64,
                    // r = b64 - Mhat^dag t64
                    prof_begin(ctx, TM_KC_OTHER);
                    launch_rel_flush(st, a, x64, 0);
                    EoArgs e1 = lin(0, true, x64, y64, nullptr, 1.0, nrhs);
                    e1.gate = a.scal;
                    launch_eo_lin(st, e1, P_F64, nr64, EO_Y);
                    EoArgs e2 = lin(1, true, y64, t64, x64, k2, nrhs);
                    e2.gate = a.scal;
                    launch_eo_lin(st, e2, P_F64, nr64, EO_T);
                    EoArgs e3 = lin(0, true, t64, y64, nullptr, 1.0, nrhs);
                    e3.gate = a.scal;
                    launch_eo_lin(st, e3, P_F64, nr64, EO_Y_DAG);
                    launch_eo_rel_resid(st, a, ec64, b64, t64, y64, nr64, prec);
                    launch_rel_fin(st, a, eo_gated_blocks(hg));
                    prof_end(ctx, TM_KC_OTHER, 0.0);
                }
                prof_begin(ctx, TM_KC_BLAS, prof_tag(prec, 1, TM_SOLVER_CG_EO, 0, rel));
                launch_cg_p(st, a, prec);
                prof_end(ctx, TM_KC_BLAS, by.p);
            }
        };
        if (ctx->use_graphs && !ctx->prof && st != nullptr) {
            char key[512];
            std::snprintf(key, sizeof(key),
                          "eo|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%d|%d|%d|%d|%d|%d|%d|%d|%llx", a0.p, a0.t,
                          a0.r, a0.x, y, a0.rho, (void*)a0.scal, (void*)a0.partials, (void*)a0.partials2, x64, t64,
                          b64, y64, (void*)a0.ahist, prec, nr, (int)track, (int)rel, nrhs, k,
                          ringm ? done % kRing : -1, (int)tiles, (unsigned long long)ctx->ws_digest);
            auto it = ctx->graphs.find(key);
            if (it == ctx->graphs.end()) {
                hipGraph_t graph;
                TM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                steps(k);
                hipError_t ce = hipStreamEndCapture(st, &graph);
                if (ce != hipSuccess) return dev_error(ctx, ce, "hipStreamEndCapture");
                hipGraphExec_t exec;
                ce = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (ce != hipSuccess) return dev_error(ctx, ce, "hipGraphInstantiate");
                it = ctx->graphs.emplace(key, exec).first;
            }
            TM_HIP(hipGraphLaunch(it->second, st));
            ctx->graph_launches++;
        } else {
            steps(k);
        }
        TM_HIP(hipGetLastError());
        done += k;
        TM_HIP(hipMemcpyAsync(ctx->scal_host, a.scal, sizeof(CgScal) * nrhs, hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
        n_active = active_count(ctx, nrhs);
        if (n_active == 0) break;
        if (done >= kIterCap) break;
    }
    remember_chunk(ctx, ckey, nrhs);
    // a caller that takes the halves of an FP16 solve gets them in FP16: the
    // last pass over the kept directions writes x_o in FP16 into y (free now)
    const bool to_halves = halves && !rel && !tiles && prec != P_F64 && !p->true_resid;
    const bool halves16 = to_halves && ringm && prec == P_F16;
    if (halves16) {
        prof_begin(ctx, TM_KC_OTHER);
        launch_eo_xflush(st, a, prec, dirs, fbh, k0, done, y, P_F16);
        prof_end(ctx, TM_KC_OTHER, 0.0);
        k0 = done;
    } else if (ringm) {
        flush(done);
    }

    // even half x_e = D^{-1} (eta_e + kappa H_eo x_o) with eta_e from the
    // hash, then the full native solution (or, for a caller that takes the
    // halves, x_e alone beside the odd half x)
    prof_begin(ctx, TM_KC_OTHER);
    if (halves16) {
        // x_e in FP16 by the FP16 half-hop, both halves handed over in FP16
        EoArgs e = lin(0, false, y, xfull, nullptr, kappa, nrhs);
        e.bnoise = 1;
        launch_eo_lin(st, e, P_F16, nr, EO_REC);
        prof_end(ctx, TM_KC_OTHER, 0.0);
        res->x = y;
        res->xe = xfull;
        res->xprec = P_F16;
        TM_HIP(hipGetLastError());
        TM_HIP(hipMemcpyAsync(ctx->scal_host, a.scal, sizeof(CgScal) * nrhs, hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
        return TM_OK;
    }
    if (to_halves) {
        EoArgs e = lin(0, false, a.x, xfull, nullptr, kappa, nrhs);
        e.gout = g32e;
        e.gin = g32o;
        e.bnoise = 1;
        for (int j0 = 0; j0 < nrhs; j0 += kRecSub) {
            EoArgs es = e;
            es.in = (const char*)a.x + field_bytes(hg, P_F32, j0);
            es.out = (char*)xfull + field_bytes(hg, P_F32, j0);
            es.ids = ids_dev + j0;
            es.nrhs = std::min(kRecSub, nrhs - j0);
            launch_eo_lin(st, es, P_F32, nr, EO_REC);
        }
        prof_end(ctx, TM_KC_OTHER, 0.0);
        res->x = a.x;
        res->xe = xfull;  // (the even halves fill the front of the full buffer)
        res->xprec = P_F32;
        TM_HIP(hipGetLastError());
        TM_HIP(hipMemcpyAsync(ctx->scal_host, a.scal, sizeof(CgScal) * nrhs, hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
        return TM_OK;
    }
    if (rel) {
        launch_rel_flush(st, a, x64, 1);
        launch_eo_rec_full(st, lin(0, true, x64, nullptr, nullptr, kappa, nrhs), P_F64, nr64, g, xfull);
    } else if (tiles) {
        launch_eot_rec(st, lin(0, false, a.x, nullptr, nullptr, kappa, nrhs), nr, g, xfull);
    } else {
        EoArgs e = lin(0, prec == P_F64, a.x, nullptr, nullptr, kappa, nrhs);
        if (prec != P_F64) {
            e.gout = g32e;
            e.gin = g32o;
            // FP32 halves of at most kRecSub sources per launch: the
            // neighbours a block gathers are then still in L2 when the blocks
            // of the next time slice need them
            for (int j0 = 0; j0 < nrhs; j0 += kRecSub) {
                EoArgs es = e;
                es.in = (const char*)a.x + field_bytes(hg, xprec, j0);
                es.ids = ids_dev + j0;
                es.nrhs = std::min(kRecSub, nrhs - j0);
                launch_eo_rec_full(st, es, xprec, nr, g, (char*)xfull + field_bytes(g, fprec, j0));
            }
        } else {
            launch_eo_rec_full(st, e, xprec, nr64, g, xfull);
        }
    }
    prof_end(ctx, TM_KC_OTHER, 0.0);
    res->x = xfull;
    res->xprec = fprec;
    if (p->true_resid) {
        CgArgs at = a;
        at.geo = g;
        at.x = xfull;
        prof_begin(ctx, TM_KC_OTHER);
        launch_true_resid(st, at, fprec, ctx->gauge64, seed_mixed, ids_dev);
        prof_end(ctx, TM_KC_OTHER, (double)g.V * (nrhs * 24.0 * (fprec == P_F64 ? 8 : 4) + 4 * 18 * 8.0));
    }
    TM_HIP(hipGetLastError());
    TM_HIP(hipMemcpyAsync(ctx->scal_host, a.scal, sizeof(CgScal) * nrhs, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    return TM_OK;
}

// Solve nrhs sources (ids on the device) with the given settings.  On
// return the stream is synchronised, ctx->scal_host[0..nrhs) holds the final
// per-source state and res the native solutions.
static tm_status solve_block(tm_ctx* ctx, const tsm_solve_params* p, uint64_t seed_mixed, const uint64_t* ids_dev,
                             int nrhs, int nr, const std::string& tag, BlockResult* res, bool halves = false) {
    if (p->solver == TM_SOLVER_FCG_LEARNED) return solve_block_fcg(ctx, p, seed_mixed, ids_dev, nrhs, nr, tag, res);
    if (p->solver == TM_SOLVER_CG_EO) return solve_block_eo(ctx, p, seed_mixed, ids_dev, nrhs, nr, tag, res, halves);
    const Geom& g = ctx->geo;
    hipStream_t st = ctx->stream;
    tm_status s = TM_OK;
    const int prec = p->prec;
    const bool rel = p->reliable != 0;
    // the recursively tracked true residual; with reliable updates the FP64
    // true residual is taken at each update instead
    const bool track = p->stop == TM_STOP_TRUE && !rel;
    const size_t nblk = (size_t)((g.V + 255) / 256);
    // buffers sized for the tag's capacity (at least nrhs)
    const int nc = ws_rhs(ctx, tag, nrhs);
    const size_t fb = field_bytes(g, prec, nc);
    const size_t fx = field_bytes(g, prec == P_F64 ? P_F64 : P_F32, nc);
    const size_t f64 = field_bytes(g, P_F64, nc);

    CgArgs a;
    std::memset(&a, 0, sizeof(a));
    a.geo = g;
    a.gauge = prec == P_F64 ? ctx->gauge64 : ctx->gauge32;
    a.kappa = ctx->lat.kappa;
    a.twist = ctx->twist;
    a.nrhs = nrhs;
    // time-marching K1 / K2 when a segment length is set for this precision
    a.tseg = march_tseg(ctx, p, nr);
    a.npart = a.tseg > 0 ? march_partials(g, a.tseg) : (uint32_t)nblk;
    const size_t npart_max = partials_per_rhs(g, ctx->hgeo, ctx->eo_ok);
    a.p = ws_get(ctx, tag + "_p", fb, &s);
    a.t = ws_get(ctx, tag + "_t", fb, &s);
    a.r = ws_get(ctx, tag + "_r", fb, &s);
    a.x = ws_get(ctx, tag + "_x", fx, &s);
    a.scal = (CgScal*)ws_get(ctx, tag + "_scal", sizeof(CgScal) * kMaxBlock, &s);
    a.partials = (double*)ws_get(ctx, "partials", sizeof(double) * npart_max * kMaxBlock, &s);
    a.partials2 = (double*)ws_get(ctx, "partials2", sizeof(double) * npart_max * kMaxBlock, &s);
    if (track) a.rho = ws_get(ctx, tag + "_rho", fb, &s);
    void* eta = nullptr;
    void *b64 = nullptr, *x64 = nullptr, *t64 = nullptr;
    if (rel) {
        eta = ws_get(ctx, tag + "_eta64", f64, &s);
        if (p->stop == TM_STOP_TRUE) a.eta64 = eta;
        b64 = ws_get(ctx, tag + "_b64", f64, &s);
        x64 = ws_get(ctx, tag + "_x64", f64, &s);
        t64 = ws_get(ctx, tag + "_t64", f64, &s);
    } else {
        eta = ws_get(ctx, tag + "_eta", fb, &s);
    }
    if (s != TM_OK) return s;
    if ((s = ensure_scal_host(ctx, nrhs)) != TM_OK) return s;

    const double tol2 = p->tol * p->tol;
    const double delta2 = rel ? p->delta * p->delta : 0.0;
    launch_scal_init(st, a.scal, nrhs, tol2, p->max_iter, p->stop, rel ? 1 : 0, delta2);

    const double gb64 = 4 * 18 * 8.0;

    // sources and right-hand side b = M^dag eta
    prof_begin(ctx, TM_KC_OTHER);
    if (rel) {
        launch_noise_native(st, g, P_F64, seed_mixed, ids_dev, nrhs, eta);
        launch_apply(st, g, P_F64, ctx->gauge64, ctx->lat.kappa, ctx->twist, 1, nrhs, eta, b64, 1, nullptr);
        launch_rel_init(st, a, b64, x64);
    } else {
        launch_noise_native(st, g, prec, seed_mixed, ids_dev, nrhs, eta);
        launch_apply(st, g, prec, a.gauge, ctx->lat.kappa, ctx->twist, 1, nrhs, eta, a.r, nr, nullptr);
        launch_cg_init(st, a, prec, track, eta);
    }
    prof_end(ctx, TM_KC_OTHER, 0.0);
    TM_HIP(hipGetLastError());

    const int vtag = prof_tag(prec, prec == P_F64 ? 1 : nr, TM_SOLVER_CG, a.tseg);
    const int dflt = rel ? 16 : 8;
    const std::string ckey = chunk_key(p, tag, nrhs);
    int chunk = first_chunk(ctx, ckey, dflt);
    int n_active = nrhs;
    if (ctx->prof) {
        TM_HIP(hipMemcpyAsync(ctx->scal_host, a.scal, sizeof(CgScal) * nrhs, hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
        n_active = active_count(ctx, nrhs);
    }
    int done = 0;
    for (;;) {
        int k = chunk;
        if (p->max_iter >= 0) k = std::max(1, std::min(chunk, p->max_iter - done));
        chunk = later_chunk(ctx, dflt);
        const CgBytes by = cg_bytes(g, prec, n_active, rel, track);
        auto steps = [&](int n) {
            for (int i = 0; i < n; i++) {
                prof_begin(ctx, TM_KC_DSLASH, vtag);
                if (a.tseg > 0)
                    launch_tm_mp(st, a, prec, nr);
                else
                    launch_cg_mp(st, a, prec, nr);
                prof_end(ctx, TM_KC_DSLASH, by.k1);
                prof_begin(ctx, TM_KC_OTHER);
                launch_cg_alpha(st, a);
                prof_end(ctx, TM_KC_OTHER, 0.0);
                prof_begin(ctx, TM_KC_DSLASH_UPD, track ? prof_tag(prec, 1, TM_SOLVER_CG, a.tseg) : vtag);
                if (a.tseg > 0)
                    launch_tm_upd(st, a, prec, nr, track);
                else
                    launch_cg_upd(st, a, prec, nr, track);
                prof_end(ctx, TM_KC_DSLASH_UPD, by.k2);
                prof_begin(ctx, TM_KC_OTHER);
                launch_cg_beta(st, a, track);
                prof_end(ctx, TM_KC_OTHER, 0.0);
                if (rel) {
                    prof_begin(ctx, TM_KC_OTHER);
                    launch_rel_flush(st, a, x64, 0);
                    launch_apply(st, g, P_F64, ctx->gauge64, ctx->lat.kappa, ctx->twist, 0, nrhs, x64, t64, 1,
                                 a.scal);
                    launch_rel_resid(st, a, ctx->gauge64, b64, t64);
                    prof_end(ctx, TM_KC_OTHER, 0.0);
                }
                prof_begin(ctx, TM_KC_BLAS, prof_tag(prec, 1, TM_SOLVER_CG));
                launch_cg_p(st, a, prec);
                prof_end(ctx, TM_KC_BLAS, by.k3);
            }
        };
        if (ctx->use_graphs && !ctx->prof && st != nullptr) {
            // the chunk's launches depend only on the buffers and the launch
            // configuration, so one captured graph serves every chunk
            char key[512];
            std::snprintf(key, sizeof(key), "cg|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%d|%d|%d|%d|%d|%d|%d|%llx", a.p,
                          a.t, a.r, a.x, a.rho, (void*)a.scal, (void*)a.partials, (void*)a.partials2, x64, t64, b64,
                          (void*)a.eta64, prec, nr, a.tseg, (int)track, (int)rel, nrhs, k,
                          (unsigned long long)ctx->ws_digest);
            auto it = ctx->graphs.find(key);
            if (it == ctx->graphs.end()) {
                hipGraph_t graph;
                TM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                steps(k);
                hipError_t ce = hipStreamEndCapture(st, &graph);
                if (ce != hipSuccess) return dev_error(ctx, ce, "hipStreamEndCapture");
                hipGraphExec_t exec;
                ce = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (ce != hipSuccess) return dev_error(ctx, ce, "hipGraphInstantiate");
                it = ctx->graphs.emplace(key, exec).first;
            }
            TM_HIP(hipGraphLaunch(it->second, st));
            ctx->graph_launches++;
        } else {
            steps(k);
        }
        TM_HIP(hipGetLastError());
        done += k;
        TM_HIP(hipMemcpyAsync(ctx->scal_host, a.scal, sizeof(CgScal) * nrhs, hipMemcpyDeviceToHost, st));
        TM_HIP(hipStreamSynchronize(st));
        n_active = active_count(ctx, nrhs);
        if (n_active == 0) break;
        if (done >= kIterCap) break;
    }
    remember_chunk(ctx, ckey, nrhs);
    if (rel) {
        launch_rel_flush(st, a, x64, 1);
        res->x = x64;
        res->xprec = P_F64;
    } else {
        res->x = a.x;
        res->xprec = prec == P_F64 ? P_F64 : P_F32;
    }
    if (p->true_resid) {
        CgArgs at = a;
        at.x = res->x;
        prof_begin(ctx, TM_KC_OTHER);
        launch_true_resid(st, at, res->xprec, ctx->gauge64, seed_mixed, ids_dev);
        prof_end(ctx, TM_KC_OTHER, (double)g.V * (nrhs * 24.0 * (res->xprec == P_F64 ? 8 : 4) + gb64));
    }
    TM_HIP(hipGetLastError());
    TM_HIP(hipMemcpyAsync(ctx->scal_host, a.scal, sizeof(CgScal) * nrhs, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    return TM_OK;
}

static void fill_stats(const CgScal& q, tsm_solve_stats* o) {
    o->iters = q.iters;
    o->converged = q.status == 1;
    o->truncated = q.status == 2;
    o->fell_back = q.fell_back;
    if (q.stop == 1)
        o->resid_iterated = q.ee > 0 ? std::sqrt(q.rho2 / q.ee) : 0.0;
    else
        o->resid_iterated = q.bb > 0 ? std::sqrt(q.rr / q.bb) * (q.reliable ? q.sigma : 1.0) : 0.0;
    o->resid_true = q.resid_true;
}

// ---------------------------------------------------------------------------
// contraction set-up
// ---------------------------------------------------------------------------
struct MomPlan {
    int np[3];
    std::vector<int> vals[3];
    std::vector<int> idx;  // [n_mom][3]
};

static tm_status plan_momenta(tm_ctx* ctx, int n_mom, const int32_t* mom, MomPlan* mp) {
    if (n_mom < 1 || !mom) return set_error(ctx, TM_EINVAL, "need at least one momentum");
    for (int d = 0; d < 3; d++) {
        mp->vals[d].clear();
        for (int m = 0; m < n_mom; m++) {
            int v = mom[3 * m + d];
            if (std::find(mp->vals[d].begin(), mp->vals[d].end(), v) == mp->vals[d].end()) mp->vals[d].push_back(v);
        }
        if (mp->vals[d].size() > 3)
            return set_error(ctx, TM_ENOTSUP, "more than 3 distinct momentum components on one axis");
        mp->np[d] = (int)mp->vals[d].size();
    }
    mp->idx.resize(3 * n_mom);
    for (int m = 0; m < n_mom; m++)
        for (int d = 0; d < 3; d++)
            mp->idx[3 * m + d] =
                (int)(std::find(mp->vals[d].begin(), mp->vals[d].end(), mom[3 * m + d]) - mp->vals[d].begin());
    return TM_OK;
}

struct Contractor {
    ContractArgs a;
};

// loop sets per source of an estimator: one per direction for the
// one-derivative loops
static int loop_sets(int est) { return est == TM_LOOP_DERIVATIVE ? 4 : 1; }

// Upload phase tables and indices; scratch sized for `maxr` sources.  est
// selects the loop form: 0 the standard eta^dag Gamma s, 1 and 2 the
// one-end loops of section 2.3 (Eqs. 5 and 6), 3 the one-derivative loops
// (four sets per source, one per direction).
static tm_status setup_contract(tm_ctx* ctx, const MomPlan& mp, int n_mom, int maxr, uint64_t seed_mixed,
                                int est, Contractor* c) {
    const Geom& g = ctx->geo;
    tm_status s = TM_OK;
    std::memset(&c->a, 0, sizeof(c->a));
    ContractArgs& a = c->a;
    a.geo = g;
    a.seed_mixed = seed_mixed;
    a.est = est;
    // isovector: Tr[X (M_u^-1 - M_d^-1)] = -2i tw <s^dag g5 X s> with tw = 2 kappa mu,
    // from M_u - M_d = 2i tw g5 (the printed sign of Eq. 5 is the opposite)
    a.coef = est == 1 ? make_double2(0.0, -2.0 * ctx->twist) : make_double2(est == 2 ? 2.0 : 1.0, 0.0);
    a.nmu = loop_sets(est);
    a.gauge64 = ctx->gauge64;
    a.gauge32 = ctx->gauge32;
    a.npx = mp.np[0];
    a.npy = mp.np[1];
    a.npz = mp.np[2];
    a.n_mom = n_mom;
    // host table: phases then indices
    const int L0 = g.L[0], L1 = g.L[1], L2 = g.L[2];
    std::vector<double> ph(2 * (a.npx * L0 + a.npy * L1 + a.npz * L2));
    size_t o = 0;
    const double twopi = 2.0 * std::acos(-1.0);
    for (int d = 0; d < 3; d++)
        for (int i = 0; i < mp.np[d]; i++)
            for (int x = 0; x < g.L[d]; x++) {
                double arg = twopi * (double)mp.vals[d][i] * x / g.L[d];
                ph[o++] = std::cos(arg);
                ph[o++] = -std::sin(arg);
            }
    double* phd = (double*)ws_get(ctx, "c_phase", sizeof(double) * ph.size(), &s);
    int* idd = (int*)ws_get(ctx, "c_momidx", sizeof(int) * mp.idx.size(), &s);
    if (s != TM_OK) return s;
    TM_COPY(phd, ph.data(), sizeof(double) * ph.size(), hipMemcpyHostToDevice);
    TM_COPY(idd, mp.idx.data(), sizeof(int) * mp.idx.size(), hipMemcpyHostToDevice);
    a.phx = (const double2*)phd;
    a.phy = a.phx + a.npx * L0;
    a.phz = a.phy + a.npy * L1;
    a.mom_idx = idd;
    a.gam_col = ctx->gam_dev + 128 * (est == 3 ? 0 : est);
    a.gam_ph = a.gam_col + 64;
    const size_t A = (size_t)maxr * a.nmu * g.L[3] * g.L[2] * a.npy * g.L[0] * 16 * 16;
    const size_t B = (size_t)maxr * a.nmu * g.L[3] * g.L[2] * a.npx * a.npy * 16 * 16;
    a.A = (double2*)ws_get(ctx, "c_A", A, &s);
    a.B = (double2*)ws_get(ctx, "c_B", B, &s);
    if (est == 2) a.dsol = ws_get(ctx, "c_dsol", field_bytes(g, P_F64, maxr), &s);
    if (s != TM_OK) return s;
    return TM_OK;
}

static void contract_block(tm_ctx* ctx, Contractor* c, const uint64_t* ids_dev, const void* x, int xprec, int nrhs,
                           double2* out, const int* slots_dev, long out_stride, const void* xe = nullptr) {
    ContractArgs a = c->a;
    a.ids = ids_dev;
    a.sol = x;
    a.sol_e = xe;  // (x and xe the two halves in xprec; standard loop only)
    a.hgeo = ctx->hgeo;
    a.nrhs = nrhs;
    a.out = out;
    a.out_slot = slots_dev;
    a.out_stride = out_stride;
    const double sb = (double)ctx->geo.V * nrhs * 24.0 * (xprec == P_F64 ? 8 : (xprec == P_F32 ? 4 : 2));
    if (a.est == 2) {
        // D s = (1 - kappa H) s: the operator at zero twist in the solution's
        // precision (FP64 links and arithmetic, or FP32 ones)
        const Geom& g = ctx->geo;
        prof_begin(ctx, TM_KC_OTHER);
        if (xprec == P_F64)
            launch_apply(ctx->stream, g, P_F64, ctx->gauge64, ctx->lat.kappa, 0.0, 0, nrhs, x, (void*)a.dsol, 1,
                         nullptr);
        else
            launch_apply(ctx->stream, g, P_F32, ctx->gauge32, ctx->lat.kappa, 0.0, 0, nrhs, x, (void*)a.dsol,
                         nrhs % 2 == 0 ? 2 : 1, nullptr);
        prof_end(ctx, TM_KC_OTHER,
                 2 * sb + (xprec == P_F64 ? (double)g.V * 144.0 * 8 : (double)g.V * 48.0 * 8));
    }
    prof_begin(ctx, TM_KC_CONTRACT);
    launch_contract(ctx->stream, a, xprec);
    // est 3 reads s at x and its eight neighbours (each reused by eight
    // sites: counted once) and the FP64 links once
    prof_end(ctx, TM_KC_CONTRACT,
             a.est == 2 ? 2 * sb
                        : (a.est == 3 ? sb + (double)ctx->geo.V * 4 * 18 * 8 : sb));
}

// Standard loops of given solutions at all Lx*Ly*Lz momenta (n_mom =
// TM_ALL_MOMENTA): Gamma traces at each site and three DFT passes; blocks of
// up to four sources (each block holds one buffer of V * 16 complex per
// source).
static tm_status contract_all_momenta(tm_ctx* ctx, uint64_t seed, int32_t nsrc, const uint64_t* ids_host,
                                      const double* sol_dev, double* loops_host) {
    const Geom& g = ctx->geo;
    hipStream_t st = ctx->stream;
    tm_status s = TM_OK;
    if (g.L[0] > 128 || g.L[1] > 128 || g.L[2] > 128)
        return set_error(ctx, TM_ENOTSUP, "tsm_contract: all momenta need spatial extents <= 128");
    const int blk = std::min(nsrc, 4);
    const long V3 = (long)g.L[0] * g.L[1] * g.L[2];
    const long nl = 16L * V3 * g.L[3];
    std::vector<double> tw;
    const double twopi = 2.0 * std::acos(-1.0);
    for (int d = 0; d < 3; d++)
        for (int m = 0; m < g.L[d]; m++) {
            tw.push_back(std::cos(twopi * m / g.L[d]));
            tw.push_back(-std::sin(twopi * m / g.L[d]));
        }
    double* twd = (double*)ws_get(ctx, "fft_tw", sizeof(double) * tw.size(), &s);
    double2* buf0 = (double2*)ws_get(ctx, "fft_buf0", sizeof(double2) * 16 * (size_t)g.V * blk, &s);
    uint64_t* ids_dev = (uint64_t*)ws_get(ctx, "contract_ids", sizeof(uint64_t) * nsrc, &s);
    int* slots = (int*)ws_get(ctx, "contract_slots", sizeof(int) * nsrc, &s);
    void* nat = ws_get(ctx, "contract_nat", field_bytes(g, P_F64, blk), &s);
    double* out = (double*)ws_get(ctx, "fft_out", sizeof(double) * 2 * nl * nsrc, &s);
    if (s != TM_OK) return s;
    std::vector<int> sl(nsrc);
    for (int i = 0; i < nsrc; i++) sl[i] = i;
    TM_COPY(twd, tw.data(), sizeof(double) * tw.size(), hipMemcpyHostToDevice);
    TM_COPY(ids_dev, ids_host, sizeof(uint64_t) * nsrc, hipMemcpyHostToDevice);
    TM_COPY(slots, sl.data(), sizeof(int) * nsrc, hipMemcpyHostToDevice);
    ContractArgs a;
    std::memset(&a, 0, sizeof(a));
    a.geo = g;
    a.seed_mixed = seed_mix(seed);
    a.gam_col = ctx->gam_dev;
    a.gam_ph = ctx->gam_dev + 64;
    a.out = (double2*)out;
    a.out_stride = nl;
    a.nmu = 1;
    for (int j0 = 0; j0 < nsrc; j0 += blk) {
        const int nb = std::min(blk, nsrc - j0);
        launch_field_convert(st, g, P_F64, nb, true, sol_dev + (size_t)j0 * g.V * 24, nat);
        a.ids = ids_dev + j0;
        a.sol = nat;
        a.nrhs = nb;
        a.out_slot = slots + j0;
        prof_begin(ctx, TM_KC_CONTRACT);
        launch_contract_all_momenta(st, a, P_F64, buf0, nullptr, (const double2*)twd);
        // the three passes: the solution read once (24 FP64), 16 complex per
        // site written by the x pass, read and written by the y pass, read
        // by the z pass, and the loops written
        prof_end(ctx, TM_KC_CONTRACT, (double)g.V * nb * (24.0 * 8 + 5 * 16 * 16.0));
        TM_HIP(hipGetLastError());
    }
    TM_HIP(hipMemcpyAsync(loops_host, out, sizeof(double) * 2 * nl * nsrc, hipMemcpyDeviceToHost, st));
    TM_HIP(hipStreamSynchronize(st));
    return TM_OK;
}

// ---- workspace bounds (tm_workspace_bytes) ----

// Scratch of one solve_block call for nc right-hand sides under settings p,
// whatever lane width, tile or time-marching choice the context makes: the
// buffers of the solver path, each rounded to 256 B.  The partial arrays
// shared by every solve of a call are counted by ws_partials.
static size_t ws_block(const Geom& g, const Geom& hg, const tsm_solve_params* p, int nc) {
    const size_t scal = align256(sizeof(CgScal) * kMaxBlock);
    const int prec = p->prec;
    const bool rel = p->reliable != 0;
    const bool track = p->stop == TM_STOP_TRUE && !rel;
    if (p->solver == TM_SOLVER_FCG_LEARNED) {
        const size_t fb = align256(field_bytes(g, P_F32, nc));
        return 7 * fb + align256(sizeof(FcgScal) * kMaxBlock) + scal + align256(field_bytes(g, P_BH, nc)) +
               ws_net_apply(g, nc);
    }
    if (p->solver == TM_SOLVER_CG_EO) {
        const int xprec = prec == P_F64 ? P_F64 : P_F32;
        const size_t fb = align256(field_bytes(hg, prec, nc));
        const bool ring = !rel && prec != P_F64;
        size_t b = ring ? align256(field_bytes(hg, prec, nc) * kEoRing) + align256(sizeof(double) * kMaxBlock * kEoRing)
                        : fb;
        b += 3 * fb + align256(field_bytes(hg, xprec, nc)) + scal + (track ? fb : 0);
        b += align256(field_bytes(g, rel ? P_F64 : xprec, nc));
        b += align256(field_bytes(hg, rel ? P_F64 : prec, nc));  // etahat
        if (rel) b += 4 * align256(field_bytes(hg, P_F64, nc));
        return b;
    }
    const size_t fb = align256(field_bytes(g, prec, nc));
    size_t b = 3 * fb + align256(field_bytes(g, prec == P_F64 ? P_F64 : P_F32, nc)) + scal + (track ? fb : 0);
    b += rel ? 4 * align256(field_bytes(g, P_F64, nc)) : fb;
    return b;
}

static size_t ws_partials(const Geom& g, const Geom& hg, bool eo_ok, bool fcg) {
    const size_t n = partials_per_rhs(g, hg, eo_ok) * kMaxBlock;
    return 2 * align256(sizeof(double) * n) + (fcg ? align256(sizeof(double) * n * 4) : 0);
}

// setup_contract for maxr sources: phase tables, momentum indices, the two
// stage buffers (nd distinct values per momentum component) and, for the
// generalized one-end loop, D s
static size_t ws_contract_setup(const Geom& g, int n_mom, int nd, int maxr, uint32_t est_mask) {
    const int nmu = (est_mask & (1u << TM_LOOP_DERIVATIVE)) ? 4 : 1;
    size_t b = align256(sizeof(double) * 2 * (size_t)nd * (g.L[0] + g.L[1] + g.L[2])) +
               align256(sizeof(int) * 3 * (size_t)n_mom);
    b += align256((size_t)maxr * nmu * g.L[3] * g.L[2] * nd * g.L[0] * 256);
    b += align256((size_t)maxr * nmu * g.L[3] * g.L[2] * nd * nd * 256);
    if (est_mask & (1u << TM_LOOP_ONEEND_GENERALIZED)) b += align256(field_bytes(g, P_F64, maxr));
    return b;
}

static size_t ws_bound(const tm_lattice* lat, const Geom& g, const Geom& hg, bool eo_ok,
                       const std::vector<tsm_solve_params>& sv, int max_sources, int max_mom, int nd,
                       uint32_t est_mask, int all_mom, int field_rhs, int train_pairs, int train_sources,
                       int loss_pairs) {
    (void)lat;
    const int N = std::max(max_sources, 1);
    const int nmu = (est_mask & (1u << TM_LOOP_DERIVATIVE)) ? 4 : 1;
    std::vector<int> blk(sv.size());
    bool fcg = false;
    int bmax = 1;
    for (size_t i = 0; i < sv.size(); i++) {
        blk[i] = std::min(default_block(&sv[i]), kMaxBlock);
        bmax = std::max(bmax, blk[i]);
        fcg = fcg || sv[i].solver == TM_SOLVER_FCG_LEARNED;
    }
    const size_t parts = ws_partials(g, hg, eo_ok, fcg);
    size_t best = ws_abi_scratch(g, field_rhs, bmax);
    // tsm_solve_batch
    for (size_t i = 0; i < sv.size(); i++)
        best = std::max(best, align256(sizeof(uint64_t) * (N + 4)) + ws_block(g, hg, &sv[i], blk[i]) + parts);
    // autotuners: a truncated solve at each listed precision and block
    for (size_t i = 0; i < sv.size(); i++) {
        tsm_solve_params t = sv[i];
        t.reliable = 0;
        t.stop = TM_STOP_NORMAL;
        const size_t ids = align256(sizeof(uint64_t) * blk[i]);
        t.solver = TM_SOLVER_CG;
        best = std::max(best, ids + ws_block(g, hg, &t, blk[i]) + parts);
        if (eo_ok) {
            t.solver = TM_SOLVER_CG_EO;
            best = std::max(best, ids + ws_block(g, hg, &t, blk[i]) + parts);
        }
    }
    // tsm_contract / tsm_contract_est at max_mom
    {
        const int b = std::min(N, kMaxBlock);
        const size_t nl = (size_t)16 * nmu * max_mom * g.L[3];
        best = std::max(best, ws_contract_setup(g, max_mom, nd, b, est_mask) + align256(sizeof(uint64_t) * N) +
                                  align256(sizeof(int) * N) + align256(field_bytes(g, P_F64, b)) +
                                  align256(sizeof(double) * 2 * nl * N));
    }
    // tsm_contract at all momenta
    if (all_mom > 0) {
        const int b = std::min(all_mom, 4);
        best = std::max(best, align256(sizeof(double) * 2 * (g.L[0] + g.L[1] + g.L[2])) +
                                  align256(sizeof(double) * 2 * 16 * (size_t)g.V * b) +
                                  align256(sizeof(uint64_t) * all_mom) + align256(sizeof(int) * all_mom) +
                                  align256(field_bytes(g, P_F64, b)) +
                                  align256(sizeof(double) * 2 * 16 * (size_t)g.V * all_mom));
    }
    // tsm_loops: any two listed settings as lp and hp
    if (!sv.empty()) {
        const size_t nl = (size_t)16 * nmu * max_mom * g.L[3];
        const size_t fixed = ws_contract_setup(g, max_mom, nd, bmax + 4, est_mask) +
                             align256(sizeof(double) * 4 * nl * N) + 2 * align256(sizeof(uint64_t) * (N + 8)) +
                             align256(sizeof(double) * 12 * nl) + parts;
        size_t pair = 0;
        for (size_t i = 0; i < sv.size(); i++)
            for (size_t j = 0; j < sv.size(); j++)
                pair = std::max(pair, ws_block(g, hg, &sv[i], blk[i]) + ws_block(g, hg, &sv[j], blk[j]));
        best = std::max(best, fixed + pair);
    }
    // network calls
    best = std::max(best, 2 * align256(field_bytes(g, P_F32, field_rhs)) + ws_net_apply(g, field_rhs));
    if (loss_pairs > 0) best = std::max(best, ws_loss_grad(g, loss_pairs));
    if (train_pairs > 0) best = std::max(best, ws_train(g, hg, eo_ok, train_pairs, std::max(train_sources, 1)));
    return ws_persistent(g, hg, eo_ok) + best + (size_t(1) << 20);
}

}  // namespace tmq

using namespace tmq;

extern "C" {

tm_status tsm_solve_batch(tm_ctx* ctx, const tsm_solve_params* params, uint64_t seed, int32_t nsrc,
                          const uint64_t* ids_host, void* sol_dev, tsm_solve_stats* stats_host) {
    if (!ctx) return TM_EINVAL;
    if (ctx->sticky) return set_error(ctx, TM_EDEVICE, "context has a sticky device error");
    WsScope scope(ctx);
    if (!ctx->gauge_loaded) return set_error(ctx, TM_ESTATE, "tsm_solve_batch: no gauge field loaded");
    tm_status s = check_solve_params(ctx, params);
    if (s != TM_OK) return s;
    if (nsrc < 0 || (nsrc > 0 && (!ids_host || !stats_host)))
        return set_error(ctx, TM_EINVAL, "tsm_solve_batch: bad source list");
    if (params->out_layout != TM_LAYOUT_CANONICAL && params->out_layout != TM_LAYOUT_NATIVE)
        return set_error(ctx, TM_EINVAL, "tsm_solve_batch: bad out_layout");
    if (params->out_prec < TM_PREC_F64 || params->out_prec > TM_PREC_BF16)
        return set_error(ctx, TM_EINVAL, "tsm_solve_batch: bad out_prec");
    if (nsrc == 0) return TM_OK;
    const Geom& g = ctx->geo;
    const int blk = default_block(params);
    const int nr = lane_rhs(ctx, params, blk);
    // ids padded to a multiple of the lane width with repeats of the last id
    const int npad = (nsrc + nr - 1) / nr * nr;
    std::vector<uint64_t> ids(ids_host, ids_host + nsrc);
    ids.resize(npad, ids_host[nsrc - 1]);
    uint64_t* ids_dev = (uint64_t*)ws_get(ctx, "solve_ids", sizeof(uint64_t) * npad, &s);
    if (!ids_dev) return s;
    TM_COPY(ids_dev, ids.data(), sizeof(uint64_t) * npad, hipMemcpyHostToDevice);
    const uint64_t sm = seed_mix(seed);
    bool warn = false;
    for (int j0 = 0; j0 < nsrc; j0 += blk) {
        const int nb = std::min(blk, nsrc - j0);
        const int nbp = (nb + nr - 1) / nr * nr;
        BlockResult res;
        s = solve_block(ctx, params, sm, ids_dev + j0, nbp, nr, "sb", &res);
        if (s != TM_OK) return s;
        for (int r = 0; r < nb; r++) {
            fill_stats(ctx->scal_host[r], stats_host + j0 + r);
            if (params->max_iter < 0 && ctx->scal_host[r].status != 1) warn = true;
        }
        if (sol_dev) {
            launch_sol_out(ctx->stream, g, res.xprec, nb, res.x, sol_dev, params->out_prec,
                           params->out_layout == TM_LAYOUT_NATIVE, j0);
            TM_HIP(hipGetLastError());
        }
    }
    TM_HIP(hipStreamSynchronize(ctx->stream));
    return warn ? TM_WARN_NOT_CONVERGED : TM_OK;
}

tm_status tsm_contract(tm_ctx* ctx, uint64_t seed, int32_t nsrc, const uint64_t* ids_host, const double* sol_dev,
                       int32_t n_mom, const int32_t* mom_host, double* loops_host) {
    return tsm_contract_est(ctx, TM_LOOP_STANDARD, seed, nsrc, ids_host, sol_dev, n_mom, mom_host, loops_host);
}

tm_status tsm_contract_est(tm_ctx* ctx, int32_t estimator, uint64_t seed, int32_t nsrc, const uint64_t* ids_host,
                           const double* sol_dev, int32_t n_mom, const int32_t* mom_host, double* loops_host) {
    if (!ctx) return TM_EINVAL;
    if (ctx->sticky) return set_error(ctx, TM_EDEVICE, "context has a sticky device error");
    WsScope scope(ctx);
    if (estimator < TM_LOOP_STANDARD || estimator > TM_LOOP_DERIVATIVE)
        return set_error(ctx, TM_EINVAL, "tsm_contract: unknown estimator");
    const bool needs_eta = estimator == TM_LOOP_STANDARD || estimator == TM_LOOP_DERIVATIVE;
    if (nsrc < 1 || !sol_dev || !loops_host || (needs_eta && !ids_host))
        return set_error(ctx, TM_EINVAL, "tsm_contract: bad argument");
    if ((estimator == TM_LOOP_ONEEND_GENERALIZED || estimator == TM_LOOP_DERIVATIVE) && !ctx->gauge_loaded)
        return set_error(ctx, TM_ESTATE, "tsm_contract: this loop needs the gauge field");
    if (n_mom == TM_ALL_MOMENTA) {
        if (estimator != TM_LOOP_STANDARD)
            return set_error(ctx, TM_ENOTSUP, "tsm_contract: all momenta only for the standard loop");
        return contract_all_momenta(ctx, seed, nsrc, ids_host, sol_dev, loops_host);
    }
    const Geom& g = ctx->geo;
    MomPlan mp;
    tm_status s = plan_momenta(ctx, n_mom, mom_host, &mp);
    if (s != TM_OK) return s;
    const int blk = std::min(nsrc, kMaxBlock);
    Contractor c;
    if ((s = setup_contract(ctx, mp, n_mom, blk, seed_mix(seed), estimator, &c)) != TM_OK) return s;
    const long nl = 16L * loop_sets(estimator) * n_mom * g.L[3];
    uint64_t* ids_dev = (uint64_t*)ws_get(ctx, "contract_ids", sizeof(uint64_t) * nsrc, &s);
    int* slots = (int*)ws_get(ctx, "contract_slots", sizeof(int) * nsrc, &s);
    void* nat = ws_get(ctx, "contract_nat", field_bytes(g, P_F64, blk), &s);
    double* out = (double*)ws_get(ctx, "contract_out", sizeof(double) * 2 * nl * nsrc, &s);
    if (s != TM_OK) return s;
    std::vector<int> sl(nsrc);
    for (int i = 0; i < nsrc; i++) sl[i] = i;
    if (ids_host)
        TM_COPY(ids_dev, ids_host, sizeof(uint64_t) * nsrc, hipMemcpyHostToDevice);
    else
        TM_HIP(hipMemsetAsync(ids_dev, 0, sizeof(uint64_t) * nsrc, ctx->stream));
    TM_COPY(slots, sl.data(), sizeof(int) * nsrc, hipMemcpyHostToDevice);
    for (int j0 = 0; j0 < nsrc; j0 += blk) {
        const int nb = std::min(blk, nsrc - j0);
        launch_field_convert(ctx->stream, g, P_F64, nb, true, sol_dev + (size_t)j0 * g.V * 24, nat);
        contract_block(ctx, &c, ids_dev + j0, nat, P_F64, nb, (double2*)out, slots + j0, nl);
        TM_HIP(hipGetLastError());
    }
    TM_HIP(hipMemcpyAsync(loops_host, out, sizeof(double) * 2 * nl * nsrc, hipMemcpyDeviceToHost, ctx->stream));
    TM_HIP(hipStreamSynchronize(ctx->stream));
    return TM_OK;
}

tm_status tsm_loops(tm_ctx* ctx, const tsm_params* P, double* loops_host, double* err_host, double* per_source_host,
                    tsm_solve_stats* stats_host, tsm_run_stats* run_stats) {
    using clk = std::chrono::steady_clock;
    if (!ctx) return TM_EINVAL;
    if (ctx->sticky) return set_error(ctx, TM_EDEVICE, "context has a sticky device error");
    WsScope scope(ctx);
    if (!ctx->gauge_loaded) return set_error(ctx, TM_ESTATE, "tsm_loops: no gauge field loaded");
    if (!P || !loops_host) return set_error(ctx, TM_EINVAL, "tsm_loops: null argument");
    if (P->n_hp < 0 || P->n_lp < 0) return set_error(ctx, TM_EINVAL, "tsm_loops: negative source count");
    tm_status s = check_solve_params(ctx, &P->lp);
    if (s != TM_OK) return s;
    if ((s = check_solve_params(ctx, &P->hp)) != TM_OK) return s;
    const Geom& g = ctx->geo;
    MomPlan mp;
    if ((s = plan_momenta(ctx, P->n_mom, P->mom_host, &mp)) != TM_OK) return s;
    const int N = P->n_hp + P->n_lp;
    if (P->estimator < TM_LOOP_STANDARD || P->estimator > TM_LOOP_DERIVATIVE)
        return set_error(ctx, TM_EINVAL, "tsm_loops: unknown estimator");
    const long nl = 16L * loop_sets(P->estimator) * P->n_mom * g.L[3];
    hipStream_t st = ctx->stream;
    const uint64_t sm = seed_mix(P->seed);

    const int blp = default_block(&P->lp), bhp = default_block(&P->hp);
    const int nr_lp = lane_rhs(ctx, &P->lp, blp), nr_hp = lane_rhs(ctx, &P->hp, bhp);
    // LP buffers sized for the LP blocks from the first (smaller) HP-set
    // block on, HP buffers for the padded HP-set blocks
    {
        const int bh0 = std::min(blp, bhp);
        ctx->ws_cap["lp"] = blp;
        ctx->ws_cap["hp"] = (bh0 + nr_hp - 1) / nr_hp * nr_hp;
    }
    Contractor c;
    if ((s = setup_contract(ctx, mp, P->n_mom, std::max(blp, bhp) + 4, sm, P->estimator, &c)) != TM_OK) return s;

    // per-source loops [N][2][nl], source ids, output slots (ids padded at the end)
    const int Npad = N + 8;
    double* ps = (double*)ws_get(ctx, "tsm_ps", sizeof(double) * 2 * 2 * nl * std::max(N, 1), &s);
    uint64_t* ids_dev = (uint64_t*)ws_get(ctx, "tsm_ids", sizeof(uint64_t) * Npad, &s);
    int* slots_dev = (int*)ws_get(ctx, "tsm_slots", sizeof(int) * 2 * Npad, &s);
    double* fin = (double*)ws_get(ctx, "tsm_fin", sizeof(double) * 2 * 2 * 3 * nl, &s);
    if (s != TM_OK) return s;
    std::vector<uint64_t> ids(Npad);
    std::vector<int> slots(2 * Npad);
    for (int j = 0; j < Npad; j++) {
        ids[j] = (uint64_t)std::min(j, std::max(N - 1, 0));
        slots[j] = 2 * std::min(j, std::max(N - 1, 0));              // LP slot
        slots[Npad + j] = 2 * std::min(j, std::max(N - 1, 0)) + 1;   // HP slot
    }
    TM_COPY(ids_dev, ids.data(), sizeof(uint64_t) * Npad, hipMemcpyHostToDevice);
    TM_COPY(slots_dev, slots.data(), sizeof(int) * 2 * Npad, hipMemcpyHostToDevice);
    TM_HIP(hipMemsetAsync(ps, 0, sizeof(double) * 2 * 2 * nl * std::max(N, 1), st));

    tsm_run_stats rs;
    std::memset(&rs, 0, sizeof(rs));
    bool warn = false;
    auto record = [&](int j0, int nb, int slot, bool hp) {
        for (int r = 0; r < nb; r++) {
            const CgScal& q = ctx->scal_host[r];
            if (stats_host) fill_stats(q, stats_host + 2 * (j0 + r) + slot);
            if (hp) {
                rs.hp_iters += q.iters;
                rs.max_hp_resid_true = std::max(rs.max_hp_resid_true, q.resid_true);
                if (q.status != 1) {
                    rs.hp_not_converged++;
                    if (P->hp.max_iter < 0) warn = true;
                }
            } else {
                rs.lp_iters += q.iters;
                rs.max_lp_resid_true = std::max(rs.max_lp_resid_true, q.resid_true);
            }
        }
    };
    if (stats_host) std::memset(stats_host, 0, sizeof(tsm_solve_stats) * 2 * N);

    // the standard loop takes the LP solutions as their two halves
    const bool halves = P->estimator == TM_LOOP_STANDARD;
    auto t0 = clk::now();
    // HP set: LP and HP solves of ids 0..n_hp-1
    const int bh = std::min(blp, bhp);
    for (int j0 = 0; j0 < P->n_hp; j0 += bh) {
        const int nb = std::min(bh, P->n_hp - j0);
        BlockResult res;
        const int nbl = (nb + nr_lp - 1) / nr_lp * nr_lp;
        if ((s = solve_block(ctx, &P->lp, sm, ids_dev + j0, nbl, nr_lp, "lp", &res, halves)) != TM_OK) return s;
        record(j0, nb, 0, false);
        contract_block(ctx, &c, ids_dev + j0, res.x, res.xprec, nb, (double2*)ps, slots_dev + j0, nl, res.xe);
        const int nbh = (nb + nr_hp - 1) / nr_hp * nr_hp;
        if ((s = solve_block(ctx, &P->hp, sm, ids_dev + j0, nbh, nr_hp, "hp", &res)) != TM_OK) return s;
        record(j0, nb, 1, true);
        contract_block(ctx, &c, ids_dev + j0, res.x, res.xprec, nb, (double2*)ps, slots_dev + Npad + j0, nl);
        TM_HIP(hipGetLastError());
    }
    TM_HIP(hipStreamSynchronize(st));
    auto t1 = clk::now();
    // LP set: ids n_hp..N-1
    for (int j0 = P->n_hp; j0 < N; j0 += blp) {
        const int nb = std::min(blp, N - j0);
        const int nbl = (nb + nr_lp - 1) / nr_lp * nr_lp;
        BlockResult res;
        if ((s = solve_block(ctx, &P->lp, sm, ids_dev + j0, nbl, nr_lp, "lp", &res, halves)) != TM_OK) return s;
        record(j0, nb, 0, false);
        contract_block(ctx, &c, ids_dev + j0, res.x, res.xprec, nb, (double2*)ps, slots_dev + j0, nl, res.xe);
        TM_HIP(hipGetLastError());
    }
    launch_tsm_final(st, ps, nl, P->n_hp, P->n_lp, fin, fin + 2 * 3 * nl);
    TM_HIP(hipGetLastError());
    TM_HIP(hipStreamSynchronize(st));
    auto t2 = clk::now();
    TM_COPY(loops_host, fin, sizeof(double) * 2 * 3 * nl, hipMemcpyDeviceToHost);
    if (err_host) TM_COPY(err_host, fin + 2 * 3 * nl, sizeof(double) * 2 * 3 * nl, hipMemcpyDeviceToHost);
    if (per_source_host && N > 0)
        TM_COPY(per_source_host, ps, sizeof(double) * 2 * 2 * nl * N, hipMemcpyDeviceToHost);
    rs.ms_hp_phase = std::chrono::duration<double, std::milli>(t1 - t0).count();
    rs.ms_lp_phase = std::chrono::duration<double, std::milli>(t2 - t1).count();
    if (run_stats) *run_stats = rs;
    return warn ? TM_WARN_NOT_CONVERGED : TM_OK;
}

tm_status tm_autotune_cg(tm_ctx* ctx, int32_t prec, int32_t nrhs, int32_t* best_nr, int32_t* best_tseg,
                         double* ms_host) {
    if (!ctx || prec < 0 || prec > 3 || nrhs < 1 || nrhs > kMaxBlock || !best_nr || !best_tseg)
        return ctx ? set_error(ctx, TM_EINVAL, "tm_autotune_cg: bad argument") : TM_EINVAL;
    if (ctx->sticky) return set_error(ctx, TM_EDEVICE, "context has a sticky device error");
    WsScope scope(ctx);
    if (!ctx->gauge_loaded) return set_error(ctx, TM_ESTATE, "tm_autotune_cg: no gauge field loaded");
    tm_status s = TM_OK;
    uint64_t* ids = (uint64_t*)ws_get(ctx, "tune_ids", sizeof(uint64_t) * nrhs, &s);
    if (!ids) return s;
    std::vector<uint64_t> idh(nrhs);
    for (int i = 0; i < nrhs; i++) idh[i] = (uint64_t)i;
    TM_COPY(ids, idh.data(), sizeof(uint64_t) * nrhs, hipMemcpyHostToDevice);
    const int keep_nr = ctx->lane_rhs[prec], keep_ts = ctx->march[prec];
    tsm_solve_params p;
    std::memset(&p, 0, sizeof(p));
    p.prec = prec;
    p.solver = TM_SOLVER_CG;
    p.tol = 0.0;  // never converges: runs max_iter steps
    p.stop = TM_STOP_NORMAL;
    p.rhs_block = nrhs;
    p.true_resid = 0;
    double best = 1e300;
    int bnr = 1, bts = 0;
    for (int c = 0; c < kTuneCandidates; c++) {
        const int nr = kTuneNr[c], ts = kTuneTseg[c];
        if (ms_host) ms_host[c] = -1.0;
        if (nrhs % nr != 0 || (prec == TM_PREC_F64 && nr != 1)) continue;
        ctx->lane_rhs[prec] = nr;
        ctx->march[prec] = ts;
        // per-iteration time: difference of a long and a short truncated
        // solve (initialisation cancels), best of two
        double per = 1e300;
        for (int rep = 0; rep < 3; rep++) {
            double t[2];
            for (int j = 0; j < 2; j++) {
                p.max_iter = j == 0 ? 2 : 10;
                BlockResult res;
                const auto t0 = std::chrono::steady_clock::now();
                s = solve_block(ctx, &p, seed_mix(12345), ids, nrhs, nr, "tune", &res);
                const auto t1 = std::chrono::steady_clock::now();
                if (s != TM_OK) break;
                t[j] = std::chrono::duration<double, std::milli>(t1 - t0).count();
            }
            if (s != TM_OK) break;
            if (rep > 0) per = std::min(per, (t[1] - t[0]) / 8.0);  // the first pass warms up
        }
        if (s != TM_OK) break;
        if (ms_host) ms_host[c] = per;
        if (per < best) {
            best = per;
            bnr = nr;
            bts = ts;
        }
    }
    if (s != TM_OK) {
        ctx->lane_rhs[prec] = keep_nr;
        ctx->march[prec] = keep_ts;
        return s;
    }
    ctx->lane_rhs[prec] = bnr;
    ctx->march[prec] = bts;
    *best_nr = bnr;
    *best_tseg = bts;
    return TM_OK;
}

tm_status tm_autotune_eo(tm_ctx* ctx, int32_t prec, int32_t nrhs, int32_t* best_nr, int32_t* best_tiles,
                         double* ms_host) {
    if (!ctx || prec < 1 || prec > 3 || nrhs < 1 || nrhs > kMaxBlock || !best_nr || !best_tiles)
        return ctx ? set_error(ctx, TM_EINVAL, "tm_autotune_eo: bad argument") : TM_EINVAL;
    if (ctx->sticky) return set_error(ctx, TM_EDEVICE, "context has a sticky device error");
    WsScope scope(ctx);
    if (!ctx->gauge_loaded) return set_error(ctx, TM_ESTATE, "tm_autotune_eo: no gauge field loaded");
    if (!ctx->eo_ok) return set_error(ctx, TM_ENOTSUP, "tm_autotune_eo: the even-odd solver needs even extents");
    tm_status s = TM_OK;
    uint64_t* ids = (uint64_t*)ws_get(ctx, "tune_ids", sizeof(uint64_t) * nrhs, &s);
    if (!ids) return s;
    std::vector<uint64_t> idh(nrhs);
    for (int i = 0; i < nrhs; i++) idh[i] = (uint64_t)i;
    TM_COPY(ids, idh.data(), sizeof(uint64_t) * nrhs, hipMemcpyHostToDevice);
    const int keep_nr = ctx->lane_rhs[prec], keep_tiles = ctx->eo_tiles[prec];
    tsm_solve_params p;
    std::memset(&p, 0, sizeof(p));
    p.prec = prec;
    p.solver = TM_SOLVER_CG_EO;
    p.tol = 0.0;  // runs max_iter steps
    p.stop = TM_STOP_NORMAL;
    p.rhs_block = nrhs;
    p.true_resid = 0;
    constexpr int kNrEo[6] = {1, 2, 4, 1, 2, 4};
    constexpr int kTilesEo[6] = {0, 0, 0, 1, 1, 1};
    double best = 1e300;
    int bnr = 1, bt = 0;
    for (int c = 0; c < 6; c++) {
        const int nr = kNrEo[c], tl = kTilesEo[c];
        if (ms_host) ms_host[c] = -1.0;
        if (nrhs % nr != 0) continue;
        ctx->lane_rhs[prec] = nr;
        ctx->eo_tiles[prec] = tl;
        // per-iteration time: difference of a long and a short truncated
        // solve (set-up and reconstruction cancel), best of two after a warm-up
        double per = 1e300;
        for (int rep = 0; rep < 3; rep++) {
            double t[2];
            for (int j = 0; j < 2; j++) {
                p.max_iter = j == 0 ? 2 : 8;
                BlockResult res;
                const auto t0 = std::chrono::steady_clock::now();
                s = solve_block(ctx, &p, seed_mix(12345), ids, nrhs, nr, "tune", &res);
                const auto t1 = std::chrono::steady_clock::now();
                if (s != TM_OK) break;
                t[j] = std::chrono::duration<double, std::milli>(t1 - t0).count();
            }
            if (s != TM_OK) break;
            if (rep > 0) per = std::min(per, (t[1] - t[0]) / 6.0);
        }
        if (s != TM_OK) break;
        if (ms_host) ms_host[c] = per;
        if (per < best) {
            best = per;
            bnr = nr;
            bt = tl;
        }
    }
    if (s != TM_OK) {
        ctx->lane_rhs[prec] = keep_nr;
        ctx->eo_tiles[prec] = keep_tiles;
        return s;
    }
    ctx->lane_rhs[prec] = bnr;
    ctx->eo_tiles[prec] = bt;
    *best_nr = bnr;
    *best_tiles = bt;
    return TM_OK;
}

size_t tm_workspace_bytes(const tm_lattice* lat, const tm_caps* caps) {
    if (!lat) return 0;
    Geom g, hg;
    bool eo_ok = false;
    std::string why;
    if (!geom_setup(lat, &g, &hg, &eo_ok, &why)) return 0;
    std::vector<tsm_solve_params> sv;
    if (!caps) {
        // every solver and storage precision at 32 sources per block
        for (int solver : {TM_SOLVER_CG, TM_SOLVER_CG_EO, TM_SOLVER_FCG_LEARNED})
            for (int prec = TM_PREC_F64; prec <= TM_PREC_BF16; prec++)
                for (int rel = 0; rel <= 1; rel++)
                    for (int stop : {TM_STOP_NORMAL, TM_STOP_TRUE}) {
                        if ((rel && prec != TM_PREC_F32) || (solver == TM_SOLVER_FCG_LEARNED && (prec == TM_PREC_F64 || rel)) ||
                            (solver == TM_SOLVER_CG_EO && !eo_ok))
                            continue;
                        tsm_solve_params p;
                        std::memset(&p, 0, sizeof(p));
                        p.prec = prec;
                        p.solver = solver;
                        p.reliable = rel;
                        p.stop = stop;
                        p.rhs_block = kMaxBlock;
                        sv.push_back(p);
                    }
        const uint32_t all_est = (1u << TM_LOOP_STANDARD) | (1u << TM_LOOP_ONEEND_ISOVECTOR) |
                                 (1u << TM_LOOP_ONEEND_GENERALIZED) | (1u << TM_LOOP_DERIVATIVE);
        return ws_bound(lat, g, hg, eo_ok, sv, 256, 27, 3, all_est, 4, kMaxBlock, 64, 64, 64);
    }
    if (caps->n_solves < 0 || caps->n_solves > TM_CAPS_MAX_SOLVES || caps->max_sources < 0 || caps->max_mom < 0 ||
        caps->mom_distinct < 0 || caps->all_mom_sources < 0 || caps->field_rhs < 0 || caps->train_pairs < 0 ||
        caps->train_sources < 0 || caps->loss_pairs < 0)
        return 0;
    for (int i = 0; i < caps->n_solves; i++) sv.push_back(caps->solves[i]);
    const int max_mom = std::max(caps->max_mom, 1);
    const int nd = caps->mom_distinct > 0 ? std::min(caps->mom_distinct, max_mom) : max_mom;
    const uint32_t est = caps->estimators ? caps->estimators : (1u << TM_LOOP_STANDARD);
    return ws_bound(lat, g, hg, eo_ok, sv, caps->max_sources, max_mom, nd, est, caps->all_mom_sources,
                    std::max(caps->field_rhs, 1), caps->train_pairs, caps->train_sources, caps->loss_pairs);
}

}  // extern "C"
