// Internal interface between the solver driver and the learned preconditioner.
#pragma once

#include <string>
#include <vector>

#include "tm_ctx.h"

namespace tmq {

// Where a replayed training solve cuts (residual, error) pairs.
struct PairSink {
    void* R;              // bfloat16 residual fields, one per pair
    void* E;              // bfloat16 error fields
    size_t fb;            // bytes per field
    int next;             // next free pair slot
    std::vector<int> ks;  // iteration counts at which pairs are cut (ascending)
    const void* xstar;    // converged solution (FP64 native)
    uint64_t seed_mixed;
    const uint64_t* id;   // source id (device)
};

// FP64 CG of one source with a host round trip per step: records
// |r_k|^2/|b|^2 (hist), stores the final solution (xstar_out) and/or cuts
// pairs (sink).  maxit = -1: run to tol.
tm_status solve_f64_history(tm_ctx* ctx, uint64_t seed_mixed, const uint64_t* id_dev, double tol, int maxit,
                            std::vector<double>* hist, void* xstar_out, PairSink* sink);

// cap: right-hand sides to size the scratch for (at least nrhs)
tm_status net_apply(tm_ctx* ctx, bool adjoint, int nrhs, const void* in, int in_prec, void* out, int out_prec,
                    const FcgScal* gate, int cap = 0);
tm_status net_precondition(tm_ctx* ctx, int nrhs, const void* r, void* z, const FcgScal* gate, int cap = 0);

// workspace bounds of the network paths (bytes of scratch, each buffer
// rounded to 256 B): one application to nrhs fields, a loss gradient over
// npairs pairs, and a training call with npairs pairs from nsrc sources
size_t ws_net_apply(const Geom& g, int nrhs);
size_t ws_loss_grad(const Geom& g, int npairs);
size_t ws_train(const Geom& g, const Geom& hg, bool eo_ok, int npairs, int nsrc);
bool net_installed(const tm_ctx* ctx);
void net_release(tm_ctx* ctx);

}  // namespace tmq
