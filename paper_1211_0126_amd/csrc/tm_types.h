// Types shared by host code and kernels (plain data only).
#pragma once

#include <stdint.h>

namespace tmq {

// Per-right-hand-side CG state, kept in device memory so that the whole
// iteration (step lengths, convergence, reliable-update decisions) runs
// without host round trips.
struct CgScal {
    double rr;      // current |r|^2 of the iterated residual
    double bb;      // |b|^2, b = M^dag eta
    double tt;      // |M p|^2
    double alpha;   // step length
    double beta;    // direction update
    double maxrr;   // largest |r|^2 since the last reliable update
    double ee;      // |eta|^2
    double rho2;    // |eta - M x|^2, tracked recursively (TM_STOP_TRUE)
    double tol2;    // tol^2
    double delta2;  // reliable-update threshold squared
    double resid_true;  // FP64 |eta - M x| / |eta| (filled at the end)
    // Reliable mode: the stored r and p are the true ones divided by sigma,
    // a power of two chosen at each reliable update so that the stored
    // residual starts every cycle at the scale of the source (the recursion
    // is invariant under a common scale of r and p; x32 accumulates alpha p
    // of the stored p and is added to x64 times sigma).  rr and maxrr are in
    // stored units, bb, rho2 and ee in true units.
    double sigma;
    double sigma_next;  // the scale of the residual stored by the pending update
    int32_t maxit;  // -1: no cap
    int32_t iters;
    int32_t active;     // 1 while iterating
    int32_t status;     // 0 running, 1 converged, 2 truncated, 3 breakdown
    int32_t rflag;      // 1: a reliable update is pending this iteration
    int32_t n_reliable;
    int32_t stop;       // 0 normal-equation residual, 1 tracked true residual
    int32_t reliable;   // 1: reliable-update mode
    int32_t fell_back;  // flexible CG only: 1 if it fell back to plain CG
    int32_t pad;
};

// Per-right-hand-side state of flexible CG (complex step scalars).
struct FcgScal {
    double zr_re, zr_im;        // <z, r>
    double alpha_re, alpha_im;
    double beta_re, beta_im;
    double rr, rr_prev, bb, tt, tol2, resid_true;
    double hist[5];             // |r|^2 of the last five steps
    int32_t maxit, iters, active, status;
    int32_t fell;               // 1 after the fallback to plain CG
    int32_t mode;               // direction update: 0 z+beta p, 1 r+beta p, 2 r, 3 z
    int32_t stagnant, pad;
};

// Lattice geometry as the kernels see it.
struct Geom {
    int32_t L[4];
    int32_t t_bc;
    int64_t V;
    int64_t Vs;     // padded plane stride of native fields (multiple of 256)
    uint32_t m[3];  // ceil(2^32 / L[d]) for exact division of site indices
    uint32_t brick; // half lattice: rows per wave of the brick order of site blocks (0: natural order)
};

enum SPrec { P_F64 = 0, P_F32 = 1, P_F16 = 2, P_BF16 = 3, P_BH = 4 /* network-internal bfloat16, half-split planes */ };

}  // namespace tmq
