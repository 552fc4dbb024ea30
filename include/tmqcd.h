/*
 * tmqcd.h -- C ABI of the MI355X (gfx950) library for the truncated solver
 * method (TSM) evaluation of disconnected quark loops with twisted-mass
 * Wilson fermions, after C. Alexandrou et al., "Evaluation of disconnected
 * contributions using GPUs", Lattice 2012 (arXiv:1211.0126).
 *
 * The problem statement follows the paper: the operator M with kappa and
 * mu (section 2.2, the twisted-mass lower bound; section 2.3, the flavour
 * identity M_u - M_d = 2 i mu a gamma_5), N_HP and N_LP Z4 noise sources
 * (Eq. 1, Eq. 4), truncation of the low-precision solves by a residual or a
 * fixed number of iterations (section 2.2), and loops Tr(M^{-1} X) estimated
 * as averages of <eta^dag X s> (section 2.3) for all 16 Dirac structures,
 * per timeslice and momentum (section 3: loops for all insertion times,
 * Fourier transformed).
 *
 * Conventions
 *  - lattice dims[4] = (Lx, Ly, Lz, Lt), each >= 2; site index
 *    x + Lx*(y + Ly*(z + Lz*t)); direction mu = 0..3 is x, y, z, t.
 *  - spinor component index 3*spin + colour; canonical spinor layout
 *    [rhs][site][spin][colour] complex, real and imaginary parts interleaved.
 *  - canonical gauge layout complex128 [site][mu][row][col]; U_mu(x)
 *    multiplies psi(x + mu).  No boundary sign is stored in the links.
 *  - time boundary factor t_bc (-1 antiperiodic, +1 periodic) on hops across
 *    t = Lt-1 <-> 0; space is periodic.
 *  - Euclidean chiral gamma basis, gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4
 *    = diag(1, 1, -1, -1); Gamma_n = g1^b0 g2^b1 g3^b2 g4^b3 for
 *    n = b0 + 2 b1 + 4 b2 + 8 b3.
 *  - hopping normalisation: M = 1 - kappa H + 2 i kappa mu gamma_5, with
 *    H psi(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu)
 *                    + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu);
 *    M is 2 kappa times the physical M_u.  M^dag = 1 - kappa H^dag
 *    - 2 i kappa mu gamma_5.
 *  - noise: Z4 components eta = i^k, k = bits (2c, 2c+1) of
 *    splitmix64mix(splitmix64mix(seed) + 0x9E3779B97F4A7C15 * (1 + id*V + site))
 *    for component c; regenerated on the fly, never stored (section 3).
 *  - loops: L_n(t, p) = sum_{x in timeslice t} exp(-i p.x)
 *    sum_{a,b,c} conj(eta(x)_{a c}) Gamma_n[a][b] s(x)_{b c},
 *    p = 2 pi (nx/Lx, ny/Ly, nz/Lz); layout [16][n_mom][Lt] complex128.
 *
 * Memory and threading
 *  - "_dev" pointers are device memory owned by the caller (16-byte
 *    aligned); "_host" pointers are host memory owned by the caller.  The
 *    library keeps its own device workspace (gauge copies, solver vectors),
 *    allocated on first use and released by tm_destroy.
 *  - all work is enqueued on the HIP stream given to tm_create.  Calls that
 *    return host results synchronise that stream; tm_dslash does not.
 *  - a context is not thread-safe: one host thread per context.
 *
 * Errors
 *  - every entry point returns tm_status: 0 success, > 0 warning, < 0 error.
 *    Nothing throws or aborts across the ABI.  Outputs are undefined after an
 *    error; tm_last_error gives the text.  TM_EDEVICE is sticky: destroy the
 *    context.  Truncation of an LP solve by the iteration cap is not an error.
 */
#ifndef TMQCD_H
#define TMQCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TM_ABI_VERSION 3

typedef int32_t tm_status;
enum {
    TM_OK = 0,
    TM_WARN_NOT_CONVERGED = 1, /* a solve with no iteration cap missed its tolerance */
    TM_WARN_FALLBACK = 2,      /* the learned preconditioner fell back to plain CG */
    TM_EINVAL = -1,            /* invalid argument */
    TM_ENOMEM = -2,            /* the workspace cannot hold the call's buffers (tm_workspace_bytes) */
    TM_EDEVICE = -3,           /* HIP runtime error (sticky) */
    TM_ESTATE = -4,            /* call out of order (e.g. no gauge field loaded) */
    TM_ENOTSUP = -5            /* combination not supported */
};

/* storage precision of spinor fields; arithmetic is FP64 for TM_PREC_F64
   and FP32 otherwise, inner products and norms are accumulated in FP64 */
typedef enum { TM_PREC_F64 = 0, TM_PREC_F32 = 1, TM_PREC_F16 = 2, TM_PREC_BF16 = 3 } tm_prec;

typedef enum {
    TM_OP_M = 0,     /* M */
    TM_OP_MDAG = 1,  /* M^dag */
    TM_OP_MDAGM = 2, /* M^dag M */
    TM_OP_HOP = 3    /* H (hopping term alone) */
} tm_op;

typedef enum {
    TM_LAYOUT_CANONICAL = 0, /* [rhs][site][spin][colour] complex of the storage precision */
    TM_LAYOUT_NATIVE = 1     /* the library's internal layout (opaque), see tm_field_bytes */
} tm_layout;

typedef enum {
    TM_STOP_NORMAL = 0, /* |M^dag eta - M^dag M s| / |M^dag eta| <= tol (CG's own residual) */
    TM_STOP_TRUE = 1    /* |eta - M s| / |eta| <= tol: tracked recursively, or with reliable
                           updates the FP64 value taken at each update (an update is also made
                           at every iteration whose normal-equation residual is below tol) */
} tm_stop;

typedef enum {
    TM_SOLVER_CG = 0,          /* conjugate gradients on M^dag M */
    TM_SOLVER_FCG_LEARNED = 1, /* flexible CG preconditioned by the learned network */
    TM_SOLVER_CG_EO = 2        /* conjugate gradients on Mhat^dag Mhat, Mhat = D - kappa^2 H_oe D^{-1} H_eo
                                  the even-odd Schur complement of M on the odd sites (D = 1 + 2i kappa mu g5);
                                  the even half of s is reconstructed.  Not in the paper; a different LP map
                                  than TM_SOLVER_CG (Eq. 4 stays unbiased for any fixed one).  Needs every
                                  extent even (TM_ENOTSUP otherwise); tol, max_iter and TM_STOP_NORMAL refer
                                  to the Schur system, TM_STOP_TRUE to |eta - M s| / |eta| of the whole
                                  system (which equals that of the Schur system) */
} tm_solver;

typedef struct {
    int32_t dims[4]; /* Lx, Ly, Lz, Lt, each >= 2 */
    double kappa;    /* hopping parameter */
    double mu;       /* twisted mass a*mu; the operator uses 2*kappa*mu */
    int32_t t_bc;    /* -1 antiperiodic, +1 periodic in time */
} tm_lattice;

typedef struct tm_ctx tm_ctx;

/* One solve configuration (the inverter of section 2.2). */
typedef struct {
    int32_t prec;       /* tm_prec: storage of the Krylov vectors */
    int32_t solver;     /* tm_solver */
    double tol;         /* relative residual target; 0 = run to max_iter */
    int32_t max_iter;   /* iteration cap, -1 = none; 0 returns s = 0 */
    int32_t stop;       /* tm_stop */
    int32_t reliable;   /* 1: FP32 iterations with FP64 reliable updates (prec F32; also F16 or BF16
                           storage with TM_SOLVER_CG_EO) */
    double delta;       /* reliable-update trigger: |r| < delta * max |r| since the last update */
    int32_t rhs_block;  /* sources per launch, 1..32; 0 = library default */
    int32_t true_resid; /* 1: compute the FP64 true residual of every solve (one FP64 M) */
    int32_t out_layout; /* tm_layout of the solutions tsm_solve_batch writes: TM_LAYOUT_CANONICAL
                           [nsrc][V][4][3] complex, or TM_LAYOUT_NATIVE (tm_field_bytes(ctx,
                           out_prec, nsrc, TM_LAYOUT_NATIVE), the input of a native tm_dslash) */
    int32_t out_prec;   /* tm_prec of those solutions (F64: complex128, F32: complex64, F16 /
                           BF16: pairs of binary16 / bfloat16), rounded from the solve's own */
} tsm_solve_params;

/* Per-source solve record. */
typedef struct {
    int32_t iters;          /* CG iterations done */
    int32_t converged;      /* 1 if stopped by the tolerance */
    int32_t truncated;      /* 1 if stopped by the iteration cap */
    int32_t fell_back;      /* 1 if the learned preconditioner was dropped */
    double resid_iterated;  /* final relative residual of the stop criterion */
    double resid_true;      /* FP64 |eta - M s| / |eta| */
} tsm_solve_stats;

/* The loop estimator of one source (section 2.3), all in the hopping
   normalisation of the operator (M = 1 - kappa H + 2i kappa mu g5 = M_u;
   M_d is the same with mu -> -mu; tw = 2 kappa mu; X = the phase-weighted
   insertion Gamma_n on one timeslice):
   STANDARD:           eta^dag Gamma_n s, whose noise average is Tr[X M_u^{-1}];
   ONEEND_ISOVECTOR:   -2i tw s^dag g5 Gamma_n s (Eq. 5), noise average
                       Tr[X M_u^{-1}] - Tr[X M_d^{-1}]; the factor follows
                       from M_u - M_d = 2i tw g5 (Eq. 5 prints the opposite
                       sign);
   ONEEND_GENERALIZED: 2 s^dag g5 Gamma_n g5 D s with D = 1 - kappa H (Eq. 6),
                       noise average Tr[X M_u^{-1}] + Tr[X M_d^{-1}]; one
                       extra FP64 stencil application per source;
   DERIVATIVE:         the one-derivative loops psibar Gamma_n Dsym_mu psi of
                       the operators of section 3 (Fig. 1), one set per
                       direction mu: (1/4) [eta^dag Gamma_n f - g^dag Gamma_n s]
                       with f = U_mu(x) s(x+mu) - U_mu(x-mu)^dag s(x-mu) and g
                       the same of eta (symmetric covariant derivative
                       (Dfwd - Dbwd)/2, hops across t carry t_bc); its
                       loop elements are [4][16][n_mom][Lt] where the
                       others have [16][n_mom][Lt]. */
typedef enum {
    TM_LOOP_STANDARD = 0,
    TM_LOOP_ONEEND_ISOVECTOR = 1,
    TM_LOOP_ONEEND_GENERALIZED = 2,
    TM_LOOP_DERIVATIVE = 3
} tm_loop_estimator;

typedef struct {
    uint64_t seed;          /* noise seed; source ids are 0..n_hp+n_lp-1 */
    int32_t n_hp;           /* sources solved to high and low precision (ids 0..n_hp-1) */
    int32_t n_lp;           /* further sources solved to low precision only */
    tsm_solve_params lp;    /* the LP solver, used for every LP solve of both sets */
    tsm_solve_params hp;    /* the HP solver */
    int32_t n_mom;          /* number of momenta (>= 1) */
    const int32_t* mom_host;/* [n_mom][3] integer momenta n, p = 2 pi n / L */
    int32_t estimator;      /* tm_loop_estimator of every per-source loop */
    int32_t reserved;
} tsm_params;

typedef struct {
    double ms_hp_phase;     /* wall time of the HP set (LP + HP solves, contractions) */
    double ms_lp_phase;     /* wall time of the LP set */
    int64_t lp_iters;       /* total LP CG iterations (both sets) */
    int64_t hp_iters;       /* total HP CG iterations */
    double max_lp_resid_true; /* largest FP64 true residual of an LP solve */
    double max_hp_resid_true; /* largest FP64 true residual of an HP solve */
    int32_t hp_not_converged; /* HP solves that missed their tolerance */
    int32_t reserved;
} tsm_run_stats;

/* What a context will be asked to do, for tm_workspace_bytes.  Every count
   is a maximum over the calls the context will see. */
#define TM_CAPS_MAX_SOLVES 4
typedef struct {
    int32_t n_solves;       /* entries of solves[] */
    tsm_solve_params solves[TM_CAPS_MAX_SOLVES]; /* the solve settings of the tsm_solve_batch calls,
                               of both the lp and the hp of tsm_loops (any two entries may pair), and
                               the precision and block (rhs_block; 0: its default) of the autotuners */
    int32_t max_sources;    /* sources of one tsm_solve_batch, tsm_loops or tsm_contract call */
    int32_t max_mom;        /* momenta of one loop call */
    int32_t mom_distinct;   /* distinct values of one momentum component among them (0: max_mom;
                               3 for the 27 momenta with components in -1..1) */
    uint32_t estimators;    /* loop estimators used: bits 1 << tm_loop_estimator (0: standard only) */
    int32_t all_mom_sources;/* sources of one tsm_contract call at TM_ALL_MOMENTA (0: none) */
    int32_t field_rhs;      /* right-hand sides of one canonical-layout tm_dslash or of one
                               tm_precond_apply call */
    int32_t train_pairs;    /* pairs of one tm_precond_train call (0: no training) */
    int32_t train_sources;  /* sources of one tm_precond_train call */
    int32_t loss_pairs;     /* pairs of one tm_precond_loss_grad call */
} tm_caps;

/* ---- lifecycle ---------------------------------------------------------- */

/* ABI version (TM_ABI_VERSION). */
int32_t tm_abi_version(void);

/* Bytes of device workspace a context of this lattice needs for the calls
   caps describes (caps NULL: every solver and storage precision, with and
   without reliable updates and true-residual stops, at 32 sources per block;
   256 sources and 27 momenta with components in 3 values per call, every
   estimator, 4 sources at all momenta, 32 right-hand sides per operator
   call, 64 training and loss pairs from 64 sources).  The links, tables and network weights the
   context keeps, plus the largest scratch of one call, each buffer rounded
   to 256 B.  0 for a lattice tm_create refuses. */
size_t tm_workspace_bytes(const tm_lattice* lat, const tm_caps* caps);

/* Create a context for one lattice on the current HIP device.  dev_ws is
   the caller's device workspace of ws_bytes (256-byte aligned; e.g. a torch
   uint8 tensor of tm_workspace_bytes(lat, caps)); it must stay allocated,
   and untouched by the caller, until tm_destroy.  Every device buffer of
   the context is carved from it: the links, tables and network weights
   from its top, the scratch of each call from its bottom (released when the
   next call begins).  The library allocates no device memory after
   tm_create; a call whose buffers do not fit returns TM_ENOMEM before it
   enqueues work.  dev_ws NULL: tm_create allocates ws_bytes itself (once;
   tm_destroy releases it).  tm_create zeroes the workspace and allocates a
   small pinned host buffer.  hip_stream is a hipStream_t (NULL: the null
   stream).  TM_EINVAL for dims < 2 or for lattices whose volume, padded to
   the plane stride (an odd multiple of 256), exceeds 7,456,512 sites
   (planes are addressed with 32-bit byte offsets: 48^3 x 64 fits, 48^3 x
   96 does not), TM_ENOMEM for a workspace below the context's own tables;
   tm_last_error(NULL) says why. */
tm_status tm_create(const tm_lattice* lat, void* dev_ws, size_t ws_bytes, void* hip_stream, tm_ctx** out);

/* Bytes of the workspace the context holds until tm_destroy (persistent),
   the most scratch one call has used since tm_create (peak_scratch), and
   the workspace size (total).  Any pointer may be NULL. */
tm_status tm_workspace_usage(const tm_ctx* ctx, size_t* persistent, size_t* peak_scratch, size_t* total);

/* Release the context (and the workspace if tm_create allocated it). */
tm_status tm_destroy(tm_ctx* ctx);

/* Text of the last error on this context (never NULL). */
const char* tm_last_error(const tm_ctx* ctx);

/* ---- gauge field -------------------------------------------------------- */

/* Load the links (canonical complex128 [V][4][3][3], host, SU(3)).  The
   library keeps an FP64 copy (full links) and an FP32 copy (two rows; the
   third is rebuilt from unitarity).  Synchronous; the caller may free its
   buffer on return.  Section 3 of the paper: one gauge configuration at a
   time. */
tm_status tm_gauge_load(tm_ctx* ctx, const double* links_host);

/* ---- operator ----------------------------------------------------------- */

/* Bytes of one field of nrhs spinors in the given precision and layout. */
size_t tm_field_bytes(const tm_ctx* ctx, int32_t prec, int32_t nrhs, int32_t layout);

/* Convert nrhs spinors between the canonical and native layouts of the same
   precision (to_native = 1: canonical -> native).  Asynchronous. */
tm_status tm_field_convert(tm_ctx* ctx, int32_t prec, int32_t nrhs, int32_t to_native,
                           const void* in_dev, void* out_dev);

/* Apply op (tm_op) to nrhs spinors: out = op(in).  in/out are device
   buffers in the given layout and storage precision (canonical complex128
   for F64, complex64 for F32, pairs of binary16 / bfloat16 for F16 / BF16);
   they must not overlap.  Arithmetic: FP64 for F64, FP32 otherwise.  The
   operator is the one defined under Conventions (section 2.2/2.3).
   Asynchronous. */
tm_status tm_dslash(tm_ctx* ctx, int32_t op, int32_t prec, int32_t nrhs, int32_t layout,
                    const void* in_dev, void* out_dev);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): tm_dslash
   with the same arguments, results and kernels, which allocates nothing.
   Its scratch (the native staging of a canonical input and output, and the
   intermediate M in of M^dag M) lives in a device array of 128 MiB that the
   library holds on every GPU it runs on until the process ends; tm_create
   looks up its address.  Needs (canonical: 2 fields, M^dag M: 1 field, each
   tm_field_bytes(ctx, prec, nrhs, TM_LAYOUT_NATIVE) rounded up to 256 B)
   beyond 128 MiB return TM_EINVAL before anything is enqueued.  Every call
   on one GPU shares that array: calls that overlap in time on one GPU (two
   streams, two host threads) race on it.  Not recorded by tm_profile_*.
   Asynchronous. */
tm_status tm_dslash_noalloc(tm_ctx* ctx, int32_t op, int32_t prec, int32_t nrhs, int32_t layout,
                            const void* in_dev, void* out_dev);

/* ---- noise -------------------------------------------------------------- */

/* Write the Z4 sources (Eq. 1) of the given ids as canonical complex128
   [nsrc][V][4][3] into out_dev.  ids_host: nsrc source ids.  Asynchronous. */
tm_status tm_noise_z4(tm_ctx* ctx, uint64_t seed, int32_t nsrc, const uint64_t* ids_host, double* out_dev);

/* ---- solves ------------------------------------------------------------- */

/* Solve M s_j = eta_j (section 2.2) for the Z4 sources of the given ids with
   CG on M^dag M from s = 0.  sol_dev (nullable, caller-owned device memory)
   receives the solutions in params->out_layout and params->out_prec
   (canonical complex128 [nsrc][V][4][3] for zeroed fields); stats_host
   receives nsrc records.  Synchronous.  Returns TM_WARN_NOT_CONVERGED if a
   solve with max_iter = -1 stopped without reaching tol (cannot happen with
   an iteration cap). */
tm_status tsm_solve_batch(tm_ctx* ctx, const tsm_solve_params* params, uint64_t seed, int32_t nsrc,
                          const uint64_t* ids_host, void* sol_dev, tsm_solve_stats* stats_host);

/* ---- loops -------------------------------------------------------------- */

/* Contract given solutions with the regenerated sources of the given ids
   (section 2.3, per timeslice and momentum).  sol_dev: canonical complex128
   [nsrc][V][4][3] (device).  loops_host: complex128 [nsrc][16][n_mom][Lt].
   Synchronous. */
tm_status tsm_contract(tm_ctx* ctx, uint64_t seed, int32_t nsrc, const uint64_t* ids_host,
                       const double* sol_dev, int32_t n_mom, const int32_t* mom_host, double* loops_host);

/* n_mom value of tsm_contract / tsm_contract_est asking for every momentum
   of the lattice (the Fourier transform of section 3): p = 2 pi n / L with
   0 <= n_i < L_i, momentum index n_x + Lx (n_y + Ly n_z), mom_host ignored;
   standard loop and spatial extents <= 128 only (TM_ENOTSUP otherwise).
   loops_host is then complex128
   [nsrc][16][Lx*Ly*Lz][Lt]. */
#define TM_ALL_MOMENTA (-1)

/* tsm_contract with the loop estimator chosen (tm_loop_estimator; section
   2.3, Eqs. 5 and 6, and the derivative loops of section 3).  The one-end
   estimators use the solutions alone: seed and ids_host are ignored and
   ids_host may be NULL.  The generalized one-end and the derivative loops
   need the gauge field (TM_ESTATE otherwise); the former applies D in FP64
   to each solution.  loops_host: complex128 [nsrc][16][n_mom][Lt], for
   TM_LOOP_DERIVATIVE [nsrc][4][16][n_mom][Lt].  TM_EINVAL for an unknown
   estimator.  Synchronous. */
tm_status tsm_contract_est(tm_ctx* ctx, int32_t estimator, uint64_t seed, int32_t nsrc, const uint64_t* ids_host,
                           const double* sol_dev, int32_t n_mom, const int32_t* mom_host, double* loops_host);

/* The whole TSM estimate of Eq. 4 for the loops L of params->estimator:
     C = (1/N_HP) sum_{j < N_HP} [L(s_j^HP) - L(s_j^LP)],
     B = (1/N_LP) sum_{N_HP <= j < N_HP+N_LP} L(s_j^LP),   T = C + B,
   with every LP solve (of both sets) done by params->lp and the HP solves by
   params->hp.  An empty set contributes zero.
   loops_host: complex128 [3][16][n_mom][Lt] (C, B, T); with
     TM_LOOP_DERIVATIVE each [16][n_mom][Lt] block is [4][16][n_mom][Lt],
     here and in err_host and per_source_host.
   err_host (nullable): same shape; real and imaginary parts are the
     standard errors of the real and imaginary parts from the per-source
     spread (sample variance / N; zero for a set of one source),
     err_T^2 = err_C^2 + err_B^2.
   per_source_host (nullable): complex128 [N_HP+N_LP][2][16][n_mom][Lt];
     slot 0 the LP loops, slot 1 the HP loops (zero for LP-only ids).
   stats_host (nullable): tsm_solve_stats [N_HP+N_LP][2] (slot 0 LP, 1 HP).
   run_stats (nullable): timings and totals.
   Synchronous.  Returns TM_WARN_NOT_CONVERGED if an HP solve missed its
   tolerance; TM_EINVAL for an unknown params->estimator. */
tm_status tsm_loops(tm_ctx* ctx, const tsm_params* params, double* loops_host, double* err_host,
                    double* per_source_host, tsm_solve_stats* stats_host, tsm_run_stats* run_stats);

/* ---- learned preconditioner --------------------------------------------- */

/* A gauge-covariant network of linear parallel-transport layers.  Layer l
   maps widths[l] spinor fields phi_b to widths[l+1] fields
     psi_a(x) = sum_b sum_p W[p][a][b] (T_p phi_b)(x),
   over nine paths p: 0 the identity, 1 + 2 mu the transport from x + mu,
   U_mu(x) phi(x + mu), 2 + 2 mu the transport from x - mu,
   U_mu(x - mu)^dag phi(x - mu) (time-boundary sign included); W[p][a][b] is
   a complex 4x4 spin matrix (identity on colour).  Weights of a layer:
   complex128 [9][widths[l+1]][widths[l]][4][4], layers back to back.
   widths[0] = widths[n_layers] = 1 and 1 <= widths[l] <= 2.  The network N
   approximates M^{-1}; flexible CG on M^dag M uses z = N(N^dag(r)).
   Transports use bfloat16 (re, im) pairs of the input and of a bfloat16
   copy of the links with FP32 accumulation; the mixing runs on the matrix
   cores in bfloat16 with FP32 accumulation; hidden activations are stored
   as bfloat16. */
#define TM_NET_MAX_LAYERS 8
typedef struct {
    int32_t n_layers;
    int32_t widths[TM_NET_MAX_LAYERS + 1];
} tm_net_shape;

/* Number of complex weights of a network shape (0 if invalid). */
size_t tm_precond_weight_count(const tm_net_shape* shape);

/* Install a network (weights_host: complex128, tm_precond_weight_count of
   them).  TM_ENOTSUP for widths outside 1..2. */
tm_status tm_precond_set(tm_ctx* ctx, const tm_net_shape* shape, const double* weights_host);

/* Read back the installed shape and weights (weights_host may be NULL). */
tm_status tm_precond_get(tm_ctx* ctx, tm_net_shape* shape_out, double* weights_host);

/* out = N(in) (adjoint = 0) or N^dag(in) (adjoint = 1) for nrhs single
   spinor fields, canonical complex128 [nrhs][V][4][3] (device).  FP32
   input and output, bfloat16 hidden activations and mixing.  Asynchronous. */
tm_status tm_precond_apply(tm_ctx* ctx, int32_t adjoint, int32_t nrhs, const double* in_dev, double* out_dev);

/* Training loss (1/npairs) sum_i |N(r_i) - e_i|^2 / |e_i|^2 over pairs given
   as canonical complex128 [npairs][V][4][3] (device), and its gradient with
   respect to conj(W) (complex128, weight layout; d loss / d Re W = 2 Re,
   d loss / d Im W = 2 Im).  Synchronous. */
tm_status tm_precond_loss_grad(tm_ctx* ctx, int32_t npairs, const double* r_dev, const double* e_dev,
                               double* loss_host, double* grad_host);

typedef struct {
    uint64_t seed;        /* noise seed of the training sources (use one disjoint from the estimator's) */
    int32_t n_sources;    /* training sources solved to hp_tol */
    int32_t n_pairs;      /* (residual, error) pairs harvested from their iterates */
    int32_t epochs;
    int32_t batch;        /* pairs per Adam step */
    double lr;            /* Adam step size */
    double hp_tol;        /* tolerance of the training solves */
    double min_rel_err;   /* harvest only iterates with |e_k| / |x*| above this */
    uint64_t init_seed;   /* seed of the noise added to the initial weights */
    double init_scale;    /* size of that noise */
    int32_t init_mode;    /* initial network: 0 identity on channel 0; 1 the third-order
                             Neumann series of M^{-1} = sum_k A^k with A = 1 - M, built as
                             psi + A (psi + A (psi + A psi)) with channel 0 carrying psi
                             (needs the default 1 -> 2 -> 2 -> 1 shape) */
    int32_t loss_mode;    /* 0: |N(r) - e|^2 / |e|^2 (the loss of tm_precond_loss_grad);
                             1: |M N(r) - r|^2 / |r|^2, the residual of the preconditioned
                             operator, which weights all modes alike */
} tm_train_params;

typedef struct {
    double loss_first;    /* mean loss of the first epoch */
    double loss_last;     /* mean loss of the last epoch */
    double ms_generate;   /* time to harvest the pairs */
    double ms_train;      /* time of the Adam epochs */
    int32_t pairs;        /* pairs used */
    int32_t steps;        /* Adam steps */
} tm_train_stats;

/* Harvest (r_k = eta - M x_k, e_k = x* - x_k) pairs from CG solves of
   training sources, store them in bfloat16, and train the installed network
   (or a new 1 -> 2 -> 2 -> 1 network initialised as init_mode says if none
   is installed) with Adam on the loss of tm_precond_loss_grad, using the
   library's forward, adjoint and weight-gradient kernels.  The trained
   weights stay installed.  n_pairs = epochs = 0 only installs the initial
   network.  Synchronous. */
tm_status tm_precond_train(tm_ctx* ctx, const tm_train_params* params, tm_train_stats* stats);

/* ---- tuning ------------------------------------------------------------- */

/* Autotuner: time the operator M on nrhs fields (native layout) of storage
   precision prec with 1, 2 and 4 right-hand sides per lane (those that
   divide nrhs; FP64 runs 1), keep the fastest for later solves in that
   precision, and report it in *best_nr and the mean milliseconds per
   application of each candidate in ms_host[3] (negative where not run).
   Needs a loaded gauge field.  Synchronous. */
tm_status tm_autotune(tm_ctx* ctx, int32_t prec, int32_t nrhs, int32_t* best_nr, double* ms_host);

/* Autotuner for the CG kernels of storage precision prec on blocks of nrhs
   sources (1..32): times truncated CG iterations (operator, reductions and
   updates) on synthetic sources for each candidate traversal, keeps the
   fastest for later solves in that precision (as tm_set_lane_rhs and
   tm_set_march would) and reports it.  Candidates, in this order, as
   (right-hand sides per lane, time slices per lane): (1,0) (2,0) (4,0)
   (1,4) (1,8) (1,16) (2,4) (2,8); those whose lane width does not divide
   nrhs are skipped (and FP64 runs lane width 1 only).  ms_host (nullable)
   receives 8 per-iteration milliseconds, negative where skipped.  Needs a
   loaded gauge field; synchronous; uses the context's workspace. */
tm_status tm_autotune_cg(tm_ctx* ctx, int32_t prec, int32_t nrhs, int32_t* best_nr, int32_t* best_tseg,
                         double* ms_host);

/* Autotuner for the even-odd solver (TM_SOLVER_CG_EO) in storage precision
   prec (F32, F16 or BF16) on blocks of nrhs sources (1..32): times
   truncated Schur-complement CG iterations on synthetic sources for each
   candidate (right-hand sides per lane, half-hop traversal), in this order:
   (1, lane per half-site) (2, lane) (4, lane) (1, LDS tiles) (2, tiles)
   (4, tiles); lane widths that do not divide nrhs are skipped.  Keeps the
   fastest for later solves in that precision (as tm_set_lane_rhs and
   tm_set_eo_tiles would) and reports it; ms_host (nullable) receives 6
   per-iteration milliseconds, negative where skipped.  TM_ENOTSUP unless
   every extent is even.  Needs a loaded gauge field; synchronous. */
tm_status tm_autotune_eo(tm_ctx* ctx, int32_t prec, int32_t nrhs, int32_t* best_nr, int32_t* best_tiles,
                         double* ms_host);

/* Set (nr = 1, 2 or 4) or reset to the built-in choice (nr = 0) the
   right-hand sides per lane used by solves in storage precision prec. */
tm_status tm_set_lane_rhs(tm_ctx* ctx, int32_t prec, int32_t nr);

/* Stencil traversal of the CG kernels in storage precision prec: tseg = 0
   gives one lane per lattice site; tseg > 0 makes each lane walk tseg time
   slices of one spatial site (time-direction hops carried between slices,
   so the time neighbours are loaded once), used with 1 or 2 right-hand
   sides per lane.  Values above the time extent act as the time extent.
   Results agree with the one-lane-per-site kernels up to rounding (the
   terms of a site are summed in another order).  TM_EINVAL for prec
   outside 0..3 or tseg outside 0..65535. */
tm_status tm_set_march(tm_ctx* ctx, int32_t prec, int32_t tseg);

/* Traversal of the even-odd solver's half-hops in storage precision prec
   (TM_SOLVER_CG_EO): on = 1 gives each block a tile of 64 half-sites and all
   right-hand sides of the launch, with the tile's links staged once in LDS;
   on = 0 (the default) one lane per half-site and one block per chunk of
   right-hand sides.  Same arithmetic; FP64 always uses on = 0.  TM_EINVAL
   for prec outside 0..3 or on outside 0..1. */
tm_status tm_set_eo_tiles(tm_ctx* ctx, int32_t prec, int32_t on);

/* CG iteration chunks are captured once into HIP graphs and replayed (on a
   non-null stream, while per-launch profiling is off).  on = 1 enables (the
   default), 0 disables, -1 leaves the setting; *replays (nullable) receives
   the number of graph replays so far. */
tm_status tm_set_graphs(tm_ctx* ctx, int32_t on, int64_t* replays);

/* ---- instrumentation ---------------------------------------------------- */

/* Kernel classes timed with HIP events on the context stream when profiling
   is enabled. */
enum {
    TM_KC_DSLASH = 0,     /* t = M p (+ |t|^2): the CG operator application (even-odd: its second
                             half t = D p - kappa^2 H_oe y) */
    TM_KC_DSLASH_UPD = 1, /* q = M^dag t fused with x, r updates (+ |r|^2) (even-odd: the second half
                             of Mhat^dag t) */
    TM_KC_BLAS = 2,       /* p = r + beta p */
    TM_KC_CONTRACT = 3,   /* loop contraction */
    TM_KC_OTHER = 4,      /* noise, initialisation, CG scalar reductions, reliable updates, residuals */
    TM_KC_APPLY = 5,      /* tm_dslash applications */
    TM_KC_EO_HOP = 6,     /* even-odd CG: y = D^{-1} H_eo p (the first half of Mhat p) */
    TM_KC_EO_HOP_DAG = 7, /* even-odd CG: y = D^{-dag} H_eo^dag t (the first half of Mhat^dag t) */
    TM_KC_COUNT = 8
};

/* Enable (1) or disable (0) per-launch event timing; enabling clears the
   accumulated figures. */
tm_status tm_profile_enable(tm_ctx* ctx, int32_t on);

/* Synchronise and read, per kernel class, the number of launches, the total
   milliseconds and the total algorithmic bytes moved (array length
   TM_KC_COUNT each; any pointer may be NULL). */
tm_status tm_profile_read(tm_ctx* ctx, int64_t* launches, double* ms, double* bytes);

/* The same figures split by kernel variant: one entry per (kernel class,
   storage precision, right-hand sides per lane, solver, reliable-update
   mode) seen since the last
   tm_profile_enable, so that an entry corresponds to one compiled kernel.
   Launches that carry no variant (initialisation, residuals, contraction,
   tm_dslash) have prec = lane_rhs = solver = -1.  Writes at most `cap`
   entries to `out` (host array) and their number to *n; TM_EINVAL if a
   pointer is NULL or cap < 0. */
typedef struct {
    int32_t kc;       /* TM_KC_* */
    int32_t prec;     /* tm_prec of the stored fields, or -1 */
    int32_t lane_rhs; /* right-hand sides per lane, or -1 */
    int32_t solver;   /* tm_solver, or -1 */
    int32_t tseg;     /* time slices per lane of a time-marching kernel, 0 if
                         one lane per site, -1 if not a CG stencil */
    int32_t reliable; /* 1: launched by a solve with reliable updates, else 0
                         (-1 if not a CG stencil) */
    int64_t launches;
    double ms;
    double bytes;
} tm_profile_entry;
tm_status tm_profile_entries(tm_ctx* ctx, tm_profile_entry* out, int32_t cap, int32_t* n);

#ifdef __cplusplus
}
#endif

#endif /* TMQCD_H */
