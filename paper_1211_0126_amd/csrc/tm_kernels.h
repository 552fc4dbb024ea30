// Host-visible launchers of the gfx950 kernels and their argument blocks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tm_types.h"

namespace tmq {

struct CgArgs {
    Geom geo;
    const void* gauge;  // native gauge of the iteration precision
    double kappa;
    double twist;       // 2 kappa mu
    void* p;
    void* t;
    void* r;
    void* x;
    void* rho;          // recursive true residual (stop on |eta - M x|)
    const void* eta64;  // reliable updates stopping on |eta - M x|: the FP64 sources
    CgScal* scal;
    double* partials;   // [nrhs][nblocks]
    double* partials2;  // [nrhs][nblocks]
    int nrhs;
    uint32_t npart;     // block partials per right-hand side written by K1 / K2
    int tseg;           // time slices per lane of the time-marching K1 / K2
    // search directions in a ring (even-odd CG without reduced-precision
    // reliable updates): K3 writes p_{k+1} to pn instead of over p, the step
    // lengths go to ahist[r][k % ring], and x is formed from them afterwards
    void* pn;           // nullable: p = r + beta p in place
    double* ahist;      // nullable: [nrhs][ring]
    int ring;
};

struct ContractArgs {
    Geom geo;
    uint64_t seed_mixed;
    const uint64_t* ids;  // [nrhs] source ids (device)
    const void* sol;      // native solutions (F64 or F32 storage), or with sol_e the odd halves
    const void* sol_e;    // (nullable) the even halves (FP32 or FP16): the solutions in the half layout of hgeo
    Geom hgeo;            // the half-lattice geometry (with sol_e)
    const void* dsol;     // est 2: native D s = (1 - kappa H) s of the same sources, in the solutions' precision
    int est;              // 0 eta^dag Gamma s; 1, 2 the one-end loops (Eqs. 5, 6)
    double2 coef;         // factor of every loop element (1; -2i 2 kappa mu; 2)
    const void* gauge64;  // est 3: FP64 links (double2 [4][9][Vs])
    const void* gauge32;  // est 3 of FP32 solutions: FP32 links (rows 0 and 1, float4 [4][3][Vs])
    int nmu;              // loop sets per source: 4 for est 3 (one per direction), else 1
    int nrhs;
    int npx, npy, npz;    // distinct momentum components per axis (<= 3)
    const double2* phx;   // [npx][Lx] exp(-2 pi i n x / Lx)
    const double2* phy;   // [npy][Ly]
    const double2* phz;   // [npz][Lz]
    int n_mom;
    const int* mom_idx;   // [n_mom][3] indices into the per-axis lists
    const int* gam_col;   // [16][4] column of the nonzero of row a of the insertion
    const int* gam_ph;    // [16][4] its value i^k as k (Gamma_n, g5 Gamma_n or g5 Gamma_n g5)
    double2* A;           // scratch [nrhs * nmu][Lt][Lz][npy][Lx][16]
    double2* B;           // scratch [nrhs * nmu][Lt][Lz][npx][npy][16]
    double2* out;         // loops, [slot][nmu][16][n_mom][Lt]
    const int* out_slot;  // [nrhs] output slot of each right-hand side (device)
    long out_stride;      // complex elements between slots
};

struct FcgArgs {
    Geom geo;
    const void* gauge;  // FP32 native links
    double kappa, twist;
    void *p, *t, *q, *r, *x, *z;  // native fields, nrhs each: p and t in prec, the rest FP32
    FcgScal* scal;
    double* partials;   // [nrhs][4][nblocks]
    int nrhs;
    int prec;           // storage of p and t (P_F32, P_F16 or P_BF16)
};

void launch_fcg_init(hipStream_t st, const FcgArgs& a, double tol2, int maxit, int fell);
void launch_fcg_mp(hipStream_t st, const FcgArgs& a);
void launch_fcg_upd(hipStream_t st, const FcgArgs& a);
void launch_fcg_dot(hipStream_t st, const FcgArgs& a, int init);
void launch_fcg_p(hipStream_t st, const FcgArgs& a);
// finalisers of F1 / F2 over nb block partials per source
void launch_fcg_mp_fin(hipStream_t st, const FcgArgs& a, uint32_t nb);
void launch_fcg_upd_fin(hipStream_t st, const FcgArgs& a, uint32_t nb);
// time-marching F1 / F2 (nr right-hand sides per lane, tseg slices per lane)
void launch_fcg_tm_mp(hipStream_t st, const FcgArgs& a, int nr, int tseg);
void launch_fcg_tm_upd(hipStream_t st, const FcgArgs& a, int nr, int tseg);

// One transport layer of the learned preconditioner (cin, cout <= 2).
struct PtArgs {
    Geom geo;
    const void* gauge;     // FP32 native links (weight gradient)
    const void* gaugebf;   // bfloat16-pair links (layer application)
    int cin, cout;
    int kpad;              // 72 * cin rounded up to 16
    const void* in;        // cin fields (per right-hand side: cin consecutive fields)
    void* out;             // cout fields (per right-hand side), FP32 or bfloat16
    const short* wfrag;    // weight fragments [kpad/16][64 lanes][4] bfloat16
    const FcgScal* gate;   // layer application: right-hand side r is skipped unless gate[r]
                           // is active and has not fallen back (nullptr: all)
    const void* g;         // weight gradient: upstream gradient (cout FP32 fields)
    float* partials;       // weight gradient: [blocks][16][kpad]
    double* partials2;     // weight gradient: [pt_chunks][16][kpad]
};

void launch_pt_layer(hipStream_t st, const PtArgs& a, int in_prec, int out_prec, int nrhs);
void launch_pt_wgrad(hipStream_t st, const PtArgs& a, int in_prec, const double* scale, double* grad);
void launch_pt_loss(hipStream_t st, const Geom& g, const void* y, const void* e, int e_prec, void* gout,
                    double* partials, double* scal, int npairs);
int pt_blocks(const Geom& g);
int pt_chunks(const Geom& g);
void launch_make_pair(hipStream_t st, const Geom& g, uint64_t seed_mixed, const uint64_t* id, const void* xk,
                      const void* xstar, const void* mxk, void* r_out, void* e_out);

// even-odd (Schur complement) kernels on half fields (hg: half geometry,
// V = sites of one parity, Vs their plane stride, L the full extents)
struct EoArgs {
    Geom hg;
    const void* gout;   // links of the output parity (native half layout)
    const void* gin;    // links of the input parity
    int pout;           // parity of the output sites
    double kappa, twist;
    const void* in;     // hop input (parity 1 - pout)
    void* out;
    const void* b;      // centre term (parity pout) or nullptr
    double c;           // coefficient of the hop
    int bnoise;         // 1: the centre term is the Z4 source of the output site
    uint64_t seed_mixed;
    const uint64_t* ids;
    const CgScal* gate; // nullable: only right-hand sides with the reliable flag
    const CgScal* act;  // nullable: skip chunks whose right-hand sides have all stopped
    int nrhs;
};
struct EoCg {
    const void* geven;  // links of the even sites
    const void* godd;   // links of the odd sites
    const void* y;      // intermediate even half field
};
// kinds of launch_eo_lin: out = POST(PRE(b) + c H in)
enum { EO_Y = 0, EO_Y_DAG = 1, EO_T = 2, EO_T_DAG = 3, EO_SRC = 4, EO_REC = 5 };
// etahat = eta_o + kappa H_oe D^{-1} eta_e on the odd sites from the Z4 hash
// (a.out, a.ids, a.nrhs, a.twist, a.kappa, a.seed_mixed; a.gout / a.gin the
// odd / even links of the arithmetic's precision)
void launch_eo_src(hipStream_t st, const EoArgs& a, int prec, int nr);
void launch_eo_lin(hipStream_t st, const EoArgs& a, int prec, int nr, int kind);
void launch_eo_rec_f32(hipStream_t st, const EoArgs& a, int nr);
void launch_eo_dinv(hipStream_t st, const Geom& hg, int prec, double twist, int nrhs, const void* in, void* out);
void launch_eo_mp(hipStream_t st, const CgArgs& a, const EoCg& e, int prec, int nr);
void launch_eo_upd(hipStream_t st, const CgArgs& a, const EoCg& e, int prec, int nr, bool track);
// K2b without the solution update (directions kept in a ring), and the
// update x += sum_k alpha_k p_k over iterations k0 <= k < min(k1, iterations
// of the source), p_k in slot k % ring of `dirs` (slot_bytes apart)
void launch_eo_upd_xfree(hipStream_t st, const CgArgs& a, const EoCg& e, int prec, int nr, bool track);
// (the sum is written to out in out_prec, P_F32 or P_F16; out nullptr: a.x)
void launch_eo_xflush(hipStream_t st, const CgArgs& a, int prec, const void* dirs, size_t slot_bytes, int k0, int k1,
                      void* out = nullptr, int out_prec = P_F32);
uint32_t eo_gated_blocks(const Geom& hg);
void launch_eo_rel_resid(hipStream_t st, const CgArgs& a, const EoCg& e, const void* b64, const void* t64,
                         const void* y64, int nr, int prec = P_F32);
// the same half-hops with the links of a tile of 64 half-sites staged in LDS
// and shared by all right-hand sides (FP32 links; FP32/FP16/BF16 storage);
// reductions write eot_tiles(hg) partials per right-hand side
uint32_t eot_tiles(const Geom& hg);
void launch_eot_y(hipStream_t st, const EoArgs& a, int prec, int nr, bool dag, const CgScal* sc);
void launch_eot_mp(hipStream_t st, const CgArgs& a, const EoCg& e, int prec, int nr, bool dag, const void* cin,
                   void* cout);
void launch_eot_upd(hipStream_t st, const CgArgs& a, const EoCg& e, int prec, int nr, bool track);
void launch_eot_src(hipStream_t st, const EoArgs& a, int prec, int nr);
void launch_eot_rec(hipStream_t st, const EoArgs& a, int nr, const Geom& g, void* full);
// the whole solution in the full native layout from the odd half a.in
void launch_eo_rec_full(hipStream_t st, const EoArgs& a, int xprec, int nr, const Geom& g, void* full);
// FP16 links of one parity (the FP16-storage hops) from its FP64 links
void launch_eo_links_h16(hipStream_t st, const Geom& hg, const void* g64, void* g16);
void launch_eo_split(hipStream_t st, const Geom& g, const Geom& hg, const void* in, int np, void* out_e, void* out_o);
void launch_eo_merge(hipStream_t st, const Geom& g, const Geom& hg, const void* in_e, const void* in_o, int np,
                     void* out);

// operator
void launch_apply(hipStream_t st, const Geom& g, int prec, const void* gauge, double kappa, double twist, int op,
                  int nrhs, const void* in, void* out, int nr, const CgScal* gate);
// CG
void launch_scal_init(hipStream_t st, CgScal* sc, int n, double tol2, int maxit, int stop, int reliable,
                      double delta2);
// ee_z4 > 0: |eta|^2 of every source (12 V of a Z4 source); else measured from eta
void launch_cg_init(hipStream_t st, const CgArgs& a, int prec, bool track, const void* eta, double ee_z4 = -1.0);
void launch_cg_mp(hipStream_t st, const CgArgs& a, int prec, int nr);
void launch_cg_upd(hipStream_t st, const CgArgs& a, int prec, int nr, bool track);
// time-marching K1 / K2 (a.tseg time slices per lane); they write
// march_partials(geo, tseg) partials per right-hand side
uint32_t march_partials(const Geom& g, int tseg);
void launch_tm_mp(hipStream_t st, const CgArgs& a, int prec, int nr);
void launch_tm_upd(hipStream_t st, const CgArgs& a, int prec, int nr, bool track);
void launch_cg_alpha(hipStream_t st, const CgArgs& a);              // after launch_cg_mp
void launch_cg_beta(hipStream_t st, const CgArgs& a, bool track);   // after launch_cg_upd
void launch_cg_p(hipStream_t st, const CgArgs& a, int prec);
// (prec: storage of r and p; x stays FP32)
void launch_rel_init(hipStream_t st, const CgArgs& a, const void* b64, void* x64, double ee_z4 = -1.0,
                     int prec = P_F32);
void launch_rel_fin(hipStream_t st, const CgArgs& a, uint32_t nb);
void launch_rel_flush(hipStream_t st, const CgArgs& a, void* x64, int force);
void launch_rel_resid(hipStream_t st, const CgArgs& a, const void* gauge64, const void* b64, const void* t64);
void launch_true_resid(hipStream_t st, const CgArgs& a, int xprec, const void* gauge64, uint64_t seed_mixed,
                       const uint64_t* ids);

// layout and noise
void launch_field_convert(hipStream_t st, const Geom& g, int prec, int nrhs, bool to_native, const void* in,
                          void* out);
// solutions (native, F64 or F32 storage) -> right-hand sides r0.. of a
// caller's field in out_prec, canonical or native
void launch_sol_out(hipStream_t st, const Geom& g, int prec, int nrhs, const void* in, void* out, int out_prec,
                    bool native, int r0);
void launch_native_to_c128(hipStream_t st, const Geom& g, int prec, int nrhs, const void* in, double* out);
void launch_c128_to_native(hipStream_t st, const Geom& g, int prec, int nrhs, const double* in, void* out);
void launch_gauge_convert(hipStream_t st, const Geom& g, const double* canon, void* g64, void* g32, void* gbf);
void launch_noise_native(hipStream_t st, const Geom& g, int prec, uint64_t seed_mixed, const uint64_t* ids, int nrhs,
                         void* out);
void launch_noise_c128(hipStream_t st, const Geom& g, uint64_t seed_mixed, const uint64_t* ids, int nrhs, double* out);

// loops
void launch_contract(hipStream_t st, const ContractArgs& a, int xprec);
// standard loops at all Lx*Ly*Lz momenta: site matrices into buf0, DFTs
// ping-ponging buf0/buf1 (each nrhs * V * 16 double2), tw the x, y, z
// phase tables exp(-2 pi i m / L) back to back
void launch_contract_all_momenta(hipStream_t st, const ContractArgs& a, int xprec, double2* buf0, double2* buf1,
                                 const double2* tw);
void launch_tsm_final(hipStream_t st, const double* ps, long nl, int n_hp, int n_lp, double* out, double* err);

}  // namespace tmq
