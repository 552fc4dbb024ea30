/*
 * tm_oracle.c -- plain, slow CPU FP64 oracle for the truncated-solver-method
 * (TSM) evaluation of disconnected quark loops with twisted-mass Wilson
 * fermions (Alexandrou et al., "Evaluation of disconnected contributions
 * using GPUs", Lattice 2012, arXiv:1211.0126).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the
 * GPU library.  Every routine is the plain definition written out: full 4x4
 * gamma matrices, full 3x3 links, direct phase sums, serial reductions.  The
 * only parallelism is an OpenMP loop over sites in the hopping term, where
 * every site is written by exactly one thread, so results do not depend on
 * the thread count.
 *
 * Conventions (readings of points the paper leaves open):
 *  - site = x + Lx*(y + Ly*(z + Lz*t)); direction mu = 0..3 is x, y, z, t.
 *  - spinor component index 3*spin + colour, complex128 interleaved.
 *  - link U_mu(x) is stored at [site][mu][row][col]; it multiplies psi(x+mu).
 *  - time boundary: a hop across t = Lt-1 <-> 0 carries the factor t_bc
 *    (-1 antiperiodic); space is periodic.
 *  - Euclidean chiral gamma basis, gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4
 *    = diag(1, 1, -1, -1); Gamma_n = g1^b0 g2^b1 g3^b2 g4^b3 for
 *    n = b0 + 2 b1 + 4 b2 + 8 b3 (Gamma_0 = 1, Gamma_15 = gamma_5).
 *  - hopping normalisation: M = 1 - kappa*H + 2i*kappa*mu*gamma_5 with
 *    H psi(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu)
 *                    + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu).
 *    This is 2*kappa times the physical M_u = D_W + i*mu*a*gamma_5 of the
 *    flavour identity M_u - M_d = 2i*mu*a*gamma_5 (section 2.3).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define NSPIN 4
#define NCOL 3
#define NCOMP 12

/* ------------------------------------------------------------------ */
/* threads                                                             */
/* ------------------------------------------------------------------ */

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* geometry                                                            */
/* ------------------------------------------------------------------ */

static long volume(const int *L) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void site_coords(const int *L, long s, int c[4])
{
    c[0] = (int)(s % L[0]); s /= L[0];
    c[1] = (int)(s % L[1]); s /= L[1];
    c[2] = (int)(s % L[2]); s /= L[2];
    c[3] = (int)s;
}

static long site_of(const int *L, const int c[4])
{
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

/* neighbour of s one step in direction mu, forward (dir=+1) or backward
   (dir=-1); *phase receives t_bc when the hop wraps in time, else 1 */
static long neighbour(const int *L, int t_bc, long s, int mu, int dir, double *phase)
{
    int c[4];
    site_coords(L, s, c);
    *phase = 1.0;
    c[mu] += dir;
    if (c[mu] == L[mu]) { c[mu] = 0; if (mu == 3) *phase = (double)t_bc; }
    if (c[mu] < 0) { c[mu] = L[mu] - 1; if (mu == 3) *phase = (double)t_bc; }
    return site_of(L, c);
}

/* ------------------------------------------------------------------ */
/* gamma matrices                                                      */
/* ------------------------------------------------------------------ */

/* Euclidean chiral basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]],
   gamma_4 = [[0, 1], [1, 0]] in 2x2 blocks. */
static void gamma_mu(int mu, cplx g[4][4])
{
    memset(g, 0, sizeof(cplx) * 16);
    switch (mu) {
    case 0: g[0][3] = -I; g[1][2] = -I; g[2][1] = I; g[3][0] = I; break;
    case 1: g[0][3] = -1; g[1][2] = 1; g[2][1] = 1; g[3][0] = -1; break;
    case 2: g[0][2] = -I; g[1][3] = I; g[2][0] = I; g[3][1] = -I; break;
    default: g[0][2] = 1; g[1][3] = 1; g[2][0] = 1; g[3][1] = 1; break;
    }
}

static void matmul4(const cplx a[4][4], const cplx b[4][4], cplx c[4][4])
{
    cplx t[4][4];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx acc = 0;
            for (int k = 0; k < 4; k++) acc += a[i][k] * b[k][j];
            t[i][j] = acc;
        }
    memcpy(c, t, sizeof(t));
}

/* Gamma_n = g1^b0 g2^b1 g3^b2 g4^b3, written into out[16] (row-major 4x4) */
void orc_gamma(int n, double *out)
{
    cplx r[4][4], g[4][4];
    memset(r, 0, sizeof(r));
    for (int i = 0; i < 4; i++) r[i][i] = 1;
    for (int mu = 0; mu < 4; mu++)
        if ((n >> mu) & 1) { gamma_mu(mu, g); matmul4(r, g, r); }
    memcpy(out, r, sizeof(r));
}

/* gamma_mu for mu = 0..3 and gamma_5 for mu = 4 */
void orc_gamma_mu(int mu, double *out)
{
    cplx g[4][4];
    if (mu < 4) gamma_mu(mu, g);
    else orc_gamma(15, (double *)g);
    memcpy(out, g, sizeof(g));
}

static void gamma5(cplx g[4][4]) { orc_gamma(15, (double *)g); }

/* ------------------------------------------------------------------ */
/* Z4 noise (Eq. 1): counter-based splitmix64                          */
/* ------------------------------------------------------------------ */

/* splitmix64 output function (Steele, Lea & Flood, OOPSLA 2014) */
static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* sequential splitmix64: advance the state by the golden-ratio increment and
   return the mixed state; exported so tests can pin it to published values */
uint64_t orc_splitmix64_next(uint64_t *state)
{
    *state += 0x9E3779B97F4A7C15ULL;
    return mix64(*state);
}

/* 64-bit hash for source id j at site s: output number 1 + j*V + s of a
   splitmix64 stream started at state mix64(seed) */
uint64_t orc_noise_hash(uint64_t seed, uint64_t j, uint64_t vol, uint64_t s)
{
    uint64_t z = mix64(seed) + 0x9E3779B97F4A7C15ULL * (1 + j * vol + s);
    return mix64(z);
}

/* Z4 codes k_c in {0,1,2,3} for every component: eta = i^k */
void orc_noise_codes(const int *L, uint64_t seed, uint64_t j, uint8_t *codes)
{
    long V = volume(L);
    for (long s = 0; s < V; s++) {
        uint64_t h = orc_noise_hash(seed, j, (uint64_t)V, (uint64_t)s);
        for (int c = 0; c < NCOMP; c++) codes[s * NCOMP + c] = (uint8_t)((h >> (2 * c)) & 3);
    }
}

/* the Z4 source eta_j itself, complex128 [V][4][3] */
void orc_noise_z4(const int *L, uint64_t seed, uint64_t j, double *eta_out)
{
    static const cplx z4[4] = {1.0, I, -1.0, -I};
    cplx *eta = (cplx *)eta_out;
    long V = volume(L);
    for (long s = 0; s < V; s++) {
        uint64_t h = orc_noise_hash(seed, j, (uint64_t)V, (uint64_t)s);
        for (int c = 0; c < NCOMP; c++) eta[s * NCOMP + c] = z4[(h >> (2 * c)) & 3];
    }
}

/* ------------------------------------------------------------------ */
/* the operator                                                        */
/* ------------------------------------------------------------------ */

/* H (dagger = 0) or its adjoint H^dag (dagger = 1).  The adjoint follows
   from transposing the hop: (1 + g_mu) U_mu(x) psi(x+mu) +
   (1 - g_mu) U_mu(x-mu)^dag psi(x-mu). */
static void hop(const int *L, int t_bc, const cplx *U, const cplx *in, cplx *out, int dagger)
{
    long V = volume(L);
    cplx gm[4][4][4];
    for (int mu = 0; mu < 4; mu++) gamma_mu(mu, gm[mu]);

#pragma omp parallel for schedule(static) if (V >= 8192)
    for (long s = 0; s < V; s++) {
        cplx acc[NSPIN][NCOL];
        memset(acc, 0, sizeof(acc));
        for (int mu = 0; mu < 4; mu++) {
            for (int dir = -1; dir <= 1; dir += 2) {
                double ph;
                long y = neighbour(L, t_bc, s, mu, dir, &ph);
                /* colour-transported neighbour, per spin */
                cplx v[NSPIN][NCOL];
                for (int a = 0; a < NSPIN; a++)
                    for (int i = 0; i < NCOL; i++) {
                        cplx t = 0;
                        for (int k = 0; k < NCOL; k++) {
                            cplx u;
                            if (dir > 0) u = U[((s * 4 + mu) * 3 + i) * 3 + k];
                            else u = conj(U[((y * 4 + mu) * 3 + k) * 3 + i]);
                            t += u * in[y * NCOMP + a * NCOL + k];
                        }
                        v[a][i] = ph * t;
                    }
                /* spin projector 1 - sgn*gamma_mu, sgn = +1 for the forward
                   hop of H and the backward hop of H^dag */
                double sgn = (dir > 0) ? 1.0 : -1.0;
                if (dagger) sgn = -sgn;
                for (int a = 0; a < NSPIN; a++)
                    for (int b = 0; b < NSPIN; b++) {
                        cplx p = (a == b ? 1.0 : 0.0) - sgn * gm[mu][a][b];
                        if (p == 0) continue;
                        for (int i = 0; i < NCOL; i++) acc[a][i] += p * v[b][i];
                    }
            }
        }
        for (int a = 0; a < NSPIN; a++)
            for (int i = 0; i < NCOL; i++) out[s * NCOMP + a * NCOL + i] = acc[a][i];
    }
}

/* M (op 0), M^dag (op 1), M^dag M (op 2), H (op 3) */
enum { ORC_M = 0, ORC_MDAG = 1, ORC_MDAGM = 2, ORC_HOP = 3 };

static void apply_m(const int *L, int t_bc, double kappa, double mu, const cplx *U,
                    const cplx *in, cplx *out, int dagger)
{
    long V = volume(L);
    cplx g5[4][4];
    gamma5(g5);
    hop(L, t_bc, U, in, out, dagger);
    /* twisted mass term +2i kappa mu gamma_5 (its adjoint has the minus sign) */
    cplx tm = (dagger ? -1.0 : 1.0) * 2.0 * I * kappa * mu;
    for (long s = 0; s < V; s++)
        for (int a = 0; a < NSPIN; a++)
            for (int i = 0; i < NCOL; i++) {
                cplx g5psi = 0;
                for (int b = 0; b < NSPIN; b++) g5psi += g5[a][b] * in[s * NCOMP + b * NCOL + i];
                long k = s * NCOMP + a * NCOL + i;
                out[k] = in[k] - kappa * out[k] + tm * g5psi;
            }
}

void orc_apply(const int *L, int t_bc, double kappa, double mu, int op,
               const double *U_, const double *in_, double *out_)
{
    const cplx *U = (const cplx *)U_;
    const cplx *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    long n = volume(L) * NCOMP;
    switch (op) {
    case ORC_M: apply_m(L, t_bc, kappa, mu, U, in, out, 0); break;
    case ORC_MDAG: apply_m(L, t_bc, kappa, mu, U, in, out, 1); break;
    case ORC_MDAGM: {
        cplx *tmp = malloc(sizeof(cplx) * n);
        apply_m(L, t_bc, kappa, mu, U, in, tmp, 0);
        apply_m(L, t_bc, kappa, mu, U, tmp, out, 1);
        free(tmp);
        break;
    }
    default: hop(L, t_bc, U, in, out, 0); break;
    }
}

/* ------------------------------------------------------------------ */
/* CG on the normal equations (the inverter of section 2.2)           */
/* ------------------------------------------------------------------ */

static double norm2(const cplx *a, long n)
{
    double s = 0;
    for (long i = 0; i < n; i++) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

enum { ORC_STOP_NORMAL = 0, ORC_STOP_TRUE = 1 };

/*
 * Solve M s = eta through M^dag M s = M^dag eta by conjugate gradients from
 * s = 0.  Stop (checked before every iteration) when the relative residual
 * is <= tol or when maxit iterations are done (maxit < 0: no cap).  The
 * residual is that of the normal equations (stop = 0) or the recursively
 * tracked residual eta - M s of the original system (stop = 1).  These are
 * the two truncation criteria of section 2.2 (a residual or a fixed number
 * of iterations).
 *
 * stats[0] iterations, [1] final normal-equation relative residual,
 * [2] true relative residual |eta - M s|/|eta| computed directly,
 * [3] 1 if stopped by the tolerance, [4] 1 if stopped by the iteration cap.
 */
int orc_cgnr(const int *L, int t_bc, double kappa, double mu, const double *U_,
             const double *eta_, double tol, int maxit, int stop,
             double *x_, double *stats)
{
    const cplx *U = (const cplx *)U_;
    const cplx *eta = (const cplx *)eta_;
    cplx *x = (cplx *)x_;
    long n = volume(L) * NCOMP;
    cplx *b = malloc(sizeof(cplx) * n), *r = malloc(sizeof(cplx) * n);
    cplx *p = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    cplx *q = malloc(sizeof(cplx) * n), *rho = malloc(sizeof(cplx) * n);

    apply_m(L, t_bc, kappa, mu, U, eta, b, 1);
    for (long i = 0; i < n; i++) { x[i] = 0; r[i] = b[i]; p[i] = b[i]; rho[i] = eta[i]; }
    double rr = norm2(r, n), bb = rr, ee = norm2(eta, n), rhorho = ee;
    int it = 0, conv = 0, trunc = 0;
    for (;;) {
        double rel = (stop == ORC_STOP_TRUE) ? sqrt(rhorho / ee) : sqrt(rr / bb);
        if (rel <= tol) { conv = 1; break; }
        if (maxit >= 0 && it >= maxit) { trunc = 1; break; }
        apply_m(L, t_bc, kappa, mu, U, p, t, 0);
        double tt = norm2(t, n);
        double alpha = rr / tt;
        for (long i = 0; i < n; i++) x[i] += alpha * p[i];
        if (stop == ORC_STOP_TRUE) {
            for (long i = 0; i < n; i++) rho[i] -= alpha * t[i];
            rhorho = norm2(rho, n);
        }
        apply_m(L, t_bc, kappa, mu, U, t, q, 1);
        for (long i = 0; i < n; i++) r[i] -= alpha * q[i];
        double rr_new = norm2(r, n);
        double beta = rr_new / rr;
        for (long i = 0; i < n; i++) p[i] = r[i] + beta * p[i];
        rr = rr_new;
        it++;
    }
    if (stats) {
        apply_m(L, t_bc, kappa, mu, U, x, t, 0);
        for (long i = 0; i < n; i++) t[i] = eta[i] - t[i];
        stats[0] = it;
        stats[1] = sqrt(rr / bb);
        stats[2] = sqrt(norm2(t, n) / ee);
        stats[3] = conv;
        stats[4] = trunc;
    }
    free(b); free(r); free(p); free(t); free(q); free(rho);
    return it;
}

/* ------------------------------------------------------------------ */
/* even-odd (Schur-complement) reduction of M                          */
/* ------------------------------------------------------------------ */

/*
 * Not in the paper: the standard even-odd reduction of the twisted-mass
 * operator, here an alternative inverter for the LP (and HP) solves.  The
 * TSM combination of Eq. 4 stays unbiased for any fixed LP map, so the
 * estimator is unchanged; only the truncated solutions differ.
 *
 * A site is even or odd by the parity of x + y + z + t.  With every extent
 * even, each hop of H changes the parity, so with the sites split by parity
 *     A = [[A_ee, A_eo], [A_oe, A_oo]]        (A = M or A = M^dag)
 * has diagonal blocks that act site by site (the twisted-mass term) and the
 * Schur complement on the odd sites is
 *     Ahat = A_oo - A_oe A_ee^{-1} A_eo.
 * M x = eta is solved as Mhat x_o = etahat_o with
 *     etahat_o = eta_o - M_oe M_ee^{-1} eta_e,
 * and the even half follows as x_e = M_ee^{-1} (eta_e - M_eo x_o).  Then
 * (eta - M x)_e = 0 and (eta - M x)_o = etahat_o - Mhat x_o.  (Mhat)^dag is
 * the same construction on A = M^dag.
 *
 * Fields are full size [V][4][3]; a field of one parity has zeros on the
 * sites of the other.
 */

static int parity_of(const int *L, long s)
{
    int c[4];
    site_coords(L, s, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

static int all_even(const int *L)
{
    for (int d = 0; d < 4; d++)
        if (L[d] % 2) return 0;
    return 1;
}

/* out = in on the sites of parity par, zero elsewhere */
static void mask_parity(const int *L, const cplx *in, cplx *out, int par)
{
    long V = volume(L);
    for (long s = 0; s < V; s++)
        for (int k = 0; k < NCOMP; k++)
            out[s * NCOMP + k] = parity_of(L, s) == par ? in[s * NCOMP + k] : 0;
}

/* v <- A_pp^{-1} v on the sites of parity par.  The diagonal block of M is
   1 + i tw gamma_5 on every site (tw = 2 kappa mu; H has no on-site term),
   that of M^dag is 1 - i tw gamma_5; gamma_5 = diag(1, 1, -1, -1), so the
   inverse divides spin component a by 1 +- i tw g5[a][a]. */
static void diag_block_inverse(const int *L, double kappa, double mu, int dagger, cplx *v, int par)
{
    long V = volume(L);
    cplx g5[4][4];
    gamma5(g5);
    double tw = (dagger ? -1.0 : 1.0) * 2.0 * kappa * mu;
    for (long s = 0; s < V; s++) {
        if (parity_of(L, s) != par) continue;
        for (int a = 0; a < NSPIN; a++)
            for (int i = 0; i < NCOL; i++) v[s * NCOMP + a * NCOL + i] /= (1.0 + I * tw * g5[a][a]);
    }
}

/* out = Ahat in (odd sites of in used, even sites of out zero), A = M or M^dag */
static void schur_apply(const int *L, int t_bc, double kappa, double mu, const cplx *U,
                        const cplx *in, cplx *out, int dagger)
{
    long n = volume(L) * NCOMP;
    cplx *a = malloc(sizeof(cplx) * n), *b = malloc(sizeof(cplx) * n);
    cplx *c = malloc(sizeof(cplx) * n), *f = malloc(sizeof(cplx) * n);
    mask_parity(L, in, a, 1);                          /* a = x_o */
    apply_m(L, t_bc, kappa, mu, U, a, b, dagger);      /* b_o = A_oo x_o, b_e = A_eo x_o */
    mask_parity(L, b, c, 0);                           /* c = A_eo x_o */
    diag_block_inverse(L, kappa, mu, dagger, c, 0);    /* c = A_ee^{-1} A_eo x_o */
    apply_m(L, t_bc, kappa, mu, U, c, f, dagger);      /* f_o = A_oe c_e */
    for (long i = 0; i < n; i++) f[i] = b[i] - f[i];
    mask_parity(L, f, out, 1);
    free(a); free(b); free(c); free(f);
}

/* Mhat (op 0), Mhat^dag (op 1), Mhat^dag Mhat (op 2) on odd-site fields;
   returns -1 (nothing written) unless every extent is even */
int orc_eo_apply(const int *L, int t_bc, double kappa, double mu, int op,
                 const double *U_, const double *in_, double *out_)
{
    if (!all_even(L)) return -1;
    const cplx *U = (const cplx *)U_;
    const cplx *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    long n = volume(L) * NCOMP;
    if (op == 2) {
        cplx *tmp = malloc(sizeof(cplx) * n);
        schur_apply(L, t_bc, kappa, mu, U, in, tmp, 0);
        schur_apply(L, t_bc, kappa, mu, U, tmp, out, 1);
        free(tmp);
    } else {
        schur_apply(L, t_bc, kappa, mu, U, in, out, op == 1);
    }
    return 0;
}

/* etahat = eta_o - M_oe M_ee^{-1} eta_e (odd-site field) */
void orc_eo_source(const int *L, int t_bc, double kappa, double mu, const double *U_,
                   const double *eta_, double *out_)
{
    const cplx *U = (const cplx *)U_;
    const cplx *eta = (const cplx *)eta_;
    cplx *out = (cplx *)out_;
    long n = volume(L) * NCOMP;
    cplx *e = malloc(sizeof(cplx) * n), *f = malloc(sizeof(cplx) * n);
    mask_parity(L, eta, e, 0);
    diag_block_inverse(L, kappa, mu, 0, e, 0);
    apply_m(L, t_bc, kappa, mu, U, e, f, 0);           /* f_o = M_oe M_ee^{-1} eta_e */
    for (long i = 0; i < n; i++) f[i] = eta[i] - f[i];
    mask_parity(L, f, out, 1);
    free(e); free(f);
}

/* x_e = M_ee^{-1} (eta_e - M_eo x_o): x holds x_o on entry and the whole
   solution on return */
void orc_eo_reconstruct(const int *L, int t_bc, double kappa, double mu, const double *U_,
                        const double *eta_, double *x_)
{
    const cplx *U = (const cplx *)U_;
    const cplx *eta = (const cplx *)eta_;
    cplx *x = (cplx *)x_;
    long n = volume(L) * NCOMP;
    cplx *a = malloc(sizeof(cplx) * n), *g = malloc(sizeof(cplx) * n), *h = malloc(sizeof(cplx) * n);
    mask_parity(L, x, a, 1);
    apply_m(L, t_bc, kappa, mu, U, a, g, 0);           /* g_e = M_eo x_o */
    for (long i = 0; i < n; i++) g[i] = eta[i] - g[i];
    mask_parity(L, g, h, 0);
    diag_block_inverse(L, kappa, mu, 0, h, 0);
    for (long i = 0; i < n; i++) x[i] = a[i] + h[i];
    free(a); free(g); free(h);
}

/*
 * Solve M x = eta by CG on the normal equations of the Schur complement,
 * Mhat^dag Mhat x_o = Mhat^dag etahat_o, from x_o = 0, then reconstruct
 * x_e.  Stop (checked before every iteration) when the relative residual is
 * <= tol or after maxit iterations (maxit < 0: no cap).  The residual is
 * that of these normal equations (stop = 0), or the recursively tracked
 * etahat_o - Mhat x_o, which is the residual eta - M x of the whole system,
 * relative to |eta| (stop = 1).  stats as orc_cgnr, with stats[1] the final
 * relative residual of the Schur normal equations.  Returns -1 unless
 * every extent is even.
 */
int orc_cgnr_eo(const int *L, int t_bc, double kappa, double mu, const double *U_,
                const double *eta_, double tol, int maxit, int stop,
                double *x_, double *stats)
{
    if (!all_even(L)) return -1;
    const cplx *U = (const cplx *)U_;
    const cplx *eta = (const cplx *)eta_;
    cplx *x = (cplx *)x_;
    long n = volume(L) * NCOMP;
    cplx *eh = malloc(sizeof(cplx) * n), *b = malloc(sizeof(cplx) * n), *r = malloc(sizeof(cplx) * n);
    cplx *p = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    cplx *q = malloc(sizeof(cplx) * n), *rho = malloc(sizeof(cplx) * n);

    orc_eo_source(L, t_bc, kappa, mu, U_, eta_, (double *)eh);
    schur_apply(L, t_bc, kappa, mu, U, eh, b, 1);
    for (long i = 0; i < n; i++) { x[i] = 0; r[i] = b[i]; p[i] = b[i]; rho[i] = eh[i]; }
    double rr = norm2(r, n), bb = rr, ee = norm2(eta, n), rhorho = norm2(eh, n);
    int it = 0, conv = 0, trunc = 0;
    for (;;) {
        double rel = (stop == ORC_STOP_TRUE) ? sqrt(rhorho / ee) : sqrt(rr / bb);
        if (rel <= tol) { conv = 1; break; }
        if (maxit >= 0 && it >= maxit) { trunc = 1; break; }
        schur_apply(L, t_bc, kappa, mu, U, p, t, 0);
        double tt = norm2(t, n);
        double alpha = rr / tt;
        for (long i = 0; i < n; i++) x[i] += alpha * p[i];
        if (stop == ORC_STOP_TRUE) {
            for (long i = 0; i < n; i++) rho[i] -= alpha * t[i];
            rhorho = norm2(rho, n);
        }
        schur_apply(L, t_bc, kappa, mu, U, t, q, 1);
        for (long i = 0; i < n; i++) r[i] -= alpha * q[i];
        double rr_new = norm2(r, n);
        double beta = rr_new / rr;
        for (long i = 0; i < n; i++) p[i] = r[i] + beta * p[i];
        rr = rr_new;
        it++;
    }
    orc_eo_reconstruct(L, t_bc, kappa, mu, U_, eta_, x_);
    if (stats) {
        apply_m(L, t_bc, kappa, mu, U, x, t, 0);
        for (long i = 0; i < n; i++) t[i] = eta[i] - t[i];
        stats[0] = it;
        stats[1] = sqrt(rr / bb);
        stats[2] = sqrt(norm2(t, n) / ee);
        stats[3] = conv;
        stats[4] = trunc;
    }
    free(eh); free(b); free(r); free(p); free(t); free(q); free(rho);
    return it;
}

/* ------------------------------------------------------------------ */
/* loops: <eta^dag Gamma s> per timeslice and momentum (section 2.3)   */
/* ------------------------------------------------------------------ */

/*
 * out[n][m][t] += sum over sites x with time t of
 *     exp(-i p_m . x) * sum_{a,b,c} conj(eta(x)_{a c}) Gamma_n[a][b] s(x)_{b c}
 * with p_m = 2 pi (mom[m][0]/Lx, mom[m][1]/Ly, mom[m][2]/Lz).  The sum runs
 * over all sites of each timeslice (the Fourier transform of the paper is
 * this sum at the chosen momenta).  out is complex128 [16][n_mom][Lt] and is
 * accumulated into, not cleared.
 */
void orc_loops(const int *L, const double *eta_, const double *s_, int n_mom,
               const int *mom, double *out_)
{
    const cplx *eta = (const cplx *)eta_;
    const cplx *sv = (const cplx *)s_;
    cplx *out = (cplx *)out_;
    long V = volume(L);
    int Lt = L[3];
    cplx G[16][4][4];
    for (int n = 0; n < 16; n++) orc_gamma(n, (double *)G[n]);
    const double twopi = 2.0 * acos(-1.0);
    for (long s = 0; s < V; s++) {
        int c[4];
        site_coords(L, s, c);
        cplx tr[16];
        for (int n = 0; n < 16; n++) {
            cplx acc = 0;
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) {
                    if (G[n][a][b] == 0) continue;
                    for (int k = 0; k < NCOL; k++)
                        acc += conj(eta[s * NCOMP + a * NCOL + k]) * G[n][a][b] * sv[s * NCOMP + b * NCOL + k];
                }
            tr[n] = acc;
        }
        for (int m = 0; m < n_mom; m++) {
            double arg = twopi * ((double)mom[3 * m] * c[0] / L[0] + (double)mom[3 * m + 1] * c[1] / L[1] +
                                  (double)mom[3 * m + 2] * c[2] / L[2]);
            cplx ph = cexp(-I * arg);
            for (int n = 0; n < 16; n++) out[((long)n * n_mom + m) * Lt + c[3]] += ph * tr[n];
        }
    }
}

/* ------------------------------------------------------------------ */
/* one-end trick loops (section 2.3, Eqs. 5 and 6)                     */
/* ------------------------------------------------------------------ */

/*
 * Loops that use the solution on both sides of the bilinear; the source
 * does not appear.  With s = M_u^{-1} eta (M_u the operator above, M_d the
 * same operator with mu -> -mu, both in hopping normalisation) and
 * tw = 2 kappa mu:
 *
 *   est 1, isovector (Eq. 5):
 *     out[n][m][t] += -2i tw sum_{x in t} exp(-i p_m.x) s(x)^dag g5 Gamma_n s(x)
 *   whose noise average is Tr over the timeslice of
 *   exp(-i p.x) Gamma_n (M_u^{-1} - M_d^{-1}).  The factor follows from
 *   M_u - M_d = 2i tw g5: M_u^{-1} - M_d^{-1} = -2i tw M_u^{-1} (M_u^{-1})^dag g5
 *   (with g5 M_u g5 = M_d^dag); the printed sign of Eq. 5 is the opposite.
 *
 *   est 2, generalized (Eq. 6):
 *     out[n][m][t] += 2 sum_{x in t} exp(-i p_m.x) s(x)^dag g5 Gamma_n g5 (D s)(x)
 *   with D = (M_u + M_d)/2 = 1 - kappa H (the operator at mu = 0), whose
 *   noise average is the same trace of Gamma_n (M_u^{-1} + M_d^{-1}).
 *
 * est 0 is the standard loop of orc_loops and est 3 the one-derivative
 * loops of orc_loops_deriv (eta must then be given).  out is complex128
 * [16][n_mom][Lt] ([4][16][n_mom][Lt] for est 3), accumulated into.
 */
void orc_loops_deriv(const int *L, int t_bc, const double *U_, const double *eta_, const double *s_, int n_mom,
                     const int *mom, double *out_);

void orc_loops_est(const int *L, int t_bc, double kappa, double mu, const double *U_, int est,
                   const double *eta_, const double *s_, int n_mom, const int *mom, double *out_)
{
    if (est == 0) {
        orc_loops(L, eta_, s_, n_mom, mom, out_);
        return;
    }
    if (est == 3) {
        orc_loops_deriv(L, t_bc, U_, eta_, s_, n_mom, mom, out_);
        return;
    }
    const cplx *sv = (const cplx *)s_;
    cplx *out = (cplx *)out_;
    long V = volume(L);
    int Lt = L[3];
    cplx *right = malloc(sizeof(cplx) * V * NCOMP);
    cplx G[16][4][4], g5[4][4], coef;
    gamma5(g5);
    for (int n = 0; n < 16; n++) {
        cplx gn[4][4];
        orc_gamma(n, (double *)gn);
        matmul4(g5, gn, G[n]);
        if (est == 2) matmul4(G[n], g5, G[n]);
    }
    if (est == 1) {
        coef = -2.0 * I * (2.0 * kappa * mu);
        memcpy(right, sv, sizeof(cplx) * V * NCOMP);
    } else {
        coef = 2.0;
        apply_m(L, t_bc, kappa, 0.0, (const cplx *)U_, sv, right, 0);
    }
    const double twopi = 2.0 * acos(-1.0);
    for (long s = 0; s < V; s++) {
        int c[4];
        site_coords(L, s, c);
        cplx tr[16];
        for (int n = 0; n < 16; n++) {
            cplx acc = 0;
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) {
                    if (G[n][a][b] == 0) continue;
                    for (int k = 0; k < NCOL; k++)
                        acc += conj(sv[s * NCOMP + a * NCOL + k]) * G[n][a][b] * right[s * NCOMP + b * NCOL + k];
                }
            tr[n] = coef * acc;
        }
        for (int m = 0; m < n_mom; m++) {
            double arg = twopi * ((double)mom[3 * m] * c[0] / L[0] + (double)mom[3 * m + 1] * c[1] / L[1] +
                                  (double)mom[3 * m + 2] * c[2] / L[2]);
            cplx ph = cexp(-I * arg);
            for (int n = 0; n < 16; n++) out[((long)n * n_mom + m) * Lt + c[3]] += ph * tr[n];
        }
    }
    free(right);
}

/* ------------------------------------------------------------------ */
/* one-derivative loops (the operators of section 3 and Fig. 1)        */
/* ------------------------------------------------------------------ */

/*
 * Loops of psibar(x) Gamma_n Dsym_mu psi(x) with the symmetric covariant
 * derivative Dsym = (Dfwd - Dbwd)/2,
 *   Dfwd_mu psi(x)   = [U_mu(x) psi(x+mu) - U_mu(x-mu)^dag psi(x-mu)] / 2,
 *   psibar Dbwd_mu(x) = [psibar(x+mu) U_mu(x)^dag - psibar(x-mu) U_mu(x-mu)] / 2,
 * with the propagator estimated by s eta^dag as in the standard loop:
 *   out[mu][n][m][t] += sum_{x in t} exp(-i p_m.x) (1/4) sum_{a,b,c}
 *       [ conj(eta_ac(x)) Gamma_n[a][b] f_bc(x) - conj(g_ac(x)) Gamma_n[a][b] s_bc(x) ],
 *   f = U_mu(x) s(x+mu) - U_mu(x-mu)^dag s(x-mu),
 *   g = U_mu(x) eta(x+mu) - U_mu(x-mu)^dag eta(x-mu),
 * hops across the time boundary carrying t_bc as in the operator.  The
 * timeslice and phase are those of x.  out: complex128
 * [4][16][n_mom][Lt], accumulated into.
 */
void orc_loops_deriv(const int *L, int t_bc, const double *U_, const double *eta_, const double *s_, int n_mom,
                     const int *mom, double *out_)
{
    const cplx *U = (const cplx *)U_, *eta = (const cplx *)eta_, *sv = (const cplx *)s_;
    cplx *out = (cplx *)out_;
    long V = volume(L);
    int Lt = L[3];
    cplx G[16][4][4];
    for (int n = 0; n < 16; n++) orc_gamma(n, (double *)G[n]);
    const double twopi = 2.0 * acos(-1.0);
    for (long x = 0; x < V; x++) {
        int c[4];
        site_coords(L, x, c);
        for (int mu = 0; mu < 4; mu++) {
            double php, phm;
            long xp = neighbour(L, t_bc, x, mu, +1, &php);
            long xm = neighbour(L, t_bc, x, mu, -1, &phm);
            cplx f[NSPIN][NCOL], g[NSPIN][NCOL];
            for (int a = 0; a < NSPIN; a++)
                for (int i = 0; i < NCOL; i++) {
                    cplx fs = 0, ge = 0;
                    for (int k = 0; k < NCOL; k++) {
                        cplx up = U[((x * 4 + mu) * 3 + i) * 3 + k];          /* U_mu(x)[i][k] */
                        cplx um = conj(U[((xm * 4 + mu) * 3 + k) * 3 + i]);   /* U_mu(x-mu)^dag[i][k] */
                        fs += php * up * sv[xp * NCOMP + a * NCOL + k] - phm * um * sv[xm * NCOMP + a * NCOL + k];
                        ge += php * up * eta[xp * NCOMP + a * NCOL + k] - phm * um * eta[xm * NCOMP + a * NCOL + k];
                    }
                    f[a][i] = fs;
                    g[a][i] = ge;
                }
            cplx tr[16];
            for (int n = 0; n < 16; n++) {
                cplx acc = 0;
                for (int a = 0; a < 4; a++)
                    for (int b = 0; b < 4; b++) {
                        if (G[n][a][b] == 0) continue;
                        for (int k = 0; k < NCOL; k++)
                            acc += G[n][a][b] * (conj(eta[x * NCOMP + a * NCOL + k]) * f[b][k] -
                                                 conj(g[a][k]) * sv[x * NCOMP + b * NCOL + k]);
                    }
                tr[n] = 0.25 * acc;
            }
            for (int m = 0; m < n_mom; m++) {
                double arg = twopi * ((double)mom[3 * m] * c[0] / L[0] + (double)mom[3 * m + 1] * c[1] / L[1] +
                                      (double)mom[3 * m + 2] * c[2] / L[2]);
                cplx ph = cexp(-I * arg);
                for (int n = 0; n < 16; n++) out[(((long)mu * 16 + n) * n_mom + m) * Lt + c[3]] += ph * tr[n];
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* TSM estimator (Eq. 4)                                               */
/* ------------------------------------------------------------------ */

/*
 * Eq. 4 applied to the loops of estimator est (0 standard, 1 and 2 the
 * one-end loops of orc_loops_est, 3 the one-derivative loops, whose
 * elements are [4][16][n_mom][Lt] where the others have [16][n_mom][Lt]):
 *   C = (1/N_HP) sum_{j in HP} [L(s_j^HP) - L(s_j^LP)]    (correction)
 *   B = (1/N_LP) sum_{j in LP} L(s_j^LP)                  (biased estimate)
 *   T = C + B
 * HP ids are 0..n_hp-1 and LP ids n_hp..n_hp+n_lp-1 (disjoint sets, n_lp of
 * them: the paper's count of N_HP + N_LP low-precision inversions).  The LP
 * solves of the HP set use exactly the LP solver settings.  An empty set
 * contributes zero.
 *
 * out: complex128 [3][16][n_mom][Lt] (C, B, T).
 * err (nullable): same shape; re/im hold the standard errors of the real and
 *   imaginary parts from the per-source spread (sample variance / N; a set
 *   with a single source contributes zero).  err_T^2 = err_C^2 + err_B^2.
 * per_src (nullable): complex128 [n_hp+n_lp][2][16][n_mom][Lt]: slot 0 the
 *   LP loops, slot 1 the HP loops (zero for LP ids).
 * src_stats (nullable): double [n_hp+n_lp][2][5] CG stats (slot 0 LP, 1 HP).
 * lp_eo, hp_eo: 1 solves that set with CG on the even-odd Schur complement
 *   (orc_cgnr_eo), 0 with CG on M^dag M (orc_cgnr).
 */
int orc_tsm(const int *L, int t_bc, double kappa, double mu, const double *U,
            uint64_t seed, int n_hp, int n_lp,
            double lp_tol, int lp_maxit, int lp_stop,
            double hp_tol, int hp_maxit, int hp_stop,
            int n_mom, const int *mom, int est,
            double *out_, double *err_, double *per_src_, double *src_stats,
            int lp_eo, int hp_eo)
{
    long V = volume(L);
    long n = V * NCOMP;
    int Lt = L[3];
    long nl = (est == 3 ? 64L : 16L) * n_mom * Lt;
    cplx *out = (cplx *)out_;
    cplx *err = (cplx *)err_;
    cplx *per_src = (cplx *)per_src_;
    cplx *eta = malloc(sizeof(cplx) * n), *s = malloc(sizeof(cplx) * n);
    cplx *l_lp = malloc(sizeof(cplx) * nl), *l_hp = malloc(sizeof(cplx) * nl);
    cplx *sumC = calloc(nl, sizeof(cplx)), *sumB = calloc(nl, sizeof(cplx));
    /* per-source values kept for the spread */
    cplx *dC = calloc((size_t)(n_hp > 0 ? n_hp : 1) * nl, sizeof(cplx));
    cplx *dB = calloc((size_t)(n_lp > 0 ? n_lp : 1) * nl, sizeof(cplx));
    double st[5];

    for (int j = 0; j < n_hp + n_lp; j++) {
        int is_hp = j < n_hp;
        orc_noise_z4(L, seed, (uint64_t)j, (double *)eta);
        if (lp_eo)
            orc_cgnr_eo(L, t_bc, kappa, mu, U, (double *)eta, lp_tol, lp_maxit, lp_stop, (double *)s, st);
        else
            orc_cgnr(L, t_bc, kappa, mu, U, (double *)eta, lp_tol, lp_maxit, lp_stop, (double *)s, st);
        if (src_stats) memcpy(src_stats + (j * 2 + 0) * 5, st, sizeof(st));
        memset(l_lp, 0, sizeof(cplx) * nl);
        orc_loops_est(L, t_bc, kappa, mu, U, est, (double *)eta, (double *)s, n_mom, mom, (double *)l_lp);
        memset(l_hp, 0, sizeof(cplx) * nl);
        if (is_hp) {
            if (hp_eo)
                orc_cgnr_eo(L, t_bc, kappa, mu, U, (double *)eta, hp_tol, hp_maxit, hp_stop, (double *)s, st);
            else
                orc_cgnr(L, t_bc, kappa, mu, U, (double *)eta, hp_tol, hp_maxit, hp_stop, (double *)s, st);
            if (src_stats) memcpy(src_stats + (j * 2 + 1) * 5, st, sizeof(st));
            orc_loops_est(L, t_bc, kappa, mu, U, est, (double *)eta, (double *)s, n_mom, mom, (double *)l_hp);
            for (long k = 0; k < nl; k++) {
                cplx d = l_hp[k] - l_lp[k];
                sumC[k] += d;
                dC[(long)j * nl + k] = d;
            }
        } else {
            if (src_stats) memset(src_stats + (j * 2 + 1) * 5, 0, sizeof(st));
            for (long k = 0; k < nl; k++) {
                sumB[k] += l_lp[k];
                dB[(long)(j - n_hp) * nl + k] = l_lp[k];
            }
        }
        if (per_src) {
            memcpy(per_src + ((long)j * 2 + 0) * nl, l_lp, sizeof(cplx) * nl);
            memcpy(per_src + ((long)j * 2 + 1) * nl, l_hp, sizeof(cplx) * nl);
        }
    }
    for (long k = 0; k < nl; k++) {
        cplx C = n_hp > 0 ? sumC[k] / n_hp : 0;
        cplx B = n_lp > 0 ? sumB[k] / n_lp : 0;
        out[k] = C;
        out[nl + k] = B;
        out[2 * nl + k] = C + B;
        if (err) {
            double vcr = 0, vci = 0, vbr = 0, vbi = 0;
            if (n_hp > 1) {
                for (int j = 0; j < n_hp; j++) {
                    cplx d = dC[(long)j * nl + k] - C;
                    vcr += creal(d) * creal(d);
                    vci += cimag(d) * cimag(d);
                }
                vcr /= (double)(n_hp - 1) * n_hp;
                vci /= (double)(n_hp - 1) * n_hp;
            }
            if (n_lp > 1) {
                for (int j = 0; j < n_lp; j++) {
                    cplx d = dB[(long)j * nl + k] - B;
                    vbr += creal(d) * creal(d);
                    vbi += cimag(d) * cimag(d);
                }
                vbr /= (double)(n_lp - 1) * n_lp;
                vbi /= (double)(n_lp - 1) * n_lp;
            }
            err[k] = sqrt(vcr) + I * sqrt(vci);
            err[nl + k] = sqrt(vbr) + I * sqrt(vbi);
            err[2 * nl + k] = sqrt(vcr + vbr) + I * sqrt(vci + vbi);
        }
    }
    free(eta); free(s); free(l_lp); free(l_hp); free(sumC); free(sumB); free(dC); free(dB);
    return 0;
}

/* ------------------------------------------------------------------ */
/* gauge-covariant parallel-transport network (learned preconditioner) */
/* ------------------------------------------------------------------ */

/*
 * A layer maps cin spinor fields phi_b to cout fields
 *     psi_a(x) = sum_b sum_p W[p][a][b] (T_p phi_b)(x),
 * where W[p][a][b] is a complex 4x4 matrix acting on spin (identity on
 * colour) and T_p runs over nine paths: p = 0 the identity, p = 1 + 2 mu
 * the transport from x + mu, U_mu(x) phi(x + mu), and p = 2 + 2 mu the
 * transport from x - mu, U_mu(x - mu)^dag phi(x - mu), both with the
 * time-boundary factor of the operator.  Transports commute with gauge
 * transformations, so the layer is gauge covariant; with
 * W[0] = 1 + 2i kappa mu gamma_5, W[1+2mu] = -kappa (1 - gamma_mu),
 * W[2+2mu] = -kappa (1 + gamma_mu) a single 1 -> 1 layer is exactly M.
 *
 * Weights of a layer: complex [9][cout][cin][4][4]; a net of nl layers
 * with widths w[0..nl] stores its layers back to back.  Fields: complex
 * [channel][V][4][3].  The net is linear (no bias, no activation), so its
 * adjoint is the reversed chain of adjoint layers, with T_{+mu}^dag =
 * T_{-mu}.
 */

static void transport(const int *L, int t_bc, const cplx *U, int p, const cplx *in, cplx *out)
{
    long V = volume(L);
    if (p == 0) {
        memcpy(out, in, sizeof(cplx) * V * NCOMP);
        return;
    }
    int mu = (p - 1) / 2;
    int dir = (p % 2 == 1) ? 1 : -1;
#pragma omp parallel for schedule(static) if (V >= 8192)
    for (long s = 0; s < V; s++) {
        double ph;
        long y = neighbour(L, t_bc, s, mu, dir, &ph);
        for (int a = 0; a < NSPIN; a++)
            for (int i = 0; i < NCOL; i++) {
                cplx t = 0;
                for (int k = 0; k < NCOL; k++) {
                    cplx u = dir > 0 ? U[((s * 4 + mu) * 3 + i) * 3 + k] : conj(U[((y * 4 + mu) * 3 + k) * 3 + i]);
                    t += u * in[y * NCOMP + a * NCOL + k];
                }
                out[s * NCOMP + a * NCOL + i] = ph * t;
            }
    }
}

static long layer_weights(int cin, int cout) { return 9L * cout * cin * 16; }

/* out (cout fields) = layer(in (cin fields)) */
void orc_pt_layer(const int *L, int t_bc, const double *U_, int cin, int cout, const double *W_,
                  const double *in_, double *out_)
{
    const cplx *U = (const cplx *)U_, *W = (const cplx *)W_, *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    long V = volume(L), n = V * NCOMP;
    cplx *tp = malloc(sizeof(cplx) * n);
    memset(out, 0, sizeof(cplx) * n * cout);
    for (int b = 0; b < cin; b++)
        for (int p = 0; p < 9; p++) {
            transport(L, t_bc, U, p, in + (long)b * n, tp);
            for (int a = 0; a < cout; a++) {
                const cplx *w = W + (((long)p * cout + a) * cin + b) * 16;
                cplx *o = out + (long)a * n;
                for (long s = 0; s < V; s++)
                    for (int so = 0; so < 4; so++)
                        for (int si = 0; si < 4; si++) {
                            cplx ww = w[so * 4 + si];
                            if (ww == 0) continue;
                            for (int c = 0; c < NCOL; c++) o[s * NCOMP + so * NCOL + c] += ww * tp[s * NCOMP + si * NCOL + c];
                        }
            }
        }
    free(tp);
}

/* out (cin fields) = layer^dag(in (cout fields)):
   out_b = sum_a sum_p T_p^dag (W[p][a][b]^dag in_a), T_{1+2mu}^dag = T_{2+2mu} */
void orc_pt_layer_adj(const int *L, int t_bc, const double *U_, int cin, int cout, const double *W_,
                      const double *in_, double *out_)
{
    const cplx *U = (const cplx *)U_, *W = (const cplx *)W_, *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    long V = volume(L), n = V * NCOMP;
    cplx *tmp = malloc(sizeof(cplx) * n), *tp = malloc(sizeof(cplx) * n);
    memset(out, 0, sizeof(cplx) * n * cin);
    for (int b = 0; b < cin; b++)
        for (int p = 0; p < 9; p++) {
            memset(tmp, 0, sizeof(cplx) * n);
            for (int a = 0; a < cout; a++) {
                const cplx *w = W + (((long)p * cout + a) * cin + b) * 16;
                const cplx *x = in + (long)a * n;
                for (long s = 0; s < V; s++)
                    for (int si = 0; si < 4; si++)
                        for (int so = 0; so < 4; so++) {
                            cplx ww = conj(w[so * 4 + si]);
                            if (ww == 0) continue;
                            for (int c = 0; c < NCOL; c++) tmp[s * NCOMP + si * NCOL + c] += ww * x[s * NCOMP + so * NCOL + c];
                        }
            }
            int padj = p == 0 ? 0 : (p % 2 == 1 ? p + 1 : p - 1);
            transport(L, t_bc, U, padj, tmp, tp);
            for (long k = 0; k < n; k++) out[(long)b * n + k] += tp[k];
        }
    free(tmp);
    free(tp);
}

/* y = net(x) (adjoint = 0) or net^dag(x) (adjoint = 1); widths[0..nl] */
void orc_pt_net(const int *L, int t_bc, const double *U, int nl, const int *widths, const double *W_,
                const double *x_, double *y_, int adjoint)
{
    const cplx *W = (const cplx *)W_;
    long n = volume(L) * NCOMP;
    int wmax = 0;
    for (int l = 0; l <= nl; l++) if (widths[l] > wmax) wmax = widths[l];
    cplx *a = malloc(sizeof(cplx) * n * wmax), *b = malloc(sizeof(cplx) * n * wmax);
    long off[64];
    off[0] = 0;
    for (int l = 0; l < nl; l++) off[l + 1] = off[l] + layer_weights(widths[l], widths[l + 1]);
    if (!adjoint) {
        memcpy(a, x_, sizeof(cplx) * n * widths[0]);
        for (int l = 0; l < nl; l++) {
            orc_pt_layer(L, t_bc, U, widths[l], widths[l + 1], (const double *)(W + off[l]), (double *)a, (double *)b);
            cplx *t = a; a = b; b = t;
        }
        memcpy(y_, a, sizeof(cplx) * n * widths[nl]);
    } else {
        memcpy(a, x_, sizeof(cplx) * n * widths[nl]);
        for (int l = nl - 1; l >= 0; l--) {
            orc_pt_layer_adj(L, t_bc, U, widths[l], widths[l + 1], (const double *)(W + off[l]), (double *)a,
                             (double *)b);
            cplx *t = a; a = b; b = t;
        }
        memcpy(y_, a, sizeof(cplx) * n * widths[0]);
    }
    free(a);
    free(b);
}

/*
 * Loss (1/npairs) sum_i |net(r_i) - e_i|^2 / |e_i|^2 over pairs of single
 * spinor fields (widths[0] = widths[nl] = 1), and its gradient with
 * respect to conj(W) (Wirtinger): the derivative of the loss with respect
 * to Re W is 2 Re(grad), with respect to Im W is 2 Im(grad).  Back
 * propagation through the linear layers: the upstream gradient of a layer's
 * input is the adjoint layer applied to that of its output, and
 *   dW[p][a][b][so][si] = sum_{x,c} g_a(x)_{so c} conj((T_p phi_b)(x)_{si c}).
 */
double orc_pt_loss_grad(const int *L, int t_bc, const double *U_, int nl, const int *widths, const double *W_,
                        int npairs, const double *r_, const double *e_, double *grad_)
{
    const cplx *U = (const cplx *)U_, *W = (const cplx *)W_, *r = (const cplx *)r_, *e = (const cplx *)e_;
    cplx *grad = (cplx *)grad_;
    long n = volume(L) * NCOMP, V = volume(L);
    long off[64];
    off[0] = 0;
    for (int l = 0; l < nl; l++) off[l + 1] = off[l] + layer_weights(widths[l], widths[l + 1]);
    memset(grad, 0, sizeof(cplx) * off[nl]);
    cplx **act = malloc(sizeof(cplx *) * (nl + 1));
    for (int l = 0; l <= nl; l++) act[l] = malloc(sizeof(cplx) * n * widths[l]);
    int wmax = 0;
    for (int l = 0; l <= nl; l++) if (widths[l] > wmax) wmax = widths[l];
    cplx *g = malloc(sizeof(cplx) * n * wmax), *g2 = malloc(sizeof(cplx) * n * wmax);
    cplx *tp = malloc(sizeof(cplx) * n);
    double loss = 0;
    for (int i = 0; i < npairs; i++) {
        memcpy(act[0], r + (long)i * n, sizeof(cplx) * n);
        for (int l = 0; l < nl; l++)
            orc_pt_layer(L, t_bc, U_, widths[l], widths[l + 1], (const double *)(W + off[l]), (double *)act[l],
                         (double *)act[l + 1]);
        const cplx *ei = e + (long)i * n;
        double ee = norm2(ei, n), d2 = 0;
        for (long k = 0; k < n; k++) {
            cplx d = act[nl][k] - ei[k];
            d2 += creal(d) * creal(d) + cimag(d) * cimag(d);
            g[k] = d / (ee * npairs);
        }
        loss += d2 / ee / npairs;
        for (int l = nl - 1; l >= 0; l--) {
            int cin = widths[l], cout = widths[l + 1];
            for (int b = 0; b < cin; b++)
                for (int p = 0; p < 9; p++) {
                    transport(L, t_bc, U, p, act[l] + (long)b * n, tp);
                    for (int a = 0; a < cout; a++) {
                        cplx *dw = grad + off[l] + (((long)p * cout + a) * cin + b) * 16;
                        const cplx *ga = g + (long)a * n;
                        for (long s = 0; s < V; s++)
                            for (int so = 0; so < 4; so++)
                                for (int si = 0; si < 4; si++) {
                                    cplx acc = 0;
                                    for (int c = 0; c < NCOL; c++)
                                        acc += ga[s * NCOMP + so * NCOL + c] * conj(tp[s * NCOMP + si * NCOL + c]);
                                    dw[so * 4 + si] += acc;
                                }
                    }
                }
            if (l > 0) {
                orc_pt_layer_adj(L, t_bc, U_, cin, cout, (const double *)(W + off[l]), (double *)g, (double *)g2);
                cplx *t = g; g = g2; g2 = t;
            }
        }
    }
    for (int l = 0; l <= nl; l++) free(act[l]);
    free(act);
    free(g);
    free(g2);
    free(tp);
    return loss;
}

static cplx cdot(const cplx *a, const cplx *b, long n)
{
    cplx s = 0;
    for (long i = 0; i < n; i++) s += conj(a[i]) * b[i];
    return s;
}

/*
 * Flexible CG on M^dag M (Notay 2000; Golub & Ye 1999) with the variable
 * preconditioner z = N(N^dag(r)) of the network N, Polak-Ribiere
 * direction update beta = <z_new, r_new - r> / <z, r>.  Falls back to plain
 * CG (from the current iterate, directions restarted) when Re<z, r> <= 0,
 * on a non-finite scalar, or when the residual norm has not dropped below
 * its value five iterations earlier.  stats as orc_cgnr plus stats[5] = 1
 * if the fallback happened.
 */
int orc_fcg(const int *L, int t_bc, double kappa, double mu, const double *U_, int nl, const int *widths,
            const double *W, const double *eta_, double tol, int maxit, double *x_, double *stats)
{
    const cplx *U = (const cplx *)U_, *eta = (const cplx *)eta_;
    cplx *x = (cplx *)x_;
    long n = volume(L) * NCOMP;
    cplx *b = malloc(sizeof(cplx) * n), *r = malloc(sizeof(cplx) * n), *z = malloc(sizeof(cplx) * n);
    cplx *p = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n), *q = malloc(sizeof(cplx) * n);
    cplx *rold = malloc(sizeof(cplx) * n), *tmp = malloc(sizeof(cplx) * n);
    apply_m(L, t_bc, kappa, mu, U, eta, b, 1);
    for (long i = 0; i < n; i++) { x[i] = 0; r[i] = b[i]; }
    double bb = norm2(b, n), rr = bb;
    double hist[5] = {rr, rr, rr, rr, rr};
    int it = 0, conv = 0, trunc = 0, fell = 0;
    orc_pt_net(L, t_bc, U_, nl, widths, W, (double *)r, (double *)tmp, 1);
    orc_pt_net(L, t_bc, U_, nl, widths, W, (double *)tmp, (double *)z, 0);
    cplx zr = cdot(z, r, n);
    if (!(creal(zr) > 0) || !isfinite(creal(zr)) || !isfinite(cimag(zr))) fell = 1;
    if (fell) { memcpy(z, r, sizeof(cplx) * n); zr = rr; }
    memcpy(p, z, sizeof(cplx) * n);
    for (;;) {
        if (sqrt(rr / bb) <= tol) { conv = 1; break; }
        if (maxit >= 0 && it >= maxit) { trunc = 1; break; }
        apply_m(L, t_bc, kappa, mu, U, p, t, 0);
        apply_m(L, t_bc, kappa, mu, U, t, q, 1);
        cplx pq = cdot(p, q, n);
        cplx alpha = zr / pq;
        memcpy(rold, r, sizeof(cplx) * n);
        for (long i = 0; i < n; i++) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        double rr_new = norm2(r, n);
        it++;
        cplx zr_new, beta;
        int drop_fail = it >= 5 && !(rr_new < hist[it % 5]);
        hist[it % 5] = rr_new;
        if (!fell && drop_fail) fell = 2;
        if (!fell) {
            orc_pt_net(L, t_bc, U_, nl, widths, W, (double *)r, (double *)tmp, 1);
            orc_pt_net(L, t_bc, U_, nl, widths, W, (double *)tmp, (double *)z, 0);
            zr_new = cdot(z, r, n);
            if (!(creal(zr_new) > 0) || !isfinite(creal(zr_new)) || !isfinite(cimag(zr_new))) fell = 2;
        }
        if (fell == 2) {
            /* drop the network: plain CG restarted from the current iterate */
            fell = 1;
            memcpy(z, r, sizeof(cplx) * n);
            memcpy(p, r, sizeof(cplx) * n);
            zr = rr_new;
            rr = rr_new;
            continue;
        }
        if (fell) {
            memcpy(z, r, sizeof(cplx) * n);
            zr_new = rr_new;
            beta = zr_new / zr;
        } else {
            for (long i = 0; i < n; i++) tmp[i] = r[i] - rold[i];
            beta = cdot(z, tmp, n) / zr;
        }
        for (long i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        zr = zr_new;
        rr = rr_new;
    }
    if (stats) {
        apply_m(L, t_bc, kappa, mu, U, x, t, 0);
        for (long i = 0; i < n; i++) t[i] = eta[i] - t[i];
        stats[0] = it;
        stats[1] = sqrt(rr / bb);
        stats[2] = sqrt(norm2(t, n) / norm2(eta, n));
        stats[3] = conv;
        stats[4] = trunc;
        stats[5] = fell ? 1 : 0;
    }
    free(b); free(r); free(z); free(p); free(t); free(q); free(rold); free(tmp);
    return it;
}

/* ------------------------------------------------------------------ */
/* flexible GMRES on M, right-preconditioned by the network            */
/* ------------------------------------------------------------------ */

/*
 * Restarted FGMRES(m) (Saad 1993) for M x = eta from x = 0, with the
 * network N as right preconditioner (z_j = N v_j, one forward pass per
 * iteration): Arnoldi on M z_j with modified Gram-Schmidt, the small least-
 * squares problem by Givens rotations, x += Z y at the end of each cycle.
 * Stops when the rotated residual |g_{j+1}| / |eta| (equal to
 * |eta - M x| / |eta| in exact arithmetic) is <= tol, or after maxit
 * iterations in total (maxit < 0: no cap).  A zero subdiagonal element
 * (the Krylov space holds the solution) ends the cycle with the exact
 * least-squares solution.  stats (nullable): iterations, final rotated
 * residual, FP64 true residual |eta - M x| / |eta|, converged, truncated.
 */
int orc_fgmres(const int *L, int t_bc, double kappa, double mu, const double *U_, int nl, const int *widths,
               const double *W, const double *eta_, double tol, int m, int maxit, double *x_, double *stats)
{
    const cplx *U = (const cplx *)U_, *eta = (const cplx *)eta_;
    cplx *x = (cplx *)x_;
    long n = volume(L) * NCOMP;
    cplx *V = malloc(sizeof(cplx) * n * (m + 1)), *Z = malloc(sizeof(cplx) * n * m);
    cplx *w = malloc(sizeof(cplx) * n);
    cplx *H = calloc((size_t)(m + 1) * m, sizeof(cplx));   /* H[i*m + j] */
    cplx *g = malloc(sizeof(cplx) * (m + 1)), *y = malloc(sizeof(cplx) * m);
    double *cs = malloc(sizeof(double) * m);
    cplx *sn = malloc(sizeof(cplx) * m);
    double eta_norm = sqrt(norm2(eta, n));
    int it = 0, conv = 0, trunc = 0;
    double res = 1.0;
    for (long i = 0; i < n; i++) x[i] = 0;
    if (eta_norm == 0) conv = 1;
    while (!conv && !trunc) {
        /* r = eta - M x, v_0 = r / |r| */
        apply_m(L, t_bc, kappa, mu, U, x, w, 0);
        for (long i = 0; i < n; i++) w[i] = eta[i] - w[i];
        double beta = sqrt(norm2(w, n));
        res = beta / eta_norm;
        if (res <= tol) { conv = 1; break; }
        if (maxit >= 0 && it >= maxit) { trunc = 1; break; }
        for (long i = 0; i < n; i++) V[i] = w[i] / beta;
        for (int i = 0; i <= m; i++) g[i] = 0;
        g[0] = beta;
        int k = 0;  /* columns of this cycle */
        for (int j = 0; j < m; j++) {
            cplx *vj = V + (long)j * n, *zj = Z + (long)j * n;
            orc_pt_net(L, t_bc, U_, nl, widths, W, (const double *)vj, (double *)zj, 0);
            apply_m(L, t_bc, kappa, mu, U, zj, w, 0);
            for (int i = 0; i <= j; i++) {
                cplx *vi = V + (long)i * n;
                cplx h = cdot(vi, w, n);
                H[i * m + j] = h;
                for (long q = 0; q < n; q++) w[q] -= h * vi[q];
            }
            double hn = sqrt(norm2(w, n));
            H[(j + 1) * m + j] = hn;
            if (hn > 0)
                for (long q = 0; q < n; q++) V[(long)(j + 1) * n + q] = w[q] / hn;
            /* previous rotations, then the one that zeroes H[j+1][j] */
            for (int i = 0; i < j; i++) {
                cplx a = H[i * m + j], b = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * b;
                H[(i + 1) * m + j] = -conj(sn[i]) * a + cs[i] * b;
            }
            cplx a = H[j * m + j];
            double bb = hn, den = sqrt(creal(a) * creal(a) + cimag(a) * cimag(a) + bb * bb);
            if (cabs(a) == 0) { cs[j] = 0; sn[j] = 1; }
            else { cs[j] = cabs(a) / den; sn[j] = (a / cabs(a)) * bb / den; }
            H[j * m + j] = cs[j] * a + sn[j] * bb;
            H[(j + 1) * m + j] = 0;
            g[j + 1] = -conj(sn[j]) * g[j];
            g[j] = cs[j] * g[j];
            it++;
            k = j + 1;
            res = cabs(g[j + 1]) / eta_norm;
            if (res <= tol) { conv = 1; break; }
            if (maxit >= 0 && it >= maxit) { trunc = 1; break; }
            if (hn == 0) break;
        }
        /* y = R^{-1} g (back substitution), x += Z y */
        for (int i = k - 1; i >= 0; i--) {
            cplx acc = g[i];
            for (int q = i + 1; q < k; q++) acc -= H[i * m + q] * y[q];
            y[i] = acc / H[i * m + i];
        }
        for (int j = 0; j < k; j++)
            for (long q = 0; q < n; q++) x[q] += y[j] * Z[(long)j * n + q];
    }
    if (stats) {
        apply_m(L, t_bc, kappa, mu, U, x, w, 0);
        for (long i = 0; i < n; i++) w[i] = eta[i] - w[i];
        stats[0] = it;
        stats[1] = res;
        stats[2] = eta_norm > 0 ? sqrt(norm2(w, n)) / eta_norm : 0.0;
        stats[3] = conv;
        stats[4] = trunc;
    }
    free(V); free(Z); free(w); free(H); free(g); free(y); free(cs); free(sn);
    return it;
}
