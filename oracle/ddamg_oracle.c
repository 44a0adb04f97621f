/*
 * ddamg_oracle.c -- plain, slow, FP64 CPU reference of DD-alpha-AMG
 * (Frommer, Kahl, Krieg, Leder, Rottmann, arXiv:1303.1377).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is used by tests/, by the smoke check
 * and by the CPU-baseline leg of bench.py.  The HIP product path never links
 * or calls it, and it shares no code, header or table with that path.
 *
 * Every routine follows a definition of the paper directly, in double
 * precision complex arithmetic, with plain loops (OpenMP only over sites,
 * blocks or aggregates whose updates are independent by construction):
 *
 *   geometry ............ Sec. 2.2/2.3  periodic 4D lattice, block decomposition
 *   gamma matrices ...... Sec. 2.2      chiral representation, gamma5 = diag(1,1,-1,-1)
 *   clover term ......... Sec. 2.2      eq. (lattice_WD) with the four-leaf Q_{mu nu}
 *   Dirac operator ...... Sec. 2.2      explicit site form of D (after the gamma matrices)
 *   SAP ................. Sec. 2.3      red-black multiplicative Schwarz, eq. (SAP_1step)
 *   block solver ........ Sec. 5        odd-even preconditioned MR (GMRES(1)), fixed steps
 *   interpolation ....... Sec. 3.1/3.2  eq. (aggInterpolation), standard aggregation,
 *                                       local orthonormalisation (Gram-Schmidt)
 *   coarse operator ..... Sec. 3.2      D_c = P^H D P (Lemma cgprops)
 *   coarse solver ....... Sec. 5        odd-even preconditioned restarted GMRES
 *   V-cycle ............. Sec. 4.2      C^(nu), eq. (iterationmatrix)
 *   outer solver ........ Sec. 4.2/5    FGMRES right-preconditioned by one V-cycle
 *   setup ............... Alg. 2        DD-alpha-AMG-setup(n_inv, nu) built on Alg. 1
 *   multilevel .......... Sec. 3, 5     recursive application on D_c
 *   comparison solvers .. Sec. 6        FGMRES preconditioned by odd-even BiCGStab;
 *                        Sec. 4.1      inexact deflation (FGMRES on D pi_R with SAP)
 *
 * Readings of points the paper leaves open are listed in the design notes of
 * the repository and repeated at the routine that takes them.
 */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define OR_MAXLEV 4

/* ------------------------------------------------------------------------ */
/* public parameter / statistics records (mirrored field-by-field in Python) */
/* ------------------------------------------------------------------------ */
typedef struct {
    int levels;               /* number of levels (2 or 3)                         */
    int n_tv[OR_MAXLEV];      /* test vectors N for the transfer level l -> l+1    */
    int agg[OR_MAXLEV][4];    /* aggregate lattice-block dims at level l           */
    int sap[OR_MAXLEV][4];    /* SAP lattice-block dims at level l                 */
    int mr_steps[OR_MAXLEV];  /* MR steps of the SAP block solver at level l       */
    int nu;                   /* post-smoothing SAP iterations                      */
    int n_inv;                /* setup iterations                                   */
    double coarse_tol;        /* coarsest GMRES relative tolerance (5e-2)          */
    int coarse_restart;       /* 30                                                 */
    int coarse_maxit;         /* iteration cap (not in the paper)                  */
    int coarse_fixed;         /* >0: exactly this many coarsest iterations         */
    double mid_tol;           /* intermediate-level FGMRES tolerance               */
    int mid_restart;
    int mid_maxit;
    int mid_fixed;            /* >0: exactly this many intermediate iterations     */
    int outer_restart;
    int outer_maxit;
    int id_setup;             /* 1: the setup is IDsetup (Sec. 4.3), not Alg. 2    */
} or_params;

typedef struct {
    int outer_iters;
    int restarts;
    long coarse_iters[OR_MAXLEV];
    double true_relres;
    int converged;
} or_stats;

/* ------------------------------------------------------------------------ */
/* geometry                                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    int d[4];
    long vol;
    long *nb;    /* [vol][8]: k<4 -> x+k, k>=4 -> x-(k-4)  (periodic) */
    int *par;    /* [vol]: (x0+x1+x2+x3) mod 2                          */
} geom;

static void coords_of(const int d[4], long i, int x[4]) {
    x[3] = (int)(i % d[3]); i /= d[3];
    x[2] = (int)(i % d[2]); i /= d[2];
    x[1] = (int)(i % d[1]); i /= d[1];
    x[0] = (int)i;
}

static long index_of(const int d[4], const int x[4]) {
    return (((long)x[0] * d[1] + x[1]) * d[2] + x[2]) * d[3] + x[3];
}

static void geom_init(geom *g, const int d[4]) {
    memcpy(g->d, d, sizeof(int) * 4);
    g->vol = (long)d[0] * d[1] * d[2] * d[3];
    g->nb = (long *)malloc(sizeof(long) * 8 * g->vol);
    g->par = (int *)malloc(sizeof(int) * g->vol);
    for (long i = 0; i < g->vol; i++) {
        int x[4], y[4];
        coords_of(d, i, x);
        g->par[i] = (x[0] + x[1] + x[2] + x[3]) & 1;
        for (int mu = 0; mu < 4; mu++) {
            memcpy(y, x, sizeof y);
            y[mu] = (x[mu] + 1) % d[mu];
            g->nb[i * 8 + mu] = index_of(d, y);
            y[mu] = (x[mu] - 1 + d[mu]) % d[mu];
            g->nb[i * 8 + 4 + mu] = index_of(d, y);
        }
    }
}

static void geom_free(geom *g) {
    free(g->nb);
    free(g->par);
    g->nb = NULL;
    g->par = NULL;
}

/* block index (lexicographic in block coordinates) and block coordinates */
static long block_of(const int d[4], const int b[4], long i, int bc[4]) {
    int x[4], nbk[4];
    coords_of(d, i, x);
    for (int mu = 0; mu < 4; mu++) {
        bc[mu] = x[mu] / b[mu];
        nbk[mu] = d[mu] / b[mu];
    }
    return index_of(nbk, bc);
}

/* ------------------------------------------------------------------------ */
/* gamma matrices, chiral representation (Sec. 2.2)                          */
/* ------------------------------------------------------------------------ */
static cplx GAMMA[4][4][4];

static void gamma_init(void) {
    memset(GAMMA, 0, sizeof GAMMA);
    /* gamma_0 */
    GAMMA[0][0][3] = I;  GAMMA[0][1][2] = I;  GAMMA[0][2][1] = -I; GAMMA[0][3][0] = -I;
    /* gamma_1 */
    GAMMA[1][0][3] = -1; GAMMA[1][1][2] = 1;  GAMMA[1][2][1] = 1;  GAMMA[1][3][0] = -1;
    /* gamma_2 */
    GAMMA[2][0][2] = I;  GAMMA[2][1][3] = -I; GAMMA[2][2][0] = -I; GAMMA[2][3][1] = I;
    /* gamma_3 */
    GAMMA[3][0][2] = 1;  GAMMA[3][1][3] = 1;  GAMMA[3][2][0] = 1;  GAMMA[3][3][1] = 1;
}

void or_gamma(cplx *out /* [4][4][4] */) {
    gamma_init();
    memcpy(out, GAMMA, sizeof GAMMA);
}

/* ------------------------------------------------------------------------ */
/* small dense helpers                                                       */
/* ------------------------------------------------------------------------ */
static void su3_mul(const cplx *a, const cplx *b, cplx *c) { /* c = a b */
    cplx t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx s = 0;
            for (int k = 0; k < 3; k++) s += a[i * 3 + k] * b[k * 3 + j];
            t[i * 3 + j] = s;
        }
    memcpy(c, t, sizeof t);
}

static void su3_dag(const cplx *a, cplx *c) {
    cplx t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) t[i * 3 + j] = conj(a[j * 3 + i]);
    memcpy(c, t, sizeof t);
}

/* Gauss-Jordan inversion with partial pivoting of an n x n complex matrix.
 * Returns 0 on success, -1 if a pivot vanishes. */
static int dense_inverse(int n, const cplx *a, cplx *inv) {
    cplx *m = (cplx *)malloc(sizeof(cplx) * n * n);
    memcpy(m, a, sizeof(cplx) * n * n);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) inv[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int c = 0; c < n; c++) {
        int p = c;
        double best = cabs(m[c * n + c]);
        for (int r = c + 1; r < n; r++)
            if (cabs(m[r * n + c]) > best) { best = cabs(m[r * n + c]); p = r; }
        if (best == 0.0) { free(m); return -1; }
        if (p != c)
            for (int j = 0; j < n; j++) {
                cplx t = m[c * n + j]; m[c * n + j] = m[p * n + j]; m[p * n + j] = t;
                t = inv[c * n + j]; inv[c * n + j] = inv[p * n + j]; inv[p * n + j] = t;
            }
        cplx piv = 1.0 / m[c * n + c];
        for (int j = 0; j < n; j++) { m[c * n + j] *= piv; inv[c * n + j] *= piv; }
        for (int r = 0; r < n; r++) {
            if (r == c) continue;
            cplx f = m[r * n + c];
            if (f == 0) continue;
            for (int j = 0; j < n; j++) {
                m[r * n + j] -= f * m[c * n + j];
                inv[r * n + j] -= f * inv[c * n + j];
            }
        }
    }
    free(m);
    return 0;
}

static void matvec(int n, const cplx *a, const cplx *x, cplx *y) { /* y = a x */
    for (int i = 0; i < n; i++) {
        cplx s = 0;
        for (int j = 0; j < n; j++) s += a[i * n + j] * x[j];
        y[i] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* vector helpers (length n complex), OpenMP over entries                    */
/* ------------------------------------------------------------------------ */
static cplx vdot(long n, const cplx *a, const cplx *b) { /* a^H b */
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (long i = 0; i < n; i++) {
        cplx t = conj(a[i]) * b[i];
        re += creal(t);
        im += cimag(t);
    }
    return re + I * im;
}

static double vnorm(long n, const cplx *a) { return sqrt(creal(vdot(n, a, a))); }

static void vaxpy(long n, cplx alpha, const cplx *x, cplx *y) {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; i++) y[i] += alpha * x[i];
}

static void vscale(long n, cplx alpha, cplx *x) {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; i++) x[i] *= alpha;
}

static void vcopy(long n, const cplx *x, cplx *y) { memcpy(y, x, sizeof(cplx) * n); }
static void vzero(long n, cplx *x) { memset(x, 0, sizeof(cplx) * n); }

static cplx *cvalloc(long n) {
    cplx *p = (cplx *)calloc((size_t)n, sizeof(cplx));
    if (!p) { fprintf(stderr, "oracle: out of memory (%ld complex)\n", n); abort(); }
    return p;
}

/* ------------------------------------------------------------------------ */
/* levels                                                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    geom g;
    int nd;          /* unknowns per site: 12 on the fine lattice, 2N on a coarse one */
    int fine;        /* 1: clover-Wilson operator applied from the links              */
    /* fine operator */
    cplx *U;         /* [vol][4][3][3]                                               */
    cplx *A;         /* [vol][2][6][6]  (m0+4) I + T(x), the two chiral blocks        */
    cplx *Ainv;      /* [vol][2][6][6]                                                */
    /* coarse operator: slot 0 self, 1+mu couples x+mu, 5+mu couples x-mu           */
    cplx *M;         /* [vol][9][nd][nd]                                              */
    cplx *Minv;      /* [vol][nd][nd]                                                 */
    int oe_ok;       /* site parity is a 2-colouring of the couplings                 */
    /* SAP block decomposition */
    int sap[4];
    int mr_steps;
    long nblk;
    long *blk_of;    /* [vol]                                                          */
    int *blk_col;    /* [nblk]: 0 red (even sum of block coordinates), 1 black        */
    long *blk_start; /* [nblk+1] into blk_sites                                       */
    long *blk_nev;   /* [nblk] number of even sites of the block                      */
    long *blk_sites; /* sites of each block: even ones first, then odd ones           */
    /* transfer to level l+1 */
    int nv;          /* number of test vectors N                                      */
    int agg[4];
    long *agg_of;    /* [vol] coarse site of each site                                */
    cplx *tv;        /* [nv][vol][nd]  test vectors                                   */
    cplx *P;         /* [nv][vol][nd]  locally orthonormalised columns                */
} level;

typedef struct {
    int nlev;
    level L[OR_MAXLEV];
    or_params p;
    int have_params;
    int have_setup;
    long coarse_count[OR_MAXLEV];
    int pre_bicg;    /* > 0: the outer FGMRES is preconditioned by this many
                        odd-even BiCGStab steps instead of the V-cycle       */
    int pre_sap;     /* > 0: ... by this many SAP iterations (M_SAP^(nu))    */
    int deflated;    /* 1: the outer FGMRES runs on D pi_R (inexact deflation) */
    char err[256];
} octx;

/* unknowns per site split into two halves: spins {0,1} / {2,3} on the fine
 * level (index sigma*3 + colour), Gamma5^c blocks on coarse levels. */
static inline int half_of(const level *L, int d) { return d >= L->nd / 2; }

/* ---- site operations -------------------------------------------------- */

/* out = A(x) in  (self coupling) */
static void site_self(const level *L, long x, const cplx *in, cplx *out) {
    if (L->fine) {
        const cplx *a = L->A + x * 72;
        matvec(6, a, in, out);
        matvec(6, a + 36, in + 6, out + 6);
    } else {
        matvec(L->nd, L->M + (x * 9) * L->nd * L->nd, in, out);
    }
}

static void site_self_inv(const level *L, long x, const cplx *in, cplx *out) {
    if (L->fine) {
        const cplx *a = L->Ainv + x * 72;
        matvec(6, a, in, out);
        matvec(6, a + 36, in + 6, out + 6);
    } else {
        matvec(L->nd, L->Minv + x * L->nd * L->nd, in, out);
    }
}

/* acc += H_k(x) in_y, where y = nb[x][k].  On the fine lattice
 *   k = mu     : H = -1/2 (I - gamma_mu) (x) U_mu(x)
 *   k = 4 + mu : H = -1/2 (I + gamma_mu) (x) U_mu(x - mu)^H
 * which are the two hopping sums of the explicit form of D. */
static void site_hop_acc(const level *L, long x, int k, const cplx *in_y, cplx *acc) {
    if (L->fine) {
        int mu = k & 3;
        cplx u[9];
        if (k < 4) {
            memcpy(u, L->U + (x * 4 + mu) * 9, sizeof u);
        } else {
            long y = L->g.nb[x * 8 + k];
            su3_dag(L->U + (y * 4 + mu) * 9, u);
        }
        double sgn = (k < 4) ? -1.0 : 1.0; /* I - gamma (forward), I + gamma (backward) */
        cplx t[4][3];
        for (int s = 0; s < 4; s++)
            for (int a = 0; a < 3; a++) {
                cplx v = 0;
                for (int b = 0; b < 3; b++) v += u[a * 3 + b] * in_y[s * 3 + b];
                t[s][a] = v;
            }
        for (int s = 0; s < 4; s++)
            for (int a = 0; a < 3; a++) {
                cplx v = 0;
                for (int r = 0; r < 4; r++) {
                    cplx proj = ((s == r) ? 1.0 : 0.0) + sgn * GAMMA[mu][s][r];
                    v += proj * t[r][a];
                }
                acc[s * 3 + a] += -0.5 * v;
            }
    } else {
        int n = L->nd;
        const cplx *m = L->M + (x * 9 + 1 + k) * n * n;
        for (int i = 0; i < n; i++) {
            cplx s = 0;
            for (int j = 0; j < n; j++) s += m[i * n + j] * in_y[j];
            acc[i] += s;
        }
    }
}

/* out = D in  on the whole lattice */
static void apply_full(const level *L, const cplx *in, cplx *out) {
    int nd = L->nd;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < L->g.vol; x++) {
        cplx acc[128];
        site_self(L, x, in + x * nd, acc);
        for (int k = 0; k < 8; k++) site_hop_acc(L, x, k, in + L->g.nb[x * 8 + k] * nd, acc);
        memcpy(out + x * nd, acc, sizeof(cplx) * nd);
    }
}

/* ------------------------------------------------------------------------ */
/* clover term (Sec. 2.2, eq. lattice_WD and the four leaves Q_{mu nu})     */
/* ------------------------------------------------------------------------ */
static const cplx *link(const level *L, long x, int mu) { return L->U + (x * 4 + mu) * 9; }

/* Q_{mu nu}(x): sum of the four plaquette leaves, transcribed term by term. */
static void clover_leaves(const level *L, long x, int mu, int nu, cplx *q) {
    const long *nb = L->g.nb;
    long xpm = nb[x * 8 + mu], xpn = nb[x * 8 + nu];
    long xmm = nb[x * 8 + 4 + mu], xmn = nb[x * 8 + 4 + nu];
    long xmm_pn = nb[xmm * 8 + nu];       /* x - mu + nu */
    long xmm_mn = nb[xmm * 8 + 4 + nu];   /* x - mu - nu */
    long xmn_pm = nb[xmn * 8 + mu];       /* x - nu + mu */
    cplx t[9], h[9];
    memset(q, 0, sizeof(cplx) * 9);
    /* U_mu(x) U_nu(x+mu) U_mu(x+nu)^H U_nu(x)^H */
    su3_mul(link(L, x, mu), link(L, xpm, nu), t);
    su3_dag(link(L, xpn, mu), h); su3_mul(t, h, t);
    su3_dag(link(L, x, nu), h);   su3_mul(t, h, t);
    for (int i = 0; i < 9; i++) q[i] += t[i];
    /* U_nu(x) U_mu(x-mu+nu)^H U_nu(x-mu)^H U_mu(x-mu) */
    su3_dag(link(L, xmm_pn, mu), h); su3_mul(link(L, x, nu), h, t);
    su3_dag(link(L, xmm, nu), h);    su3_mul(t, h, t);
    su3_mul(t, link(L, xmm, mu), t);
    for (int i = 0; i < 9; i++) q[i] += t[i];
    /* U_mu(x-mu)^H U_nu(x-mu-nu)^H U_mu(x-mu-nu) U_nu(x-nu) */
    su3_dag(link(L, xmm, mu), t);
    su3_dag(link(L, xmm_mn, nu), h); su3_mul(t, h, t);
    su3_mul(t, link(L, xmm_mn, mu), t);
    su3_mul(t, link(L, xmn, nu), t);
    for (int i = 0; i < 9; i++) q[i] += t[i];
    /* U_nu(x-nu)^H U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^H */
    su3_dag(link(L, xmn, nu), t);
    su3_mul(t, link(L, xmn, mu), t);
    su3_mul(t, link(L, xmn_pm, nu), t);
    su3_dag(link(L, x, mu), h); su3_mul(t, h, t);
    for (int i = 0; i < 9; i++) q[i] += t[i];
}

/* T(x) = -(csw/32) sum_{mu,nu} (gamma_mu gamma_nu) (x) (Q_{mu nu} - Q_{nu mu}) as a
 * full 12 x 12 matrix in the (spin, colour) index sigma*3 + c. */
static void clover_T(const level *L, long x, double csw, cplx *T /* [12][12] */) {
    memset(T, 0, sizeof(cplx) * 144);
    for (int mu = 0; mu < 4; mu++)
        for (int nu = 0; nu < 4; nu++) {
            if (mu == nu) continue; /* Q_{mu mu} - Q_{mu mu} = 0 */
            cplx qmn[9], qnm[9], gg[16];
            clover_leaves(L, x, mu, nu, qmn);
            clover_leaves(L, x, nu, mu, qnm);
            for (int s = 0; s < 4; s++)
                for (int r = 0; r < 4; r++) {
                    cplx v = 0;
                    for (int k = 0; k < 4; k++) v += GAMMA[mu][s][k] * GAMMA[nu][k][r];
                    gg[s * 4 + r] = v;
                }
            for (int s = 0; s < 4; s++)
                for (int r = 0; r < 4; r++)
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++)
                            T[(s * 3 + a) * 12 + r * 3 + b] +=
                                -(csw / 32.0) * gg[s * 4 + r] * (qmn[a * 3 + b] - qnm[a * 3 + b]);
        }
}

/* Fill A = (m0+4) I + T and its inverse.  T either computed from the links or
 * supplied as packed blocks [vol][2][6][6].  Returns the largest magnitude of an
 * entry of T outside the two chiral 6x6 blocks (must be 0). */
static double build_clover(level *L, double m0, double csw, const cplx *Tgiven, int *fail) {
    double offmax = 0;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(max : offmax) reduction(| : bad)
    for (long x = 0; x < L->g.vol; x++) {
        cplx T[144];
        cplx *a = L->A + x * 72;
        if (Tgiven) {
            memcpy(a, Tgiven + x * 72, sizeof(cplx) * 72);
        } else {
            clover_T(L, x, csw, T);
            for (int i = 0; i < 12; i++)
                for (int j = 0; j < 12; j++) {
                    int bi = i / 6, bj = j / 6;
                    if (bi == bj) a[bi * 36 + (i % 6) * 6 + (j % 6)] = T[i * 12 + j];
                    else if (cabs(T[i * 12 + j]) > offmax) offmax = cabs(T[i * 12 + j]);
                }
        }
        for (int h = 0; h < 2; h++)
            for (int i = 0; i < 6; i++) a[h * 36 + i * 6 + i] += m0 + 4.0;
        if (dense_inverse(6, a, L->Ainv + x * 72)) bad |= 1;
        if (dense_inverse(6, a + 36, L->Ainv + x * 72 + 36)) bad |= 1;
    }
    *fail = bad;
    return offmax;
}

/* ------------------------------------------------------------------------ */
/* SAP block decomposition and red-black multiplicative Schwarz (Sec. 2.3)  */
/* ------------------------------------------------------------------------ */
static int valid_blocks(const int d[4], const int b[4]) {
    for (int mu = 0; mu < 4; mu++) {
        if (b[mu] <= 0 || d[mu] % b[mu]) return 0;
        int n = d[mu] / b[mu];
        if (n != 1 && (n & 1)) return 0; /* two colours need an even block count (or 1) */
    }
    return 1;
}

static void sap_free(level *L) {
    free(L->blk_of); free(L->blk_col); free(L->blk_start); free(L->blk_nev); free(L->blk_sites);
    L->blk_of = NULL; L->blk_col = NULL; L->blk_start = NULL; L->blk_nev = NULL; L->blk_sites = NULL;
    L->nblk = 0;
}

static void sap_init(level *L, const int b[4], int mr_steps) {
    sap_free(L);
    memcpy(L->sap, b, sizeof(int) * 4);
    L->mr_steps = mr_steps;
    const int *d = L->g.d;
    L->nblk = (long)(d[0] / b[0]) * (d[1] / b[1]) * (d[2] / b[2]) * (d[3] / b[3]);
    L->blk_of = (long *)malloc(sizeof(long) * L->g.vol);
    L->blk_col = (int *)malloc(sizeof(int) * L->nblk);
    L->blk_start = (long *)calloc(L->nblk + 1, sizeof(long));
    L->blk_nev = (long *)calloc(L->nblk, sizeof(long));
    L->blk_sites = (long *)malloc(sizeof(long) * L->g.vol);
    long *cnt = (long *)calloc(L->nblk, sizeof(long));
    for (long x = 0; x < L->g.vol; x++) {
        int bc[4];
        long bi = block_of(d, b, x, bc);
        L->blk_of[x] = bi;
        L->blk_col[bi] = (bc[0] + bc[1] + bc[2] + bc[3]) & 1;
        cnt[bi]++;
        if (L->g.par[x] == 0) L->blk_nev[bi]++;
    }
    for (long i = 0; i < L->nblk; i++) L->blk_start[i + 1] = L->blk_start[i] + cnt[i];
    long *fill_e = (long *)calloc(L->nblk, sizeof(long));
    long *fill_o = (long *)calloc(L->nblk, sizeof(long));
    for (long x = 0; x < L->g.vol; x++) {
        long bi = L->blk_of[x];
        if (L->g.par[x] == 0) L->blk_sites[L->blk_start[bi] + fill_e[bi]++] = x;
        else L->blk_sites[L->blk_start[bi] + L->blk_nev[bi] + fill_o[bi]++] = x;
    }
    free(cnt); free(fill_e); free(fill_o);
}

/* Approximate block solve e = B_i r on block `bi` (eq. localsystem): odd-even
 * preconditioned minimal residual with a fixed number of steps (Sec. 5).
 * Schur complement on the block's odd sites S = A_oo - D_oe A_ee^{-1} D_eo,
 * block-internal couplings only; back-substitution on the even sites.
 * Adds e to z on the block.  t, rho, s, e are lattice-size scratch arrays of
 * which only this block's sites are touched. */
static void block_solve(const level *L, long bi, const cplx *r, cplx *z,
                        cplx *t, cplx *rho, cplx *s, cplx *e) {
    const int nd = L->nd;
    const long *sites = L->blk_sites + L->blk_start[bi];
    const long ne = L->blk_nev[bi];
    const long nt = L->blk_start[bi + 1] - L->blk_start[bi];
    const long *nb = L->g.nb;
    cplx u[128];

    /* t_e = A_ee^{-1} r_e */
    for (long i = 0; i < ne; i++) site_self_inv(L, sites[i], r + sites[i] * nd, t + sites[i] * nd);
    /* f_o = r_o - D_oe t_e ;  rho = f_o ; e_o = 0 */
    for (long i = ne; i < nt; i++) {
        long x = sites[i];
        for (int c = 0; c < nd; c++) u[c] = 0;
        for (int k = 0; k < 8; k++) {
            long y = nb[x * 8 + k];
            if (L->blk_of[y] == bi) site_hop_acc(L, x, k, t + y * nd, u);
        }
        for (int c = 0; c < nd; c++) {
            rho[x * nd + c] = r[x * nd + c] - u[c];
            e[x * nd + c] = 0;
        }
    }
    for (int it = 0; it < L->mr_steps; it++) {
        /* s = S rho */
        for (long i = 0; i < ne; i++) {
            long y = sites[i];
            for (int c = 0; c < nd; c++) u[c] = 0;
            for (int k = 0; k < 8; k++) {
                long w = nb[y * 8 + k];
                if (L->blk_of[w] == bi) site_hop_acc(L, y, k, rho + w * nd, u);
            }
            site_self_inv(L, y, u, t + y * nd);
        }
        double num_re = 0, num_im = 0, den = 0;
        for (long i = ne; i < nt; i++) {
            long x = sites[i];
            cplx v[128];
            for (int c = 0; c < nd; c++) u[c] = 0;
            for (int k = 0; k < 8; k++) {
                long y = nb[x * 8 + k];
                if (L->blk_of[y] == bi) site_hop_acc(L, x, k, t + y * nd, u);
            }
            site_self(L, x, rho + x * nd, v);
            for (int c = 0; c < nd; c++) {
                cplx sv = v[c] - u[c];
                s[x * nd + c] = sv;
                cplx pr = conj(sv) * rho[x * nd + c];
                num_re += creal(pr);
                num_im += cimag(pr);
                den += creal(conj(sv) * sv);
            }
        }
        if (den == 0.0) break;
        cplx alpha = (num_re + I * num_im) / den; /* alpha = s^H rho / s^H s */
        for (long i = ne; i < nt; i++) {
            long x = sites[i];
            for (int c = 0; c < nd; c++) {
                e[x * nd + c] += alpha * rho[x * nd + c];
                rho[x * nd + c] -= alpha * s[x * nd + c];
            }
        }
    }
    /* e_e = A_ee^{-1} (r_e - D_eo e_o) */
    for (long i = 0; i < ne; i++) {
        long y = sites[i];
        cplx v[128];
        for (int c = 0; c < nd; c++) u[c] = 0;
        for (int k = 0; k < 8; k++) {
            long w = nb[y * 8 + k];
            if (L->blk_of[w] == bi) site_hop_acc(L, y, k, e + w * nd, u);
        }
        for (int c = 0; c < nd; c++) v[c] = r[y * nd + c] - u[c];
        site_self_inv(L, y, v, e + y * nd);
    }
    for (long i = 0; i < nt; i++) {
        long x = sites[i];
        for (int c = 0; c < nd; c++) z[x * nd + c] += e[x * nd + c];
    }
}

/* nsweeps iterations of red-black SAP (eq. SAP_1step) on D z = rhs, z in/out.
 * One iteration: r = rhs - D z, red blocks z += B_i r; r = rhs - D z, black
 * blocks z += B_i r.  Red = even sum of block coordinates (reading: the paper
 * does not say which colour is first). */
static void sap_sweeps(const level *L, const cplx *rhs, cplx *z, int nsweeps) {
    long n = L->g.vol * L->nd;
    cplx *r = cvalloc(n), *t = cvalloc(n), *rho = cvalloc(n), *s = cvalloc(n), *e = cvalloc(n);
    for (int sw = 0; sw < nsweeps; sw++) {
        for (int col = 0; col < 2; col++) {
            apply_full(L, z, r);
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; i++) r[i] = rhs[i] - r[i];
#pragma omp parallel for schedule(dynamic)
            for (long bi = 0; bi < L->nblk; bi++)
                if (L->blk_col[bi] == col) block_solve(L, bi, r, z, t, rho, s, e);
        }
    }
    free(r); free(t); free(rho); free(s); free(e);
}

/* ------------------------------------------------------------------------ */
/* aggregation, interpolation P, restriction P^H, D_c = P^H D P (Sec. 3)    */
/* ------------------------------------------------------------------------ */

/* Standard aggregation: lattice block j gives two aggregates, one per half of
 * the site unknowns.  For each aggregate the restrictions of v_1..v_N are
 * orthonormalised by Gram-Schmidt in the order 1..N (modified form), which
 * gives P^H P = I and leaves range(P) unchanged (Sec. 3.1). */
static int build_P(level *F, long nagg) {
    const int nd = F->nd, nv = F->nv;
    const long vol = F->g.vol;
    int bad = 0;
    /* sites of each aggregate */
    long *start = (long *)calloc(nagg + 1, sizeof(long));
    long *list = (long *)malloc(sizeof(long) * vol);
    long *fill = (long *)calloc(nagg, sizeof(long));
    for (long x = 0; x < vol; x++) start[F->agg_of[x] + 1]++;
    for (long a = 0; a < nagg; a++) start[a + 1] += start[a];
    for (long x = 0; x < vol; x++) list[start[F->agg_of[x]] + fill[F->agg_of[x]]++] = x;
    int h0 = nd / 2;
#pragma omp parallel for schedule(dynamic) reduction(| : bad)
    for (long a = 0; a < nagg; a++) {
        for (int h = 0; h < 2; h++) {
            for (int k = 0; k < nv; k++) {
                cplx *qk = F->P + (long)k * vol * nd;
                const cplx *vk = F->tv + (long)k * vol * nd;
                for (long i = start[a]; i < start[a + 1]; i++) {
                    long x = list[i];
                    for (int d = h * h0; d < (h + 1) * h0; d++) qk[x * nd + d] = vk[x * nd + d];
                }
                for (int j = 0; j < k; j++) {
                    const cplx *qj = F->P + (long)j * vol * nd;
                    cplx hh = 0;
                    for (long i = start[a]; i < start[a + 1]; i++) {
                        long x = list[i];
                        for (int d = h * h0; d < (h + 1) * h0; d++) hh += conj(qj[x * nd + d]) * qk[x * nd + d];
                    }
                    for (long i = start[a]; i < start[a + 1]; i++) {
                        long x = list[i];
                        for (int d = h * h0; d < (h + 1) * h0; d++) qk[x * nd + d] -= hh * qj[x * nd + d];
                    }
                }
                double nrm = 0;
                for (long i = start[a]; i < start[a + 1]; i++) {
                    long x = list[i];
                    for (int d = h * h0; d < (h + 1) * h0; d++) nrm += creal(conj(qk[x * nd + d]) * qk[x * nd + d]);
                }
                nrm = sqrt(nrm);
                if (nrm == 0.0) { bad |= 1; nrm = 1.0; }
                for (long i = start[a]; i < start[a + 1]; i++) {
                    long x = list[i];
                    for (int d = h * h0; d < (h + 1) * h0; d++) qk[x * nd + d] /= nrm;
                }
            }
        }
    }
    free(start); free(list); free(fill);
    return bad ? -1 : 0;
}

/* coarse index of (half h, vector k) is h*N + k */
static void restrict_to(const level *F, const level *C, const cplx *in, cplx *out) {
    const int nd = F->nd, nv = F->nv, ndc = C->nd, h0 = nd / 2;
    const long vol = F->g.vol;
    vzero(C->g.vol * ndc, out);
    /* sequential accumulation over fine sites keeps this obviously correct */
    for (long x = 0; x < vol; x++) {
        long c = F->agg_of[x];
        for (int k = 0; k < nv; k++) {
            const cplx *p = F->P + ((long)k * vol + x) * nd;
            for (int d = 0; d < nd; d++) out[c * ndc + (d / h0) * nv + k] += conj(p[d]) * in[x * nd + d];
        }
    }
}

static void prolong_from(const level *F, const level *C, const cplx *in, cplx *out) {
    const int nd = F->nd, nv = F->nv, ndc = C->nd, h0 = nd / 2;
    const long vol = F->g.vol;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < vol; x++) {
        long c = F->agg_of[x];
        for (int d = 0; d < nd; d++) {
            cplx s = 0;
            for (int k = 0; k < nv; k++) s += F->P[((long)k * vol + x) * nd + d] * in[c * ndc + (d / h0) * nv + k];
            out[x * nd + d] = s;
        }
    }
}

/* D_c = P^H D P written as a nearest-neighbour stencil on the coarse lattice:
 * the self block collects all couplings inside an aggregate's lattice block,
 * slot 1+mu the couplings reaching the block at c+mu through a forward hop and
 * slot 5+mu those reaching c-mu through a backward hop (Sec. 3.2). */
static void assemble_Dc(const level *F, level *C) {
    const int nd = F->nd, nv = F->nv, ndc = C->nd, h0 = nd / 2;
    const long vol = F->g.vol, volc = C->g.vol;
    vzero(volc * 9 * ndc * ndc, C->M);
    long *start = (long *)calloc(volc + 1, sizeof(long));
    long *list = (long *)malloc(sizeof(long) * vol);
    long *fill = (long *)calloc(volc, sizeof(long));
    for (long x = 0; x < vol; x++) start[F->agg_of[x] + 1]++;
    for (long a = 0; a < volc; a++) start[a + 1] += start[a];
    for (long x = 0; x < vol; x++) list[start[F->agg_of[x]] + fill[F->agg_of[x]]++] = x;
#pragma omp parallel for schedule(dynamic)
    for (long c = 0; c < volc; c++) {
        cplx *Pb = (cplx *)malloc(sizeof(cplx) * ndc * nd); /* P columns at one site */
        cplx *W = (cplx *)malloc(sizeof(cplx) * ndc * nd);  /* D applied to them     */
        for (long i = start[c]; i < start[c + 1]; i++) {
            long x = list[i];
            for (int slot = -1; slot < 8; slot++) {
                long y = (slot < 0) ? x : F->g.nb[x * 8 + slot];
                long cy = F->agg_of[y];
                int target;
                if (slot < 0) target = 0;
                else target = (cy == c) ? 0 : 1 + slot;
                /* columns b = h*N + k of P at site y, zero outside half h */
                for (int b = 0; b < ndc; b++) {
                    int h = b / nv, k = b % nv;
                    for (int d = 0; d < nd; d++)
                        Pb[b * nd + d] = (d / h0 == h) ? F->P[((long)k * vol + y) * nd + d] : 0.0;
                    if (slot < 0) site_self(F, x, Pb + b * nd, W + b * nd);
                    else {
                        for (int d = 0; d < nd; d++) W[b * nd + d] = 0;
                        site_hop_acc(F, x, slot, Pb + b * nd, W + b * nd);
                    }
                }
                cplx *Mt = C->M + (c * 9 + target) * ndc * ndc;
                for (int a = 0; a < ndc; a++) {
                    int ha = a / nv, ka = a % nv;
                    const cplx *pa = F->P + ((long)ka * vol + x) * nd;
                    for (int b = 0; b < ndc; b++) {
                        cplx s = 0;
                        for (int d = ha * h0; d < (ha + 1) * h0; d++) s += conj(pa[d]) * W[b * nd + d];
                        Mt[a * ndc + b] += s;
                    }
                }
            }
        }
        free(Pb); free(W);
    }
    free(start); free(list); free(fill);
}

static int coarse_inverses(level *C) {
    int bad = 0, n = C->nd;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long c = 0; c < C->g.vol; c++)
        if (dense_inverse(n, C->M + c * 9 * n * n, C->Minv + c * n * n)) bad |= 1;
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* coarsest-level solver: odd-even preconditioned restarted GMRES (Sec. 5)  */
/* ------------------------------------------------------------------------ */

/* out_o = S in_o,  S = A_oo - D_oe A_ee^{-1} D_eo ; even entries of out are 0 */
static void schur_apply(const level *C, const cplx *in, cplx *out, cplx *t) {
    const int nd = C->nd;
    const long *nb = C->g.nb;
#pragma omp parallel for schedule(static)
    for (long y = 0; y < C->g.vol; y++) {
        if (C->g.par[y] != 0) continue;
        cplx u[128];
        for (int c = 0; c < nd; c++) u[c] = 0;
        for (int k = 0; k < 8; k++) site_hop_acc(C, y, k, in + nb[y * 8 + k] * nd, u);
        site_self_inv(C, y, u, t + y * nd);
    }
#pragma omp parallel for schedule(static)
    for (long x = 0; x < C->g.vol; x++) {
        if (C->g.par[x] != 1) { for (int c = 0; c < nd; c++) out[x * nd + c] = 0; continue; }
        cplx u[128], v[128];
        for (int c = 0; c < nd; c++) u[c] = 0;
        for (int k = 0; k < 8; k++) site_hop_acc(C, x, k, t + nb[x * 8 + k] * nd, u);
        site_self(C, x, in + x * nd, v);
        for (int c = 0; c < nd; c++) out[x * nd + c] = v[c] - u[c];
    }
}

typedef void (*lin_op)(void *ctx, const cplx *in, cplx *out);

typedef struct { const level *C; cplx *t; } schur_ctx;
static void schur_cb(void *p, const cplx *in, cplx *out) {
    schur_ctx *s = (schur_ctx *)p;
    schur_apply(s->C, in, out, s->t);
}
static void full_cb(void *p, const cplx *in, cplx *out) { apply_full((const level *)p, in, out); }

/* Restarted GMRES(m) with modified Gram-Schmidt Arnoldi and Givens rotations,
 * zero initial guess.  Stops when the Arnoldi residual estimate is at most
 * tol*||rhs|| (or after exactly `fixed` iterations if fixed > 0, or at maxit).
 * Returns the number of iterations. */
static long gmres(long n, lin_op A, void *actx, const cplx *rhs, cplx *x,
                  double tol, int m, long maxit, long fixed) {
    cplx **V = (cplx **)malloc(sizeof(cplx *) * (m + 1));
    for (int i = 0; i <= m; i++) V[i] = cvalloc(n);
    cplx *H = (cplx *)calloc((size_t)(m + 1) * m, sizeof(cplx));
    cplx *g = (cplx *)calloc(m + 1, sizeof(cplx));
    cplx *cs = (cplx *)calloc(m, sizeof(cplx)), *sn = (cplx *)calloc(m, sizeof(cplx));
    cplx *y = (cplx *)calloc(m, sizeof(cplx));
    cplx *w = cvalloc(n);
    vzero(n, x);
    double bnorm = vnorm(n, rhs);
    long its = 0;
    if (bnorm == 0.0) goto done;
    vcopy(n, rhs, w); /* r = rhs - A x with x = 0 */
    for (;;) {
        double beta = vnorm(n, w);
        if (beta == 0.0) break;
        memset(H, 0, sizeof(cplx) * (m + 1) * m);
        memset(g, 0, sizeof(cplx) * (m + 1));
        g[0] = beta;
        vcopy(n, w, V[0]);
        vscale(n, 1.0 / beta, V[0]);
        int j, jend = 0;
        int stop = 0;
        for (j = 0; j < m; j++) {
            A(actx, V[j], w);
            for (int i = 0; i <= j; i++) {
                cplx h = vdot(n, V[i], w);
                H[i * m + j] = h;
                vaxpy(n, -h, V[i], w);
            }
            double hn = vnorm(n, w);
            H[(j + 1) * m + j] = hn;
            if (hn != 0.0) { vcopy(n, w, V[j + 1]); vscale(n, 1.0 / hn, V[j + 1]); }
            for (int i = 0; i < j; i++) { /* previous rotations */
                cplx a = H[i * m + j], b = H[(i + 1) * m + j];
                H[i * m + j] = conj(cs[i]) * a + conj(sn[i]) * b;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            cplx a = H[j * m + j], b = H[(j + 1) * m + j];
            double den = sqrt(creal(conj(a) * a) + creal(conj(b) * b));
            if (den == 0.0) { cs[j] = 1; sn[j] = 0; }
            else { cs[j] = a / den; sn[j] = b / den; }
            H[j * m + j] = conj(cs[j]) * a + conj(sn[j]) * b;
            H[(j + 1) * m + j] = 0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = conj(cs[j]) * g[j];
            its++;
            jend = j + 1;
            double res = cabs(g[j + 1]);
            if (fixed > 0) { if (its >= fixed) { stop = 1; break; } }
            else if (res <= tol * bnorm || its >= maxit) { stop = 1; break; }
            if (hn == 0.0) { stop = 1; break; } /* exact solution reached */
        }
        for (int i = jend - 1; i >= 0; i--) {
            cplx s = g[i];
            for (int k = i + 1; k < jend; k++) s -= H[i * m + k] * y[k];
            y[i] = s / H[i * m + i];
        }
        for (int i = 0; i < jend; i++) vaxpy(n, y[i], V[i], x);
        if (stop) break;
        A(actx, x, w); /* restart from the true residual */
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; i++) w[i] = rhs[i] - w[i];
    }
done:
    for (int i = 0; i <= m; i++) free(V[i]);
    free(V); free(H); free(g); free(cs); free(sn); free(y); free(w);
    return its;
}

/* D_c e = r on the coarsest level: odd-even reduction when site parity
 * 2-colours the couplings, GMRES on the Schur complement to relative residual
 * tol, back-substitution on the even sites.  Otherwise GMRES on D_c itself. */
static long coarse_solve(const level *C, const or_params *p, const cplx *r, cplx *e) {
    const int nd = C->nd;
    const long n = C->g.vol * nd;
    const long *nb = C->g.nb;
    long its;
    if (!C->oe_ok) {
        return gmres(n, full_cb, (void *)C, r, e, p->coarse_tol, p->coarse_restart, p->coarse_maxit, p->coarse_fixed);
    }
    cplx *f = cvalloc(n), *t = cvalloc(n), *eo = cvalloc(n);
    /* t_e = A_ee^{-1} r_e ; f_o = r_o - D_oe t_e */
#pragma omp parallel for schedule(static)
    for (long y = 0; y < C->g.vol; y++)
        if (C->g.par[y] == 0) site_self_inv(C, y, r + y * nd, t + y * nd);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < C->g.vol; x++) {
        if (C->g.par[x] != 1) continue;
        cplx u[128];
        for (int c = 0; c < nd; c++) u[c] = 0;
        for (int k = 0; k < 8; k++) site_hop_acc(C, x, k, t + nb[x * 8 + k] * nd, u);
        for (int c = 0; c < nd; c++) f[x * nd + c] = r[x * nd + c] - u[c];
    }
    schur_ctx sc = {C, cvalloc(n)};
    its = gmres(n, schur_cb, &sc, f, eo, p->coarse_tol, p->coarse_restart, p->coarse_maxit, p->coarse_fixed);
    free(sc.t);
    /* e_e = A_ee^{-1} (r_e - D_eo e_o) ; e_o as solved */
#pragma omp parallel for schedule(static)
    for (long y = 0; y < C->g.vol; y++) {
        if (C->g.par[y] == 0) {
            cplx u[128], v[128];
            for (int c = 0; c < nd; c++) u[c] = 0;
            for (int k = 0; k < 8; k++) site_hop_acc(C, y, k, eo + nb[y * 8 + k] * nd, u);
            for (int c = 0; c < nd; c++) v[c] = r[y * nd + c] - u[c];
            site_self_inv(C, y, v, e + y * nd);
        } else {
            for (int c = 0; c < nd; c++) e[y * nd + c] = eo[y * nd + c];
        }
    }
    free(f); free(t); free(eo);
    return its;
}

/* ------------------------------------------------------------------------ */
/* comparison solver of Sec. 6: odd-even preconditioned BiCGStab            */
/* ------------------------------------------------------------------------ */

/* x = approximate D^{-1} b on level L by the odd-even reduction (Sec. 6):
 * f_o = b_o - D_oe A_ee^{-1} b_e, `steps` steps of BiCGStab (van der Vorst,
 * SIAM J. Sci. Stat. Comput. 13 (1992)) from zero on S x_o = f_o with
 * S = A_oo - D_oe A_ee^{-1} D_eo, then x_e = A_ee^{-1} (b_e - D_eo x_o).
 * The reduced vectors are full-length with zero even entries.  Returns the
 * steps taken (fewer on an exact breakdown). */
static long bicgstab_oe(const level *L, const cplx *b, cplx *x, int steps) {
    const int nd = L->nd;
    const long n = L->g.vol * nd;
    const long *nb = L->g.nb;
    cplx *t = cvalloc(n), *r = cvalloc(n), *rh = cvalloc(n), *p = cvalloc(n), *v = cvalloc(n);
    cplx *s = cvalloc(n), *tt = cvalloc(n), *xo = cvalloc(n), *w = cvalloc(n);
    /* t_e = A_ee^{-1} b_e ; r_o = b_o - D_oe t_e ; even entries of r stay 0 */
#pragma omp parallel for schedule(static)
    for (long y = 0; y < L->g.vol; y++)
        if (L->g.par[y] == 0) site_self_inv(L, y, b + y * nd, t + y * nd);
#pragma omp parallel for schedule(static)
    for (long y = 0; y < L->g.vol; y++) {
        if (L->g.par[y] != 1) continue;
        cplx u[128];
        for (int c = 0; c < nd; c++) u[c] = 0;
        for (int k = 0; k < 8; k++) site_hop_acc(L, y, k, t + nb[y * 8 + k] * nd, u);
        for (int c = 0; c < nd; c++) r[y * nd + c] = b[y * nd + c] - u[c];
    }
    vcopy(n, r, rh);
    cplx rho_old = 1, alpha = 1, omega = 1;
    long it = 0;
    for (; it < steps; it++) {
        cplx rho = vdot(n, rh, r);
        if (rho == 0) break;
        cplx beta = (rho / rho_old) * (alpha / omega);
        for (long i = 0; i < n; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        schur_apply(L, p, v, w);
        cplx rv = vdot(n, rh, v);
        if (rv == 0) break;
        alpha = rho / rv;
        for (long i = 0; i < n; i++) s[i] = r[i] - alpha * v[i];
        schur_apply(L, s, tt, w);
        double tn = creal(vdot(n, tt, tt));
        vaxpy(n, alpha, p, xo);
        if (tn == 0) { it++; break; }
        omega = vdot(n, tt, s) / tn;
        if (omega == 0) { it++; break; }   /* breakdown: the next beta would divide by omega */
        vaxpy(n, omega, s, xo);
        for (long i = 0; i < n; i++) r[i] = s[i] - omega * tt[i];
        rho_old = rho;
    }
    /* x_e = A_ee^{-1} (b_e - D_eo x_o) ; x_o as solved */
#pragma omp parallel for schedule(static)
    for (long y = 0; y < L->g.vol; y++) {
        if (L->g.par[y] == 0) {
            cplx u[128], q[128];
            for (int c = 0; c < nd; c++) u[c] = 0;
            for (int k = 0; k < 8; k++) site_hop_acc(L, y, k, xo + nb[y * 8 + k] * nd, u);
            for (int c = 0; c < nd; c++) q[c] = b[y * nd + c] - u[c];
            site_self_inv(L, y, q, x + y * nd);
        } else {
            for (int c = 0; c < nd; c++) x[y * nd + c] = xo[y * nd + c];
        }
    }
    free(t); free(r); free(rh); free(p); free(v); free(s); free(tt); free(xo); free(w);
    return it;
}

/* ------------------------------------------------------------------------ */
/* V-cycle and FGMRES                                                        */
/* ------------------------------------------------------------------------ */
static void vcycle(octx *X, int l, int bottom, const cplx *r, cplx *z);

/* Inexact deflation (Sec. 4.1): out = pi_R in = in - P D_c^{-1} P^H D in with the
 * coarse system solved by the coarsest solver of level 1 (to the tolerance of
 * the parameters: high accuracy for this method). */
static void pi_R(octx *X, const cplx *in, cplx *out) {
    level *F = &X->L[0], *C = &X->L[1];
    const long n = F->g.vol * F->nd, nc = C->g.vol * C->nd;
    cplx *t = cvalloc(n), *rc = cvalloc(nc), *ec = cvalloc(nc);
    apply_full(F, in, t);
    restrict_to(F, C, t, rc);
    X->coarse_count[1] += coarse_solve(C, &X->p, rc, ec);
    prolong_from(F, C, ec, t);
    for (long i = 0; i < n; i++) out[i] = in[i] - t[i];
    free(t); free(rc); free(ec);
}

/* The operator of the outer FGMRES on level 0: D, or D pi_R for inexact deflation. */
static void outer_op(octx *X, int l, const cplx *in, cplx *out) {
    const level *L = &X->L[l];
    if (l == 0 && X->deflated) {
        cplx *t = cvalloc(L->g.vol * L->nd);
        pi_R(X, in, t);
        apply_full(L, t, out);
        free(t);
    } else {
        apply_full(L, in, out);
    }
}

static void outer_op_deflated(octx *X, const cplx *in, cplx *out) {
    int d = X->deflated;
    X->deflated = 1;
    outer_op(X, 0, in, out);
    X->deflated = d;
}

/* Flexible GMRES(m) on level l, right-preconditioned by one V-cycle of level l
 * whose coarsest level is `bottom`.  Arnoldi by modified Gram-Schmidt with one
 * re-orthogonalisation pass.  Convergence is decided on the true residual
 * ||rhs - D x|| <= tol ||rhs|| at the end of each restart cycle. */
static long fgmres(octx *X, int l, int bottom, const cplx *rhs, cplx *x, double tol,
                   int m, long maxit, long fixed, int *restarts, int *converged) {
    const level *L = &X->L[l];
    const long n = L->g.vol * L->nd;
    cplx **V = (cplx **)malloc(sizeof(cplx *) * (m + 1));
    cplx **Z = (cplx **)malloc(sizeof(cplx *) * m);
    for (int i = 0; i <= m; i++) V[i] = cvalloc(n);
    for (int i = 0; i < m; i++) Z[i] = cvalloc(n);
    cplx *H = (cplx *)calloc((size_t)(m + 1) * m, sizeof(cplx));
    cplx *g = (cplx *)calloc(m + 1, sizeof(cplx));
    cplx *cs = (cplx *)calloc(m, sizeof(cplx)), *sn = (cplx *)calloc(m, sizeof(cplx));
    cplx *y = (cplx *)calloc(m, sizeof(cplx));
    cplx *w = cvalloc(n);
    vzero(n, x);
    double bnorm = vnorm(n, rhs);
    long its = 0;
    int nrest = 0, conv = 0;
    if (bnorm == 0.0) { conv = 1; goto done; }
    vcopy(n, rhs, w);
    for (;;) {
        double beta = vnorm(n, w);
        if (beta <= tol * bnorm) { conv = 1; break; }
        if (fixed > 0 ? its >= fixed : its >= maxit) break;
        memset(H, 0, sizeof(cplx) * (m + 1) * m);
        memset(g, 0, sizeof(cplx) * (m + 1));
        g[0] = beta;
        vcopy(n, w, V[0]);
        vscale(n, 1.0 / beta, V[0]);
        int jend = 0;
        for (int j = 0; j < m; j++) {
            if (X->pre_bicg > 0 && l == 0) bicgstab_oe(L, V[j], Z[j], X->pre_bicg);
            else if (X->pre_sap > 0 && l == 0) { vzero(n, Z[j]); sap_sweeps(L, V[j], Z[j], X->pre_sap); }
            else vcycle(X, l, bottom, V[j], Z[j]);
            outer_op(X, l, Z[j], w);
            for (int pass = 0; pass < 2; pass++)
                for (int i = 0; i <= j; i++) {
                    cplx h = vdot(n, V[i], w);
                    H[i * m + j] += h;
                    vaxpy(n, -h, V[i], w);
                }
            double hn = vnorm(n, w);
            H[(j + 1) * m + j] = hn;
            if (hn != 0.0) { vcopy(n, w, V[j + 1]); vscale(n, 1.0 / hn, V[j + 1]); }
            for (int i = 0; i < j; i++) {
                cplx a = H[i * m + j], b = H[(i + 1) * m + j];
                H[i * m + j] = conj(cs[i]) * a + conj(sn[i]) * b;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            cplx a = H[j * m + j], b = H[(j + 1) * m + j];
            double den = sqrt(creal(conj(a) * a) + creal(conj(b) * b));
            if (den == 0.0) { cs[j] = 1; sn[j] = 0; }
            else { cs[j] = a / den; sn[j] = b / den; }
            H[j * m + j] = conj(cs[j]) * a + conj(sn[j]) * b;
            H[(j + 1) * m + j] = 0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = conj(cs[j]) * g[j];
            its++;
            jend = j + 1;
            if (fixed > 0) { if (its >= fixed) break; }
            else if (cabs(g[j + 1]) <= tol * bnorm || its >= maxit) break;
            if (hn == 0.0) break;
        }
        for (int i = jend - 1; i >= 0; i--) {
            cplx s = g[i];
            for (int k = i + 1; k < jend; k++) s -= H[i * m + k] * y[k];
            y[i] = s / H[i * m + i];
        }
        for (int i = 0; i < jend; i++) vaxpy(n, y[i], Z[i], x);
        outer_op(X, l, x, w);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; i++) w[i] = rhs[i] - w[i];
        if (fixed > 0 && its >= fixed) { conv = vnorm(n, w) <= tol * bnorm; break; }
        nrest++;
    }
done:
    for (int i = 0; i <= m; i++) free(V[i]);
    for (int i = 0; i < m; i++) free(Z[i]);
    free(V); free(Z); free(H); free(g); free(cs); free(sn); free(y); free(w);
    if (restarts) *restarts = nrest;
    if (converged) *converged = conv;
    return its;
}

/* One V-cycle with no pre- and nu post-smoothing steps (Sec. 4.2, eq.
 * iterationmatrix):  e_c = D_c^{-1} P^H r (approximately), z = P e_c, then nu
 * SAP iterations on D z = r starting from z.  The coarse equation is solved by
 * odd-even GMRES on the bottom level, otherwise recursively by FGMRES
 * preconditioned with the next level's V-cycle. */
static void vcycle(octx *X, int l, int bottom, const cplx *r, cplx *z) {
    level *F = &X->L[l], *C = &X->L[l + 1];
    long nc = C->g.vol * C->nd;
    cplx *rc = cvalloc(nc), *ec = cvalloc(nc);
    restrict_to(F, C, r, rc);
    if (l + 1 == bottom) {
        X->coarse_count[l + 1] += coarse_solve(C, &X->p, rc, ec);
    } else {
        X->coarse_count[l + 1] += fgmres(X, l + 1, bottom, rc, ec, X->p.mid_tol, X->p.mid_restart,
                                         X->p.mid_maxit, X->p.mid_fixed, NULL, NULL);
    }
    prolong_from(F, C, ec, z);
    sap_sweeps(F, r, z, X->p.nu);
    free(rc); free(ec);
}

/* ------------------------------------------------------------------------ */
/* context, levels                                                           */
/* ------------------------------------------------------------------------ */
static void level_free(level *L) {
    geom_free(&L->g);
    free(L->U); free(L->A); free(L->Ainv); free(L->M); free(L->Minv);
    sap_free(L);
    free(L->agg_of); free(L->tv); free(L->P);
    memset(L, 0, sizeof *L);
}

static int oe_possible(const int d[4]) {
    for (int mu = 0; mu < 4; mu++)
        if (d[mu] != 1 && (d[mu] & 1)) return 0;
    return 1;
}

void *or_create(const int dims[4], const cplx *gauge, const cplx *clover_T, double m0, double csw) {
    gamma_init();
    for (int mu = 0; mu < 4; mu++)
        if (dims[mu] < 2 || (dims[mu] & 1)) return NULL;
    octx *X = (octx *)calloc(1, sizeof(octx));
    level *L = &X->L[0];
    geom_init(&L->g, dims);
    L->nd = 12;
    L->fine = 1;
    L->oe_ok = 1;
    L->U = cvalloc(L->g.vol * 36);
    memcpy(L->U, gauge, sizeof(cplx) * 36 * L->g.vol);
    L->A = cvalloc(L->g.vol * 72);
    L->Ainv = cvalloc(L->g.vol * 72);
    int fail = 0;
    build_clover(L, m0, csw, clover_T, &fail);
    X->nlev = 1;
    if (fail) snprintf(X->err, sizeof X->err, "singular clover block");
    return X;
}

void or_destroy(void *p) {
    octx *X = (octx *)p;
    if (!X) return;
    for (int l = 0; l < OR_MAXLEV; l++) level_free(&X->L[l]);
    free(X);
}

const char *or_error(void *p) { return ((octx *)p)->err; }

/* Largest |entry| of the clover term outside its two chiral 6x6 blocks. */
double or_clover_offblock(const int dims[4], const cplx *gauge, double csw) {
    gamma_init();
    level L;
    memset(&L, 0, sizeof L);
    geom_init(&L.g, dims);
    L.nd = 12; L.fine = 1;
    L.U = (cplx *)gauge;
    double off = 0;
    for (long x = 0; x < L.g.vol; x++) {
        cplx T[144];
        clover_T(&L, x, csw, T);
        for (int i = 0; i < 12; i++)
            for (int j = 0; j < 12; j++)
                if (i / 6 != j / 6 && cabs(T[i * 12 + j]) > off) off = cabs(T[i * 12 + j]);
    }
    geom_free(&L.g);
    return off;
}

/* Full 12x12 clover term T(x) at one site. */
void or_clover_site(const int dims[4], const cplx *gauge, double csw, long x, cplx *T) {
    gamma_init();
    level L;
    memset(&L, 0, sizeof L);
    geom_init(&L.g, dims);
    L.nd = 12; L.fine = 1;
    L.U = (cplx *)gauge;
    clover_T(&L, x, csw, T);
    geom_free(&L.g);
}

void or_get_clover(void *p, cplx *A, cplx *Ainv) {
    octx *X = (octx *)p;
    long v = X->L[0].g.vol;
    if (A) memcpy(A, X->L[0].A, sizeof(cplx) * 72 * v);
    if (Ainv) memcpy(Ainv, X->L[0].Ainv, sizeof(cplx) * 72 * v);
}

/* Change m0 keeping the clover term: A -> A + (m0' - m0) I on every site. */
void or_shift_mass(void *p, double dm) {
    octx *X = (octx *)p;
    level *L = &X->L[0];
    for (long x = 0; x < L->g.vol; x++) {
        for (int h = 0; h < 2; h++)
            for (int i = 0; i < 6; i++) L->A[x * 72 + h * 36 + i * 6 + i] += dm;
        dense_inverse(6, L->A + x * 72, L->Ainv + x * 72);
        dense_inverse(6, L->A + x * 72 + 36, L->Ainv + x * 72 + 36);
    }
}

int or_level_info(void *p, int l, int *dims, int *nd) {
    octx *X = (octx *)p;
    if (l < 0 || l >= X->nlev) return -1;
    memcpy(dims, X->L[l].g.d, sizeof(int) * 4);
    *nd = X->L[l].nd;
    return 0;
}

void or_apply(void *p, int l, const cplx *in, cplx *out) { apply_full(&((octx *)p)->L[l], in, out); }

/* Configure SAP / aggregation geometry for every level from the parameters and
 * allocate the coarse levels (their operators are filled by the setup). */
int or_configure(void *p, const or_params *prm) {
    octx *X = (octx *)p;
    X->p = *prm;
    if (prm->levels < 2 || prm->levels > OR_MAXLEV) { snprintf(X->err, sizeof X->err, "levels"); return -1; }
    for (int l = 1; l < OR_MAXLEV; l++) level_free(&X->L[l]);
    for (int l = 0; l < prm->levels; l++) {
        level *F = &X->L[l];
        if (l < prm->levels - 1) {
            if (!valid_blocks(F->g.d, prm->sap[l])) { snprintf(X->err, sizeof X->err, "SAP blocks at level %d", l); return -1; }
            sap_init(F, prm->sap[l], prm->mr_steps[l]);
            int dc[4];
            for (int mu = 0; mu < 4; mu++) {
                if (prm->agg[l][mu] <= 0 || F->g.d[mu] % prm->agg[l][mu]) { snprintf(X->err, sizeof X->err, "aggregates at level %d", l); return -1; }
                dc[mu] = F->g.d[mu] / prm->agg[l][mu];
            }
            F->nv = prm->n_tv[l];
            memcpy(F->agg, prm->agg[l], sizeof(int) * 4);
            free(F->agg_of); free(F->tv); free(F->P);
            F->agg_of = (long *)malloc(sizeof(long) * F->g.vol);
            for (long x = 0; x < F->g.vol; x++) { int bc[4]; F->agg_of[x] = block_of(F->g.d, F->agg, x, bc); }
            F->tv = cvalloc((long)F->nv * F->g.vol * F->nd);
            F->P = cvalloc((long)F->nv * F->g.vol * F->nd);
            level *C = &X->L[l + 1];
            geom_init(&C->g, dc);
            C->nd = 2 * F->nv;
            C->fine = 0;
            C->oe_ok = oe_possible(dc);
            C->M = cvalloc(C->g.vol * 9 * C->nd * C->nd);
            C->Minv = cvalloc(C->g.vol * C->nd * C->nd);
        }
    }
    X->nlev = prm->levels;
    X->have_params = 1;
    X->have_setup = 0;
    return 0;
}

/* test vectors of the transfer l -> l+1: [N][vol_l][nd_l] */
void or_set_vectors(void *p, int l, const cplx *v) {
    level *F = &((octx *)p)->L[l];
    memcpy(F->tv, v, sizeof(cplx) * (long)F->nv * F->g.vol * F->nd);
}

void or_get_vectors(void *p, int l, cplx *v) {
    level *F = &((octx *)p)->L[l];
    memcpy(v, F->tv, sizeof(cplx) * (long)F->nv * F->g.vol * F->nd);
}

/* P, D_c and the coarse self-block inverses from the current test vectors */
int or_build(void *p, int l) {
    octx *X = (octx *)p;
    level *F = &X->L[l], *C = &X->L[l + 1];
    if (build_P(F, C->g.vol)) { snprintf(X->err, sizeof X->err, "rank-deficient aggregate"); return -1; }
    assemble_Dc(F, C);
    if (coarse_inverses(C)) { snprintf(X->err, sizeof X->err, "singular coarse self block"); return -1; }
    return 0;
}

void or_get_P(void *p, int l, cplx *out) {
    level *F = &((octx *)p)->L[l];
    memcpy(out, F->P, sizeof(cplx) * (long)F->nv * F->g.vol * F->nd);
}

/* Install explicitly given interpolation columns (already orthonormal) and build D_c. */
int or_set_P(void *p, int l, const cplx *in) {
    octx *X = (octx *)p;
    level *F = &X->L[l], *C = &X->L[l + 1];
    memcpy(F->P, in, sizeof(cplx) * (long)F->nv * F->g.vol * F->nd);
    assemble_Dc(F, C);
    return coarse_inverses(C);
}

void or_get_coarse(void *p, int l, cplx *M, cplx *Minv) {
    level *C = &((octx *)p)->L[l];
    long n = C->nd;
    if (M) memcpy(M, C->M, sizeof(cplx) * C->g.vol * 9 * n * n);
    if (Minv) memcpy(Minv, C->Minv, sizeof(cplx) * C->g.vol * n * n);
}

void or_restrict(void *p, int l, const cplx *in, cplx *out) {
    octx *X = (octx *)p;
    restrict_to(&X->L[l], &X->L[l + 1], in, out);
}

void or_prolong(void *p, int l, const cplx *in, cplx *out) {
    octx *X = (octx *)p;
    prolong_from(&X->L[l], &X->L[l + 1], in, out);
}

/* z = M_SAP^(nsweeps) rhs if zero_start, else nsweeps SAP iterations from z */
void or_sap(void *p, int l, const cplx *rhs, cplx *z, int nsweeps, int zero_start) {
    level *L = &((octx *)p)->L[l];
    if (zero_start) vzero(L->g.vol * L->nd, z);
    sap_sweeps(L, rhs, z, nsweeps);
}

/* single block solve on block bi with residual r (z += B_i r) */
void or_block_solve(void *p, int l, long bi, const cplx *r, cplx *z) {
    level *L = &((octx *)p)->L[l];
    long n = L->g.vol * L->nd;
    cplx *t = cvalloc(n), *rho = cvalloc(n), *s = cvalloc(n), *e = cvalloc(n);
    block_solve(L, bi, r, z, t, rho, s, e);
    free(t); free(rho); free(s); free(e);
}

long or_coarse_solve(void *p, int l, const cplx *r, cplx *e) {
    octx *X = (octx *)p;
    return coarse_solve(&X->L[l], &X->p, r, e);
}

void or_schur(void *p, int l, const cplx *in, cplx *out) {
    level *C = &((octx *)p)->L[l];
    cplx *t = cvalloc(C->g.vol * C->nd);
    schur_apply(C, in, out, t);
    free(t);
}

void or_vcycle(void *p, int l, int bottom, const cplx *r, cplx *z) { vcycle((octx *)p, l, bottom, r, z); }

/* The intermediate-level solve of a V-cycle on level l (1 <= l < levels-1):
 * FGMRES preconditioned by the level-l V-cycle, with the intermediate-level
 * tolerance, restart and iteration counts; returns the iteration count. */
long or_fgmres_level(void *p, int l, const cplx *rhs, cplx *x) {
    octx *X = (octx *)p;
    return fgmres(X, l, X->nlev - 1, rhs, x, X->p.mid_tol, X->p.mid_restart, X->p.mid_maxit, X->p.mid_fixed,
                  NULL, NULL);
}

/* Algorithm 2 (DD-alpha-AMG-setup(n_inv, nu)) on level l with the test vectors
 * already installed by or_set_vectors; with id_setup, the inexact-deflation
 * setup of Sec. 4.3 instead, which differs only in the update of the second
 * half (the V-cycle applied to v_j from a zero start replaces v_j).  The V-cycles inside use level l+1 as
 * the coarsest level.  Readings: the vectors are normalised after each of the
 * three initial SAP passes (the passes are homogeneous, so only the scale
 * changes), and P, D_c are rebuilt once more from the final vectors. */
int or_setup_level(void *p, int l) {
    octx *X = (octx *)p;
    level *F = &X->L[l];
    const long n = F->g.vol * F->nd;
    cplx *z = cvalloc(n), *r = cvalloc(n), *c = cvalloc(n);
    int rc = 0;
    for (int eta = 1; eta <= 3; eta++) {
        for (int j = 0; j < F->nv; j++) {
            cplx *v = F->tv + (long)j * n;
            vzero(n, z);
            sap_sweeps(F, v, z, eta);
            vcopy(n, z, v);
            vscale(n, 1.0 / vnorm(n, v), v);
        }
    }
    for (int it = 0; it < X->p.n_inv; it++) {
        if ((rc = or_build(p, l))) goto out;
        for (int j = 0; j < F->nv; j++) {
            cplx *v = F->tv + (long)j * n;
            if (X->p.id_setup) {
                /* IDsetup: v_j <- (M_SAP^(nu) pi_L + P D_c^{-1} P^H) v_j, the V-cycle from zero */
                vcycle(X, l, l + 1, v, c);
                vcopy(n, c, v);
            } else {
                apply_full(F, v, r);
#pragma omp parallel for schedule(static)
                for (long i = 0; i < n; i++) r[i] = v[i] - r[i];
                vcycle(X, l, l + 1, r, c);
                vaxpy(n, 1.0, c, v);
            }
            vscale(n, 1.0 / vnorm(n, v), v);
        }
    }
    rc = or_build(p, l);
out:
    free(z); free(r); free(c);
    return rc;
}

/* Full setup: Algorithm 2 on each level in turn, coarser levels after finer
 * ones.  tv[l] holds the initial random vectors of level l. */
int or_setup(void *p, const cplx *const *tv) {
    octx *X = (octx *)p;
    if (!X->have_params) return -1;
    for (int l = 0; l < X->nlev - 1; l++) {
        or_set_vectors(p, l, tv[l]);
        int rc = or_setup_level(p, l);
        if (rc) return rc;
    }
    X->have_setup = 1;
    return 0;
}

/* FGMRES on level 0 preconditioned by the full V-cycle, x0 = 0. */
int or_solve(void *p, const cplx *b, cplx *x, double tol, long fixed, or_stats *st) {
    octx *X = (octx *)p;
    if (!X->have_setup) return -5;
    memset(X->coarse_count, 0, sizeof X->coarse_count);
    int restarts = 0, conv = 0;
    long its = fgmres(X, 0, X->nlev - 1, b, x, tol, X->p.outer_restart, X->p.outer_maxit, fixed, &restarts, &conv);
    if (st) {
        level *L = &X->L[0];
        long n = L->g.vol * L->nd;
        cplx *r = cvalloc(n);
        apply_full(L, x, r);
        for (long i = 0; i < n; i++) r[i] = b[i] - r[i];
        st->true_relres = vnorm(n, r) / vnorm(n, b);
        free(r);
        st->outer_iters = (int)its;
        st->restarts = restarts;
        st->converged = conv;
        for (int l = 0; l < OR_MAXLEV; l++) st->coarse_iters[l] = X->coarse_count[l];
    }
    return conv ? 0 : -3;
}

/* x = BiCGStab preconditioner (odd-even, `steps` steps from zero) applied to b
 * on the fine level. */
long or_bicgstab(void *p, const cplx *b, cplx *x, int steps) {
    return bicgstab_oe(&((octx *)p)->L[0], b, x, steps);
}

/* The comparison solver: FGMRES(outer_restart) on the fine level,
 * right-preconditioned by `steps` odd-even BiCGStab steps (needs
 * or_configure for the outer parameters; no multigrid setup is used). */
int or_solve_bicgstab(void *p, const cplx *b, cplx *x, double tol, int steps, or_stats *st) {
    octx *X = (octx *)p;
    if (!X->have_params) return -5;
    X->pre_bicg = steps;
    int restarts = 0, conv = 0;
    long its = fgmres(X, 0, 0, b, x, tol, X->p.outer_restart, X->p.outer_maxit, 0, &restarts, &conv);
    X->pre_bicg = 0;
    if (st) {
        level *L = &X->L[0];
        long n = L->g.vol * L->nd;
        cplx *r = cvalloc(n);
        apply_full(L, x, r);
        for (long i = 0; i < n; i++) r[i] = b[i] - r[i];
        st->true_relres = vnorm(n, r) / vnorm(n, b);
        free(r);
        st->outer_iters = (int)its;
        st->restarts = restarts;
        st->converged = conv;
        memset(st->coarse_iters, 0, sizeof st->coarse_iters);
    }
    return conv ? 0 : -3;
}

/* Inexact deflation (Sec. 4.1), the other comparison solver: with the two-level
 * hierarchy as built (P, D_c), chi' = P D_c^{-1} P^H b, then FGMRES(outer_restart)
 * on D pi_R chi = pi_L b = b - D chi' right-preconditioned by nu SAP iterations
 * M_SAP^(nu) (the paper uses GCR, the same minimal-residual iterates), and
 * z = pi_R chi + chi'.  The coarse systems are solved to the coarsest solver's
 * tolerance of the parameters, which this method needs small.  tol applies to
 * the deflated system; the true residual of z is reported. */
int or_solve_id(void *p, const cplx *b, cplx *x, double tol, int nu, or_stats *st) {
    octx *X = (octx *)p;
    if (!X->have_setup || X->nlev != 2) return -5;
    level *F = &X->L[0], *C = &X->L[1];
    const long n = F->g.vol * F->nd, nc = C->g.vol * C->nd;
    memset(X->coarse_count, 0, sizeof X->coarse_count);
    cplx *rc = cvalloc(nc), *ec = cvalloc(nc), *chi1 = cvalloc(n), *bd = cvalloc(n), *chi = cvalloc(n);
    restrict_to(F, C, b, rc);
    X->coarse_count[1] += coarse_solve(C, &X->p, rc, ec);
    prolong_from(F, C, ec, chi1);
    apply_full(F, chi1, bd);
    for (long i = 0; i < n; i++) bd[i] = b[i] - bd[i];
    X->deflated = 1;
    X->pre_sap = nu;
    int restarts = 0, conv = 0;
    long its = fgmres(X, 0, 1, bd, chi, tol, X->p.outer_restart, X->p.outer_maxit, 0, &restarts, &conv);
    X->deflated = 0;
    X->pre_sap = 0;
    pi_R(X, chi, x);
    vaxpy(n, 1.0, chi1, x);
    if (st) {
        cplx *r = cvalloc(n);
        apply_full(F, x, r);
        for (long i = 0; i < n; i++) r[i] = b[i] - r[i];
        st->true_relres = vnorm(n, r) / vnorm(n, b);
        free(r);
        st->outer_iters = (int)its;
        st->restarts = restarts;
        st->converged = conv;
        for (int l = 0; l < OR_MAXLEV; l++) st->coarse_iters[l] = X->coarse_count[l];
    }
    free(rc); free(ec); free(chi1); free(bd); free(chi);
    return conv ? 0 : -3;
}

/* out = D pi_R in on level 0 (the inexact-deflation operator). */
void or_apply_deflated(void *p, const cplx *in, cplx *out) { outer_op_deflated((octx *)p, in, out); }

/* Mark the hierarchy as complete after components were installed piecewise. */
void or_mark_setup(void *p) { ((octx *)p)->have_setup = 1; }

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
