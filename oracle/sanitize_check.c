/*
 * sanitize_check.c -- memory and undefined-behaviour check of the oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Built by the CPU test suite together with
 * ddamg_oracle.c under gcc's AddressSanitizer and UndefinedBehaviorSanitizer
 * and run as a separate program: it drives every public routine of the oracle
 * once on tiny lattices (two and three levels, odd-even and plain coarsest
 * GMRES, SAP with a block spanning a dimension) and exits non-zero if a solve
 * misses its residual.  The links are arbitrary complex 3x3 matrices near the
 * identity (memory safety does not need SU(3)); m0 = 0.8 keeps D well
 * conditioned.
 */
#include "ddamg_oracle.c"

static unsigned long long rng_state = 88172645463325252ULL;
static double urand(void) { /* xorshift64, uniform in [-0.5, 0.5) */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) / 9007199254740992.0 - 0.5;
}

static cplx *links(const int d[4]) {
    long vol = (long)d[0] * d[1] * d[2] * d[3];
    cplx *U = cvalloc(vol * 36);
    for (long i = 0; i < vol * 4; i++)
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) U[i * 9 + a * 3 + b] = (a == b) + 0.3 * (urand() + I * urand());
    return U;
}

static cplx *vectors(long n) {
    cplx *v = cvalloc(n);
    for (long i = 0; i < n; i++) v[i] = urand() + I * urand();
    return v;
}

static int run(const int d[4], int levels, const int agg[2][4], const int sap[2][4], int n_tv) {
    long vol = (long)d[0] * d[1] * d[2] * d[3];
    cplx *U = links(d);
    void *X = or_create(d, U, NULL, 0.8, 1.0);
    if (!X) return 1;
    or_params p;
    memset(&p, 0, sizeof p);
    p.levels = levels;
    for (int l = 0; l < OR_MAXLEV; l++) {
        p.n_tv[l] = n_tv;
        p.mr_steps[l] = 3;
        for (int mu = 0; mu < 4; mu++) {
            p.agg[l][mu] = agg[l < 2 ? l : 1][mu];
            p.sap[l][mu] = sap[l < 2 ? l : 1][mu];
        }
    }
    p.nu = 2; p.n_inv = 1;
    p.coarse_tol = 5e-2; p.coarse_restart = 10; p.coarse_maxit = 200;
    p.mid_tol = 5e-2; p.mid_restart = 5; p.mid_maxit = 20;
    p.outer_restart = 10; p.outer_maxit = 400;
    if (or_configure(X, &p)) { fprintf(stderr, "configure: %s\n", or_error(X)); return 1; }
    const cplx *tv[OR_MAXLEV] = {0};
    cplx *keep[OR_MAXLEV] = {0};
    long nl = vol * 12;
    for (int l = 0; l < levels - 1; l++) {
        int dl[4], nd;
        or_level_info(X, l, dl, &nd);
        long vl = (long)dl[0] * dl[1] * dl[2] * dl[3];
        keep[l] = vectors((long)n_tv * vl * nd);
        tv[l] = keep[l];
    }
    if (or_setup(X, tv)) { fprintf(stderr, "setup: %s\n", or_error(X)); return 1; }
    cplx *b = vectors(nl), *x = cvalloc(nl), *y = cvalloc(nl);
    or_stats st;
    int rc = or_solve(X, b, x, 1e-10, 0, &st);
    if (rc || st.true_relres > 1e-10) { fprintf(stderr, "solve rc %d relres %g\n", rc, st.true_relres); return 1; }
    or_apply(X, 0, b, y);
    or_sap(X, 0, b, y, 2, 1);
    or_vcycle(X, 0, levels - 1, b, y);
    int dc[4], ndc;
    or_level_info(X, 1, dc, &ndc);
    long nc = (long)dc[0] * dc[1] * dc[2] * dc[3] * ndc;
    cplx *rc1 = cvalloc(nc), *ec1 = cvalloc(nc);
    or_restrict(X, 0, b, rc1);
    or_prolong(X, 0, rc1, y);
    if (levels == 2) {
        or_coarse_solve(X, 1, rc1, ec1);
        or_schur(X, 1, rc1, ec1);
        /* the comparison solvers: odd-even BiCGStab, inexact deflation and its setup */
        or_bicgstab(X, b, y, 5);
        rc = or_solve_bicgstab(X, b, x, 1e-8, 10, &st);
        if (rc || st.true_relres > 1e-8) { fprintf(stderr, "bicgstab rc %d relres %g\n", rc, st.true_relres); return 1; }
        /* inexact deflation needs its coarse systems solved accurately */
        p.id_setup = 1;
        p.coarse_tol = 1e-12;
        p.coarse_maxit = 4000;
        if (or_configure(X, &p) || or_setup(X, tv)) { fprintf(stderr, "id setup: %s\n", or_error(X)); return 1; }
        or_apply_deflated(X, b, y);
        rc = or_solve_id(X, b, x, 1e-8, 3, &st);
        if (rc || st.true_relres > 1e-7) { fprintf(stderr, "id rc %d relres %g\n", rc, st.true_relres); return 1; }
    } else {
        or_fgmres_level(X, 1, rc1, ec1);
        or_sap(X, 1, rc1, ec1, 1, 1);
    }
    cplx *A = cvalloc(vol * 72), *Ai = cvalloc(vol * 72);
    or_get_clover(X, A, Ai);
    or_shift_mass(X, 0.05);
    or_apply(X, 0, b, y);
    free(A); free(Ai); free(rc1); free(ec1);
    free(b); free(x); free(y);
    for (int l = 0; l < OR_MAXLEV; l++) free(keep[l]);
    free(U);
    or_destroy(X);
    return 0;
}

int main(void) {
    /* two levels, odd-even coarsest */
    int d1[4] = {4, 4, 2, 2};
    int a1[2][4] = {{2, 2, 2, 2}, {2, 2, 1, 1}};
    int s1[2][4] = {{2, 2, 2, 2}, {1, 1, 1, 1}};
    if (run(d1, 2, a1, s1, 4)) return 1;
    /* two levels, a SAP block spanning dimension 2 and a coarsest lattice with
     * an odd extent (plain GMRES) */
    int d2[4] = {4, 4, 6, 2};
    int a2[2][4] = {{2, 2, 2, 2}, {1, 1, 1, 1}};
    int s2[2][4] = {{2, 2, 6, 2}, {1, 1, 1, 1}};
    if (run(d2, 2, a2, s2, 3)) return 1;
    /* three levels */
    int d3[4] = {8, 4, 4, 4};
    int a3[2][4] = {{2, 2, 2, 2}, {2, 2, 2, 2}};
    int s3[2][4] = {{2, 2, 2, 2}, {2, 2, 2, 2}};
    if (run(d3, 3, a3, s3, 3)) return 1;
    printf("sanitize_check ok\n");
    return 0;
}
