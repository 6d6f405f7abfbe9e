/*
 * Drives every entry point of the test oracle (oracle/modal_oracle.c) on a
 * small synthetic problem, built together with it under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py.  Any invalid
 * access, overflow or undefined operation aborts the run; the driver itself
 * only checks that every output is finite and that bad sizes are refused.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int or_gauss_legendre(int n, double *x, double *w);
void or_legendre_table(int lmax, int nmu, const double *mu, double *P);
int or_sph_bessel_table(int lmax, int64_t nx, const double *x, double *J);
int or_beta(int lmin, int lmax, int nk, const double *k, const double *wk, int nr, const double *r, int np,
            const double *qk, const double *delta, int nsel, const int32_t *psel, double *beta);
int or_S(int lmin, int lmax, const double *cl, double v_power, int na, const double *ql, int nr, int nmu,
         const double *P, int nb, const double *beta, int npairs, const int32_t *pairs, double *S);
int or_gamma_entries(int kind, int nr, const double *r, const double *wr, int nmu, const double *wmu, int nS,
                     const double *S, int64_t ne, const int32_t *sidx, double *gamma, double *scale);
int or_gamma_adjoint(int kind, int nr, const double *r, const double *wr, int nmu, const double *wmu, int nS,
                     const double *S, int64_t ne, const int32_t *sidx, const double *g, double *Shat);
int or_S_adjoint(int lmin, int lmax, const double *cl, double v_power, int na, const double *ql, int nr, int nmu,
                 const double *P, int nb, int npairs, const int32_t *pairs, const double *Shat, double *bhat);
int or_beta_adjoint(int lmin, int lmax, int nk, const double *k, const double *wk, int nr, const double *r, int np,
                    const double *qk, const double *delta, const double *bhat, double *dq, double *ddelta);
int or_num_threads(void);

static int bad = 0;

static void finite(const char *what, const double *a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) {
            fprintf(stderr, "%s[%zu] not finite\n", what, i);
            bad = 1;
            return;
        }
}

static double *arr(size_t n)
{
    double *p = (double *)calloc(n ? n : 1, sizeof(double));
    if (!p) exit(2);
    return p;
}

int main(void)
{
    enum { LMIN = 2, LMAX = 20, L = LMAX - LMIN + 1, NK = 30, NR = 4, NMU = 32, N1 = 3, NP = N1, NA = N1 };
    double *k = arr(NK), *wk = arr(NK), *r = arr(NR), *wr = arr(NR), *cl = arr(L);
    double *qk = arr((size_t)NP * NK), *delta = arr((size_t)L * NK), *ql = arr((size_t)NA * L);
    for (int i = 0; i < NK; ++i) {
        k[i] = 1e-4 * pow(400.0, (double)i / (NK - 1));
        wk[i] = 1e-4;
    }
    for (int j = 0; j < NR; ++j) {
        r[j] = 13900.0 + 60.0 * j;
        wr[j] = 60.0;
    }
    for (int l = 0; l < L; ++l) {
        const double ll = l + LMIN;
        cl[l] = 1e3 / (ll * (ll + 1.0));
        for (int i = 0; i < NK; ++i) delta[(size_t)l * NK + i] = sin(0.3 * ll + 0.1 * i) * exp(-0.01 * i);
        for (int a = 0; a < NA; ++a) ql[(size_t)a * L + l] = cos(0.2 * a * l);
    }
    for (int p = 0; p < NP; ++p)
        for (int i = 0; i < NK; ++i) qk[(size_t)p * NK + i] = cos(0.1 * p * i);

    double *mu = arr(NMU), *wmu = arr(NMU);
    if (or_gauss_legendre(NMU, mu, wmu) != 0) bad = 1;
    if (or_gauss_legendre(0, mu, wmu) == 0) bad = 1;               /* refused */
    finite("mu", mu, NMU);
    double *P = arr((size_t)NMU * (LMAX + 1));
    or_legendre_table(LMAX, NMU, mu, P);
    finite("P", P, (size_t)NMU * (LMAX + 1));

    double x[6] = {0.0, 1e-8, 0.5, 3.0, 25.0, 300.0};
    double *J = arr(6 * (LMAX + 1));
    if (or_sph_bessel_table(LMAX, 6, x, J) != 0) bad = 1;
    finite("J", J, 6 * (LMAX + 1));

    int32_t psel[NP];
    for (int p = 0; p < NP; ++p) psel[p] = p;
    double *beta = arr((size_t)NP * L * NR);
    if (or_beta(LMIN, LMAX, NK, k, wk, NR, r, NP, qk, delta, NP, psel, beta) != 0) bad = 1;
    finite("beta", beta, (size_t)NP * L * NR);

    int32_t pairs[2 * NA * NP];
    for (int a = 0; a < NA; ++a)
        for (int p = 0; p < NP; ++p) {
            pairs[2 * (a * NP + p)] = a;
            pairs[2 * (a * NP + p) + 1] = p;
        }
    const int nS = NA * NP;
    double *S = arr((size_t)nS * NR * NMU);
    if (or_S(LMIN, LMAX, cl, 1.0 / 6.0, NA, ql, NR, NMU, P, NP, beta, nS, pairs, S) != 0) bad = 1;
    finite("S", S, (size_t)nS * NR * NMU);

    enum { NE = 20 };
    int32_t sidx[9 * NE];
    for (int e = 0; e < 9 * NE; ++e) sidx[e] = (e * 7 + 3) % nS;
    double g[NE], sc[NE], dg[NE];
    for (int kind = 0; kind < 2; ++kind) {
        if (or_gamma_entries(kind, NR, r, wr, NMU, wmu, nS, S, NE, sidx, g, sc) != 0) bad = 1;
        if (or_gamma_entries(kind, NR, r, wr, NMU, wmu, nS, S, NE, sidx, g, NULL) != 0) bad = 1;
        finite("gamma", g, NE);
        finite("scale", sc, NE);
        for (int e = 0; e < NE; ++e) dg[e] = 1.0 / (1.0 + e);
        double *Shat = arr((size_t)nS * NR * NMU);
        if (or_gamma_adjoint(kind, NR, r, wr, NMU, wmu, nS, S, NE, sidx, dg, Shat) != 0) bad = 1;
        finite("Shat", Shat, (size_t)nS * NR * NMU);
        double *bhat = arr((size_t)NP * L * NR);
        if (or_S_adjoint(LMIN, LMAX, cl, 1.0 / 6.0, NA, ql, NR, NMU, P, NP, nS, pairs, Shat, bhat) != 0) bad = 1;
        finite("bhat", bhat, (size_t)NP * L * NR);
        double *dq = arr((size_t)NP * NK), *dd = arr((size_t)L * NK);
        if (or_beta_adjoint(LMIN, LMAX, NK, k, wk, NR, r, NP, qk, delta, bhat, dq, dd) != 0) bad = 1;
        finite("dq", dq, (size_t)NP * NK);
        finite("ddelta", dd, (size_t)L * NK);
        free(Shat);
        free(bhat);
        free(dq);
        free(dd);
    }
    sidx[4] = nS;                                                    /* index out of range: refused */
    if (or_gamma_entries(1, NR, r, wr, NMU, wmu, nS, S, NE, sidx, g, sc) == 0) bad = 1;
    if (or_num_threads() < 1) bad = 1;

    free(k); free(wk); free(r); free(wr); free(cl); free(qk); free(delta); free(ql);
    free(mu); free(wmu); free(P); free(J); free(beta); free(S);
    printf(bad ? "FAILED\n" : "sanitized oracle run OK\n");
    return bad;
}
