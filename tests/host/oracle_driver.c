/* Host driver of the CPU oracle (oracle/emri_oracle.c, compiled into this
 * program) for the address and undefined-behaviour sanitizers
 * (tests/test_host_sanitizers.py).  It calls every entry point on small
 * inputs -- valid walkers, edge rows (circular, spinless, spin along the
 * ecliptic pole, plunging) and invalid ones -- in each orbit convention and
 * integrator, and checks that what must be finite is finite and what must
 * be -inf is.  Numerical correctness is the business of the pinned Python
 * tests; this program is about memory and undefined behaviour. */
#include "../../oracle/emri_oracle.c"

#include <stdio.h>
#include <stdlib.h>

#define CHECK(c)                                                                   \
    do {                                                                           \
        if (!(c)) {                                                                \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c);  \
            abort();                                                               \
        }                                                                          \
    } while (0)

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static double uniform01(void)
{
    g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
    return ((g_state >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}
static double normal(void)
{
    const double u = uniform01(), v = uniform01();
    return sqrt(-2.0 * log(u)) * cos(2.0 * 3.141592653589793 * v);
}

enum { B = 8 };

static void rows(double *P)
{
    const double inj[17] = {1e6, 10.0, 0.5, 0.3, 1e-3, 1.0, 1.0, 1.0, 0.5,
                            0.8, 0.8, 0.8, 0.8, 1.0, 0.9, 2.0, 0.0};
    for (int w = 0; w < B; ++w)
        for (int j = 0; j < 17; ++j) P[w * 17 + j] = inj[j] * (1.0 + (w ? 1e-4 * normal() : 0.0));
    P[1 * 17 + 3] = 0.0;               /* circular */
    P[2 * 17 + 2] = 0.0;               /* spinless */
    P[3 * 17 + 11] = 0.0;              /* spin along the ecliptic pole */
    P[4 * 17 + 4] = 1.62e-3;           /* just below the LSO: plunges inside the window */
    P[5 * 17 + 1] = 2e6;               /* mu > M: invalid */
    P[6 * 17 + 3] = 1.2;               /* e0 >= 1: invalid */
    P[7 * 17 + 16] = 1e-16;            /* tiny constant delay */
}

static void run(int ic_lso, int ode)
{
    oracle_cfg c;
    memset(&c, 0, sizeof c);
    c.T_obs = 2.5 * 86400.0;
    c.dt = 10.0;
    c.N = 1 << 15;
    c.n_harm = 8;
    c.coarse_log2 = 10;
    c.ic_lso = ic_lso;
    c.ode = ode;
    c.rtol = 1e-10;
    c.atol = 1e-10;
    const int64_t N = c.N, H = N / 2 + 1, K = n_intervals_of(&c);
    double P[B * 17];
    rows(P);

    double sc[B * 8];
    CHECK(oracle_scalars(P, B, sc) == 0);
    double *orb = calloc((size_t)B * (K + 1) * 10, sizeof(double));
    int32_t kw[B];
    CHECK(oracle_orbit(P, B, &c, orb, kw) == 0);
    int32_t steps[B * 2];
    if (ode == 1) CHECK(oracle_orbit_steps(P, B, &c, steps) == 0);

    double *x = calloc((size_t)B * 2 * N, sizeof(double));
    CHECK(oracle_waveform(P, B, &c, x) == 0);
    double *X = calloc((size_t)B * 2 * H * 2, sizeof(double));
    CHECK(oracle_rfft(x, 2 * B, N, c.dt, X) == 0);
    double *diag = calloc((size_t)N * 16, sizeof(double));
    double *x1 = calloc((size_t)2 * N, sizeof(double));
    CHECK(oracle_waveform_diag(P, &c, x1, diag) == 0);

    double *f = malloc((size_t)H * sizeof(double));
    double *S = malloc((size_t)H * sizeof(double));
    for (int64_t k = 0; k < H; ++k) f[k] = (double)k / ((double)N * c.dt);
    CHECK(oracle_psd_bc04(f, H, S) == 0);
    double *S2 = malloc((size_t)H * sizeof(double));
    for (int conf = -1; conf < 4; ++conf) CHECK(oracle_psd_rcl(f, H, conf, S2) == 0);

    double *g = malloc((size_t)2 * H * 2 * sizeof(double));
    for (int64_t i = 0; i < 2 * H * 2; ++i) g[i] = normal();
    double *d = calloc((size_t)2 * H * 2, sizeof(double));
    CHECK(oracle_make_data(X, P, S, g, N, c.dt, d) == 0);
    double *d0 = calloc((size_t)2 * H * 2, sizeof(double));
    CHECK(oracle_make_data(X, P, S, NULL, N, c.dt, d0) == 0);

    double lnL[B];
    CHECK(oracle_loglike(P, B, d, S, &c, lnL) == 0);
    for (int w = 0; w < B; ++w) {
        if (w == 5 || w == 6) CHECK(isinf(lnL[w]) && lnL[w] < 0);
        else if (ic_lso == 0) CHECK(isfinite(lnL[w]));
    }
    double *sets = malloc((size_t)2 * 2 * H * 2 * sizeof(double));
    memcpy(sets, d, (size_t)2 * H * 2 * sizeof(double));
    memcpy(sets + 2 * H * 2, d0, (size_t)2 * H * 2 * sizeof(double));
    double lnL2[B * 2];
    CHECK(oracle_loglike_sets(P, B, sets, 2, S, &c, lnL2, NULL) == 0);
    for (int w = 0; w < B; ++w) CHECK(lnL2[w * 2] == lnL[w] || (isnan(lnL[w]) && isnan(lnL2[w * 2])));
    double *spec = malloc((size_t)B * 2 * H * 2 * sizeof(double));
    CHECK(oracle_loglike_sets(P, B, sets, 2, S, &c, lnL2, spec) == 0);
    for (int w = 0; w < B; ++w) CHECK(lnL2[w * 2] == lnL[w] || (isnan(lnL[w]) && isnan(lnL2[w * 2])));
    free(spec);

    double coef[B * 2 * 3];
    for (int i = 0; i < B * 2 * 3; ++i) coef[i] = 1e-3 * normal();
    double lf[B];
    CHECK(oracle_loglike_fmg(P, B, coef, 3, 1e-2, d, S, &c, lf) == 0);
    CHECK(oracle_loglike_fmg(P, B, NULL, 0, 1e-2, d, S, &c, lf) == 0);

    /* ensemble sampler: two halves of 4 walkers, three free coordinates */
    const int W = 4;
    double Xe[2 * 4 * 17], lnp[2 * 4];
    for (int i = 0; i < 2 * W; ++i) memcpy(Xe + i * 17, P, 17 * sizeof(double));
    int32_t fi[3] = {0, 3, 13};
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = P[fi[k]] * 0.99;
        hi[k] = P[fi[k]] * 1.01;
    }
    for (int i = 1; i < 2 * W; ++i)
        for (int k = 0; k < 3; ++k) Xe[i * 17 + fi[k]] *= 1.0 + 1e-3 * normal();
    CHECK(oracle_ensemble_lnprob(Xe, 2 * W, fi, 3, lo, hi, d, S, &c, lnp) == 0);
    double u[2 * 4 * 3];
    for (int i = 0; i < 2 * W * 3; ++i) u[i] = uniform01();
    int32_t acc[2 * 4];
    CHECK(oracle_stretch_step(Xe, lnp, W, fi, 3, lo, hi, 2.0, u, d, S, &c, acc) == 0);

    free(orb); free(x); free(X); free(diag); free(x1); free(f); free(S); free(S2);
    free(g); free(d); free(d0); free(sets);
}

int main(void)
{
    double tab[77], out3[3], out2[2], dy[5];
    CHECK(oracle_dp5_tableau(tab) == 0);
    for (int n = -4; n <= 70; ++n) {
        const double v = oracle_besselj(n, 0.37 * (n < 0 ? -n : n) + 0.1);
        CHECK(isfinite(v));
    }
    for (int n = 1; n <= 64; ++n) CHECK(oracle_pm_coeffs(n, 0.7, out3) == 0);
    CHECK(oracle_antenna(0.3, 1.1, 0.7, out2) == 0);
    CHECK(isfinite(oracle_hermite(1.0, 0.5, 2.0, -0.5, 3.0, 0.25)));
    CHECK(fabs(oracle_dl_of_z(oracle_z_of_dl(1e17)) - 1e17) < 1e3);
    const double y[5] = {0.0, 1e-3, 0.0, 0.3, 0.0};
    const double prow[17] = {1e6, 10.0, 0.5, 0.3, 1e-3, 1, 1, 1, 0.5, 0.8, 0.8, 0.8, 0.8, 1, 1, 0, 0};
    CHECK(oracle_rhs(y, prow, 0, dy) == 0);
    CHECK(oracle_rhs(y, prow, 1, dy) == 0);
    for (int ic = 0; ic < 2; ++ic)
        for (int ode = 0; ode < 2; ++ode) {
            run(ic, ode);
            printf("oracle ic=%d ode=%d ok\n", ic, ode);
        }
    printf("ALL OK\n");
    return 0;
}
