/*
 * emri_oracle.c -- plain FP64 CPU oracle for the batched EMRI log-likelihood
 * of Saltas & Oliveri, "emri_mc: A GPU-based Python code for Bayesian
 * inference of EMRI waveforms" (arXiv:2311.17174).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP product
 * path.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or constant with
 * the HIP library; its constants are written out here on purpose.
 *
 * Everything is FP64, written for a reader to check against the paper and
 * against the Analytic Kludge (AK) formulas of Barack & Cutler 2004
 * (Phys. Rev. D 69, 082005; "BC04" below), which the paper cites for the
 * orbital equations, the harmonic amplitudes and the LISA response without
 * printing them (Sec. 2 "Waveform generation").
 *
 * Steps, in the paper's order (Sec. 3 "Overview"):
 *   1. per-walker scalars: validity, z(d_L), Xi(z) [Eq. (6)], propagation
 *      delay Delta T [Eqs. (4)-(5)], overall factor 1/(Xi d_L)
 *   2. orbit: Eq. (1) with Y = {Phi, nu, gamma~, e, alpha}, classical RK4
 *      with a fixed coarse step, stopped at the last stable orbit
 *      (nu_LSO of Sec. 3 "Waveform computation"); or, optionally, an
 *      adaptive embedded Runge-Kutta pair whose continuous extension gives
 *      the same coarse nodes (Sec. 3 "Computational overhead": the ODE
 *      solver is the method's main cost and its choice is open)
 *   3. time-domain waveform: Eq. (2), Peters-Mathews harmonics n=1..n_max,
 *      projected on the two low-frequency LISA channels with Doppler phase
 *      modulation; the orbit is read between coarse nodes by cubic Hermite
 *      interpolation; Bessel functions evaluated per sample
 *   4. FFT: h~(f_k) = dt * sum_j x_j exp(-2 pi i j k / N)  (Sec. 3)
 *   5. likelihood, Eq. (8) read as -1/2 <d - m | d - m> with the noise
 *      weighted inner product, m = (1/Xi d_L) exp(-2 pi i f Delta T) h~
 *      (Eq. (4); the distance factor enters only here, Sec. 3 file list)
 *
 * Readings where the paper is silent or garbled are listed in the design
 * notes of the repository; each is marked "reading" at the place it is used.
 *
 * Parity pins: see tests/test_oracle_*.py.  The spin-orbit and the
 * eccentricity-dependent 1PN terms of dnu/dt and de/dt in the BC04 orbital
 * equations are parity unpinned (no printed values exist to check, and the
 * AK's spin-orbit chirp does not reduce to the test-mass one, so that limit
 * cannot pin it); the 1PN terms at e = 0, the 1PN pericentre advance and the
 * Lense-Thirring precessions are pinned against their textbook forms.  The
 * response (Doppler phase, detector-frame angles, polarisation angle, beta)
 * is pinned against vector constructions of the same geometry, up to the
 * constant orientation offsets, which are a convention.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#else
static int omp_in_parallel(void) { return 1; }
#endif

/* ---- parameter row layout (17 doubles per walker) ---------------------- */
enum {
    I_M = 0,      /* central mass M [Msun]                                   */
    I_MU = 1,     /* compact-object mass mu [Msun]                           */
    I_A = 2,      /* spin S/M^2                                              */
    I_E0 = 3,     /* eccentricity at t = 0                                   */
    I_NU0 = 4,    /* orbital frequency nu at t = 0 [Hz]                      */
    I_PHI0 = 5,   /* mean anomaly Phi at t = 0 [rad]                         */
    I_GT0 = 6,    /* gamma~ at t = 0 [rad]                                   */
    I_AL0 = 7,    /* alpha at t = 0 [rad]                                    */
    I_CLAM = 8,   /* cos(lambda), L-S inclination                            */
    I_THS = 9,    /* source polar angle theta_S (ecliptic) [rad]             */
    I_PHS = 10,   /* source azimuth phi_S [rad]                              */
    I_THK = 11,   /* spin polar angle theta_K [rad]                          */
    I_PHK = 12,   /* spin azimuth phi_K [rad]                                */
    I_DL = 13,    /* luminosity distance d_L [Gpc]                           */
    I_XI0 = 14,   /* Xi_0 of Eq. (6)                                         */
    I_NXI = 15,   /* n of Eq. (6)                                            */
    I_AT = 16,    /* alpha_T of Eq. (3): c_T^2 = 1 + alpha_T, constant       */
    NPAR = 17
};

/* ---- physical constants (SI-derived; masses and distances in seconds) -- */
#define O_PI 3.14159265358979323846
static const double O_TSUN = 4.925490947641267e-6;   /* G Msun / c^3 [s]   */
static const double O_CLIGHT = 299792458.0;           /* [m/s]              */
static const double O_PARSEC = 3.0856775814913673e16; /* [m]                */
static const double O_AU = 1.495978707e11;            /* [m]                */
static const double O_YEAR = 31557600.0;              /* Julian year [s]    */
static const double O_H0 = 67.66;                     /* [km/s/Mpc]         */
static const double O_OMEGA_M = 0.3111;               /* flat LCDM          */

typedef struct {
    double T_obs;        /* observation time [s]                            */
    double dt;           /* sampling interval [s]                           */
    int64_t N;           /* transform length, power of two >= N_valid        */
    int32_t n_harm;      /* n_max of Eq. (2)                                 */
    int32_t coarse_log2; /* coarse ODE step = dt * 2^coarse_log2            */
    int32_t lo_only;     /* test hook: leading-order (Peters-Mathews) ODE    */
    int32_t ic_lso;      /* 1: initial conditions at the LSO, integrated backward */
    int32_t ode;         /* 0: classical RK4 on the nodes; 1: adaptive Dormand-Prince 5(4);
                          * 2: Fehlberg 7(8), node to node */
    int32_t reserved;
    double rtol, atol;   /* tolerances of the adaptive integrators (ode = 1, 2) */
} oracle_cfg;

int oracle_num_threads(void);

static int64_t n_valid_of(const oracle_cfg *c) { return (int64_t)llround(c->T_obs / c->dt); }
static int64_t n_intervals_of(const oracle_cfg *c)
{
    int64_t m = (int64_t)1 << c->coarse_log2;
    return (n_valid_of(c) + m - 1) / m;
}

/* ======================================================================== */
/* Cosmology: d_L(z) for flat LCDM (reading; the paper does not give it).   */
/* ======================================================================== */
static double inv_E(double z)
{
    double a = 1.0 + z;
    return 1.0 / sqrt(O_OMEGA_M * a * a * a + 1.0 - O_OMEGA_M);
}

/* integral_0^z dz'/E(z'): Romberg integration (trapezoid rule with
 * Richardson extrapolation), run until two diagonal estimates agree to
 * 1e-15 relative; the integrand is analytic on [0, z]. */
static double comoving_integral(double z)
{
    if (z <= 0.0) return 0.0;
    double R[2][24];
    double *prev = R[0], *cur = R[1];
    double h = z;
    prev[0] = 0.5 * h * (inv_E(0.0) + inv_E(z));
    for (int k = 1; k < 24; ++k) {
        h *= 0.5;
        double s = 0.0;
        int64_t n = (int64_t)1 << (k - 1);
        for (int64_t i = 0; i < n; ++i) s += inv_E((2 * i + 1) * h);
        cur[0] = 0.5 * prev[0] + h * s;
        double f = 1.0;
        for (int j = 1; j <= k; ++j) {
            f *= 4.0;
            cur[j] = cur[j - 1] + (cur[j - 1] - prev[j - 1]) / (f - 1.0);
        }
        if (k >= 4 && fabs(cur[k] - prev[k - 1]) <= 1e-15 * fabs(cur[k])) return cur[k];
        double *t = prev; prev = cur; cur = t;
    }
    return prev[23];
}

/* Hubble distance c/H0 in seconds of light travel */
static double hubble_distance_s(void)
{
    return (O_CLIGHT / 1000.0 / O_H0) * 1e6 * O_PARSEC / O_CLIGHT;
}

/* d_L(z) in seconds */
double oracle_dl_of_z(double z)
{
    return (1.0 + z) * hubble_distance_s() * comoving_integral(z);
}

/* invert d_L(z) = D (seconds) by Newton's method; d_L is convex increasing,
 * so starting to the right of the root converges monotonically. */
double oracle_z_of_dl(double D)
{
    double DH = hubble_distance_s();
    if (!(D > 0.0)) return 0.0;
    double z = D / DH; /* d_L(D/DH) >= D: right of the root */
    for (int it = 0; it < 200; ++it) {
        double I = comoving_integral(z);
        double f = (1.0 + z) * DH * I - D;
        double fp = DH * I + (1.0 + z) * DH * inv_E(z);
        double dz = f / fp;
        z -= dz;
        if (fabs(dz) <= 1e-16 * (1.0 + z)) break;
    }
    return z;
}

/* ======================================================================== */
/* Step 1: per-walker scalars.                                              */
/* out[8] = {valid, z, Xi, chi [s], DeltaT [s], g = 1/(Xi D), D [s], 0}     */
/* ======================================================================== */
static double nu_lso(double M_s, double e)
{
    /* Sec. 3 "Waveform computation": nu_LSO = c^3/(2 pi G M) ((1-e^2)/(6+2e))^{3/2} */
    return pow((1.0 - e * e) / (6.0 + 2.0 * e), 1.5) / (2.0 * O_PI * M_s);
}

/* ic_lso: the row gives e, Phi, gamma~, alpha at the LSO and nu0 is unused */
static void walker_scalars(const double *p, int ic_lso, double out[8])
{
    memset(out, 0, 8 * sizeof(double));
    for (int i = 0; i < NPAR; ++i)
        if (!isfinite(p[i])) return;
    double M = p[I_M], mu = p[I_MU], a = p[I_A], e0 = p[I_E0], nu0 = p[I_NU0];
    double dl = p[I_DL], at = p[I_AT], cl = p[I_CLAM];
    int ok = (mu > 0.0) && (mu < M) && (a >= 0.0) && (a <= 1.0) && (e0 >= 0.0) &&
             (e0 < 1.0) && (ic_lso || nu0 > 0.0) && (dl > 0.0) && (at > -1.0) && (cl >= -1.0) &&
             (cl <= 1.0);
    if (!ok) return;
    double M_s = M * O_TSUN;
    if (!ic_lso && !(nu0 < nu_lso(M_s, e0))) return;
    double D = dl * 1e9 * O_PARSEC / O_CLIGHT;
    double z = oracle_z_of_dl(D);
    /* Eq. (6) */
    double Xi = p[I_XI0] + (1.0 - p[I_XI0]) / pow(1.0 + z, p[I_NXI]);
    if (!(Xi > 0.0) || !isfinite(Xi)) return;
    double chi = D / (1.0 + z);
    /* reading of Eqs. (3)-(5) for constant alpha_T: the wave crosses the
     * comoving distance chi at speed c_T = sqrt(1 + alpha_T), so it arrives
     * later by (1/c_T - 1) chi/c.  1/c_T - 1 is written without cancellation
     * as -alpha_T / (c_T (1 + c_T)). */
    double ct = sqrt(1.0 + at);
    double dT = -at / (ct * (1.0 + ct)) * chi;
    out[0] = 1.0;
    out[1] = z;
    out[2] = Xi;
    out[3] = chi;
    out[4] = dT;
    out[5] = 1.0 / (Xi * D);
    out[6] = D;
}

int oracle_scalars(const double *params, int64_t B, double *out)
{
    for (int64_t w = 0; w < B; ++w) walker_scalars(params + w * NPAR, 0, out + w * 8);
    return 0;
}

/* ======================================================================== */
/* Step 2: orbital ODE, Eq. (1), right-hand side of BC04 (reading R1).      */
/* y = {Phi, nu, gamma~, e, alpha}                                          */
/* ======================================================================== */
static void ak_rhs(const double y[5], double M_s, double mu_s, double a, double cl,
                   int lo_only, double dy[5])
{
    double nu = y[1], e = y[3];
    double x = 2.0 * O_PI * M_s * nu;          /* PN parameter, Sec. 2 */
    double e2 = e * e, e4 = e2 * e2, e6 = e4 * e2;
    double eps = 1.0 - e2;
    double x23 = pow(x, 2.0 / 3.0);

    dy[0] = 2.0 * O_PI * nu;

    /* d nu / dt */
    double brace = (1.0 + 73.0 / 24.0 * e2 + 37.0 / 96.0 * e4) * eps;
    if (!lo_only) {
        brace += x23 * (1273.0 / 336.0 - 2561.0 / 224.0 * e2 - 3885.0 / 128.0 * e4 -
                        13147.0 / 5376.0 * e6);
        brace -= x * a * cl * pow(eps, -0.5) *
                 (73.0 / 12.0 + 1211.0 / 24.0 * e2 + 3143.0 / 96.0 * e4 + 65.0 / 64.0 * e6);
    }
    dy[1] = 96.0 / (10.0 * O_PI) * (mu_s / (M_s * M_s * M_s)) * pow(x, 11.0 / 3.0) *
            pow(eps, -4.5) * brace;

    /* d gamma~ / dt */
    dy[2] = 6.0 * O_PI * nu * x23 / eps * (1.0 + 0.25 * x23 / eps * (26.0 - 15.0 * e2)) -
            12.0 * O_PI * nu * a * cl * x * pow(eps, -1.5);

    /* d e / dt */
    double inner = (304.0 + 121.0 * e2) * eps;
    if (!lo_only) {
        inner = (304.0 + 121.0 * e2) * eps * (1.0 + 12.0 * x23) -
                x23 / 56.0 * (8.0 * 16705.0 + 12.0 * 9082.0 * e2 - 25211.0 * e4);
    }
    double de = -(e / 15.0) * (mu_s / (M_s * M_s)) * pow(eps, -3.5) * pow(x, 8.0 / 3.0) * inner;
    if (!lo_only) {
        de += e * (mu_s / (M_s * M_s)) * a * cl * pow(x, 11.0 / 3.0) * pow(eps, -4.0) *
              (1364.0 / 5.0 + 5032.0 / 15.0 * e2 + 263.0 / 10.0 * e4);
    }
    dy[3] = de;

    /* d alpha / dt */
    dy[4] = 4.0 * O_PI * nu * a * x * pow(eps, -1.5);
}

/* exported for tests: right-hand side at a state, for one parameter row */
int oracle_rhs(const double *y5, const double *prow, int lo_only, double *dy5)
{
    ak_rhs(y5, prow[I_M] * O_TSUN, prow[I_MU] * O_TSUN, prow[I_A], prow[I_CLAM], lo_only, dy5);
    return 0;
}

/* node k is before the last stable orbit: nu < nu_LSO(e), i.e.
 * x^{2/3} (6 + 2e) < 1 - e^2 (Sec. 3), with a finite state and 0 <= e < 1 */
static int node_ok(const double y[5], double M_s)
{
    double nu = y[1], e = y[3];
    if (!isfinite(y[0]) || !isfinite(nu) || !isfinite(y[2]) || !isfinite(e) || !isfinite(y[4]))
        return 0;
    if (!(e >= 0.0 && e < 1.0 && nu > 0.0)) return 0;
    double x = 2.0 * O_PI * M_s * nu;
    return pow(x, 2.0 / 3.0) * (6.0 + 2.0 * e) < 1.0 - e * e;
}

/* Classical RK4 on t_k = k h, h = dt 2^coarse_log2 (reading R3).
 * orb[(K+1)][10]: Y_k then f(Y_k).  Returns K_w, the index of the last node
 * before the LSO (reading R5); nodes after it are zero. */
/* a finite state with 0 <= e < 1 and nu > 0 (the backward integration has
 * no LSO to stop at) */
static int node_sane(const double y[5])
{
    for (int i = 0; i < 5; ++i)
        if (!isfinite(y[i])) return 0;
    return y[3] >= 0.0 && y[3] < 1.0 && y[1] > 0.0;
}

/* The paper's convention (Sec. 3 "Waveform computation"): the state is given
 * at the last stable orbit, nu = nu_LSO(e_LSO), and the orbit is integrated
 * backward over the window.  Reading: the LSO is node K (the end of the last
 * coarse interval covering the window); classical RK4 with step -h fills
 * nodes K-1 .. 0.  Returns K, or -1 if the state leaves the physical range
 * on the way back. */
static int64_t walker_orbit_lso(const double *p, const oracle_cfg *c, double *orb)
{
    int64_t K = n_intervals_of(c);
    double h = -c->dt * (double)((int64_t)1 << c->coarse_log2);
    double M_s = p[I_M] * O_TSUN, mu_s = p[I_MU] * O_TSUN, a = p[I_A], cl = p[I_CLAM];
    memset(orb, 0, (size_t)(K + 1) * 10 * sizeof(double));
    double y[5] = {p[I_PHI0], nu_lso(M_s, p[I_E0]), p[I_GT0], p[I_E0], p[I_AL0]};
    double k1[5], k2[5], k3[5], k4[5], yt[5];
    ak_rhs(y, M_s, mu_s, a, cl, c->lo_only, k1);
    for (int i = 0; i < 5; ++i) { orb[K * 10 + i] = y[i]; orb[K * 10 + 5 + i] = k1[i]; }
    for (int64_t k = K; k > 0; --k) {
        for (int i = 0; i < 5; ++i) yt[i] = y[i] + 0.5 * h * k1[i];
        ak_rhs(yt, M_s, mu_s, a, cl, c->lo_only, k2);
        for (int i = 0; i < 5; ++i) yt[i] = y[i] + 0.5 * h * k2[i];
        ak_rhs(yt, M_s, mu_s, a, cl, c->lo_only, k3);
        for (int i = 0; i < 5; ++i) yt[i] = y[i] + h * k3[i];
        ak_rhs(yt, M_s, mu_s, a, cl, c->lo_only, k4);
        for (int i = 0; i < 5; ++i) y[i] = y[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        if (!node_sane(y)) return -1;
        ak_rhs(y, M_s, mu_s, a, cl, c->lo_only, k1);
        double *o = orb + (k - 1) * 10;
        for (int i = 0; i < 5; ++i) { o[i] = y[i]; o[5 + i] = k1[i]; }
    }
    return K;
}

static int64_t walker_orbit_dp5(const double *p, const oracle_cfg *c, double *orb, int32_t *stats);
static int64_t walker_orbit_rk78(const double *p, const oracle_cfg *c, double *orb, int32_t *stats);
static int cfg_ok(const oracle_cfg *c);

static int64_t walker_orbit(const double *p, const oracle_cfg *c, double *orb)
{
    if (c->ode == 1) return walker_orbit_dp5(p, c, orb, NULL);
    if (c->ode == 2) return walker_orbit_rk78(p, c, orb, NULL);
    if (c->ic_lso) return walker_orbit_lso(p, c, orb);
    int64_t K = n_intervals_of(c);
    double h = c->dt * (double)((int64_t)1 << c->coarse_log2);
    double M_s = p[I_M] * O_TSUN, mu_s = p[I_MU] * O_TSUN, a = p[I_A], cl = p[I_CLAM];
    memset(orb, 0, (size_t)(K + 1) * 10 * sizeof(double));
    double y[5] = {p[I_PHI0], p[I_NU0], p[I_GT0], p[I_E0], p[I_AL0]};
    double k1[5], k2[5], k3[5], k4[5], yt[5];
    ak_rhs(y, M_s, mu_s, a, cl, c->lo_only, k1);
    for (int i = 0; i < 5; ++i) { orb[i] = y[i]; orb[5 + i] = k1[i]; }
    int64_t Kw = K;
    for (int64_t k = 0; k < K; ++k) {
        for (int i = 0; i < 5; ++i) yt[i] = y[i] + 0.5 * h * k1[i];
        ak_rhs(yt, M_s, mu_s, a, cl, c->lo_only, k2);
        for (int i = 0; i < 5; ++i) yt[i] = y[i] + 0.5 * h * k2[i];
        ak_rhs(yt, M_s, mu_s, a, cl, c->lo_only, k3);
        for (int i = 0; i < 5; ++i) yt[i] = y[i] + h * k3[i];
        ak_rhs(yt, M_s, mu_s, a, cl, c->lo_only, k4);
        for (int i = 0; i < 5; ++i) y[i] = y[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        if (!node_ok(y, M_s)) { Kw = k; break; }   /* node k+1 is past the LSO */
        ak_rhs(y, M_s, mu_s, a, cl, c->lo_only, k1);
        double *o = orb + (k + 1) * 10;
        for (int i = 0; i < 5; ++i) { o[i] = y[i]; o[5 + i] = k1[i]; }
    }
    return Kw;
}

/* ------------------------------------------------------------------------ */
/* Adaptive orbit (cfg.ode = 1).  Reading: the paper integrates Eq. (1)     */
/* with a standard adaptive Runge-Kutta solver and names the solver as the  */
/* main cost (Sec. 3 "Waveform computation", "Computational overhead").     */
/* Here: the embedded 5(4) pair of Dormand & Prince (J. Comput. Appl. Math. */
/* 6 (1980) 19), local extrapolation (the order-5 solution is kept), the    */
/* standard step-size control of Hairer, Norsett & Wanner, "Solving ODEs I" */
/* Sec. II.4, and the order-4 continuous extension of the pair (Shampine    */
/* 1986, in the form of HNW Sec. II.6) evaluated at the coarse nodes         */
/* t_k = k h_c, so that the orbit reaches the waveform step in the same      */
/* layout as the RK4 path: Y_k and f(Y_k), with f evaluated at the           */
/* interpolated state.                                                      */
/*   error norm    sqrt(mean_i (err_i / sc_i)^2) over the five components,  */
/*                 err = H sum_j (b_j - b*_j) k_j,                          */
/*                 sc_i = atol + rtol max(|y_i|, |y1_i|), except nu: rtol    */
/*                 max(|nu|, |nu1|) alone (nu is a frequency, always > 0)   */
/*   accept        err <= 1; then H <- H min(5, max(0.2, 0.9 err^(-1/5)))   */
/*                 (factor at most 1 right after a rejection)               */
/*   reject        H <- H max(0.2, 0.9 err^(-1/5)) (a non-finite err: 0.2)  */
/*   first step    one coarse interval; the last step is cut to end exactly */
/*                 on the end of the window                                 */
/*   stop          forward: at the first node past the LSO (K_w = the one   */
/*                 before it, as with RK4); backward from the LSO: a node   */
/*                 outside the physical range makes the walker invalid      */
/*   budget        4 K + 64 step attempts, else the walker is invalid       */
/* ------------------------------------------------------------------------ */
static const double DP_C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
static const double DP_A[7][6] = {
    {0.0},
    {1.0 / 5.0},
    {3.0 / 40.0, 9.0 / 40.0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0}};
/* order-5 weights (the last row of A: the seventh stage is f(y1)) */
static const double DP_B[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0,
                               -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
/* b - b*, b* the embedded order-4 weights */
static const double DP_E[7] = {71.0 / 57600.0, 0.0, -71.0 / 16695.0, 71.0 / 1920.0,
                               -17253.0 / 339200.0, 22.0 / 525.0, -1.0 / 40.0};
/* continuous extension, fifth coefficient vector */
static const double DP_D[7] = {-12715105075.0 / 11282082432.0, 0.0,
                               87487479700.0 / 32700410799.0, -10690763975.0 / 1880347072.0,
                               701980252875.0 / 199316789632.0, -1453857185.0 / 822651844.0,
                               69997945.0 / 29380423.0};

int oracle_dp5_tableau(double *out /* [77]: c[7], A[7][7], b[7], b - b*[7], d[7] */)
{
    for (int i = 0; i < 7; ++i) {
        out[i] = DP_C[i];
        for (int j = 0; j < 7; ++j) out[7 + 7 * i + j] = (j < 6) ? DP_A[i][j] : 0.0;
        out[56 + i] = DP_B[i];
        out[63 + i] = DP_E[i];
        out[70 + i] = DP_D[i];
    }
    return 0;
}

/* stats (optional): [0] accepted steps, [1] rejected steps */
static int64_t walker_orbit_dp5(const double *p, const oracle_cfg *c, double *orb, int32_t *stats)
{
    const int64_t K = n_intervals_of(c);
    const double hc = c->dt * (double)((int64_t)1 << c->coarse_log2);
    const double M_s = p[I_M] * O_TSUN, mu_s = p[I_MU] * O_TSUN, a = p[I_A], cl = p[I_CLAM];
    const int back = c->ic_lso != 0;
    const double t_end = back ? 0.0 : (double)K * hc;
    const int64_t budget = 4 * K + 64;
    memset(orb, 0, (size_t)(K + 1) * 10 * sizeof(double));
    if (stats) stats[0] = stats[1] = 0;

    double y[5], f[5];
    int64_t node;     /* the next node to fill */
    double t;
    if (back) {
        y[0] = p[I_PHI0]; y[1] = nu_lso(M_s, p[I_E0]); y[2] = p[I_GT0]; y[3] = p[I_E0];
        y[4] = p[I_AL0];
        t = (double)K * hc;
        node = K - 1;
    } else {
        y[0] = p[I_PHI0]; y[1] = p[I_NU0]; y[2] = p[I_GT0]; y[3] = p[I_E0]; y[4] = p[I_AL0];
        t = 0.0;
        node = 1;
    }
    ak_rhs(y, M_s, mu_s, a, cl, c->lo_only, f);
    double *o0 = orb + (back ? K : 0) * 10;
    for (int i = 0; i < 5; ++i) { o0[i] = y[i]; o0[5 + i] = f[i]; }

    double H = back ? -hc : hc;
    int rejected = 0;
    for (int64_t att = 0; att < budget; ++att) {
        /* the step, cut to end on the end of the window */
        double Hs = H;
        int last = 0;
        if (back ? (t + Hs <= t_end) : (t + Hs >= t_end)) { Hs = t_end - t; last = 1; }

        double k[7][5], ys[5];
        for (int i = 0; i < 5; ++i) k[0][i] = f[i];
        for (int s = 1; s < 7; ++s) {
            for (int i = 0; i < 5; ++i) {
                double acc = 0.0;
                for (int j = 0; j < s; ++j) acc += DP_A[s][j] * k[j][i];
                ys[i] = y[i] + Hs * acc;
            }
            ak_rhs(ys, M_s, mu_s, a, cl, c->lo_only, k[s]);
        }
        /* ys now holds y1, the order-5 solution (seventh stage state), and
         * k[6] = f(y1) */
        double sum = 0.0;
        for (int i = 0; i < 5; ++i) {
            double err = 0.0;
            for (int j = 0; j < 7; ++j) err += DP_E[j] * k[j][i];
            err *= Hs;
            double sc = (i == 1 ? 0.0 : c->atol) + c->rtol * fmax(fabs(y[i]), fabs(ys[i]));
            sum += (err / sc) * (err / sc);
        }
        double en = sqrt(sum / 5.0);
        double fac = fmax(0.2, 0.9 * pow(en, -0.2));
        if (!(en <= 1.0)) {            /* rejected (a NaN norm too) */
            H = Hs * fac;
            rejected = 1;
            if (stats) stats[1]++;
            continue;
        }
        if (stats) stats[0]++;
        double t1 = last ? t_end : t + Hs;

        /* continuous extension on [t, t1]:
         * y(th) = r1 + th (r2 + (1 - th) (r3 + th (r4 + (1 - th) r5))) */
        double r1[5], r2[5], r3[5], r4[5], r5[5];
        for (int i = 0; i < 5; ++i) {
            r1[i] = y[i];
            r2[i] = ys[i] - y[i];
            r3[i] = Hs * k[0][i] - r2[i];
            r4[i] = r2[i] - Hs * k[6][i] - r3[i];
            double dd = 0.0;
            for (int j = 0; j < 7; ++j) dd += DP_D[j] * k[j][i];
            r5[i] = Hs * dd;
        }
        /* the coarse nodes in (t, t1] */
        while (back ? (node >= 0 && (double)node * hc >= t1)
                    : (node <= K && (double)node * hc <= t1)) {
            double th = ((double)node * hc - t) / Hs, yk[5], fk[5];
            for (int i = 0; i < 5; ++i)
                yk[i] = r1[i] + th * (r2[i] + (1.0 - th) * (r3[i] + th * (r4[i] + (1.0 - th) * r5[i])));
            if (back) {
                if (!node_sane(yk)) return -1;
            } else if (!node_ok(yk, M_s)) {
                return node - 1;       /* node is past the LSO */
            }
            ak_rhs(yk, M_s, mu_s, a, cl, c->lo_only, fk);
            double *o = orb + node * 10;
            for (int i = 0; i < 5; ++i) { o[i] = yk[i]; o[5 + i] = fk[i]; }
            node += back ? -1 : 1;
        }
        if (last) return K;
        for (int i = 0; i < 5; ++i) { y[i] = ys[i]; f[i] = k[6][i]; }
        t = t1;
        H = Hs * fmin(rejected ? 1.0 : 5.0, fac);
        rejected = 0;
    }
    return -1;                         /* step budget exhausted */
}

/* ------------------------------------------------------------------------ */
/* Seventh-order orbit (cfg.ode = 2).  Reading: the "7th-order Runge-Kutta   */
/* scheme" of Sec. 3 ("Waveform computation") is taken as Fehlberg's         */
/* embedded 7(8) pair (NASA TR R-287, 1968; 13 stages), the order-7          */
/* solution kept and the order-8 one used for the error estimate only.       */
/* The integration runs node to node: a step never passes the next coarse   */
/* node t_k = k h_c, so every node value is a step end of the method itself */
/* and no continuous extension enters.                                      */
/*   error estimate err = H (b7 - b8) . k = H 41/840 (k1 + k11 - k12 - k13)  */
/*   error norm    as for ode = 1 (rms over the five components, nu on rtol */
/*                 alone)                                                   */
/*   accept        err <= 1; then H <- H min(5, max(0.2, 0.9 err^(-1/8)))   */
/*                 (factor at most 1 right after a rejection), H the step   */
/*                 just taken                                               */
/*   reject        H <- H max(0.2, 0.9 err^(-1/8)) (a non-finite err: 0.2)  */
/*   first step    one coarse interval; a step that would pass the next     */
/*                 node is cut to end on it                                 */
/*   stop          forward: at the first step end past the LSO (K_w = the   */
/*                 last node filled before it); backward from the LSO: a    */
/*                 step end outside the physical range makes the walker     */
/*                 invalid                                                  */
/*   budget        4 K + 64 step attempts, else the walker is invalid       */
/* ------------------------------------------------------------------------ */
static const double F78_C[13] = {0.0,       2.0 / 27.0, 1.0 / 9.0, 1.0 / 6.0, 5.0 / 12.0,
                                 1.0 / 2.0, 5.0 / 6.0,  1.0 / 6.0, 2.0 / 3.0, 1.0 / 3.0,
                                 1.0,       0.0,        1.0};
static const double F78_A[13][12] = {
    {0.0},
    {2.0 / 27.0},
    {1.0 / 36.0, 1.0 / 12.0},
    {1.0 / 24.0, 0.0, 1.0 / 8.0},
    {5.0 / 12.0, 0.0, -25.0 / 16.0, 25.0 / 16.0},
    {1.0 / 20.0, 0.0, 0.0, 1.0 / 4.0, 1.0 / 5.0},
    {-25.0 / 108.0, 0.0, 0.0, 125.0 / 108.0, -65.0 / 27.0, 125.0 / 54.0},
    {31.0 / 300.0, 0.0, 0.0, 0.0, 61.0 / 225.0, -2.0 / 9.0, 13.0 / 900.0},
    {2.0, 0.0, 0.0, -53.0 / 6.0, 704.0 / 45.0, -107.0 / 9.0, 67.0 / 90.0, 3.0},
    {-91.0 / 108.0, 0.0, 0.0, 23.0 / 108.0, -976.0 / 135.0, 311.0 / 54.0, -19.0 / 60.0,
     17.0 / 6.0, -1.0 / 12.0},
    {2383.0 / 4100.0, 0.0, 0.0, -341.0 / 164.0, 4496.0 / 1025.0, -301.0 / 82.0,
     2133.0 / 4100.0, 45.0 / 82.0, 45.0 / 164.0, 18.0 / 41.0},
    {3.0 / 205.0, 0.0, 0.0, 0.0, 0.0, -6.0 / 41.0, -3.0 / 205.0, -3.0 / 41.0, 3.0 / 41.0,
     6.0 / 41.0},
    {-1777.0 / 4100.0, 0.0, 0.0, -341.0 / 164.0, 4496.0 / 1025.0, -289.0 / 82.0,
     2193.0 / 4100.0, 51.0 / 82.0, 33.0 / 164.0, 12.0 / 41.0, 0.0, 1.0}};
/* order-7 weights (kept) and order-8 weights (error estimate) */
static const double F78_B7[13] = {41.0 / 840.0, 0.0, 0.0, 0.0, 0.0, 34.0 / 105.0, 9.0 / 35.0,
                                  9.0 / 35.0, 9.0 / 280.0, 9.0 / 280.0, 41.0 / 840.0, 0.0, 0.0};
static const double F78_B8[13] = {0.0, 0.0, 0.0, 0.0, 0.0, 34.0 / 105.0, 9.0 / 35.0,
                                  9.0 / 35.0, 9.0 / 280.0, 9.0 / 280.0, 0.0, 41.0 / 840.0,
                                  41.0 / 840.0};

int oracle_rk78_tableau(double *out /* [195]: c[13], A[13][12], b7[13], b8[13] */)
{
    for (int i = 0; i < 13; ++i) {
        out[i] = F78_C[i];
        for (int j = 0; j < 12; ++j) out[13 + 12 * i + j] = F78_A[i][j];
        out[169 + i] = F78_B7[i];
        out[182 + i] = F78_B8[i];
    }
    return 0;
}

/* stats (optional): [0] accepted steps, [1] rejected steps */
static int64_t walker_orbit_rk78(const double *p, const oracle_cfg *c, double *orb, int32_t *stats)
{
    const int64_t K = n_intervals_of(c);
    const double hc = c->dt * (double)((int64_t)1 << c->coarse_log2);
    const double M_s = p[I_M] * O_TSUN, mu_s = p[I_MU] * O_TSUN, a = p[I_A], cl = p[I_CLAM];
    const int back = c->ic_lso != 0;
    const int64_t budget = 4 * K + 64;
    memset(orb, 0, (size_t)(K + 1) * 10 * sizeof(double));
    if (stats) stats[0] = stats[1] = 0;

    double y[5], f[5];
    int64_t node;     /* the next node to fill */
    double t;
    if (back) {
        y[0] = p[I_PHI0]; y[1] = nu_lso(M_s, p[I_E0]); y[2] = p[I_GT0]; y[3] = p[I_E0];
        y[4] = p[I_AL0];
        t = (double)K * hc;
        node = K - 1;
    } else {
        y[0] = p[I_PHI0]; y[1] = p[I_NU0]; y[2] = p[I_GT0]; y[3] = p[I_E0]; y[4] = p[I_AL0];
        t = 0.0;
        node = 1;
    }
    ak_rhs(y, M_s, mu_s, a, cl, c->lo_only, f);
    double *o0 = orb + (back ? K : 0) * 10;
    for (int i = 0; i < 5; ++i) { o0[i] = y[i]; o0[5 + i] = f[i]; }
    if (K == 0) return 0;

    double H = back ? -hc : hc;
    int rejected = 0;
    for (int64_t att = 0; att < budget; ++att) {
        /* the step, cut to end on the next node */
        const double tn = (double)node * hc;
        double Hs = H;
        int land = 0;
        if (back ? (t + Hs <= tn) : (t + Hs >= tn)) { Hs = tn - t; land = 1; }

        double k[13][5], ys[5], y1[5];
        for (int i = 0; i < 5; ++i) k[0][i] = f[i];
        for (int s = 1; s < 13; ++s) {
            for (int i = 0; i < 5; ++i) {
                double acc = 0.0;
                for (int j = 0; j < s; ++j) acc += F78_A[s][j] * k[j][i];
                ys[i] = y[i] + Hs * acc;
            }
            ak_rhs(ys, M_s, mu_s, a, cl, c->lo_only, k[s]);
        }
        double sum = 0.0;
        for (int i = 0; i < 5; ++i) {
            double acc = 0.0, err = 0.0;
            for (int j = 0; j < 13; ++j) {
                acc += F78_B7[j] * k[j][i];
                err += (F78_B7[j] - F78_B8[j]) * k[j][i];
            }
            y1[i] = y[i] + Hs * acc;
            err *= Hs;
            double sc = (i == 1 ? 0.0 : c->atol) + c->rtol * fmax(fabs(y[i]), fabs(y1[i]));
            sum += (err / sc) * (err / sc);
        }
        double en = sqrt(sum / 5.0);
        double fac = fmax(0.2, 0.9 * pow(en, -0.125));
        if (!(en <= 1.0)) {            /* rejected (a NaN norm too) */
            H = Hs * fac;
            rejected = 1;
            if (stats) stats[1]++;
            continue;
        }
        if (stats) stats[0]++;
        if (back) {
            if (!node_sane(y1)) return -1;
        } else if (!node_ok(y1, M_s)) {
            return node - 1;           /* past the LSO before node `node` */
        }
        for (int i = 0; i < 5; ++i) y[i] = y1[i];
        ak_rhs(y, M_s, mu_s, a, cl, c->lo_only, f);
        t = land ? tn : t + Hs;
        if (land) {
            double *o = orb + node * 10;
            for (int i = 0; i < 5; ++i) { o[i] = y[i]; o[5 + i] = f[i]; }
            if (back ? node == 0 : node == K) return K;
            node += back ? -1 : 1;
        }
        H = Hs * fmin(rejected ? 1.0 : 5.0, fac);
        rejected = 0;
    }
    return -1;                         /* step budget exhausted */
}

int oracle_orbit_steps(const double *params, int64_t B, const oracle_cfg *c, int32_t *steps /* [B][2] */)
{
    if (!cfg_ok(c) || (c->ode != 1 && c->ode != 2)) return -1;
    int64_t K = n_intervals_of(c);
    double *orb = (double *)malloc((size_t)(K + 1) * 10 * sizeof(double));
    for (int64_t w = 0; w < B; ++w) {
        steps[2 * w] = steps[2 * w + 1] = 0;
        double s[8];
        walker_scalars(params + w * NPAR, c->ic_lso, s);
        if (s[0] == 0.0) continue;
        if (c->ode == 1) walker_orbit_dp5(params + w * NPAR, c, orb, steps + 2 * w);
        else walker_orbit_rk78(params + w * NPAR, c, orb, steps + 2 * w);
    }
    free(orb);
    return 0;
}

int oracle_orbit(const double *params, int64_t B, const oracle_cfg *c, double *orb, int32_t *Kw)
{
    if (!cfg_ok(c)) return -1;
    int64_t K = n_intervals_of(c);
    for (int64_t w = 0; w < B; ++w) {
        double s[8];
        walker_scalars(params + w * NPAR, c->ic_lso, s);
        double *o = orb + w * (K + 1) * 10;
        if (s[0] == 0.0) {
            memset(o, 0, (size_t)(K + 1) * 10 * sizeof(double));
            Kw[w] = -1;
            continue;
        }
        Kw[w] = (int32_t)walker_orbit(params + w * NPAR, c, o);
    }
    return 0;
}

/* cubic Hermite on [t_k, t_k + h] from values and derivatives, u in [0,1] */
static double hermite(double y0, double d0, double y1, double d1, double h, double u)
{
    double u2 = u * u, u3 = u2 * u;
    return (2.0 * u3 - 3.0 * u2 + 1.0) * y0 + (u3 - 2.0 * u2 + u) * h * d0 +
           (-2.0 * u3 + 3.0 * u2) * y1 + (u3 - u2) * h * d1;
}

double oracle_hermite(double y0, double d0, double y1, double d1, double h, double u)
{
    return hermite(y0, d0, y1, d1, h, u);
}

/* ======================================================================== */
/* Bessel functions J_k(x), k = 0..kmax, by Miller's backward recurrence    */
/* J_{k-1} = (2k/x) J_k - J_{k+1}, normalised with J_0 + 2 sum J_{2k} = 1   */
/* (Abramowitz & Stegun 9.1.27 and 9.1.46).                                  */
/* ======================================================================== */
static void bessel_j_upto(double x, int kmax, double *J /* [kmax+1] */)
{
    for (int k = 0; k <= kmax; ++k) J[k] = 0.0;
    if (x == 0.0) { J[0] = 1.0; return; }
    double ax = fabs(x);
    int top = (kmax > (int)ax ? kmax : (int)ax);
    int start = top + 24 + (int)sqrt(160.0 * (top + 1));
    if (start & 1) start += 1;
    double jp1 = 0.0, jk = 1e-300, norm = 0.0;
    for (int k = start; k >= 1; --k) {
        double jm1 = (2.0 * k / ax) * jk - jp1;   /* J_{k-1} */
        jp1 = jk;
        jk = jm1;
        if ((k - 1) <= kmax) J[k - 1] = jk;
        if (((k - 1) & 1) == 0 && (k - 1) > 0) norm += 2.0 * jk;
        if (fabs(jk) > 1e250) {                   /* rescale everything kept */
            jk *= 1e-250; jp1 *= 1e-250; norm *= 1e-250;
            for (int i = 0; i <= kmax; ++i) J[i] *= 1e-250;
        }
    }
    norm += jk; /* + J_0 */
    for (int k = 0; k <= kmax; ++k) J[k] /= norm;
    if (x < 0.0)
        for (int k = 1; k <= kmax; k += 2) J[k] = -J[k];
}

/* J_n(x) for any integer n (J_{-n} = (-1)^n J_n) */
double oracle_besselj(int n, double x)
{
    int an = n < 0 ? -n : n;
    double *J = (double *)malloc((size_t)(an + 1) * sizeof(double));
    bessel_j_upto(x, an, J);
    double v = J[an];
    free(J);
    if (n < 0 && (an & 1)) v = -v;
    return v;
}

static double jn_signed(const double *J, int k)
{
    if (k >= 0) return J[k];
    return (k & 1) ? -J[-k] : J[-k];
}

/* Peters-Mathews harmonic coefficients as used by BC04 (Eq. (2) of the
 * paper with amplitudes of Peters & Mathews): for X = n e,
 *   P_n = J_{n-2} - 2e J_{n-1} + (2/n) J_n + 2e J_{n+1} - J_{n+2}
 *   Q_n = sqrt(1-e^2) (J_{n-2} - 2 J_n + J_{n+2})
 *   R_n = J_n
 * J holds J_0..J_{n+2}(X). */
static void pm_coeffs_from(int n, double e, const double *J, double *P, double *Q, double *R)
{
    double jm2 = jn_signed(J, n - 2), jm1 = jn_signed(J, n - 1), j0 = J[n], jp1 = J[n + 1],
           jp2 = J[n + 2];
    *P = jm2 - 2.0 * e * jm1 + (2.0 / n) * j0 + 2.0 * e * jp1 - jp2;
    *Q = sqrt(1.0 - e * e) * (jm2 - 2.0 * j0 + jp2);
    *R = j0;
}

int oracle_pm_coeffs(int n, double e, double *out3)
{
    double J[128];
    if (n < 1 || n + 2 >= 128) return -1;
    bessel_j_upto(n * e, n + 2, J);
    pm_coeffs_from(n, e, J, &out3[0], &out3[1], &out3[2]);
    return 0;
}

/* LISA low-frequency antenna patterns (BC04, after Cutler 1998) */
static void antenna(double cth, double phi, double psi, double *Fp, double *Fx)
{
    double a = 0.5 * (1.0 + cth * cth);
    *Fp = a * cos(2.0 * phi) * cos(2.0 * psi) - cth * sin(2.0 * phi) * sin(2.0 * psi);
    *Fx = a * cos(2.0 * phi) * sin(2.0 * psi) + cth * sin(2.0 * phi) * cos(2.0 * psi);
}

int oracle_antenna(double cth, double phi, double psi, double *out2)
{
    antenna(cth, phi, psi, &out2[0], &out2[1]);
    return 0;
}

/* ======================================================================== */
/* Step 3: time-domain waveform of one walker at unit distance, GR.         */
/* Writes channels I and II, x[2][N]; optional diagnostics per sample       */
/* diag[N][16] = {h+, hx, A, c_iota, Phi', gamma, cos theta_d, phi_d, psi,   */
/* beta, Phi, nu, gamma~, alpha, e, 0}.                                       */
/* ======================================================================== */
static void walker_waveform(const double *p, const oracle_cfg *c, const double *orb, int64_t Kw,
                            double *x /* [2][N] */, double *diag /* [N][8] or NULL */)
{
    int64_t N = c->N, Nv = n_valid_of(c);
    int64_t m = (int64_t)1 << c->coarse_log2;
    double h = c->dt * (double)m;
    int nh = c->n_harm;
    memset(x, 0, (size_t)(2 * N) * sizeof(double));
    if (diag) memset(diag, 0, (size_t)(16 * N) * sizeof(double));
    if (Kw <= 0) return;

    double M_s = p[I_M] * O_TSUN, mu_s = p[I_MU] * O_TSUN;
    double cl = p[I_CLAM], sl = sqrt(1.0 - cl * cl);
    double thS = p[I_THS], phS = p[I_PHS], thK = p[I_THK], phK = p[I_PHK];
    /* source direction N, spin direction S and the basis e1, e2 orthogonal to S */
    double Nv3[3] = {sin(thS) * cos(phS), sin(thS) * sin(phS), cos(thS)};
    double Sv[3] = {sin(thK) * cos(phK), sin(thK) * sin(phK), cos(thK)};
    double e1[3] = {-cos(thK) * cos(phK), -cos(thK) * sin(phK), sin(thK)};
    double e2[3] = {sin(phK), -cos(phK), 0.0};
    double NS = Nv3[0] * Sv[0] + Nv3[1] * Sv[1] + Nv3[2] * Sv[2];
    double R = O_AU / O_CLIGHT; /* 1 AU in light seconds */
    double s3 = sqrt(3.0);

    int64_t jend = Kw * m;
    if (jend > Nv) jend = Nv;
    /* samples are independent: spread them over threads unless this walker
     * already runs inside a walker-parallel region */
#pragma omp parallel if (!omp_in_parallel())
    {
    double *J = (double *)malloc((size_t)(nh + 3) * sizeof(double));
#pragma omp for schedule(static)
    for (int64_t j = 0; j < jend; ++j) {
        int64_t k = j / m;
        double u = (double)(j - k * m) / (double)m;
        const double *o0 = orb + k * 10, *o1 = orb + (k + 1) * 10;
        double Y[5];
        for (int i = 0; i < 5; ++i) Y[i] = hermite(o0[i], o0[5 + i], o1[i], o1[5 + i], h, u);
        double Phi = Y[0], nu = Y[1], gt = Y[2], e = Y[3], al = Y[4];
        double t = (double)j * c->dt;

        /* orbital angular momentum direction, precessing about S */
        double L[3];
        for (int i = 0; i < 3; ++i) L[i] = cl * Sv[i] + sl * (cos(al) * e1[i] + sin(al) * e2[i]);
        double ci = L[0] * Nv3[0] + L[1] * Nv3[1] + L[2] * Nv3[2];
        /* beta: angle from L x N to L x S in the orbital plane */
        double SxL[3] = {Sv[1] * L[2] - Sv[2] * L[1], Sv[2] * L[0] - Sv[0] * L[2],
                         Sv[0] * L[1] - Sv[1] * L[0]};
        double sb = Nv3[0] * SxL[0] + Nv3[1] * SxL[1] + Nv3[2] * SxL[2];
        double cb = NS - ci * cl;
        /* beta is undefined when L is parallel to S or to N (sb = cb = 0 up
         * to rounding); it is taken as 0 there (reading R4) */
        double beta = (sb * sb + cb * cb < 1e-24) ? 0.0 : atan2(sb, cb);
        double gam = gt + beta;

        /* detector position and Doppler phase (BC04) */
        double phib = 2.0 * O_PI * t / O_YEAR;
        double Phid = Phi + 2.0 * O_PI * nu * R * sin(thS) * cos(phib - phS);
        /* detector-plane normal, tilted by 60 degrees */
        double zd[3] = {-0.5 * s3 * cos(phib), -0.5 * s3 * sin(phib), 0.5};
        double cthd = Nv3[0] * zd[0] + Nv3[1] * zd[1] + Nv3[2] * zd[2];
        double phid = phib + atan2(s3 * cos(thS) + sin(thS) * cos(phib - phS),
                                   2.0 * sin(thS) * sin(phib - phS));
        double Lz = L[0] * zd[0] + L[1] * zd[1] + L[2] * zd[2];
        double Lxz[3] = {L[1] * zd[2] - L[2] * zd[1], L[2] * zd[0] - L[0] * zd[2],
                         L[0] * zd[1] - L[1] * zd[0]};
        double NLz = Nv3[0] * Lxz[0] + Nv3[1] * Lxz[1] + Nv3[2] * Lxz[2];
        /* psi is undefined for a face-on or face-off source (L parallel to
         * N); it is taken as 0 there, like beta */
        double yps = Lz - ci * cthd;
        double psi = (yps * yps + NLz * NLz < 1e-24) ? 0.0 : atan2(yps, NLz);
        double FpI, FxI, FpII, FxII;
        antenna(cthd, phid, psi, &FpI, &FxI);
        antenna(cthd, phid - 0.25 * O_PI, psi, &FpII, &FxII);

        /* harmonic sum (Peters-Mathews; unit distance, no 1/d_L) */
        double A = pow(2.0 * O_PI * M_s * nu, 2.0 / 3.0) * mu_s;
        double c2g = cos(2.0 * gam), s2g = sin(2.0 * gam);
        double hp = 0.0, hx = 0.0;
        for (int n = 1; n <= nh; ++n) {
            double P, Q, Rn;
            bessel_j_upto(n * e, n + 2, J);
            pm_coeffs_from(n, e, J, &P, &Q, &Rn);
            double an = -n * A * P * cos(n * Phid);
            double bn = -n * A * Q * sin(n * Phid);
            double cn = 2.0 * A * Rn * cos(n * Phid);
            hp += -(1.0 + ci * ci) * (an * c2g - bn * s2g) + (1.0 - ci * ci) * cn;
            hx += 2.0 * ci * (bn * c2g + an * s2g);
        }
        x[j] = 0.5 * s3 * (FpI * hp + FxI * hx);
        x[N + j] = 0.5 * s3 * (FpII * hp + FxII * hx);
        if (diag) {
            double *d = diag + 16 * j;
            d[0] = hp; d[1] = hx; d[2] = A; d[3] = ci; d[4] = Phid; d[5] = gam; d[6] = cthd;
            d[7] = phid; d[8] = psi; d[9] = beta; d[10] = Phi; d[11] = nu; d[12] = gt;
            d[13] = al; d[14] = e;
        }
    }
    free(J);
    }
}

static int cfg_ok(const oracle_cfg *c)
{
    if (!(c->dt > 0.0) || !(c->T_obs > 0.0) || c->N < 2 || (c->N & (c->N - 1))) return 0;
    if (n_valid_of(c) > c->N || n_valid_of(c) < 1) return 0;
    if (c->n_harm < 1 || c->n_harm > 100 || c->coarse_log2 < 0 || c->coarse_log2 > 30) return 0;
    if (c->ode != 0 && c->ode != 1 && c->ode != 2) return 0;
    if (c->ode != 0 && !(c->rtol >= 1e-13 && c->rtol <= 1e-3 && c->atol >= 0.0 && isfinite(c->atol)))
        return 0;
    return 1;
}

int oracle_waveform(const double *params, int64_t B, const oracle_cfg *c, double *x /* [B][2][N] */)
{
    if (!cfg_ok(c)) return -1;
    int64_t K = n_intervals_of(c);
#pragma omp parallel for schedule(dynamic, 1) if (B >= oracle_num_threads())
    for (int64_t w = 0; w < B; ++w) {
        double s[8];
        const double *p = params + w * NPAR;
        walker_scalars(p, c->ic_lso, s);
        double *xw = x + w * 2 * c->N;
        if (s[0] == 0.0) { memset(xw, 0, (size_t)(2 * c->N) * sizeof(double)); continue; }
        double *orb = (double *)malloc((size_t)(K + 1) * 10 * sizeof(double));
        int64_t Kw = walker_orbit(p, c, orb);
        if (Kw >= 0) walker_waveform(p, c, orb, Kw, xw, NULL);
        else memset(xw, 0, (size_t)(2 * c->N) * sizeof(double));
        free(orb);
    }
    return 0;
}

/* single walker waveform with per-sample diagnostics, for pin tests */
int oracle_waveform_diag(const double *p, const oracle_cfg *c, double *x, double *diag)
{
    if (!cfg_ok(c)) return -1;
    double s[8];
    walker_scalars(p, c->ic_lso, s);
    if (s[0] == 0.0) return -2;
    int64_t K = n_intervals_of(c);
    double *orb = (double *)malloc((size_t)(K + 1) * 10 * sizeof(double));
    int64_t Kw = walker_orbit(p, c, orb);
    if (Kw < 0) { free(orb); return -2; }
    walker_waveform(p, c, orb, Kw, x, diag);
    free(orb);
    return 0;
}

/* ======================================================================== */
/* Step 4: discrete Fourier transform, iterative radix-2 Cooley-Tukey.       */
/* ======================================================================== */
static void fft_inplace(double *re, double *im, int64_t n)
{
    /* bit reversal */
    for (int64_t i = 1, j = 0; i < n; ++i) {
        int64_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double t = re[i]; re[i] = re[j]; re[j] = t;
            t = im[i]; im[i] = im[j]; im[j] = t;
        }
    }
    /* twiddles exp(-2 pi i k / n), k < n/2, from the library cos / sin */
    double *wr = (double *)malloc((size_t)(n / 2 + 1) * sizeof(double));
    double *wi = (double *)malloc((size_t)(n / 2 + 1) * sizeof(double));
    for (int64_t k = 0; k < n / 2; ++k) {
        double ang = 2.0 * O_PI * (double)k / (double)n;
        wr[k] = cos(ang);
        wi[k] = -sin(ang);
    }
    for (int64_t len = 2; len <= n; len <<= 1) {
        int64_t half = len >> 1, step = n / len;
        for (int64_t s = 0; s < n; s += len) {
            for (int64_t q = 0; q < half; ++q) {
                double c = wr[q * step], d = wi[q * step];
                int64_t a = s + q, b = s + q + half;
                double tr = re[b] * c - im[b] * d;
                double ti = re[b] * d + im[b] * c;
                re[b] = re[a] - tr; im[b] = im[a] - ti;
                re[a] += tr; im[a] += ti;
            }
        }
    }
    free(wr);
    free(wi);
}

/* X[m][N/2+1][2] = dt * DFT of each real row x[m][N], bins 0..N/2 */
int oracle_rfft(const double *x, int64_t M, int64_t N, double dt, double *X)
{
    if (N < 2 || (N & (N - 1))) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < M; ++r) {
        double *re = (double *)malloc((size_t)N * sizeof(double));
        double *im = (double *)calloc((size_t)N, sizeof(double));
        memcpy(re, x + r * N, (size_t)N * sizeof(double));
        fft_inplace(re, im, N);
        double *o = X + r * (N / 2 + 1) * 2;
        for (int64_t k = 0; k <= N / 2; ++k) { o[2 * k] = dt * re[k]; o[2 * k + 1] = dt * im[k]; }
        free(re);
        free(im);
    }
    return 0;
}

/* ======================================================================== */
/* Step 5: likelihood.                                                      */
/* ======================================================================== */

/* exp(-2 pi i k phi) with phi = Delta T / (N dt); k*phi is reduced mod 1
 * exactly (the product's rounding error is recovered with an FMA). */
static void delay_phase(int64_t k, double phi_frac, double *cr, double *ci)
{
    double kk = (double)k;
    double p = kk * phi_frac;
    double err = fma(kk, phi_frac, -p);
    double f = (p - floor(p)) + err;
    f -= floor(f);
    *cr = cos(2.0 * O_PI * f);
    *ci = -sin(2.0 * O_PI * f);
}

typedef struct { double s, c; } neumaier;
static void nsum_add(neumaier *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

/* Scalars, orbit, waveform and both channels' spectra of one walker: the
 * spectra (dt * DFT, bins 0..N/2, re/im interleaved) are left at
 * scratch_X + 2N, channel I then II.  Returns 0, or -1 for an invalid walker
 * (outside the physical domain, or an orbit that leaves it backward). */
static int walker_spectrum(const double *p, const oracle_cfg *c, double s[8], double *scratch_x,
                           double *scratch_X)
{
    walker_scalars(p, c->ic_lso, s);
    if (s[0] == 0.0) return -1;
    int64_t N = c->N, K = n_intervals_of(c), H = N / 2 + 1;
    double *orb = (double *)malloc((size_t)(K + 1) * 10 * sizeof(double));
    int64_t Kw = walker_orbit(p, c, orb);
    if (Kw < 0) { free(orb); return -1; }   /* left the physical range backward */
    walker_waveform(p, c, orb, Kw, scratch_x, NULL);
    free(orb);
    /* FFT both channels */
    for (int ch = 0; ch < 2; ++ch) {
        double *re = scratch_X, *im = scratch_X + N;
        memcpy(re, scratch_x + ch * N, (size_t)N * sizeof(double));
        memset(im, 0, (size_t)N * sizeof(double));
        fft_inplace(re, im, N);
        /* keep bins 0..N/2, scaled by dt, interleaved re/im */
        double *spec = scratch_X + 2 * N + ch * 2 * H;
        for (int64_t k = 0; k < H; ++k) { spec[2 * k] = c->dt * re[k]; spec[2 * k + 1] = c->dt * im[k]; }
    }
    return 0;
}

/* lnL = -1/2 sum_{channels} sum_{k=1}^{N/2-1} (4 df / S_k) |d_k - m_k|^2
 * (reading R8) from a walker's spectra (walker_spectrum) and scalars */
static double spectrum_loglike(const double s[8], const double *spectra, const double *data,
                               const double *psd, const oracle_cfg *c)
{
    int64_t N = c->N, H = N / 2 + 1;
    double g = s[5], dT = s[4];
    double df = 1.0 / ((double)N * c->dt);
    double phi = dT / ((double)N * c->dt);
    phi -= floor(phi);
    neumaier acc = {0.0, 0.0};
    for (int ch = 0; ch < 2; ++ch) {
        const double *spec = spectra + ch * 2 * H;
        const double *d = data + ch * 2 * H;
        for (int64_t k = 1; k < N / 2; ++k) {
            double cr, ci;
            delay_phase(k, phi, &cr, &ci);
            double hr = spec[2 * k], hi = spec[2 * k + 1];
            double mr = g * (cr * hr - ci * hi);
            double mi = g * (cr * hi + ci * hr);
            double rr = d[2 * k] - mr, ri = d[2 * k + 1] - mi;
            nsum_add(&acc, (4.0 * df / psd[k]) * (rr * rr + ri * ri));
        }
    }
    return -0.5 * (acc.s + acc.c);
}

static double walker_loglike(const double *p, const double *data, const double *psd,
                             const oracle_cfg *c, double *scratch_x, double *scratch_X)
{
    double s[8];
    if (walker_spectrum(p, c, s, scratch_x, scratch_X)) return -INFINITY;
    return spectrum_loglike(s, scratch_X + 2 * c->N, data, psd, c);
}

/* ------------------------------------------------------------------------ */
/* Frequency-dependent propagation (the variant of Sec. 2 "Waveform           */
/* propagation" where alpha_M and alpha_T depend on f, given there as power   */
/* series in f / f*).  Reading: the series coefficients are constant in z,    */
/*   alpha_M(f) = sum_n m_n (f/f*)^n,                                         */
/*   alpha_T(f) = alpha_T(row) + sum_n t_n (f/f*)^n.                          */
/* The friction integral of Eq. (5), (1/2) int_0^z alpha_M / (1 + z') dz',    */
/* is then alpha_M(f) ln(1 + z) / 2, so the amplitude carries the extra       */
/* factor (1 + z)^(-alpha_M(f)/2) on top of Eq. (6); the delay is the         */
/* constant-speed reading of Eqs. (4)-(5) at each frequency,                  */
/* Delta T(f) = (1/c_T(f) - 1) chi / c with c_T(f)^2 = 1 + alpha_T(f).        */
/* A bin with 1 + alpha_T(f) <= 0 makes the walker invalid (lnL = -inf).      */
/* ------------------------------------------------------------------------ */
static double walker_loglike_fmg(const double *p, const double *coef, int P, double f_star,
                                 const double *data, const double *psd, const oracle_cfg *c,
                                 double *scratch_x, double *scratch_X)
{
    double s[8];
    walker_scalars(p, c->ic_lso, s);
    if (s[0] == 0.0) return -INFINITY;
    int64_t N = c->N, K = n_intervals_of(c), H = N / 2 + 1;
    double *orb = (double *)malloc((size_t)(K + 1) * 10 * sizeof(double));
    int64_t Kw = walker_orbit(p, c, orb);
    if (Kw < 0) { free(orb); return -INFINITY; }   /* left the physical range backward */
    walker_waveform(p, c, orb, Kw, scratch_x, NULL);
    free(orb);
    for (int ch = 0; ch < 2; ++ch) {
        double *re = scratch_X, *im = scratch_X + N;
        memcpy(re, scratch_x + ch * N, (size_t)N * sizeof(double));
        memset(im, 0, (size_t)N * sizeof(double));
        fft_inplace(re, im, N);
        double *spec = scratch_X + 2 * N + ch * 2 * H;
        for (int64_t k = 0; k < H; ++k) { spec[2 * k] = c->dt * re[k]; spec[2 * k + 1] = c->dt * im[k]; }
    }
    const double z = s[1], chi = s[3], g = s[5];
    const double *mM = coef, *mT = coef + P;
    double df = 1.0 / ((double)N * c->dt);
    /* the same summation order as the constant-propagation likelihood */
    neumaier acc = {0.0, 0.0};
    for (int ch = 0; ch < 2; ++ch) {
        const double *spec = scratch_X + 2 * N + ch * 2 * H;
        const double *d = data + ch * 2 * H;
        for (int64_t k = 1; k < N / 2; ++k) {
            double f = (double)k * df, x = f / f_star;
            /* the two power series, by Horner's rule */
            double aM = 0.0, aT = 0.0;
            for (int n = P - 1; n >= 0; --n) {
                aM = aM * x + mM[n];
                aT = aT * x + mT[n];
            }
            aT += p[I_AT];
            if (!(1.0 + aT > 0.0)) return -INFINITY;
            double amp = g * exp(-0.5 * aM * log1p(z));
            double ct = sqrt(1.0 + aT);
            double dT = -aT / (ct * (1.0 + ct)) * chi;   /* (1/c_T - 1) chi as for constant alpha_T */
            double cyc = f * dT;
            cyc -= floor(cyc);
            double cr = cos(2.0 * O_PI * cyc), ci = -sin(2.0 * O_PI * cyc);
            double hr = spec[2 * k], hi = spec[2 * k + 1];
            double mr = amp * (cr * hr - ci * hi);
            double mi = amp * (cr * hi + ci * hr);
            double rr = d[2 * k] - mr, ri = d[2 * k + 1] - mi;
            nsum_add(&acc, (4.0 * df / psd[k]) * (rr * rr + ri * ri));
        }
    }
    return -0.5 * (acc.s + acc.c);
}

/* lnL with the frequency-dependent propagation: coef [B][2][P] holds per
 * walker m_0..m_{P-1} then t_0..t_{P-1}; 0 <= P <= 8, f_star > 0. */
int oracle_loglike_fmg(const double *params, int64_t B, const double *coef, int32_t P,
                       double f_star, const double *data, const double *psd, const oracle_cfg *c,
                       double *lnL)
{
    if (!cfg_ok(c) || P < 0 || P > 8 || !(f_star > 0.0)) return -1;
    int64_t N = c->N, H = N / 2 + 1;
#pragma omp parallel if (B >= oracle_num_threads())
    {
        double *sx = (double *)malloc((size_t)(2 * N) * sizeof(double));
        double *sX = (double *)malloc((size_t)(2 * N + 4 * H) * sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int64_t w = 0; w < B; ++w)
            lnL[w] = walker_loglike_fmg(params + w * NPAR, coef + w * 2 * P, P, f_star, data, psd,
                                        c, sx, sX);
        free(sx);
        free(sX);
    }
    return 0;
}

int oracle_loglike(const double *params, int64_t B, const double *data /* [2][N/2+1][2] */,
                   const double *psd /* [N/2+1] */, const oracle_cfg *c, double *lnL)
{
    if (!cfg_ok(c)) return -1;
    int64_t N = c->N, H = N / 2 + 1;
#pragma omp parallel if (B >= oracle_num_threads())
    {
        double *sx = (double *)malloc((size_t)(2 * N) * sizeof(double));
        double *sX = (double *)malloc((size_t)(2 * N + 4 * H) * sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int64_t w = 0; w < B; ++w)
            lnL[w] = walker_loglike(params + w * NPAR, data, psd, c, sx, sX);
        free(sx);
        free(sX);
    }
    return 0;
}

/* The likelihood of each walker against several data sets (data
 * [nset][2][N/2+1][2]) from one evaluation of its spectrum: lnL[B][nset].
 * Each entry equals oracle_loglike's for that data set.  If spec is not
 * NULL, each walker's unit-distance GR spectra (as oracle_rfft of its
 * waveform, [B][2][N/2+1][2]) are copied there too (zeros for an invalid
 * walker). */
int oracle_loglike_sets(const double *params, int64_t B, const double *data, int32_t nset,
                        const double *psd, const oracle_cfg *c, double *lnL, double *spec)
{
    if (!cfg_ok(c) || nset < 1) return -1;
    int64_t N = c->N, H = N / 2 + 1;
#pragma omp parallel if (B >= oracle_num_threads())
    {
        double *sx = (double *)malloc((size_t)(2 * N) * sizeof(double));
        double *sX = (double *)malloc((size_t)(2 * N + 4 * H) * sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int64_t w = 0; w < B; ++w) {
            double s[8];
            int bad = walker_spectrum(params + w * NPAR, c, s, sx, sX);
            for (int32_t q = 0; q < nset; ++q)
                lnL[w * nset + q] = bad ? -INFINITY
                                        : spectrum_loglike(s, sX + 2 * N, data + q * 4 * H, psd, c);
            if (spec) {
                if (bad) memset(spec + w * 4 * H, 0, (size_t)(4 * H) * sizeof(double));
                else memcpy(spec + w * 4 * H, sX + 2 * N, (size_t)(4 * H) * sizeof(double));
            }
        }
        free(sx);
        free(sX);
    }
    return 0;
}

/* ======================================================================== */
/* Data set helpers (inputs of the likelihood).                             */
/* ======================================================================== */

/* LISA instrumental noise of BC04 (the paper's example noise model, Sec. 3),
 * one-sided, in Hz^-1; confusion noise omitted (reading R12). */
int oracle_psd_bc04(const double *f, int64_t n, double *S)
{
    for (int64_t i = 0; i < n; ++i) {
        double v = f[i];
        S[i] = (v > 0.0) ? 9.18e-52 / (v * v * v * v) + 1.59e-41 + 9.18e-38 * v * v : INFINITY;
    }
    return 0;
}

/* The second noise model of the paper (Sec. 3, `get_noise()`): the LISA
 * sensitivity of Robson, Cornish & Liu 2019 (CQG 36, 105011), sky-averaged,
 * one-sided, in Hz^-1:
 *   S_n = 10/(3 L^2) [P_OMS + 2 (1 + cos^2(f/f*)) P_acc / (2 pi f)^4]
 *         (1 + (6/10) (f/f*)^2) + S_c,
 * L = 2.5e9 m, f* = c / (2 pi L),
 * P_OMS = (1.5e-11 m)^2 (1 + (2 mHz / f)^4),
 * P_acc = (3e-15 m s^-2)^2 (1 + (0.4 mHz / f)^2) (1 + (f / 8 mHz)^4),
 * and the galactic confusion noise
 *   S_c = A f^(-7/3) exp(-f^al + be f sin(ka f)) (1 + tanh(ga (f_k - f))),
 * A = 9e-45, (al, be, ka, ga, f_k) for 0.5, 1, 2 and 4 years of
 * observation.  conf = -1: no confusion noise; 0..3: those four periods.
 * Parity unpinned in its constants (no printed values are at hand); the
 * tests pin its limits and shape. */
int oracle_psd_rcl(const double *f, int64_t n, int32_t conf, double *S)
{
    static const double tab[4][5] = {
        {0.133, 243.0, 482.0, 917.0, 0.00258},
        {0.171, 292.0, 1020.0, 1680.0, 0.00215},
        {0.165, 299.0, 611.0, 1340.0, 0.00173},
        {0.138, -221.0, 521.0, 1680.0, 0.00113},
    };
    if (conf < -1 || conf > 3) return -1;
    const double L = 2.5e9, fs = O_CLIGHT / (2.0 * O_PI * L);
    for (int64_t i = 0; i < n; ++i) {
        double v = f[i];
        if (!(v > 0.0)) { S[i] = INFINITY; continue; }
        double poms = 1.5e-11 * 1.5e-11 * (1.0 + pow(2e-3 / v, 4.0));
        double pacc = 3e-15 * 3e-15 * (1.0 + pow(0.4e-3 / v, 2.0)) * (1.0 + pow(v / 8e-3, 4.0));
        double cs = cos(v / fs);
        double w4 = pow(2.0 * O_PI * v, 4.0);
        double sn = 10.0 / (3.0 * L * L) * (poms + 2.0 * (1.0 + cs * cs) * pacc / w4) *
                    (1.0 + 0.6 * (v / fs) * (v / fs));
        if (conf >= 0) {
            const double *t = tab[conf];
            sn += 9e-45 * pow(v, -7.0 / 3.0) * exp(-pow(v, t[0]) + t[1] * v * sin(t[2] * v)) *
                  (1.0 + tanh(t[3] * (t[4] - v)));
        }
        S[i] = sn;
    }
    return 0;
}

/* data = m[theta_inj] + n, with n_k = sqrt(S_k N dt / 4) (x_k + i y_k) for the
 * standard normal draws gauss[2][N/2+1][2] (NULL: noise-less data); bins 0
 * and N/2 carry no noise.  hinj is the unit-distance GR spectrum. */
int oracle_make_data(const double *hinj, const double *pinj, const double *psd,
                     const double *gauss, int64_t N, double dt, double *data)
{
    double s[8];
    /* only the propagation scalars (Eqs. (3)-(6)) enter here: the orbit, and
     * with it the initial frequency, is already in hinj, so the injection's
     * nu0 is not checked (an injection whose state is given at the LSO
     * carries none) */
    walker_scalars(pinj, 1, s);
    if (s[0] == 0.0) return -2;
    int64_t H = N / 2 + 1;
    double g = s[5];
    double phi = s[4] / ((double)N * dt);
    phi -= floor(phi);
    for (int ch = 0; ch < 2; ++ch) {
        for (int64_t k = 0; k < H; ++k) {
            double cr, ci;
            delay_phase(k, phi, &cr, &ci);
            const double *hk = hinj + (ch * H + k) * 2;
            double mr = g * (cr * hk[0] - ci * hk[1]);
            double mi = g * (cr * hk[1] + ci * hk[0]);
            double nr = 0.0, ni = 0.0;
            if (gauss && k > 0 && k < N / 2) {
                double sig = sqrt(psd[k] * (double)N * dt / 4.0);
                nr = sig * gauss[(ch * H + k) * 2];
                ni = sig * gauss[(ch * H + k) * 2 + 1];
            }
            data[(ch * H + k) * 2] = mr + nr;
            data[(ch * H + k) * 2 + 1] = mi + ni;
        }
    }
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ======================================================================== */
/* Ensemble sampler step: the affine-invariant stretch move of Goodman &    */
/* Weare (2010) that the paper's sampler (emcee, Sec. 1 iii and Sec. 3      */
/* "Posterior sampling") applies to the walker matrix, in its parallel form */
/* where the ensemble of 2W walkers is split into two halves updated in     */
/* turn, each against the other.                                             */
/*                                                                           */
/* For walker k of half h: a partner j is drawn uniformly from the other     */
/* half; the stretch z has density proportional to 1/sqrt(z) on [1/a, a],    */
/* drawn by inverting its distribution function, F(z) = (sqrt(a z) - 1) /   */
/* (a - 1); the proposal moves the free coordinates to X_j + z (X_k - X_j)   */
/* and keeps the others; it is accepted with probability                     */
/* min(1, z^(D-1) p(Y) / p(X_k)), D the number of free coordinates.          */
/* Readings: the log-prior is flat inside a box on the free coordinates and  */
/* -inf outside (the paper's priors are not printed); a proposal with log-   */
/* posterior -inf is rejected, a walker at -inf accepts any finite proposal. */
/* The random numbers are inputs, three per walker and half: u0 picks the    */
/* partner, u1 the stretch, u2 decides acceptance (all in [0, 1)).           */
/* ======================================================================== */

/* proposals, their (D-1) ln z and log-prior, for half h of 2W walkers */
int oracle_stretch_propose(const double *X, int64_t W, int32_t h, const int32_t *free_idx,
                           int32_t D, const double *lo, const double *hi, double a,
                           const double *u /* [W][3] */, double *Y /* [W][NPAR] */,
                           double *lnz /* [W] */, double *lnprior /* [W] */)
{
    if (W < 1 || h < 0 || h > 1 || D < 1 || D > NPAR || !(a > 1.0)) return -1;
    for (int64_t k = 0; k < W; ++k) {
        const double *xk = X + (h * W + k) * NPAR;
        int64_t j = (int64_t)floor(u[3 * k] * (double)W);
        if (j < 0) j = 0;
        if (j > W - 1) j = W - 1;
        const double *xj = X + ((1 - h) * W + j) * NPAR;
        const double s = (a - 1.0) * u[3 * k + 1] + 1.0;   /* s = sqrt(a z) */
        const double z = s * s / a;
        double *y = Y + k * NPAR;
        for (int i = 0; i < NPAR; ++i) y[i] = xk[i];
        int inside = 1;
        for (int d = 0; d < D; ++d) {
            const int i = free_idx[d];
            y[i] = xj[i] + z * (xk[i] - xj[i]);
            if (!(y[i] >= lo[d] && y[i] <= hi[d])) inside = 0;
        }
        lnz[k] = (double)(D - 1) * log(z);
        lnprior[k] = inside ? 0.0 : -INFINITY;
    }
    return 0;
}

/* acceptance for half h, given the proposals' log-posteriors lnpY */
int oracle_stretch_accept(double *X, double *lnp, int64_t W, int32_t h, const double *Y,
                          const double *lnpY, const double *lnz, const double *u /* [W][3] */,
                          int32_t *accepted /* [2W] */)
{
    if (W < 1 || h < 0 || h > 1) return -1;
    for (int64_t k = 0; k < W; ++k) {
        const int64_t g = h * W + k;
        const double lold = lnp[g], lnew = lnpY[k];
        int take;
        if (!(lnew > -INFINITY)) take = 0;            /* -inf or NaN */
        else if (!(lold > -INFINITY)) take = 1;
        else take = log(u[3 * k + 2]) < lnz[k] + lnew - lold;
        if (take) {
            for (int i = 0; i < NPAR; ++i) X[g * NPAR + i] = Y[k * NPAR + i];
            lnp[g] = lnew;
        }
        accepted[g] = take;
    }
    return 0;
}

static double box_lnprior(const double *p, const int32_t *free_idx, int32_t D, const double *lo,
                          const double *hi)
{
    for (int d = 0; d < D; ++d) {
        const double v = p[free_idx[d]];
        if (!(v >= lo[d] && v <= hi[d])) return -INFINITY;
    }
    return 0.0;
}

/* log-posterior of n walkers: box prior plus log-likelihood */
int oracle_ensemble_lnprob(const double *X, int64_t n, const int32_t *free_idx, int32_t D,
                           const double *lo, const double *hi, const double *data,
                           const double *psd, const oracle_cfg *c, double *lnp)
{
    if (n < 1 || D < 1 || D > NPAR) return -1;
    int rc = oracle_loglike(X, n, data, psd, c, lnp);
    if (rc) return rc;
    for (int64_t k = 0; k < n; ++k) lnp[k] += box_lnprior(X + k * NPAR, free_idx, D, lo, hi);
    return 0;
}

/* one step of the ensemble of 2W walkers: half 0 against half 1, then half
 * 1 against the updated half 0; u is [2][W][3] */
int oracle_stretch_step(double *X, double *lnp, int64_t W, const int32_t *free_idx, int32_t D,
                        const double *lo, const double *hi, double a, const double *u,
                        const double *data, const double *psd, const oracle_cfg *c,
                        int32_t *accepted)
{
    if (W < 1 || D < 1 || D > NPAR || !(a > 1.0)) return -1;
    double *Y = (double *)malloc((size_t)W * NPAR * sizeof(double));
    double *lnz = (double *)malloc((size_t)W * sizeof(double));
    double *lpr = (double *)malloc((size_t)W * sizeof(double));
    double *lnL = (double *)malloc((size_t)W * sizeof(double));
    int rc = (Y && lnz && lpr && lnL) ? 0 : -2;
    for (int h = 0; h < 2 && rc == 0; ++h) {
        const double *uh = u + (int64_t)h * W * 3;
        rc = oracle_stretch_propose(X, W, h, free_idx, D, lo, hi, a, uh, Y, lnz, lpr);
        if (rc == 0) rc = oracle_loglike(Y, W, data, psd, c, lnL);
        if (rc == 0) {
            for (int64_t k = 0; k < W; ++k) lnL[k] += lpr[k];
            rc = oracle_stretch_accept(X, lnp, W, h, Y, lnL, lnz, uh, accepted);
        }
    }
    free(Y);
    free(lnz);
    free(lpr);
    free(lnL);
    return rc;
}
