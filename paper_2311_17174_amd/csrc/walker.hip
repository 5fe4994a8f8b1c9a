// walker.hip -- per-walker stages of the likelihood: scalars, orbit, tables.
//
//  k_walker_setup   one lane per walker (FP64): validity, z(d_L), Xi(z),
//                   propagation delay, geometry constants, then the orbital
//                   ODE of Eq. (1) by classical RK4 on the coarse grid,
//                   stopped at the last node before the LSO (Sec. 3);
//                   k_walker_resume continues it segment by segment
//  k_walker_setup_adaptive, k_orbit_dp5, k_orbit_rk78
//                   the same constants, then the ODE by the adaptive
//                   Dormand-Prince 5(4) pair sampled at the same nodes by its
//                   continuous extension (one wave per walker), or by
//                   Fehlberg's 7(8) pair stepped node to node (one lane per
//                   walker)
//  k_amp_tables     one workgroup per (walker, range of coarse intervals,
//                   group of harmonics): Bessel functions of the
//                   Peters-Mathews amplitudes and their time derivatives at
//                   the range's nodes (in LDS), folded into cubic Hermite
//                   polynomials in the interval coordinate u
#include "internal.hpp"

#include <math.h>

namespace emri {

struct GL8 {            // 8-point Gauss-Legendre rule on [-1, 1], both halves
    double x[4], w[4];  // positive nodes and weights
};

// ---------------------------------------------------------------------------
// cosmology (flat LCDM, Planck 2018 H0 and Omega_m): d_L = (1+z) D_H I(z),
// I(z) = int_0^z dz'/E(z'), E = sqrt(Om (1+z)^3 + 1 - Om).
// I(z) by composite 8-point Gauss-Legendre on 16 panels.
// ---------------------------------------------------------------------------
__device__ inline double inv_hubble_rate(double z)
{
    double a = 1.0 + z;
    return rsqrt(kOmegaM * a * a * a + (1.0 - kOmegaM));
}

__device__ double comoving_integral(double z, const GL8& g)
{
    const int panels = 16;
    double h = z / panels, acc = 0.0;
    for (int p = 0; p < panels; ++p) {
        double c = (p + 0.5) * h, r = 0.5 * h, s = 0.0;
        for (int i = 0; i < 4; ++i)
            s += g.w[i] * (inv_hubble_rate(c - r * g.x[i]) + inv_hubble_rate(c + r * g.x[i]));
        acc += r * s;
    }
    return acc;
}

// ---------------------------------------------------------------------------
// Eq. (1): right-hand side of the AK orbital system (Barack & Cutler 2004),
// written with x = 2 pi M nu, eps = 1 - e^2.  Depends only on (nu, e).
// ---------------------------------------------------------------------------
struct Rhs { double dPhi, dnu, dgt, de, dal; };

// x13 = cbrt(2 pi M nu) is passed in: the state after a step shares it with
// the plunge test.  Constant divisors are applied as reciprocal products and
// 1/eps as rsqrt(eps)^2 (a few ulp from the quotients; no IEEE division on
// the step's dependency chain).
__device__ inline Rhs ak_rhs_x(double nu, double x13, double e, double Ms, double mus, double a,
                               double cl)
{
    const double x = 2.0 * kPi * Ms * nu;
    const double x23 = x13 * x13;
    const double e2 = e * e, e4 = e2 * e2, e6 = e4 * e2;
    const double eps = 1.0 - e2;
    const double rse = rsqrt(eps);          // eps^{-1/2}
    const double ie = rse * rse;
    const double ie2 = ie * ie, ie4 = ie2 * ie2;
    const double acl = a * cl;
    const double M2 = Ms * Ms;
    Rhs r;
    r.dPhi = 2.0 * kPi * nu;
    double b = (1.0 + (73.0 / 24.0) * e2 + (37.0 / 96.0) * e4) * eps +
               x23 * (1273.0 / 336.0 - (2561.0 / 224.0) * e2 - (3885.0 / 128.0) * e4 -
                      (13147.0 / 5376.0) * e6) -
               x * acl * rse *
                   (73.0 / 12.0 + (1211.0 / 24.0) * e2 + (3143.0 / 96.0) * e4 +
                    (65.0 / 64.0) * e6);
    const double x113 = x * x * x * x23;    // x^{11/3}
    r.dnu = (96.0 / (10.0 * kPi)) * (mus / (M2 * Ms)) * x113 * ie4 * rse * b;
    r.dgt = 6.0 * kPi * nu * x23 * ie * (1.0 + 0.25 * x23 * ie * (26.0 - 15.0 * e2)) -
            12.0 * kPi * nu * acl * x * ie * rse;
    const double x83 = x * x * x23;         // x^{8/3}
    double br = (304.0 + 121.0 * e2) * eps * (1.0 + 12.0 * x23) -
                (x23 * (1.0 / 56.0)) * (133640.0 + 108984.0 * e2 - 25211.0 * e4);
    r.de = -(e * (1.0 / 15.0)) * (mus / M2) * ie2 * ie * rse * x83 * br +
           e * (mus / M2) * acl * x113 * ie4 *
               (1364.0 / 5.0 + (5032.0 / 15.0) * e2 + (263.0 / 10.0) * e4);
    r.dal = 4.0 * kPi * nu * a * x * ie * rse;
    return r;
}

__device__ inline Rhs ak_rhs(double nu, double e, double Ms, double mus, double a, double cl)
{
    return ak_rhs_x(nu, cbrt(2.0 * kPi * Ms * nu), e, Ms, mus, a, cl);
}

// before the last stable orbit: nu < nu_LSO(e) of Sec. 3, on a sane state;
// *x13 receives cbrt(2 pi M nu)
__device__ inline bool before_lso(double Phi, double nu, double gt, double e, double al, double Ms,
                                  double* x13)
{
    *x13 = cbrt(2.0 * kPi * Ms * nu);
    if (!(isfinite(Phi) && isfinite(nu) && isfinite(gt) && isfinite(e) && isfinite(al)))
        return false;
    if (!(nu > 0.0 && e >= 0.0 && e < 1.0)) return false;
    return *x13 * *x13 * (6.0 + 2.0 * e) < (1.0 - e) * (1.0 + e);
}

// ---------------------------------------------------------------------------
// k_walker_setup: one lane per walker
// ---------------------------------------------------------------------------
// RK4 steps k0 .. k1-1 from the state Y at node k0 with derivative f;
// writes nodes k0+1 .. to o (10 values each: Y, then dY/dt) and returns the
// index of the last node before the LSO (k1 if every step stays before it)
__device__ __forceinline__ int64_t rk4_steps(double& Y0, double& Y1, double& Y2, double& Y3,
                                             double& Y4, Rhs f, int64_t k0, int64_t k1, double h,
                                             double Ms, double mus, double a, double cl,
                                             double* __restrict__ o)
{
    const double hh = 0.5 * h, h6 = h / 6.0;
    for (int64_t k = k0; k < k1; ++k) {
        const Rhs k2 = ak_rhs(Y1 + hh * f.dnu, Y3 + hh * f.de, Ms, mus, a, cl);
        const Rhs k3 = ak_rhs(Y1 + hh * k2.dnu, Y3 + hh * k2.de, Ms, mus, a, cl);
        const Rhs k4 = ak_rhs(Y1 + h * k3.dnu, Y3 + h * k3.de, Ms, mus, a, cl);
        Y0 += h6 * (f.dPhi + 2.0 * k2.dPhi + 2.0 * k3.dPhi + k4.dPhi);
        Y1 += h6 * (f.dnu + 2.0 * k2.dnu + 2.0 * k3.dnu + k4.dnu);
        Y2 += h6 * (f.dgt + 2.0 * k2.dgt + 2.0 * k3.dgt + k4.dgt);
        Y3 += h6 * (f.de + 2.0 * k2.de + 2.0 * k3.de + k4.de);
        Y4 += h6 * (f.dal + 2.0 * k2.dal + 2.0 * k3.dal + k4.dal);
        double x13;
        if (!before_lso(Y0, Y1, Y2, Y3, Y4, Ms, &x13)) return k;
        f = ak_rhs_x(Y1, x13, Y3, Ms, mus, a, cl);
        double* q = o + (k + 1) * 10;
        q[0] = Y0; q[1] = Y1; q[2] = Y2; q[3] = Y3; q[4] = Y4;
        q[5] = f.dPhi; q[6] = f.dnu; q[7] = f.dgt; q[8] = f.de; q[9] = f.dal;
    }
    return k1;
}

// From the LSO backward: RK4 steps with -h from the state Y at node K (f its
// derivative) down to node k_stop, writing nodes K-1 .. k_stop.  false if
// the state leaves the physical range (finite, 0 <= e < 1, nu > 0) on the
// way.
__device__ __forceinline__ bool rk4_back(double Y0, double Y1, double Y2, double Y3, double Y4,
                                         Rhs f, int64_t K, int64_t k_stop, double h, double Ms,
                                         double mus, double a, double cl,
                                         double* __restrict__ o)
{
    const double hb = -h, hh = 0.5 * hb, h6 = hb / 6.0;
    for (int64_t k = K; k > k_stop; --k) {
        const Rhs k2 = ak_rhs(Y1 + hh * f.dnu, Y3 + hh * f.de, Ms, mus, a, cl);
        const Rhs k3 = ak_rhs(Y1 + hh * k2.dnu, Y3 + hh * k2.de, Ms, mus, a, cl);
        const Rhs k4 = ak_rhs(Y1 + hb * k3.dnu, Y3 + hb * k3.de, Ms, mus, a, cl);
        Y0 += h6 * (f.dPhi + 2.0 * k2.dPhi + 2.0 * k3.dPhi + k4.dPhi);
        Y1 += h6 * (f.dnu + 2.0 * k2.dnu + 2.0 * k3.dnu + k4.dnu);
        Y2 += h6 * (f.dgt + 2.0 * k2.dgt + 2.0 * k3.dgt + k4.dgt);
        Y3 += h6 * (f.de + 2.0 * k2.de + 2.0 * k3.de + k4.de);
        Y4 += h6 * (f.dal + 2.0 * k2.dal + 2.0 * k3.dal + k4.dal);
        if (!(isfinite(Y0) && isfinite(Y1) && isfinite(Y2) && isfinite(Y3) && isfinite(Y4) &&
              Y3 >= 0.0 && Y3 < 1.0 && Y1 > 0.0))
            return false;
        f = ak_rhs(Y1, Y3, Ms, mus, a, cl);
        double* q = o + (k - 1) * 10;
        q[0] = Y0; q[1] = Y1; q[2] = Y2; q[3] = Y3; q[4] = Y4;
        q[5] = f.dPhi; q[6] = f.dnu; q[7] = f.dgt; q[8] = f.de; q[9] = f.dal;
    }
    return true;
}

// ---------------------------------------------------------------------------
// Adaptive orbit (emri_cfg.ode = EMRI_ODE_DP5): the embedded Dormand-Prince
// 5(4) pair (J. Comput. Appl. Math. 6 (1980) 19), the order-5 solution kept,
// step control as in Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.4,
// and the pair's order-4 continuous extension (Shampine 1986, in the form
// of HNW Sec. II.6) evaluated at the coarse nodes t_k = k h.  The nodes
// carry Y_k and f(Y_k) as on the RK4 path, so the tables and synthesis do
// not know which integrator ran.  The right-hand side depends on (nu, e)
// alone: a stage only forms those two components of its state.
// ---------------------------------------------------------------------------
namespace dp5 {
constexpr double A21 = 1.0 / 5.0;
constexpr double A31 = 3.0 / 40.0, A32 = 9.0 / 40.0;
constexpr double A41 = 44.0 / 45.0, A42 = -56.0 / 15.0, A43 = 32.0 / 9.0;
constexpr double A51 = 19372.0 / 6561.0, A52 = -25360.0 / 2187.0, A53 = 64448.0 / 6561.0,
                 A54 = -212.0 / 729.0;
constexpr double A61 = 9017.0 / 3168.0, A62 = -355.0 / 33.0, A63 = 46732.0 / 5247.0,
                 A64 = 49.0 / 176.0, A65 = -5103.0 / 18656.0;
// order-5 weights; the seventh stage is f(y1) (its b is 0)
constexpr double B1 = 35.0 / 384.0, B3 = 500.0 / 1113.0, B4 = 125.0 / 192.0,
                 B5 = -2187.0 / 6784.0, B6 = 11.0 / 84.0;
// b - b*, b* the embedded order-4 weights
constexpr double E1 = 71.0 / 57600.0, E3 = -71.0 / 16695.0, E4 = 71.0 / 1920.0,
                 E5 = -17253.0 / 339200.0, E6 = 22.0 / 525.0, E7 = -1.0 / 40.0;
// continuous extension, fifth coefficient vector
constexpr double D1 = -12715105075.0 / 11282082432.0, D3 = 87487479700.0 / 32700410799.0,
                 D4 = -10690763975.0 / 1880347072.0, D5 = 701980252875.0 / 199316789632.0,
                 D6 = -1453857185.0 / 822651844.0, D7 = 69997945.0 / 29380423.0;
constexpr double kSafety = 0.9, kFacMin = 0.2, kFacMax = 5.0;

enum { GO = 0, END = 1, FAIL = 2 };

struct State {
    double t, H;       // time of Y; proposed step (signed)
    double Y[5];       // Phi, nu, gamma~, e, alpha
    Rhs f;             // f(Y)
    int64_t node;      // next coarse node to fill
    int64_t att;       // step attempts so far
    int rej;           // the last attempt was rejected
};

__device__ inline double comp(const Rhs& r, int i)
{
    return i == 0 ? r.dPhi : i == 1 ? r.dnu : i == 2 ? r.dgt : i == 3 ? r.de : r.dal;
}

// steps until node `stop` is filled (forward: nodes up to stop; backward:
// down to stop).  END: the orbit is complete, *kw its last node (forward:
// the last before the LSO); FAIL: budget exhausted, or (backward) a node
// outside the physical range
// Run by all 64 lanes of a wave for one walker: every lane takes the same
// steps (the state is the same in each); the nodes of an accepted step are
// shared out over the lanes.  R: this lane's kLdsSlots LDS slots of the
// continuous extension, stride 64.
constexpr int kLdsSlots = 20;
__device__ int advance(State& s, int64_t stop, int64_t K, double hc, bool back, double rtol,
                       double atol, double Ms, double mus, double a, double cl,
                       double* __restrict__ o, int64_t* kw, double* __restrict__ R)
{
    const int lane = threadIdx.x;
    const double t_end = back ? 0.0 : (double)K * hc;
    const int64_t budget = 4 * K + 64;
    while (back ? s.node >= stop : s.node <= stop) {
        if (s.att >= budget) return FAIL;
        ++s.att;
        double Hs = s.H;
        bool last = false;
        if (back ? (s.t + Hs <= t_end) : (s.t + Hs >= t_end)) {
            Hs = t_end - s.t;
            last = true;
        }
        // stage j adds b_j k_j, (b_j - b*_j) k_j and d_j k_j to running sums
        // (the order of the sums is j = 1..7); later stages need only the nu
        // and e components of earlier ones
        double sB[5], sE[5], sD[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const double k = comp(s.f, i);
            sB[i] = B1 * k;
            sE[i] = E1 * k;
            sD[i] = D1 * k;
        }
        const double n0 = s.Y[1], e0 = s.Y[3];
        const double n1 = s.f.dnu, m1 = s.f.de;
        const Rhs k2 = ak_rhs(n0 + Hs * (A21 * n1), e0 + Hs * (A21 * m1), Ms, mus, a, cl);
        const double n2 = k2.dnu, m2 = k2.de;
        Rhs k = ak_rhs(n0 + Hs * (A31 * n1 + A32 * n2), e0 + Hs * (A31 * m1 + A32 * m2), Ms, mus,
                       a, cl);
        const double n3 = k.dnu, m3 = k.de;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            sB[i] += B3 * comp(k, i);
            sE[i] += E3 * comp(k, i);
            sD[i] += D3 * comp(k, i);
        }
        k = ak_rhs(n0 + Hs * (A41 * n1 + A42 * n2 + A43 * n3),
                   e0 + Hs * (A41 * m1 + A42 * m2 + A43 * m3), Ms, mus, a, cl);
        const double n4 = k.dnu, m4 = k.de;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            sB[i] += B4 * comp(k, i);
            sE[i] += E4 * comp(k, i);
            sD[i] += D4 * comp(k, i);
        }
        k = ak_rhs(n0 + Hs * (A51 * n1 + A52 * n2 + A53 * n3 + A54 * n4),
                   e0 + Hs * (A51 * m1 + A52 * m2 + A53 * m3 + A54 * m4), Ms, mus, a, cl);
        const double n5 = k.dnu, m5 = k.de;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            sB[i] += B5 * comp(k, i);
            sE[i] += E5 * comp(k, i);
            sD[i] += D5 * comp(k, i);
        }
        k = ak_rhs(n0 + Hs * (A61 * n1 + A62 * n2 + A63 * n3 + A64 * n4 + A65 * n5),
                   e0 + Hs * (A61 * m1 + A62 * m2 + A63 * m3 + A64 * m4 + A65 * m5), Ms, mus, a,
                   cl);
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            sB[i] += B6 * comp(k, i);
            sE[i] += E6 * comp(k, i);
            sD[i] += D6 * comp(k, i);
        }
        double y1[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) y1[i] = s.Y[i] + Hs * sB[i];
        const Rhs k7 = ak_rhs(y1[1], y1[3], Ms, mus, a, cl);
        double sum = 0.0;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const double err = Hs * (sE[i] + E7 * comp(k7, i));
            const double sc = (i == 1 ? 0.0 : atol) + rtol * fmax(fabs(s.Y[i]), fabs(y1[i]));
            const double q = err / sc;
            sum += q * q;
        }
        const double en = sqrt(sum / 5.0);
        const double fac = fmax(kFacMin, kSafety * pow(en, -0.2));
        if (!(en <= 1.0)) {              // rejected (a NaN norm too)
            s.H = Hs * fac;
            s.rej = 1;
            continue;
        }
        const double t1 = last ? t_end : s.t + Hs;
        // y(th) = r1 + th (r2 + (1 - th) (r3 + th (r4 + (1 - th) r5))) on [t, t1];
        // r2..r5 wait in this lane's LDS slots while the nodes are filled
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const double r2 = y1[i] - s.Y[i];
            const double r3 = Hs * comp(s.f, i) - r2;
            R[(0 * 5 + i) * 64] = r2;
            R[(1 * 5 + i) * 64] = r3;
            R[(2 * 5 + i) * 64] = r2 - Hs * comp(k7, i) - r3;
            R[(3 * 5 + i) * 64] = Hs * (sD[i] + D7 * comp(k7, i));
        }
        // the nodes in (t, t1], 64 at a time: lane l takes the l-th; they
        // form a prefix of the lanes (the node times increase with l)
        for (;;) {
            const int64_t n = back ? s.node - lane : s.node + lane;
            const bool inside = back ? (n >= 0 && (double)n * hc >= t1)
                                     : (n <= K && (double)n * hc <= t1);
            const uint64_t in_mask = __ballot(inside);
            if (in_mask == 0) break;
            double yk[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            double x13 = 0.0;
            bool bad = false;
            if (inside) {
                const double th = ((double)n * hc - s.t) / Hs;
#pragma unroll
                for (int i = 0; i < 5; ++i)
                    yk[i] = s.Y[i] + th * (R[i * 64] +
                                           (1.0 - th) * (R[(5 + i) * 64] +
                                                         th * (R[(10 + i) * 64] +
                                                               (1.0 - th) * R[(15 + i) * 64])));
                if (back)
                    bad = !(isfinite(yk[0]) && isfinite(yk[1]) && isfinite(yk[2]) &&
                            isfinite(yk[3]) && isfinite(yk[4]) && yk[3] >= 0.0 && yk[3] < 1.0 &&
                            yk[1] > 0.0);
                else
                    bad = !before_lso(yk[0], yk[1], yk[2], yk[3], yk[4], Ms, &x13);
            }
            const uint64_t bad_mask = __ballot(inside && bad);
            if (back && bad_mask) return FAIL;
            const int nin = __popcll(in_mask);
            // forward: the nodes before the first one past the LSO
            const int nok = bad_mask ? __ffsll((unsigned long long)bad_mask) - 1 : nin;
            if (lane < nok) {
                const Rhs fk = back ? ak_rhs(yk[1], yk[3], Ms, mus, a, cl)
                                    : ak_rhs_x(yk[1], x13, yk[3], Ms, mus, a, cl);
                double* q = o + n * 10;
                q[0] = yk[0]; q[1] = yk[1]; q[2] = yk[2]; q[3] = yk[3]; q[4] = yk[4];
                q[5] = fk.dPhi; q[6] = fk.dnu; q[7] = fk.dgt; q[8] = fk.de; q[9] = fk.dal;
            }
            if (bad_mask) {
                *kw = s.node + nok - 1;
                return END;
            }
            s.node += back ? -nin : nin;
            if (nin < 64) break;
        }
        if (last) {
            *kw = K;
            return END;
        }
#pragma unroll
        for (int i = 0; i < 5; ++i) s.Y[i] = y1[i];
        s.f = k7;
        s.t = t1;
        s.H = Hs * fmin(s.rej ? 1.0 : kFacMax, fac);
        s.rej = 0;
    }
    return GO;
}

__device__ inline void save(const State& s, double* __restrict__ c)
{
    c[WC_OT] = s.t;
    c[WC_OH] = s.H;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        c[WC_OY + i] = s.Y[i];
        c[WC_OF + i] = comp(s.f, i);
    }
    c[WC_ONODE] = (double)s.node;
    c[WC_OATT] = (double)s.att;
    c[WC_OREJ] = (double)s.rej;
}

__device__ inline State load(const double* __restrict__ c)
{
    State s;
    s.t = c[WC_OT];
    s.H = c[WC_OH];
#pragma unroll
    for (int i = 0; i < 5; ++i) s.Y[i] = c[WC_OY + i];
    s.f = Rhs{c[WC_OF], c[WC_OF + 1], c[WC_OF + 2], c[WC_OF + 3], c[WC_OF + 4]};
    s.node = (int64_t)c[WC_ONODE];
    s.att = (int64_t)c[WC_OATT];
    s.rej = (int)c[WC_OREJ];
    return s;
}

// after segment seg: K_w as known, and the state for the next segment
// (backward from the LSO every node up to K is valid while the walker is)
__device__ inline void finish_segment(int r, const State& s, int64_t kw, int seg, bool back,
                                      int64_t K, double* __restrict__ c)
{
    if (r == FAIL) {
        c[WC_VALID] = 0.0;
        c[WC_KSEG + seg] = -1.0;
        c[WC_KW] = -1.0;
        c[WC_ODONE] = 1.0;
        return;
    }
    const int64_t known = back ? K : (r == END) ? kw : s.node - 1;
    c[WC_KSEG + seg] = (double)known;
    c[WC_KW] = (double)known;
    c[WC_ODONE] = (r == END) ? 1.0 : 0.0;
    save(s, c);
}
}  // namespace dp5

// ---------------------------------------------------------------------------
// Seventh-order orbit (emri_cfg.ode = EMRI_ODE_RK78): Fehlberg's embedded
// 7(8) pair (NASA TR R-287, 1968; 13 stages), the order-7 solution kept and
// the order-8 one entering the error estimate alone, which reduces to
// H 41/840 (k1 + k11 - k12 - k13).  The steps run node to node: a step that
// would pass the next coarse node is cut to end on it, so each node is a
// step end of the method and no continuous extension is needed, and one lane
// integrates one walker.  Step control as for the 5(4) pair with the
// exponent 1/8; the state between segments is the 5(4) pair's (dp5::State).
// ---------------------------------------------------------------------------
namespace rk78 {
constexpr double kA[13][12] = {
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
// order-7 weights; b7 - b8 (b8 the order-8 weights)
constexpr double kB[13] = {41.0 / 840.0, 0.0, 0.0, 0.0, 0.0, 34.0 / 105.0, 9.0 / 35.0,
                           9.0 / 35.0, 9.0 / 280.0, 9.0 / 280.0, 41.0 / 840.0, 0.0, 0.0};
constexpr double kE[13] = {41.0 / 840.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0,
                           0.0, 0.0, 0.0, 41.0 / 840.0, -41.0 / 840.0, -41.0 / 840.0};

// steps until node `stop` is filled (forward: nodes up to stop; backward:
// down to stop); the return codes and *kw are those of dp5::advance
__device__ int advance(dp5::State& s, int64_t stop, int64_t K, double hc, bool back,
                       double rtol, double atol, double Ms, double mus, double a, double cl,
                       double* __restrict__ o, int64_t* kw)
{
    const int64_t budget = 4 * K + 64;
    while (back ? s.node >= stop : s.node <= stop) {
        if (s.att >= budget) return dp5::FAIL;
        ++s.att;
        const double tn = (double)s.node * hc;
        double Hs = s.H;
        bool land = false;
        if (back ? (s.t + Hs <= tn) : (s.t + Hs >= tn)) {
            Hs = tn - s.t;
            land = true;
        }
        // a stage's state needs only the nu and e components of the earlier
        // stages; the weight sums take all five, in stage order
        double kn[13], ke[13], sB[5], sE[5];
        kn[0] = s.f.dnu;
        ke[0] = s.f.de;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            sB[i] = kB[0] * dp5::comp(s.f, i);
            sE[i] = kE[0] * dp5::comp(s.f, i);
        }
        const double n0 = s.Y[1], e0 = s.Y[3];
#pragma unroll
        for (int st = 1; st < 13; ++st) {
            double an = 0.0, ae = 0.0;
#pragma unroll
            for (int j = 0; j < st; ++j) {
                if (kA[st][j] != 0.0) {
                    an += kA[st][j] * kn[j];
                    ae += kA[st][j] * ke[j];
                }
            }
            const Rhs k = ak_rhs(n0 + Hs * an, e0 + Hs * ae, Ms, mus, a, cl);
            kn[st] = k.dnu;
            ke[st] = k.de;
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                if (kB[st] != 0.0) sB[i] += kB[st] * dp5::comp(k, i);
                if (kE[st] != 0.0) sE[i] += kE[st] * dp5::comp(k, i);
            }
        }
        double y1[5], sum = 0.0;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            y1[i] = s.Y[i] + Hs * sB[i];
            const double err = Hs * sE[i];
            const double sc = (i == 1 ? 0.0 : atol) + rtol * fmax(fabs(s.Y[i]), fabs(y1[i]));
            const double q = err / sc;
            sum += q * q;
        }
        const double en = sqrt(sum / 5.0);
        const double fac = fmax(dp5::kFacMin, dp5::kSafety * pow(en, -0.125));
        if (!(en <= 1.0)) {              // rejected (a NaN norm too)
            s.H = Hs * fac;
            s.rej = 1;
            continue;
        }
        double x13 = 0.0;
        if (back) {
            if (!(isfinite(y1[0]) && isfinite(y1[1]) && isfinite(y1[2]) && isfinite(y1[3]) &&
                  isfinite(y1[4]) && y1[3] >= 0.0 && y1[3] < 1.0 && y1[1] > 0.0))
                return dp5::FAIL;
        } else if (!before_lso(y1[0], y1[1], y1[2], y1[3], y1[4], Ms, &x13)) {
            *kw = s.node - 1;            // past the LSO before node s.node
            return dp5::END;
        }
        const Rhs f1 = back ? ak_rhs(y1[1], y1[3], Ms, mus, a, cl)
                            : ak_rhs_x(y1[1], x13, y1[3], Ms, mus, a, cl);
#pragma unroll
        for (int i = 0; i < 5; ++i) s.Y[i] = y1[i];
        s.f = f1;
        s.t = land ? tn : s.t + Hs;
        if (land) {
            double* q = o + s.node * 10;
            q[0] = y1[0]; q[1] = y1[1]; q[2] = y1[2]; q[3] = y1[3]; q[4] = y1[4];
            q[5] = f1.dPhi; q[6] = f1.dnu; q[7] = f1.dgt; q[8] = f1.de; q[9] = f1.dal;
            if (back ? s.node == 0 : s.node == K) {
                *kw = K;
                return dp5::END;
            }
            s.node += back ? -1 : 1;
        }
        s.H = Hs * fmin(s.rej ? 1.0 : dp5::kFacMax, fac);
        s.rej = 0;
    }
    return dp5::GO;
}
}  // namespace rk78

// The orbit kernels run a few waves for the whole batch (one lane, or for
// the adaptive integrator one wave, per walker) beside the table and
// synthesis kernels of earlier segments: they raise their waves' issue
// priority so those do not stretch the integration.
template <int ODE>
__device__ __forceinline__ void walker_setup(const double* __restrict__ params, int64_t B,
                                             int64_t K, double h, double Ndt, const GL8& gl,
                                             int64_t k1, int ic, double* __restrict__ wc,
                                             double* __restrict__ orb)
{
    __builtin_amdgcn_s_setprio(3);
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= B) return;
    const double* p = params + w * EMRI_NPAR;
    double* c = wc + w * WC;
    for (int i = 0; i < WC; ++i) c[i] = 0.0;
    c[WC_KW] = -1.0;

    bool ok = true;
    for (int i = 0; i < EMRI_NPAR; ++i) ok = ok && isfinite(p[i]);
    const double M = p[0], mu = p[1], a = p[2], e0 = p[3], nu0 = p[4];
    const double cl = p[8], dl = p[13], xi0 = p[14], nxi = p[15], at = p[16];
    const bool lso = ic == EMRI_IC_LSO;
    ok = ok && mu > 0.0 && mu < M && a >= 0.0 && a <= 1.0 && e0 >= 0.0 && e0 < 1.0 &&
         (lso || nu0 > 0.0) && dl > 0.0 && at > -1.0 && cl >= -1.0 && cl <= 1.0;
    const double Ms = M * kSunSeconds, mus = mu * kSunSeconds;
    double x13_0;
    ok = ok && (lso || before_lso(p[5], nu0, p[6], e0, p[7], Ms, &x13_0));
    if (!ok) return;

    // distance, redshift, Eq. (6), delay, overall factor
    const double D = dl * 1e9 * kParsecM / kLightSpeed;
    const double DH = (kLightSpeed / 1000.0 / kHubble) * 1e6 * kParsecM / kLightSpeed;
    double z = D / DH;
    for (int it = 0; it < 40; ++it) {
        const double I = comoving_integral(z, gl);
        const double f = (1.0 + z) * DH * I - D;
        const double fp = DH * I + (1.0 + z) * DH * inv_hubble_rate(z);
        const double dz = f / fp;
        z -= dz;
        if (fabs(dz) <= 4e-16 * (1.0 + z)) break;
    }
    const double Xi = xi0 + (1.0 - xi0) * exp(-nxi * log1p(z));
    if (!(Xi > 0.0) || !isfinite(Xi)) return;
    const double chi = D / (1.0 + z);
    const double cT = sqrt(1.0 + at);
    const double dT = -at / (cT * (1.0 + cT)) * chi;
    double ph = dT / Ndt;
    ph -= floor(ph);

    const double thS = p[9], phS = p[10], thK = p[11], phK = p[12];
    double sts, cts, sps, cps, stk, ctk, spk, cpk;
    sincos(thS, &sts, &cts);
    sincos(phS, &sps, &cps);
    sincos(thK, &stk, &ctk);
    sincos(phK, &spk, &cpk);

    c[WC_MS] = Ms;
    c[WC_MUS] = mus;
    c[WC_A] = a;
    c[WC_CL] = cl;
    c[WC_SL] = sqrt(fmax(0.0, (1.0 - cl) * (1.0 + cl)));
    c[WC_G] = 1.0 / (Xi * D);
    c[WC_PHI] = ph;
    c[WC_NX] = sts * cps; c[WC_NY] = sts * sps; c[WC_NZ] = cts;
    c[WC_SX] = stk * cpk; c[WC_SY] = stk * spk; c[WC_SZ] = ctk;
    c[WC_E1X] = -ctk * cpk; c[WC_E1Y] = -ctk * spk; c[WC_E1Z] = stk;
    c[WC_E2X] = spk; c[WC_E2Y] = -cpk;
    c[WC_NS] = sts * stk * (cps * cpk + sps * spk) + cts * ctk;
    c[WC_CTS] = cts; c[WC_STS] = sts; c[WC_CPS] = cps; c[WC_SPS] = sps;
    c[WC_DOP] = 2.0 * kPi * kAuSeconds * sts;
    c[WC_Z] = z; c[WC_XI] = Xi; c[WC_DT] = dT; c[WC_D] = D;
    c[WC_HASDT] = (dT != 0.0) ? 1.0 : 0.0;
    c[WC_AT] = at;

    double* o = orb + w * (K + 1) * 10;
    if (lso) {
        // nu_LSO(e) = ((1 - e^2)/(6 + 2e))^{3/2} / (2 pi M) at node K, then backward
        const double r = (1.0 - e0) * (1.0 + e0) / (6.0 + 2.0 * e0);
        const double nuL = r * sqrt(r) / (2.0 * kPi * Ms);
        const Rhs f = ak_rhs(nuL, e0, Ms, mus, a, cl);
        double* q = o + K * 10;
        q[0] = p[5]; q[1] = nuL; q[2] = p[6]; q[3] = e0; q[4] = p[7];
        q[5] = f.dPhi; q[6] = f.dnu; q[7] = f.dgt; q[8] = f.de; q[9] = f.dal;
        if constexpr (ODE != EMRI_ODE_RK4) {
            // the integration itself is k_orbit_dp5's or k_orbit_rk78's
            dp5::save(dp5::State{(double)K * h, -h, {p[5], nuL, p[6], e0, p[7]}, f, K - 1, 0, 0},
                      c);
            c[WC_ODONE] = 0.0;
            c[WC_VALID] = 1.0;
            return;
        } else {
            // k1: the last node of the first (backward) segment
            if (!rk4_back(p[5], nuL, p[6], e0, p[7], f, K, k1, h, Ms, mus, a, cl, o)) return;
        }
        c[WC_KSEG] = (double)K;
        c[WC_KW] = (double)K;
        c[WC_VALID] = 1.0;
        return;
    }
    // orbit: classical RK4, nodes t_k = k h
    double Y0 = p[5], Y1 = nu0, Y2 = p[6], Y3 = e0, Y4 = p[7];
    Rhs f = ak_rhs(Y1, Y3, Ms, mus, a, cl);
    o[0] = Y0; o[1] = Y1; o[2] = Y2; o[3] = Y3; o[4] = Y4;
    o[5] = f.dPhi; o[6] = f.dnu; o[7] = f.dgt; o[8] = f.de; o[9] = f.dal;
    if constexpr (ODE != EMRI_ODE_RK4) {
        dp5::save(dp5::State{0.0, h, {Y0, Y1, Y2, Y3, Y4}, f, 1, 0, 0}, c);
        c[WC_ODONE] = 0.0;
        c[WC_VALID] = 1.0;
    } else {
        const int64_t Kw = rk4_steps(Y0, Y1, Y2, Y3, Y4, f, 0, k1, h, Ms, mus, a, cl, o);
        c[WC_KSEG] = (double)Kw;
        c[WC_KW] = (double)Kw;
        c[WC_VALID] = 1.0;
    }
}

// One set of kernels per integrator, each with its own register budget: the
// orbit runs beside the synthesis waves of earlier segments and its waves
// must find room between them (the RK4 kernels hold 130 and 110 VGPRs).
__global__ void __launch_bounds__(64) k_walker_setup(const double* __restrict__ params, int64_t B,
                                                     int64_t K, double h, double Ndt, GL8 gl,
                                                     int64_t k1, int ic, double* __restrict__ wc,
                                                     double* __restrict__ orb)
{
    walker_setup<EMRI_ODE_RK4>(params, B, K, h, Ndt, gl, k1, ic, wc, orb);
}

// constants and an adaptive integrator's starting state (one lane per
// walker); the integration is k_orbit_dp5's or k_orbit_rk78's
__global__ void __launch_bounds__(64) k_walker_setup_adaptive(const double* __restrict__ params,
                                                              int64_t B, int64_t K, double h,
                                                              double Ndt, GL8 gl, int ic,
                                                              double* __restrict__ wc,
                                                              double* __restrict__ orb)
{
    walker_setup<EMRI_ODE_DP5>(params, B, K, h, Ndt, gl, K, ic, wc, orb);
}

// adaptive orbit segment seg: one wave per walker continues from the saved
// integrator state until node k1 is filled (backward: down to node k1), so
// the step sequence does not depend on where the segments end.  Every lane
// of the wave takes the same steps; the nodes of an accepted step are
// shared out over the lanes.  The waves are held to three per SIMD (168
// VGPRs, some spills): they start beside the synthesis waves of earlier
// segments and wait for room on a SIMD, and with about 230 VGPRs they waited
// several times longer.
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3)))
k_orbit_dp5(int64_t K, double h, int64_t k1, int seg, int back, double rtol, double atol,
            double* __restrict__ wc, double* __restrict__ orb)
{
    __builtin_amdgcn_s_setprio(3);
    __shared__ double dense[dp5::kLdsSlots * 64];
    const int64_t w = blockIdx.x;
    double* c = wc + w * WC;
    if (c[WC_VALID] == 0.0) return;                  // the same in every lane
    if (c[WC_ODONE] != 0.0) {
        if (threadIdx.x == 0) c[WC_KSEG + seg] = c[WC_KW];
        return;
    }
    dp5::State st = dp5::load(c);
    int64_t kw = -1;
    const int r = dp5::advance(st, k1, K, h, back != 0, rtol, atol, c[WC_MS], c[WC_MUS],
                               c[WC_A], c[WC_CL], orb + w * (K + 1) * 10, &kw,
                               dense + threadIdx.x);
    if (threadIdx.x == 0) dp5::finish_segment(r, st, kw, seg, back != 0, K, c);
}

// seventh-order orbit segment seg: one lane per walker continues from the
// saved integrator state until node k1 is filled (backward: down to node
// k1), so the step sequence does not depend on where the segments end
__global__ void __launch_bounds__(64) k_orbit_rk78(int64_t B, int64_t K, double h, int64_t k1,
                                                   int seg, int back, double rtol, double atol,
                                                   double* __restrict__ wc,
                                                   double* __restrict__ orb)
{
    __builtin_amdgcn_s_setprio(3);
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= B) return;
    double* c = wc + w * WC;
    if (c[WC_VALID] == 0.0) return;
    if (c[WC_ODONE] != 0.0) {
        c[WC_KSEG + seg] = c[WC_KW];
        return;
    }
    dp5::State st = dp5::load(c);
    int64_t kw = -1;
    const int r = rk78::advance(st, k1, K, h, back != 0, rtol, atol, c[WC_MS], c[WC_MUS],
                                c[WC_A], c[WC_CL], orb + w * (K + 1) * 10, &kw);
    dp5::finish_segment(r, st, kw, seg, back != 0, K, c);
}

// backward orbit segment seg >= 1 (RK4, from the LSO): steps from node k0
// (stored by segment seg - 1) down to node k1 < k0
__global__ void __launch_bounds__(64) k_walker_resume_back(int64_t B, int64_t K, double h,
                                                           int64_t k0, int64_t k1, int seg,
                                                           double* __restrict__ wc,
                                                           double* __restrict__ orb)
{
    __builtin_amdgcn_s_setprio(3);
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= B) return;
    double* c = wc + w * WC;
    if (c[WC_VALID] == 0.0) return;
    double* o = orb + w * (K + 1) * 10;
    const double* q = o + k0 * 10;
    const Rhs f{q[5], q[6], q[7], q[8], q[9]};
    if (!rk4_back(q[0], q[1], q[2], q[3], q[4], f, k0, k1, h, c[WC_MS], c[WC_MUS], c[WC_A],
                  c[WC_CL], o)) {
        c[WC_VALID] = 0.0;
        c[WC_KSEG + seg] = -1.0;
        c[WC_KW] = -1.0;
        return;
    }
    c[WC_KSEG + seg] = (double)K;
}

// orbit segment seg >= 1 (RK4): steps [k0, k1) from node k0 (stored by
// segment seg - 1), unless the orbit reached the LSO before k0
__global__ void __launch_bounds__(64) k_walker_resume(int64_t B, int64_t K, double h, int64_t k0,
                                                      int64_t k1, int seg,
                                                      double* __restrict__ wc,
                                                      double* __restrict__ orb)
{
    __builtin_amdgcn_s_setprio(3);
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= B) return;
    double* c = wc + w * WC;
    if (c[WC_VALID] == 0.0) return;
    const int64_t Kp = (int64_t)c[WC_KSEG + seg - 1];
    if (Kp < k0) {
        c[WC_KSEG + seg] = (double)Kp;
        return;
    }
    const double Ms = c[WC_MS], mus = c[WC_MUS], a = c[WC_A], cl = c[WC_CL];
    double* o = orb + w * (K + 1) * 10;
    const double* q = o + k0 * 10;
    double Y0 = q[0], Y1 = q[1], Y2 = q[2], Y3 = q[3], Y4 = q[4];
    const Rhs f{q[5], q[6], q[7], q[8], q[9]};
    const int64_t Kw = rk4_steps(Y0, Y1, Y2, Y3, Y4, f, k0, k1, h, Ms, mus, a, cl, o);
    c[WC_KSEG + seg] = (double)Kw;
    c[WC_KW] = (double)Kw;
}

// ---------------------------------------------------------------------------
// Bessel functions J_{n-3..n+3}(X), X = n e >= 0, by Miller's downward
// recurrence J_{q-1} = (2q/X) J_q - J_{q+1} from a trial start, normalised
// with J_0 + 2 (J_2 + J_4 + ...) = 1.
//
// Start order S: above the turning point the recurrence amplifies the
// unwanted solution against J by at least (2k - X)/X per step, and the
// relative error of the orders kept is about the inverse square of the
// product of those factors from top = max(n + 3, ceil X) to S.  S is the
// first order where that product exceeds 1e11 (error ~1e-22), capped at
// top + 10 + sqrt(40 top).  The recurrence runs in three loops: down to
// order n + 3 (two values live), the seven orders kept, then down to 0;
// each step is one product, one FMA and the norm update.
// ---------------------------------------------------------------------------
__device__ void bessel7(int n, double X, double J[7])
{
    if (X == 0.0) {
        for (int i = 0; i < 7; ++i) J[i] = (n - 3 + i == 0) ? 1.0 : 0.0;
        return;
    }
    const int hi = n + 3, lo = n - 3;
    const int top = max(hi, (int)ceil(X));
    const double iX = 1.0 / X, iX2 = 2.0 * iX;
    const int cap = top + 10 + (int)sqrt(40.0 * top);
    int S = top;
    double prod = 1.0;
    while (S < cap && prod < 1e11) {
        ++S;
        prod *= (2.0 * S - X) * iX;
    }
    S += S & 1;                       // even: J_S enters the norm
    // a = J_q, b = J_{q+1} (unnormalised), dq = q.  Orders are produced
    // one step at a time, J_{q-1} = (2q/X) J_q - J_{q+1}; the even ones
    // enter the norm with weight 2.  The steps run in pairs (odd order, then
    // even), with the running scale checked once per pair: between checks
    // the values grow by at most (2S/X)^2, which stays inside the FP64 range
    // above the 1e150 threshold for X down to about 1e-75.
    double a = 1e-280, b = 0.0, dq = (double)S, norm = 2.0 * a;
    double w[7] = {0, 0, 0, 0, 0, 0, 0};
    auto step = [&]() {
        const double next = (dq * iX2) * a - b;
        dq -= 1.0;
        b = a;
        a = next;
    };
    auto rescale = [&]() {            // keep the values on the running scale
        if (fabs(a) > 1e150) {
            const double r = 1e-200;
            a *= r; b *= r; norm *= r;
#pragma unroll
            for (int k = 0; k < 7; ++k) w[k] *= r;
        }
    };
    // orders S-1 .. hi (S even): with an odd count the first step stands
    // alone and the pairs run (even, odd), else they run (odd, even)
    int q = S;
    if ((S - hi) & 1) {
        step();
        rescale();
        --q;
#pragma unroll 1
        for (; q > hi; q -= 2) {
            step();
            norm = fma(2.0, a, norm);
            step();
            rescale();
        }
    } else {
#pragma unroll 1
        for (; q > hi; q -= 2) {
            step();
            step();
            norm = fma(2.0, a, norm);
            rescale();
        }
    }
    w[6] = a;                         // J_{n+3}
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        if (lo + i >= 0) {
            step();
            norm = fma(((lo + i) & 1) ? 0.0 : 2.0, a, norm);
            w[i] = a;                 // J_{n-3+i}
            rescale();
        }
    }
    // orders lo-1 .. 0
    q = lo;
    if (q > 0 && ((q - 1) & 1) == 0) {   // an even order first
        step();
        norm = fma(2.0, a, norm);
        rescale();
        --q;
    }
#pragma unroll 1
    for (; q >= 2; q -= 2) {
        step();
        step();
        norm = fma(2.0, a, norm);
        rescale();
    }
    norm -= a;                        // a = J_0 was counted twice
    // orders below zero (n < 3): J_{-k} = (-1)^k J_k
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const int o = lo + i;
        if (o < 0) w[i] = ((-o) & 1 ? -1.0 : 1.0) * w[-o - lo];
    }
    const double in = 1.0 / norm;
#pragma unroll
    for (int i = 0; i < 7; ++i) J[i] = w[i] * in;
}

// values and e-derivatives of n P_n, n Q_n, 2 J_n at (n, e); A factor applied
// by the caller.  J holds J_{n-3..n+3}(n e).
struct PM { double a, b, c, da, db, dc; };

__device__ inline PM pm_amplitudes(int n, double e, const double J[7])
{
    // J[3] = J_n; derivative dJ_k/dX = (J_{k-1} - J_{k+1})/2, X = n e
    const double jm2 = J[1], jm1 = J[2], j0 = J[3], jp1 = J[4], jp2 = J[5];
    const double dm2 = 0.5 * (J[0] - J[2]), dm1 = 0.5 * (J[1] - J[3]), d0 = 0.5 * (J[2] - J[4]),
                 dp1 = 0.5 * (J[3] - J[5]), dp2 = 0.5 * (J[4] - J[6]);
    const double dn = (double)n;
    const double P = jm2 - 2.0 * e * jm1 + (2.0 / dn) * j0 + 2.0 * e * jp1 - jp2;
    const double dP = dn * (dm2 - 2.0 * e * dm1 + (2.0 / dn) * d0 + 2.0 * e * dp1 - dp2) -
                      2.0 * jm1 + 2.0 * jp1;
    const double s = sqrt((1.0 - e) * (1.0 + e));
    const double qb = jm2 - 2.0 * j0 + jp2;
    const double Q = s * qb;
    const double dQ = (s > 0.0 ? -e / s : 0.0) * qb + s * dn * (dm2 - 2.0 * d0 + dp2);
    PM r;
    r.a = dn * P;  r.da = dn * dP;
    r.b = dn * Q;  r.db = dn * dQ;
    r.c = 2.0 * j0; r.dc = 2.0 * dn * d0;
    return r;
}

// cubic Hermite in u from values/derivatives (derivatives per unit time)
__device__ inline void hermite_coeffs(double y0, double d0, double y1, double d1, double h,
                                      double c[4])
{
    c[0] = y0;
    c[1] = h * d0;
    c[2] = 3.0 * (y1 - y0) - h * (2.0 * d0 + d1);
    c[3] = 2.0 * (y0 - y1) + h * (d0 + d1);
}

// amplitude tables, one workgroup per (walker, range of up to kTabI coarse
// intervals of the segment, group of up to kTabH harmonics):
//  1. the node values of the range's nodes -- the three amplitudes A n P_n,
//     A n Q_n, 2 A J_n(ne) and their time derivatives -- go to LDS, one
//     harmonic per wave of 64 nodes, so that every lane of a wave runs
//     Miller's recurrence for the same order and the lanes' trip counts
//     agree (one lane per (node, harmonic) with the harmonics fastest left
//     most lanes of a wave idle behind the highest order);
//  2. each lane folds the values at the ends of an interval into the
//     power-basis Hermite cubics of (interval, harmonic), harmonics fastest,
//     so a wave writes whole runs of the table; the n = 1 group also
//     tabulates Phi, nu, gamma~, alpha.
// A range's last node is its successor's first and is evaluated by both;
// nothing passes between segments.
constexpr int kTabNodes = 64;              // nodes per range
constexpr int kTabI = kTabNodes - 1;       // intervals per range
constexpr int kTabH = 16;                  // harmonics per group
constexpr int kTabPad = kTabNodes + 1;     // LDS row (no bank conflicts in step 2)

template <typename HT>
__global__ void __launch_bounds__(256) k_amp_tables(int64_t K, int nh, double h, int64_t k0,
                                                    int64_t k1, int seg,
                                                    const double* __restrict__ wc,
                                                    const double* __restrict__ orb,
                                                    double* __restrict__ co,
                                                    HT* __restrict__ ch,
                                                    float2* __restrict__ hb)
{
    __shared__ double sv[6 * kTabH * kTabPad];   // [value][harmonic][node]
    const int64_t w = blockIdx.y;
    const int ng = (nh + kTabH - 1) / kTabH;
    const int64_t r = blockIdx.x / ng;
    const int grp = (int)(blockIdx.x - r * ng);
    const double* c = wc + w * WC;
    if (c[WC_VALID] == 0.0) return;
    const int64_t kb = k0 + r * kTabI;                           // first interval
    const int64_t ke = min(k1, (int64_t)c[WC_KSEG + seg]);       // intervals end (< K_w)
    if (kb >= ke) return;                                         // uniform over the block
    const int ni = (int)min((int64_t)kTabI, ke - kb);            // intervals of the range
    const int n_lo = grp * kTabH + 1;
    const int nhb = min(kTabH, nh - grp * kTabH);
    const double Ms = c[WC_MS], mus = c[WC_MUS];

    // 1. node values, node fastest
    for (int p = threadIdx.x; p < kTabNodes * nhb; p += 256) {
        const int hn = p / kTabNodes, i = p - hn * kTabNodes;
        if (i > ni) continue;
        const int n = n_lo + hn;
        const double* o = orb + (w * (K + 1) + kb + i) * 10;
        const double nu = o[1], e = o[3], dnu = o[6], de = o[8];
        const double x13 = cbrt(2.0 * kPi * Ms * nu);
        const double A = x13 * x13 * mus;
        const double dA = (2.0 / 3.0) * A * dnu / nu;
        double J[7];
        bessel7(n, n * e, J);
        const PM pm = pm_amplitudes(n, e, J);
        double* q = sv + hn * kTabPad + i;
        q[0 * kTabH * kTabPad] = A * pm.a;
        q[1 * kTabH * kTabPad] = dA * pm.a + A * pm.da * de;
        q[2 * kTabH * kTabPad] = A * pm.b;
        q[3 * kTabH * kTabPad] = dA * pm.b + A * pm.db * de;
        q[4 * kTabH * kTabPad] = A * pm.c;
        q[5 * kTabH * kTabPad] = dA * pm.c + A * pm.dc * de;
    }

    // orbital interpolants of the range's intervals: Phi, nu, gamma~, alpha
    if (grp == 0 && (int)threadIdx.x < ni) {
        const int64_t k = kb + threadIdx.x;
        const double* o0 = orb + (w * (K + 1) + k) * 10;
        const double* o1 = o0 + 10;
        double* q = co + (w * K + k) * 16;
        const int comp[4] = {0, 1, 2, 4};
        for (int i = 0; i < 4; ++i) {
            double cc[4];
            hermite_coeffs(o0[comp[i]], o0[5 + comp[i]], o1[comp[i]], o1[5 + comp[i]], h, cc);
            q[4 * i + 0] = cc[0]; q[4 * i + 1] = cc[1]; q[4 * i + 2] = cc[2]; q[4 * i + 3] = cc[3];
        }
    }
    __syncthreads();

    // 2. interval cubics, harmonic fastest
    for (int p = threadIdx.x; p < ni * nhb; p += 256) {
        const int i = p / nhb, hn = p - i * nhb;
        const int64_t k = kb + i;
        const int n = n_lo + hn;
        const double* v = sv + hn * kTabPad + i;
        HT* q = ch + ((w * K + k) * nh + (n - 1)) * 12;
        float bnd = 0.f, c3 = 0.f;
        for (int a = 0; a < 3; ++a) {
            const double* y = v + 2 * a * kTabH * kTabPad;
            const double* d = y + kTabH * kTabPad;
            double cc[4];
            hermite_coeffs(y[0], d[0], y[1], d[1], h, cc);
            float sa = 0.f;
            for (int j = 0; j < 4; ++j) {
                q[4 * a + j] = (HT)cc[j];
                sa += fabsf((float)(HT)cc[j]);
            }
            bnd = fmaxf(bnd, sa);
            c3 = fmaxf(c3, fabsf((float)(HT)cc[3]));
        }
        // the amplitude bound over u in [0, 1] and the largest cubic
        // coefficient of this harmonic, for the synthesis to leave out what
        // cannot change an FP32 sum
        if (hb) hb[(w * K + k) * nh + (n - 1)] = float2{bnd, c3};
    }
}

// FP32 synthesis: per (walker, interval) of the segment, the number of
// harmonics to sum and whether the cubic amplitude terms matter.  With M the
// largest amplitude bound of the interval's harmonics (k_amp_tables: the sum of
// a cubic's absolute coefficients, which bounds it over u in [0, 1]), the
// harmonics past the last one whose bound reaches kTiny M are left out, and
// the cubic terms are dropped when every harmonic's cubic coefficients are
// below kTiny M.  kTiny = 2^-24 is FP32's unit roundoff: past their peak
// the Peters-Mathews amplitudes decay monotonically, so what is left out
// stays within a few kTiny M, the size of the FP32 sum's own rounding.
__global__ void __launch_bounds__(256) k_harm_extent(int64_t K, int nh, int64_t k0, int64_t k1,
                                                     int seg, const double* __restrict__ wc,
                                                     const float2* __restrict__ hb,
                                                     int2* __restrict__ hx)
{
    constexpr float kTiny = 5.960464477539063e-08f;   // 2^-24
    const int64_t w = blockIdx.y;
    const int64_t k = k0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= k1) return;
    const double* c = wc + w * WC;
    if (c[WC_VALID] == 0.0 || k >= (int64_t)c[WC_KSEG + seg]) return;
    const float2* b = hb + (w * K + k) * nh;
    float M = 0.f, c3 = 0.f;
    for (int n = 0; n < nh; ++n) {
        M = fmaxf(M, b[n].x);
        c3 = fmaxf(c3, b[n].y);
    }
    int nsum = 0;
    for (int n = 0; n < nh; ++n)
        if (b[n].x >= kTiny * M) nsum = n + 1;
    // M = 0 (no signal) or a non-finite bound: sum everything
    if (!(M > 0.f) || !(M <= 3.4e38f)) nsum = nh;
    hx[w * K + k] = int2{nsum, (c3 < kTiny * M) ? 0 : 1};
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static GL8 make_gl8()
{
    // roots of the Legendre polynomial P_8 by Newton's method in long double
    GL8 g;
    const int n = 8;
    for (int i = 0; i < 4; ++i) {
        long double x = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
        long double dp = 0;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = x;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1);
            long double dx = p1 / dp;
            x -= dx;
            if (fabsl(dx) < 1e-19L) break;
        }
        g.x[i] = (double)x;
        g.w[i] = (double)(2.0L / ((1 - x * x) * dp * dp));
    }
    return g;
}

hipError_t launch_walker_setup(const Plan& p, const double* params, int64_t B, void* ws,
                               int64_t k1, hipStream_t s)
{
    static const GL8 gl = make_gl8();
    const bool back = p.ic == EMRI_IC_LSO;
    // forward: nodes 0 .. k1; backward from the LSO: nodes K .. k1 (k1 = K:
    // an empty first segment, node K alone)
    if (k1 < 0 || k1 > p.K) return hipErrorInvalidValue;
    char* base = (char*)ws;
    const double h = p.dt * (double)p.L;
    dim3 grid((unsigned)((B + 63) / 64));
    trace_mark(ST_SETUP, s, true);
    if (p.ode == EMRI_ODE_DP5 || p.ode == EMRI_ODE_RK78) {
        hipLaunchKernelGGL(k_walker_setup_adaptive, grid, dim3(64), 0, s, params, B, p.K, h,
                           (double)p.N * p.dt, gl, p.ic, (double*)(base + p.off_wc),
                           (double*)(base + p.off_orb));
        if (B > 0 && p.ode == EMRI_ODE_DP5)
            hipLaunchKernelGGL(k_orbit_dp5, dim3((unsigned)B), dim3(64), 0, s, p.K, h, k1, 0,
                               back ? 1 : 0, p.rtol, p.atol, (double*)(base + p.off_wc),
                               (double*)(base + p.off_orb));
        if (B > 0 && p.ode == EMRI_ODE_RK78)
            hipLaunchKernelGGL(k_orbit_rk78, grid, dim3(64), 0, s, B, p.K, h, k1, 0,
                               back ? 1 : 0, p.rtol, p.atol, (double*)(base + p.off_wc),
                               (double*)(base + p.off_orb));
    } else
        hipLaunchKernelGGL(k_walker_setup, grid, dim3(64), 0, s, params, B, p.K, h,
                           (double)p.N * p.dt, gl, k1, p.ic, (double*)(base + p.off_wc),
                           (double*)(base + p.off_orb));
    trace_mark(ST_SETUP, s, false);
    return hipGetLastError();
}

hipError_t launch_walker_resume(const Plan& p, int64_t B, void* ws, int64_t k0, int64_t k1,
                                int seg, hipStream_t s)
{
    const bool back = p.ic == EMRI_IC_LSO;
    // forward: steps from node k0 up to node k1; backward: from k0 down to k1
    // (k0 = k1: an empty segment)
    if (seg < 1 || seg >= kMaxSeg ||
        (back ? (k1 < 0 || k0 < k1 || k0 > p.K) : (k0 < 0 || k1 < k0 || k1 > p.K)))
        return hipErrorInvalidValue;
    char* base = (char*)ws;
    const double h = p.dt * (double)p.L;
    dim3 grid((unsigned)((B + 63) / 64));
    trace_mark(ST_SETUP, s, true);
    if (p.ode == EMRI_ODE_DP5) {
        if (B > 0)
            hipLaunchKernelGGL(k_orbit_dp5, dim3((unsigned)B), dim3(64), 0, s, p.K, h, k1, seg,
                               back ? 1 : 0, p.rtol, p.atol, (double*)(base + p.off_wc),
                               (double*)(base + p.off_orb));
    } else if (p.ode == EMRI_ODE_RK78) {
        if (B > 0)
            hipLaunchKernelGGL(k_orbit_rk78, grid, dim3(64), 0, s, B, p.K, h, k1, seg,
                               back ? 1 : 0, p.rtol, p.atol, (double*)(base + p.off_wc),
                               (double*)(base + p.off_orb));
    } else if (back) {
        hipLaunchKernelGGL(k_walker_resume_back, grid, dim3(64), 0, s, B, p.K, h, k0, k1, seg,
                           (double*)(base + p.off_wc), (double*)(base + p.off_orb));
    } else {
        hipLaunchKernelGGL(k_walker_resume, grid, dim3(64), 0, s, B, p.K, h, k0, k1, seg,
                           (double*)(base + p.off_wc), (double*)(base + p.off_orb));
    }
    trace_mark(ST_SETUP, s, false);
    return hipGetLastError();
}

// one lane per (walker, node)
__global__ void __launch_bounds__(256) k_orbit_out(int64_t B, int64_t K,
                                                   const double* __restrict__ wc,
                                                   const double* __restrict__ src,
                                                   double* __restrict__ dst, int32_t* __restrict__ kw)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * (K + 1)) return;
    const int64_t w = i / (K + 1), k = i - w * (K + 1);
    const double* c = wc + w * WC;
    const int64_t last = (c[WC_VALID] != 0.0) ? (int64_t)c[WC_KW] : -1;
    const double* q = src + i * 10;
    double* o = dst + i * 10;
#pragma unroll
    for (int j = 0; j < 10; ++j) o[j] = (k <= last) ? q[j] : 0.0;
    if (k == 0) kw[w] = (int32_t)last;
}

hipError_t launch_orbit_out(const Plan& p, int64_t B, const void* ws, double* orb, int32_t* kw,
                            hipStream_t s)
{
    const char* base = (const char*)ws;
    const int64_t n = B * (p.K + 1);
    if (n > 0)
        hipLaunchKernelGGL(k_orbit_out, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, B,
                           p.K, (const double*)(base + p.off_wc),
                           (const double*)(base + p.off_orb), orb, kw);
    return hipGetLastError();
}

hipError_t launch_tables(const Plan& p, int64_t B, void* ws, int64_t k0, int64_t k1, int seg,
                         hipStream_t s)
{
    if (seg < 0 || seg >= kMaxSeg || k0 < 0 || k1 < k0 || k1 > p.K) return hipErrorInvalidValue;
    char* base = (char*)ws;
    const double h = p.dt * (double)p.L;
    const double* wc = (const double*)(base + p.off_wc);
    const double* orb = (const double*)(base + p.off_orb);
    trace_mark(ST_TABLES, s, true);
    const int64_t n = k1 - k0;
    if (n > 0) {
        const int ng = (p.nh + kTabH - 1) / kTabH;
        const dim3 grid((unsigned)(((n + kTabI - 1) / kTabI) * ng), (unsigned)B);
        if (p.prec == EMRI_FP64) {
            hipLaunchKernelGGL(k_amp_tables<double>, grid, dim3(256), 0, s, p.K, p.nh, h, k0, k1,
                               seg, wc, orb, (double*)(base + p.off_co),
                               (double*)(base + p.off_ch), (float2*)nullptr);
        } else {
            hipLaunchKernelGGL(k_amp_tables<float>, grid, dim3(256), 0, s, p.K, p.nh, h, k0, k1,
                               seg, wc, orb, (double*)(base + p.off_co),
                               (float*)(base + p.off_ch), (float2*)(base + p.off_hb));
            if (hipPeekAtLastError() == hipSuccess)
                hipLaunchKernelGGL(k_harm_extent,
                                   dim3((unsigned)((k1 - k0 + 255) / 256), (unsigned)B), dim3(256),
                                   0, s, p.K, p.nh, k0, k1, seg, wc,
                                   (const float2*)(base + p.off_hb), (int2*)(base + p.off_hx));
        }
    }
    trace_mark(ST_TABLES, s, false);
    return hipGetLastError();
}

}  // namespace emri
