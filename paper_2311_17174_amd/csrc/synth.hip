// synth.hip -- stage (b): time-domain AK waveform on the fine sampling grid.
//
// One workgroup of LANES lanes (256; 128 for FP32 at 2^10 samples per
// interval) per (coarse interval k, walker w), over the intervals [k0, k1) of
// one orbit segment; each lane produces SPT = 2^coarse_log2 / LANES
// consecutive samples j = k 2^cl + lane SPT + s.  Everything a wave needs
// from the orbit and the amplitude tables is uniform over the interval and is
// read with scalar loads.  When
// the phases advance by less than 0.25 rad per sample (checked per interval
// from the Hermite coefficients), a lane evaluates sin/cos once and rotates
// by small-angle factors for its next samples.
//
// Per sample (Eq. (2) with the BC04 response; the oracle spells out the same
// quantities with angles and atan2, here double angles come from the
// tangent-pair identities cos 2x = (c^2 - s^2)/(c^2 + s^2) and
// sin 2x = 2 s c / (c^2 + s^2), so no inverse trigonometry is evaluated):
//   Phi, nu, gamma~, alpha      cubic Hermite in u (FP64)
//   Phi' = Phi + 2 pi nu R sin(theta_S) cos(phibar - phi_S)  Doppler phase
//   L = cos(lambda) S + sin(lambda) (cos(alpha) e1 + sin(alpha) e2)
//   S_a = sum_n A n P_n cos(n Phi'), S_b = sum_n A n Q_n sin(n Phi'),
//   S_c = sum_n 2 A J_n cos(n Phi')   (cos, sin of n Phi' by the three-term
//                                       recurrence; in FP32 the terms below
//                                       its rounding are left out)
//   h+ = (1 + c^2)(S_a cos 2g - S_b sin 2g) + (1 - c^2) S_c
//   hx = -2 c (S_b cos 2g + S_a sin 2g),  c = L.N, g = gamma~ + beta
//   h_I/II = sqrt(3)/2 (F+ h+ + Fx hx), channel II at phi_d - pi/4
#include "internal.hpp"

namespace emri {

template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

// sin/cos of a small angle by Taylor series: |d| <= 0.3 gives full FP64
// accuracy (the first omitted term is below 1e-19); the FP32 variant stops
// at d^9 (below 1e-10 relative)
__device__ __forceinline__ void small_sincos(double d, double* s, double* c)
{
    const double d2 = d * d;
    *s = d * (1.0 - d2 * (1.0 / 6 - d2 * (1.0 / 120 - d2 * (1.0 / 5040 - d2 * (1.0 / 362880 -
             d2 * (1.0 / 39916800 - d2 * (1.0 / 6227020800.0)))))));
    *c = 1.0 - d2 * (0.5 - d2 * (1.0 / 24 - d2 * (1.0 / 720 - d2 * (1.0 / 40320 -
             d2 * (1.0 / 3628800 - d2 * (1.0 / 479001600.0 - d2 * (1.0 / 87178291200.0)))))));
}
__device__ __forceinline__ void small_sincos(float d, float* s, float* c)
{
    const float d2 = d * d;
    *s = d * (1.f - d2 * (1.f / 6 - d2 * (1.f / 120 - d2 * (1.f / 5040 - d2 * (1.f / 362880)))));
    *c = 1.f - d2 * (0.5f - d2 * (1.f / 24 - d2 * (1.f / 720 - d2 * (1.f / 40320))));
}

// degenerate-angle thresholds for the squared norm of a tangent pair: 1e-24 in
// FP64, 1e-10 in FP32, where rounding residues themselves reach ~1e-14
template <typename R> struct Degenerate;
template <> struct Degenerate<double> { static constexpr double v = 1e-24; };
template <> struct Degenerate<float> { static constexpr float v = 1e-10f; };

// 1/x for the normalisation of the tangent pairs (x is a product of squared
// norms in [1e-72, 1e3]): the hardware reciprocal refined by Newton steps,
// two in FP64 (from about 2^-29 to full precision), one in FP32
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float recip(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// sin/cos of an FP64 angle in precision R: FP64 uses the library sincos;
// FP32 reduces the angle modulo 2 pi in FP64 first.
__device__ inline void angle_sincos(double a, double* s, double* c) { sincos(a, s, c); }
__device__ inline void angle_sincos(double a, float* s, float* c)
{
    double r = a * (0.5 / kPi);
    r -= rint(r);                      // r in [-1/2, 1/2]
    sincospif((float)(2.0 * r), s, c);
}

// e^{i a_s} for the SPT consecutive angles a_s of one lane: on a smooth
// interval (every step |a_s - a_{s-1}| < 0.25 rad) one sincos, then
// rotations by the small steps; otherwise one sincos per sample.
template <typename R, int SPT>
__device__ __forceinline__ void angle_run(const double (&a)[SPT], bool smooth, R (&c)[SPT],
                                          R (&s)[SPT])
{
    angle_sincos(a[0], &s[0], &c[0]);
#pragma unroll
    for (int k = 1; k < SPT; ++k) {
        if (smooth) {
            R sd, cd;
            small_sincos((R)(a[k] - a[k - 1]), &sd, &cd);
            c[k] = c[k - 1] * cd - s[k - 1] * sd;
            s[k] = s[k - 1] * cd + c[k - 1] * sd;
        } else {
            angle_sincos(a[k], &s[k], &c[k]);
        }
    }
}

// up to 4 samples per lane the register budget is capped at 128 (4 waves
// per SIMD; a few spills outside the harmonic loop are cheaper than the
// lost occupancy); longer runs keep their registers
template <typename R, typename HT, int SPT, int LANES>
__global__ void __launch_bounds__(LANES) __attribute__((amdgpu_waves_per_eu(SPT <= 4 ? 4 : 1)))
k_synth(int64_t K, int64_t Nv, int64_t N, int nh,
                                               int64_t k0, int seg, int zfill,
                                               double dt, const double* __restrict__ wc,
                                               const double* __restrict__ co,
                                               const HT* __restrict__ ch,
                                               const int2* __restrict__ hx,
                                               const double2* __restrict__ az,
                                               typename V2<R>::T* __restrict__ out)
{
    using R2 = typename V2<R>::T;
    constexpr int L = LANES * SPT;
    const int64_t k = k0 + blockIdx.x;
    const int64_t w = blockIdx.y;
    const int lane = threadIdx.x;
    R2* zw = out + w * N;
    const int64_t j0 = k * L;
    const int64_t jl = j0 + (int64_t)lane * SPT;      // this lane's first sample
    const double* c = wc + w * WC;
    const int64_t Kw = (int64_t)c[WC_KSEG + seg];
    if (c[WC_VALID] == 0.0 || k >= Kw || j0 >= Nv) {
        if (zfill) {
#pragma unroll
            for (int s = 0; s < SPT; ++s) zw[jl + s] = R2{R(0), R(0)};
        }
        return;
    }

    // ---- uniform per interval --------------------------------------------
    const double* q = co + (w * K + k) * 16;
    const double dop = c[WC_DOP];
    const double cps = c[WC_CPS], sps = c[WC_SPS];
    const double2 a0 = az[k];                          // detector azimuth at j0
    const double cb0 = a0.x, sb0 = a0.y;
    const double dphi = 2.0 * kPi * dt / kYearSeconds;   // per sample
    const double invL = 1.0 / (double)L;
    // largest per-sample step of Phi' (plus a Doppler margin), 2 gamma~, alpha
    const double stepPhi = (fabs(q[1]) + 2.0 * fabs(q[2]) + 3.0 * fabs(q[3])) * invL + 1e-3;
    const double stepG = 2.0 * (fabs(q[9]) + 2.0 * fabs(q[10]) + 3.0 * fabs(q[11])) * invL;
    const double stepA = (fabs(q[13]) + 2.0 * fabs(q[14]) + 3.0 * fabs(q[15])) * invL;
    const bool smooth = stepPhi < 0.25 && stepG < 0.25 && stepA < 0.25;

    // ---- per sample: phases ------------------------------------------------
    R u[SPT];                               // interval coordinate
    R c1[SPT], s1[SPT];                     // e^{i Phi'}
    double ph[SPT];
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
        const int off = lane * SPT + s;
        const double ud = (double)off * invL;
        u[s] = (R)ud;
        const double Phi = ((q[3] * ud + q[2]) * ud + q[1]) * ud + q[0];
        const double nu = ((q[7] * ud + q[6]) * ud + q[5]) * ud + q[4];
        R sd, cd;
        small_sincos((R)(dphi * (double)off), &sd, &cd);
        const R cb = (R)cb0 * cd - (R)sb0 * sd;
        const R sb = (R)sb0 * cd + (R)cb0 * sd;
        const double cdel = (double)cb * cps + (double)sb * sps;   // cos(phibar - phi_S)
        ph[s] = Phi + dop * nu * cdel;                              // Doppler-shifted phase
    }
    angle_run<R, SPT>(ph, smooth, c1, s1);
    if constexpr (sizeof(R) == 4) {
        // the FP32 rotation chain leaves |e^{i Phi'}| a few rounding units
        // off 1, an error of cos(Phi') that the recurrence below carries
        // n^2-fold into harmonic n: renormalise by one Newton step for
        // 1/sqrt(q) at q = 1 (r = (3 - q)/2, exact to O((q - 1)^2) and, with
        // round-to-nearest arithmetic only, free of a systematic scale)
#pragma unroll
        for (int s = 1; s < SPT; ++s) {
            const R q = fmaf(c1[s], c1[s], s1[s] * s1[s]);
            const R r = fmaf(-0.5f, q, 1.5f);
            c1[s] *= r;
            s1[s] *= r;
        }
    }

    // ---- harmonic sum ------------------------------------------------------
    // cos/sin(n Phi') for n = 1..nh by the three-term recurrence
    // x_{n+1} = 2 cos(Phi') x_n - x_{n-1}: one FMA per value.  An error made
    // at step m is carried forward at most (n - m + 1)-fold (|U_k| <= k + 1),
    // which sums to n^2/2 rounding units; an error dc of cos(Phi') itself
    // moves T_n by at most n |U_{n-1}| |dc| <= n^2 |dc|.  Harmonic n so
    // carries at most about (3/2) n^2 rounding units of its own amplitude; the
    // sum's error is set by the strong harmonics
    R Sa[SPT], Sb[SPT], Sc[SPT], cn[SPT], sn[SPT], cq[SPT], sq[SPT], tc[SPT];
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
        Sa[s] = Sb[s] = Sc[s] = R(0);
        cn[s] = c1[s];
        sn[s] = s1[s];
        cq[s] = R(1);
        sq[s] = R(0);
        tc[s] = R(2) * c1[s];
    }
    const HT* hq = ch + (w * K + k) * (int64_t)nh * 12;
    int nsum = nh;           // harmonics summed
    bool cubic = true;       // amplitude polynomials of degree 3 (else 2)
    if constexpr (sizeof(R) == 4) {
        // FP32: the harmonics and cubic terms that cannot change the sum at
        // its precision are left out (k_harm_extent: the number of
        // harmonics to sum and whether the cubic terms matter, per walker
        // and interval)
        const int2 x = hx[w * K + k];
        nsum = x.x;
        cubic = x.y != 0;
    }
    if (cubic) {
#pragma unroll 2
        for (int n = 0; n < nsum; ++n) {
            const HT* t = hq + 12 * n;
            const R a0 = (R)t[0], a1 = (R)t[1], a2 = (R)t[2], a3 = (R)t[3];
            const R b0 = (R)t[4], b1 = (R)t[5], b2 = (R)t[6], b3 = (R)t[7];
            const R e0 = (R)t[8], e1 = (R)t[9], e2 = (R)t[10], e3 = (R)t[11];
#pragma unroll
            for (int s = 0; s < SPT; ++s) {
                const R x = u[s];
                const R ua = ((a3 * x + a2) * x + a1) * x + a0;
                const R ub = ((b3 * x + b2) * x + b1) * x + b0;
                const R uc = ((e3 * x + e2) * x + e1) * x + e0;
                Sa[s] += ua * cn[s];
                Sb[s] += ub * sn[s];
                Sc[s] += uc * cn[s];
                const R cc = tc[s] * cn[s] - cq[s];
                const R ss = tc[s] * sn[s] - sq[s];
                cq[s] = cn[s];
                sq[s] = sn[s];
                cn[s] = cc;
                sn[s] = ss;
            }
        }
    } else {
        // the same with the cubic terms left out (FP32 only); the table row
        // is read in the same 16-byte pieces as above
#pragma unroll 2
        for (int n = 0; n < nsum; ++n) {
            const float4* t = (const float4*)(hq + 12 * n);
            const float4 ta = t[0], tb = t[1], te = t[2];
            const R a0 = (R)ta.x, a1 = (R)ta.y, a2 = (R)ta.z;
            const R b0 = (R)tb.x, b1 = (R)tb.y, b2 = (R)tb.z;
            const R e0 = (R)te.x, e1 = (R)te.y, e2 = (R)te.z;
#pragma unroll
            for (int s = 0; s < SPT; ++s) {
                const R x = u[s];
                const R ua = (a2 * x + a1) * x + a0;
                const R ub = (b2 * x + b1) * x + b0;
                const R uc = (e2 * x + e1) * x + e0;
                Sa[s] += ua * cn[s];
                Sb[s] += ub * sn[s];
                Sc[s] += uc * cn[s];
                const R cc = tc[s] * cn[s] - cq[s];
                const R ss = tc[s] * sn[s] - sq[s];
                cq[s] = cn[s];
                sq[s] = sn[s];
                cn[s] = cc;
                sn[s] = ss;
            }
        }
    }

    // ---- geometry, response, store -----------------------------------------
    // one sample at a time, with the angles carried from sample to sample
    // (the same rotations as for Phi'), so that only the three harmonic sums
    // stay live from the loop above
    const R Nx = (R)c[WC_NX], Ny = (R)c[WC_NY], Nz = (R)c[WC_NZ];
    const R Sx = (R)c[WC_SX], Sy = (R)c[WC_SY], Sz = (R)c[WC_SZ];
    const R E1x = (R)c[WC_E1X], E1y = (R)c[WC_E1Y], E1z = (R)c[WC_E1Z];
    const R E2x = (R)c[WC_E2X], E2y = (R)c[WC_E2Y];
    const R cl = (R)c[WC_CL], sl = (R)c[WC_SL], NS = (R)c[WC_NS];
    const R cts = (R)c[WC_CTS], sts = (R)c[WC_STS];
    const R Rcps = (R)cps, Rsps = (R)sps;
    // N x S, for sin(beta) = L . (N x S)
    const R NSx = Ny * Sz - Nz * Sy, NSy = Nz * Sx - Nx * Sz, NSz = Nx * Sy - Ny * Sx;
    const R h3 = (R)0.8660254037844386467637231707529362;  // sqrt(3)/2
    const R thr = Degenerate<R>::v;
    R sdp, cdp;                                   // azimuth step per sample
    small_sincos((R)dphi, &sdp, &cdp);
    R cb = R(0), sb = R(0), c2g = R(0), s2g = R(0), ca = R(0), sa = R(0);
    double gprev = 0.0, aprev = 0.0;
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
        const int64_t j = jl + s;
        const double ud = (double)(lane * SPT + s) * invL;
        const double gam2 = 2.0 * (((q[11] * ud + q[10]) * ud + q[9]) * ud + q[8]);
        const double alp = ((q[15] * ud + q[14]) * ud + q[13]) * ud + q[12];
        if (s == 0) {
            R sd, cd;
            small_sincos((R)(dphi * (double)(lane * SPT)), &sd, &cd);
            cb = (R)cb0 * cd - (R)sb0 * sd;
            sb = (R)sb0 * cd + (R)cb0 * sd;
            angle_sincos(gam2, &s2g, &c2g);
            angle_sincos(alp, &sa, &ca);
        } else {
            const R t = cb * cdp - sb * sdp;
            sb = sb * cdp + cb * sdp;
            cb = t;
            if (smooth) {
                R sd, cd;
                small_sincos((R)(gam2 - gprev), &sd, &cd);
                const R tg = c2g * cd - s2g * sd;
                s2g = s2g * cd + c2g * sd;
                c2g = tg;
                small_sincos((R)(alp - aprev), &sd, &cd);
                const R ta = ca * cd - sa * sd;
                sa = sa * cd + ca * sd;
                ca = ta;
            } else {
                angle_sincos(gam2, &s2g, &c2g);
                angle_sincos(alp, &sa, &ca);
            }
        }
        gprev = gam2;
        aprev = alp;
        if (j >= Nv) {
            zw[j] = R2{R(0), R(0)};
            continue;
        }
        const R Lx = cl * Sx + sl * (ca * E1x + sa * E2x);
        const R Ly = cl * Sy + sl * (ca * E1y + sa * E2y);
        const R Lz = cl * Sz + sl * (ca * E1z);
        const R ci = Lx * Nx + Ly * Ny + Lz * Nz;
        // the three angles beta, phi_d - phibar and psi as tangent pairs
        // (x, y) = (|.| cos, |.| sin); beta is undefined (0) when sin(lambda) = 0
        const R bx = NS - ci * cl, by = Lx * NSx + Ly * NSy + Lz * NSz;
        const R cdel = cb * Rcps + sb * Rsps;         // cos(phibar - phi_S)
        const R sdel = sb * Rcps - cb * Rsps;         // sin(phibar - phi_S)
        const R cthd = R(0.5) * cts - h3 * sts * cdel;
        const R dx = R(2) * sts * sdel, dy = R(2) * h3 * cts + sts * cdel;
        const R zx = -h3 * cb, zy = -h3 * sb, zz = R(0.5);
        const R Lzd = Lx * zx + Ly * zy + Lz * zz;
        const R NLx = Ny * Lz - Nz * Ly, NLy = Nz * Lx - Nx * Lz, NLz = Nx * Ly - Ny * Lx;
        const R px_ = zx * NLx + zy * NLy + zz * NLz, py_ = Lzd - ci * cthd;
        // one reciprocal for the three squared norms; a degenerate pair
        // becomes (1, 0) (angle 0)
        R nb = bx * bx + by * by, nd = dx * dx + dy * dy, np = px_ * px_ + py_ * py_;
        const bool okb = (sl != R(0)) && nb >= thr, okd = nd >= thr, okp = np >= thr;
        if (!okb) nb = R(1);
        if (!okd) nd = R(1);
        if (!okp) np = R(1);
        const R inv = recip(nb * nd * np);
        const R ib = nd * np * inv, idd = nb * np * inv, ip = nb * nd * inv;
        const R c2b = okb ? (bx * bx - by * by) * ib : R(1);
        const R s2b = okb ? R(2) * bx * by * ib : R(0);
        const R c2d = okd ? (dx * dx - dy * dy) * idd : R(1);
        const R s2d = okd ? R(2) * dx * dy * idd : R(0);
        const R c2s = okp ? (px_ * px_ - py_ * py_) * ip : R(1);
        const R s2s = okp ? R(2) * px_ * py_ * ip : R(0);

        const R c2 = c2g * c2b - s2g * s2b;     // cos 2 gamma, gamma = gamma~ + beta
        const R s2 = s2g * c2b + c2g * s2b;     // sin 2 gamma
        const R ci2 = ci * ci;
        const R hp = (R(1) + ci2) * (Sa[s] * c2 - Sb[s] * s2) + (R(1) - ci2) * Sc[s];
        const R hx = R(-2) * ci * (Sb[s] * c2 + Sa[s] * s2);
        const R c2pb = cb * cb - sb * sb, s2pb = R(2) * sb * cb;
        const R c2p = c2pb * c2d - s2pb * s2d;        // cos 2 phi_d
        const R s2p = s2pb * c2d + c2pb * s2d;        // sin 2 phi_d
        const R aa = R(0.5) * (R(1) + cthd * cthd);
        const R FpI = aa * c2p * c2s - cthd * s2p * s2s;
        const R FxI = aa * c2p * s2s + cthd * s2p * c2s;
        const R FpII = aa * s2p * c2s + cthd * c2p * s2s;
        const R FxII = aa * s2p * s2s - cthd * c2p * c2s;
        zw[j] = R2{h3 * (FpI * hp + FxI * hx), h3 * (FpII * hp + FxII * hx)};
    }
}

template <typename R, typename HT>
static hipError_t synth_dispatch(const Plan& p, int64_t B, const char* base, void* out,
                                 int64_t k0, int64_t k1, int seg, int zfill, hipStream_t s)
{
    dim3 grid((unsigned)(k1 - k0), (unsigned)B);
    using R2 = typename V2<R>::T;
    const double* wc = (const double*)(base + p.off_wc);
    const double* co = (const double*)(base + p.off_co);
    const HT* ch = (const HT*)(base + p.off_ch);
    const int2* hx = (p.prec == EMRI_MIXED) ? (const int2*)(base + p.off_hx) : nullptr;
    const double2* az = (const double2*)(base + p.off_az);
    R2* o = (R2*)out;
#define EMRI_SYNTH(SPT, LANES)                                                                 \
    hipLaunchKernelGGL((k_synth<R, HT, SPT, LANES>), grid, dim3(LANES), 0, s, p.K, p.Nv, p.N, p.nh, k0, \
                       seg, zfill, p.dt, wc, co, ch, hx, az, o)
    switch (p.cl) {
    case 8: EMRI_SYNTH(1, 256); break;
    case 9: EMRI_SYNTH(2, 256); break;
    case 10:
        // FP32 at 8 samples per lane (116 VGPRs, still four waves per SIMD)
        // shares each lane's fixed cost over twice the samples; FP64 at 8
        // would take 166 VGPRs (three waves) and leave no room beside it for
        // the amplitude tables of the next orbit segment
        if constexpr (sizeof(R) == 4) EMRI_SYNTH(8, 128);
        else EMRI_SYNTH(4, 256);
        break;
    case 11: EMRI_SYNTH(8, 256); break;
    case 12: EMRI_SYNTH(16, 256); break;
    default: return hipErrorInvalidValue;
    }
#undef EMRI_SYNTH
    return hipGetLastError();
}

hipError_t launch_synth(const Plan& p, int64_t B, void* ws, void* out, int64_t k0, int64_t k1,
                        int seg, bool zfill, hipStream_t s)
{
    if (seg < 0 || seg >= kMaxSeg || k0 < 0 || k1 < k0 || k1 > p.N / p.L)
        return hipErrorInvalidValue;
    if (k1 == k0) return hipSuccess;
    const char* base = (const char*)ws;
    trace_mark(ST_SYNTH, s, true);
    const hipError_t e =
        (p.prec == EMRI_FP64)
            ? synth_dispatch<double, double>(p, B, base, out, k0, k1, seg, zfill ? 1 : 0, s)
            : synth_dispatch<float, float>(p, B, base, out, k0, k1, seg, zfill ? 1 : 0, s);
    trace_mark(ST_SYNTH, s, false);
    return e;
}

// detector azimuth phibar = 2 pi t / yr at the first sample of each coarse
// interval: az[k] = (cos, sin) of it, shared by all walkers of a batch
__global__ void __launch_bounds__(256) k_azimuth(int64_t K, int64_t L, double dt,
                                                 double2* __restrict__ az)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    double s, c;
    sincospi(2.0 * (double)(k * L) * dt / kYearSeconds, &s, &c);
    az[k] = double2{c, s};
}

hipError_t launch_azimuth(const Plan& p, void* ws, hipStream_t s)
{
    double2* az = (double2*)((char*)ws + p.off_az);
    hipLaunchKernelGGL(k_azimuth, dim3((unsigned)((p.K + 255) / 256)), dim3(256), 0, s, p.K, p.L,
                       p.dt, az);
    return hipGetLastError();
}

}  // namespace emri
