// fft_lds.hpp -- in-LDS Stockham FFT building blocks shared by the FFT
// passes (fft.hip) and the fused row-FFT + likelihood kernel (like.hip).
//
// A column of L = 2^lgL complex values lives in LDS as two arrays re[], im[]
// indexed through px<R>(i) = i + i/16 (one pad slot per 16 elements), which makes
// the stride-8 writes of the first radix-8 stage bank-conflict free.  L/8
// lanes transform one column: radix-8 Stockham stages (one radix-4 or radix-2
// stage for the remainder), twiddles W_L^e from a device table, three table
// loads per radix-8 butterfly (w, w^2, w^4; the other powers by products).
// The first stage runs on values the lanes loaded into registers, and the
// last may leave its outputs there, so an L-point transform with S stages
// makes S-1 round trips through LDS.
#pragma once

#include "internal.hpp"

namespace emri {

template <typename R> struct C2;
template <> struct C2<double> { using T = double2; };
template <> struct C2<float> { using T = float2; };

// pad one slot per 2^PadShift<R> elements (one per 16: other paddings lowered
// the bank-conflict counters of some stages on MI355X but not the time)
template <typename R> struct PadShift { static constexpr int v = 4; };
template <typename R>
__device__ __host__ inline int px(int i) { return i + (i >> PadShift<R>::v); }
// LDS elements (per re or im array) of a padded column of length L
template <typename R>
__host__ __device__ inline int padded_len(int L) { return ((L + (L >> PadShift<R>::v)) + 15) & ~15; }

// ---------------------------------------------------------------------------
// small DFTs in registers, natural order out: b_q = sum_t a_t W_R^{t q}
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void dft2(R& ar, R& ai, R& br, R& bi)
{
    const R tr = ar - br, ti = ai - bi;
    ar += br; ai += bi;
    br = tr; bi = ti;
}

template <typename R>
__device__ __forceinline__ void dft4(R* xr, R* xi)  // 4 values, in place
{
    const R t0r = xr[0] + xr[2], t0i = xi[0] + xi[2];
    const R t1r = xr[0] - xr[2], t1i = xi[0] - xi[2];
    const R t2r = xr[1] + xr[3], t2i = xi[1] + xi[3];
    const R t3r = xi[1] - xi[3], t3i = xr[3] - xr[1];   // (a1 - a3) * (-i)
    xr[0] = t0r + t2r; xi[0] = t0i + t2i;
    xr[2] = t0r - t2r; xi[2] = t0i - t2i;
    xr[1] = t1r + t3r; xi[1] = t1i + t3i;
    xr[3] = t1r - t3r; xi[3] = t1i - t3i;
}

template <typename R>
__device__ __forceinline__ void dft8(R* xr, R* xi)
{
    // even / odd radix-4 halves, in scalars (no local arrays)
    const R a0r = xr[0] + xr[4], a0i = xi[0] + xi[4], a1r = xr[0] - xr[4], a1i = xi[0] - xi[4];
    const R a2r = xr[2] + xr[6], a2i = xi[2] + xi[6], a3r = xi[2] - xi[6], a3i = xr[6] - xr[2];
    const R e0r = a0r + a2r, e0i = a0i + a2i, e2r = a0r - a2r, e2i = a0i - a2i;
    const R e1r = a1r + a3r, e1i = a1i + a3i, e3r = a1r - a3r, e3i = a1i - a3i;
    const R b0r = xr[1] + xr[5], b0i = xi[1] + xi[5], b1r = xr[1] - xr[5], b1i = xi[1] - xi[5];
    const R b2r = xr[3] + xr[7], b2i = xi[3] + xi[7], b3r = xi[3] - xi[7], b3i = xr[7] - xr[3];
    const R o0r = b0r + b2r, o0i = b0i + b2i, o2r = b0r - b2r, o2i = b0i - b2i;
    const R o1r = b1r + b3r, o1i = b1i + b3i, o3r = b1r - b3r, o3i = b1i - b3i;
    const R h = (R)0.70710678118654752440084436210484903928;
    // W_8^1 = (1 - i)/sqrt2, W_8^2 = -i, W_8^3 = -(1 + i)/sqrt2
    const R w1r = h * (o1r + o1i), w1i = h * (o1i - o1r);
    const R w2r = o2i, w2i = -o2r;
    const R w3r = h * (o3i - o3r), w3i = -h * (o3r + o3i);
    xr[0] = e0r + o0r; xi[0] = e0i + o0i;
    xr[4] = e0r - o0r; xi[4] = e0i - o0i;
    xr[1] = e1r + w1r; xi[1] = e1i + w1i;
    xr[5] = e1r - w1r; xi[5] = e1i - w1i;
    xr[2] = e2r + w2r; xi[2] = e2i + w2i;
    xr[6] = e2r - w2r; xi[6] = e2i - w2i;
    xr[3] = e3r + w3r; xi[3] = e3i + w3i;
    xr[7] = e3r - w3r; xi[7] = e3i - w3i;
}

template <typename R>
__device__ __forceinline__ void cmul(R& xr, R& xi, R wr, R wi)
{
    const R t = xr * wr - xi * wi;
    xi = xr * wi + xi * wr;
    xr = t;
}

// One Stockham stage of radix RR over an L-point column in LDS: lane t
// handles 8/RR butterflies j = t + b L/8; Ns is the product of the radices
// of the previous stages.  W_{Ns RR}^{r k} = W_L^{r k tws}.
template <typename R, int RR>
__device__ __forceinline__ void lds_stage(R* re, R* im, int L, int Ns, int t,
                                 const typename C2<R>::T* __restrict__ tw)
{
    using T2 = typename C2<R>::T;
    constexpr int NB = 8 / RR;
    const int stride = L / RR;
    const int tws = L / (Ns * RR);
    R vr[8], vi[8];
    asm volatile("" ::: "memory");   // no hoisting of twiddle loads across stages
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * (L / 8);
        const int k = j & (Ns - 1);
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            vr[b * RR + r] = re[px<R>(j + r * stride)];
            vi[b * RR + r] = im[px<R>(j + r * stride)];
        }
        if (k > 0) {
            // twiddle powers w^r, r = 1..RR-1, w = W_L^{k tws}
            R wr[8], wi[8];
            const T2 w1 = tw[k * tws];
            wr[1] = w1.x; wi[1] = w1.y;
            if constexpr (RR >= 4) {
                const T2 w2 = tw[2 * k * tws];
                wr[2] = w2.x; wi[2] = w2.y;
                wr[3] = w1.x * w2.x - w1.y * w2.y; wi[3] = w1.x * w2.y + w1.y * w2.x;
            }
            if constexpr (RR == 8) {
                const T2 w4 = tw[4 * k * tws];
                wr[4] = w4.x; wi[4] = w4.y;
                wr[5] = w1.x * w4.x - w1.y * w4.y; wi[5] = w1.x * w4.y + w1.y * w4.x;
                wr[6] = wr[2] * w4.x - wi[2] * w4.y; wi[6] = wr[2] * w4.y + wi[2] * w4.x;
                wr[7] = wr[3] * w4.x - wi[3] * w4.y; wi[7] = wr[3] * w4.y + wi[3] * w4.x;
            }
#pragma unroll
            for (int r = 1; r < RR; ++r) cmul(vr[b * RR + r], vi[b * RR + r], wr[r], wi[r]);
        }
    }
    __syncthreads();
    if constexpr (RR == 8) {
        dft8(vr, vi);
    } else if constexpr (RR == 4) {
        dft4(vr, vi);
        dft4(vr + 4, vi + 4);
    } else {
#pragma unroll
        for (int b = 0; b < 4; ++b) dft2(vr[2 * b], vi[2 * b], vr[2 * b + 1], vi[2 * b + 1]);
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * (L / 8);
        const int k = j & (Ns - 1);
        const int base = (j - k) * RR + k;
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            re[px<R>(base + r * Ns)] = vr[b * RR + r];
            im[px<R>(base + r * Ns)] = vi[b * RR + r];
        }
    }
    __syncthreads();
}

// L-point FFT (L = 2^lgL >= 8) of one padded column already in LDS, every
// stage through LDS, by lane t of L/8.  Every lane of the workgroup must
// call it (it contains barriers).
template <typename R>
__device__ __forceinline__ void lds_fft(R* re, R* im, int L, int lgL, int t,
                                        const typename C2<R>::T* __restrict__ tw)
{
    const int n8 = lgL / 3, rem = lgL - 3 * n8;
    int Ns = 1;
    for (int st = 0; st < n8; ++st) {
        lds_stage<R, 8>(re, im, L, Ns, t, tw);
        Ns *= 8;
    }
    if (rem == 2) lds_stage<R, 4>(re, im, L, Ns, t, tw);
    else if (rem == 1) lds_stage<R, 2>(re, im, L, Ns, t, tw);
}

// Last Stockham stage (radix RR, Ns = L/RR) from LDS into registers: lane t
// receives the outputs at positions t + i L/8, i = 0..7, in x[i].
template <typename R, int RR>
__device__ __forceinline__ void last_stage_to_regs(const R* re, const R* im, int L, int t,
                                                   const typename C2<R>::T* __restrict__ tw,
                                                   R (&xr)[8], R (&xi)[8])
{
    using T2 = typename C2<R>::T;
    constexpr int NB = 8 / RR;
    const int stride = L / RR;       // = Ns of this stage: tws = 1
    R vr[8], vi[8];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * (L / 8);   // j < Ns: k = j
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            vr[b * RR + r] = re[px<R>(j + r * stride)];
            vi[b * RR + r] = im[px<R>(j + r * stride)];
        }
        if (j > 0) {
            R wr[8], wi[8];
            const T2 w1 = tw[j];
            wr[1] = w1.x; wi[1] = w1.y;
            if constexpr (RR >= 4) {
                const T2 w2 = tw[2 * j];
                wr[2] = w2.x; wi[2] = w2.y;
                wr[3] = w1.x * w2.x - w1.y * w2.y; wi[3] = w1.x * w2.y + w1.y * w2.x;
            }
            if constexpr (RR == 8) {
                const T2 w4 = tw[4 * j];
                wr[4] = w4.x; wi[4] = w4.y;
                wr[5] = w1.x * w4.x - w1.y * w4.y; wi[5] = w1.x * w4.y + w1.y * w4.x;
                wr[6] = wr[2] * w4.x - wi[2] * w4.y; wi[6] = wr[2] * w4.y + wi[2] * w4.x;
                wr[7] = wr[3] * w4.x - wi[3] * w4.y; wi[7] = wr[3] * w4.y + wi[3] * w4.x;
            }
#pragma unroll
            for (int r = 1; r < RR; ++r) cmul(vr[b * RR + r], vi[b * RR + r], wr[r], wi[r]);
        }
    }
    if constexpr (RR == 8) {
        dft8(vr, vi);
    } else if constexpr (RR == 4) {
        dft4(vr, vi);
        dft4(vr + 4, vi + 4);
    } else {
#pragma unroll
        for (int b = 0; b < 4; ++b) dft2(vr[2 * b], vi[2 * b], vr[2 * b + 1], vi[2 * b + 1]);
    }
    // output q of butterfly b sits at t + (b + q NB) L/8
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int q = 0; q < RR; ++q) {
            xr[b + q * NB] = vr[b * RR + q];
            xi[b + q * NB] = vi[b * RR + q];
        }
}

// L-point FFT (L = 2^lgL >= 8) of one column whose lane t holds, on entry,
// the elements at positions t + i L/8 (i = 0..7) in x.  The first radix-8
// stage runs on those registers, the middle stages in LDS; with OUT_REGS the
// last stage leaves the outputs at positions t + i L/8 in x, otherwise the
// transform is left in LDS (padded).  Every lane of the workgroup must call
// it; with OUT_REGS the caller synchronises before LDS is written again.
template <typename R, bool OUT_REGS>
__device__ __forceinline__ void fft_regs(R* re, R* im, int L, int lgL, int t,
                                         const typename C2<R>::T* __restrict__ tw, R (&xr)[8],
                                         R (&xi)[8])
{
    const int n8 = lgL / 3, rem = lgL - 3 * n8;
    const int nst = n8 + (rem ? 1 : 0);
    dft8(xr, xi);                          // stage 1: Ns = 1, no twiddles
    if (nst == 1) {                        // L = 8: outputs already at t + i
        if (!OUT_REGS) {
#pragma unroll
            for (int r = 0; r < 8; ++r) { re[px<R>(r)] = xr[r]; im[px<R>(r)] = xi[r]; }
            __syncthreads();
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        re[px<R>(8 * t + r)] = xr[r];
        im[px<R>(8 * t + r)] = xi[r];
    }
    __syncthreads();
    int Ns = 8;
    for (int st = 1; st < nst - 1; ++st) {   // middle stages are radix 8
        lds_stage<R, 8>(re, im, L, Ns, t, tw);
        Ns *= 8;
    }
    const int RR = (rem == 0) ? 8 : (rem == 2 ? 4 : 2);
    if (OUT_REGS) {
        if (RR == 8) last_stage_to_regs<R, 8>(re, im, L, t, tw, xr, xi);
        else if (RR == 4) last_stage_to_regs<R, 4>(re, im, L, t, tw, xr, xi);
        else last_stage_to_regs<R, 2>(re, im, L, t, tw, xr, xi);
    } else {
        if (RR == 8) lds_stage<R, 8>(re, im, L, Ns, t, tw);
        else if (RR == 4) lds_stage<R, 4>(re, im, L, Ns, t, tw);
        else lds_stage<R, 2>(re, im, L, Ns, t, tw);
    }
}

// ===========================================================================
// 16 values per lane.  A column of L = 2^lgL >= 16 points is transformed by
// L/16 lanes: radix-16 Stockham stages, then one radix-2/4/8 stage for the
// remainder.  Lane t holds, on entry, the positions t + i L/16 (i = 0..15),
// runs the first stage on them, exchanges through LDS between stages, and
// keeps the last stage's outputs (again positions t + i L/16) in registers.
// ===========================================================================

// 16-point DFT in registers, natural order in and out, as 4 x 4:
// X[k1 + 4 k2] = sum_n2 W4^{n2 k2} W16^{n2 k1} sum_n1 a[4 n1 + n2] W4^{n1 k1}
template <typename R>
__device__ __forceinline__ void dft16(R* xr, R* xi)
{
    const R c1 = (R)0.92387953251128675612818318939678828682;   // cos(pi/8)
    const R s1 = (R)0.38268343236508977172845998403039886676;   // sin(pi/8)
    const R h = (R)0.70710678118654752440084436210484903928;
    R yr[16], yi[16];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        R tr[4] = {xr[n2], xr[4 + n2], xr[8 + n2], xr[12 + n2]};
        R ti[4] = {xi[n2], xi[4 + n2], xi[8 + n2], xi[12 + n2]};
        dft4(tr, ti);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) { yr[4 * k1 + n2] = tr[k1]; yi[4 * k1 + n2] = ti[k1]; }
    }
    // y[4 k1 + n2] *= W16^{n2 k1}, W16^m = cos(2 pi m/16) - i sin(2 pi m/16)
    cmul(yr[5], yi[5], c1, -s1);                                  // m = 1
    { const R a = yr[6], b = yi[6]; yr[6] = h * (a + b); yi[6] = h * (b - a); }    // m = 2
    cmul(yr[7], yi[7], s1, -c1);                                  // m = 3
    { const R a = yr[9], b = yi[9]; yr[9] = h * (a + b); yi[9] = h * (b - a); }    // m = 2
    { const R a = yr[10]; yr[10] = yi[10]; yi[10] = -a; }         // m = 4
    { const R a = yr[11], b = yi[11]; yr[11] = h * (b - a); yi[11] = -h * (a + b); } // m = 6
    cmul(yr[13], yi[13], s1, -c1);                                // m = 3
    { const R a = yr[14], b = yi[14]; yr[14] = h * (b - a); yi[14] = -h * (a + b); } // m = 6
    cmul(yr[15], yi[15], -c1, s1);                                // m = 9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        R tr[4] = {yr[4 * k1], yr[4 * k1 + 1], yr[4 * k1 + 2], yr[4 * k1 + 3]};
        R ti[4] = {yi[4 * k1], yi[4 * k1 + 1], yi[4 * k1 + 2], yi[4 * k1 + 3]};
        dft4(tr, ti);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) { xr[k1 + 4 * k2] = tr[k2]; xi[k1 + 4 * k2] = ti[k2]; }
    }
}

// radix-RR DFTs of the lane's 16/RR butterflies (slots b RR .. b RR + RR-1)
template <typename R, int RR>
__device__ __forceinline__ void dft_slots16(R (&xr)[16], R (&xi)[16])
{
    if constexpr (RR == 16) {
        dft16(xr, xi);
    } else if constexpr (RR == 8) {
        dft8(xr, xi);
        dft8(xr + 8, xi + 8);
    } else if constexpr (RR == 4) {
#pragma unroll
        for (int b = 0; b < 4; ++b) dft4(xr + 4 * b, xi + 4 * b);
    } else {
#pragma unroll
        for (int b = 0; b < 8; ++b) dft2(xr[2 * b], xi[2 * b], xr[2 * b + 1], xi[2 * b + 1]);
    }
}

// twiddles of a stage with Ns > 1: input r of butterfly b times w^r,
// w = W_L^{k tws}; w, w^2, w^4, w^8 from the table, the other powers as
// products (at most three factors), applied as they are formed
template <typename R, int RR>
__device__ __forceinline__ void twiddle_slots16(R (&xr)[16], R (&xi)[16], int L, int Ns, int t,
                                                const typename C2<R>::T* __restrict__ tw)
{
    using T2 = typename C2<R>::T;
    constexpr int NB = 16 / RR;
    const int tws = L / (Ns * RR);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * (L / 16);
        const int k = j & (Ns - 1);
        if (k == 0) continue;
        R* vr = xr + b * RR;
        R* vi = xi + b * RR;
        const T2 w1 = tw[k * tws];
        cmul(vr[1], vi[1], w1.x, w1.y);
        if constexpr (RR >= 4) {
            const T2 w2 = tw[2 * k * tws];
            cmul(vr[2], vi[2], w2.x, w2.y);
            const R w3r = w1.x * w2.x - w1.y * w2.y, w3i = w1.x * w2.y + w1.y * w2.x;
            cmul(vr[3], vi[3], w3r, w3i);
            if constexpr (RR >= 8) {
                const T2 w4 = tw[4 * k * tws];
                cmul(vr[4], vi[4], w4.x, w4.y);
                const R w5r = w1.x * w4.x - w1.y * w4.y, w5i = w1.x * w4.y + w1.y * w4.x;
                cmul(vr[5], vi[5], w5r, w5i);
                const R w6r = w2.x * w4.x - w2.y * w4.y, w6i = w2.x * w4.y + w2.y * w4.x;
                cmul(vr[6], vi[6], w6r, w6i);
                const R w7r = w3r * w4.x - w3i * w4.y, w7i = w3r * w4.y + w3i * w4.x;
                cmul(vr[7], vi[7], w7r, w7i);
                if constexpr (RR == 16) {
                    const T2 w8 = tw[8 * k * tws];
                    cmul(vr[8], vi[8], w8.x, w8.y);
                    const R a[7][2] = {{w1.x, w1.y}, {w2.x, w2.y}, {w3r, w3i}, {w4.x, w4.y},
                                       {w5r, w5i}, {w6r, w6i}, {w7r, w7i}};
#pragma unroll
                    for (int r = 0; r < 7; ++r) {
                        const R pr = a[r][0] * w8.x - a[r][1] * w8.y;
                        const R pi = a[r][0] * w8.y + a[r][1] * w8.x;
                        cmul(vr[9 + r], vi[9 + r], pr, pi);
                    }
                }
            }
        }
    }
}

// stage outputs to LDS: output r of butterfly b (j = t + b L/16, k = j mod
// Ns) goes to position (j - k) RR + k + r Ns
template <typename R, int RR>
__device__ __forceinline__ void put_slots16(R* buf, const R (&x)[16], int L, int Ns, int t)
{
#pragma unroll
    for (int b = 0; b < 16 / RR; ++b) {
        const int j = t + b * (L / 16);
        const int k = j & (Ns - 1);
        const int base = (j - k) * RR + k;
#pragma unroll
        for (int r = 0; r < RR; ++r) buf[px<R>(base + r * Ns)] = x[b * RR + r];
    }
}

// stage inputs from LDS: input r of butterfly b sits at position j + r L/RR
template <typename R, int RR>
__device__ __forceinline__ void get_slots16(const R* buf, R (&x)[16], int L, int t)
{
#pragma unroll
    for (int b = 0; b < 16 / RR; ++b) {
        const int j = t + b * (L / 16);
#pragma unroll
        for (int r = 0; r < RR; ++r) x[b * RR + r] = buf[px<R>(j + r * (L / RR))];
    }
}

// exchange between a stage of radix RA (outputs) and one of radix RB
// (inputs) through the two LDS arrays.  Starts with a barrier, so the
// caller's previous reads of the arrays are complete before they are reused.
template <typename R, int RA, int RB>
__device__ __forceinline__ void exchange16(R* re, R* im, R (&xr)[16], R (&xi)[16], int L, int Ns,
                                           int t)
{
    __syncthreads();
    put_slots16<R, RA>(re, xr, L, Ns, t);
    put_slots16<R, RA>(im, xi, L, Ns, t);
    __syncthreads();
    get_slots16<R, RB>(re, xr, L, t);
    get_slots16<R, RB>(im, xi, L, t);
}

// radix of the last stage of an L = 2^lgL point transform (16 if lgL is a
// multiple of 4), and the position index i (position t + i L/16) that slot
// s holds after it: s = b RR + r holds i = b + r 16/RR
__host__ __device__ inline int last_radix16(int lgL) { return 1 << ((lgL & 3) ? (lgL & 3) : 4); }
__device__ __forceinline__ int slot_pos16(int s, int RL) { return (s % RL) * (16 / RL) + s / RL; }

// The whole L-point transform (L = 2^lgL, 16 <= L <= 4096) of lane t's
// column: on entry x holds positions t + i L/16 (i = 0..15); on exit slot s
// holds the transform at position t + slot_pos16(s, last_radix16(lgL)) L/16.
// Stage radices: 16 as often as fits, then the remainder (2, 4 or 8).
// Every lane of the workgroup must call it with the same L (barriers).
template <typename R>
__device__ __forceinline__ void fft16_regs(R* re, R* im, int L, int lgL, int t,
                                           const typename C2<R>::T* __restrict__ tw,
                                           R (&xr)[16], R (&xi)[16])
{
    const int n16 = lgL / 4, rem = lgL - 4 * n16;
    dft_slots16<R, 16>(xr, xi);              // stage 1: Ns = 1, no twiddles
    int Ns = 16;                             // product of the radices so far
    for (int st = 1; st < n16; ++st) {
        exchange16<R, 16, 16>(re, im, xr, xi, L, Ns / 16, t);
        twiddle_slots16<R, 16>(xr, xi, L, Ns, t, tw);
        dft_slots16<R, 16>(xr, xi);
        Ns *= 16;
    }
    if (rem == 1) {
        exchange16<R, 16, 2>(re, im, xr, xi, L, Ns / 16, t);
        twiddle_slots16<R, 2>(xr, xi, L, Ns, t, tw);
        dft_slots16<R, 2>(xr, xi);
    } else if (rem == 2) {
        exchange16<R, 16, 4>(re, im, xr, xi, L, Ns / 16, t);
        twiddle_slots16<R, 4>(xr, xi, L, Ns, t, tw);
        dft_slots16<R, 4>(xr, xi);
    } else if (rem == 3) {
        exchange16<R, 16, 8>(re, im, xr, xi, L, Ns / 16, t);
        twiddle_slots16<R, 8>(xr, xi, L, Ns, t, tw);
        dft_slots16<R, 8>(xr, xi);
    }
}

}  // namespace emri
