// fft_lds.hpp -- in-LDS Stockham FFT building blocks shared by the FFT
// passes (fft.hip) and the fused row-FFT + likelihood kernel (like.hip).
//
// A column of L = 2^lgL complex values lives in LDS as two arrays re[], im[]
// indexed through px(i) = i + i/16 (one pad slot per 16 elements), which makes
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

__device__ __host__ inline int px(int i) { return i + (i >> 4); }
// LDS elements (per re or im array) of a padded column of length L
__host__ __device__ inline int padded_len(int L) { return ((L + (L >> 4)) + 15) & ~15; }

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
            vr[b * RR + r] = re[px(j + r * stride)];
            vi[b * RR + r] = im[px(j + r * stride)];
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
            re[px(base + r * Ns)] = vr[b * RR + r];
            im[px(base + r * Ns)] = vi[b * RR + r];
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
            vr[b * RR + r] = re[px(j + r * stride)];
            vi[b * RR + r] = im[px(j + r * stride)];
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
            for (int r = 0; r < 8; ++r) { re[px(r)] = xr[r]; im[px(r)] = xi[r]; }
            __syncthreads();
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        re[px(8 * t + r)] = xr[r];
        im[px(8 * t + r)] = xi[r];
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

}  // namespace emri
