// like.hip -- stage (d): noise-weighted inner product and the walker sum.
//
// lnL = -1/2 sum_{I,II} sum_{k=1}^{N/2-1} w_k |d_k - m_k|^2,  w_k = 4 df / S_k,
// m_k = g dt exp(-2 pi i k phi) X_k,  g = 1/(Xi d_L), phi = Delta T/(N dt),
// where X is the unnormalised DFT of each channel (Eq. (8) with Eqs. (4)-(6)).
//
// The FFT leaves the packed spectrum in transposed order z[k2 R1 + k1] =
// Z[k2 + R2 k1].  The lower bins k = k2 + R2 k1 < N/2 are exactly those with
// k1 < R1/2; bin k pairs with N - k, which sits in row (R2 - k2) mod R2.  The
// data set stores data and weights at index b = k2 (R1/2) + k1, so every
// stream is read contiguously.
//
// FP64 path: sum of w |d - m|^2 in FP64.
// Mixed path: whitened FP32 data d^ = d sqrt(w) and weights sqrt(w); per bin
// Re(conj(d^) m^) and |m^|^2 with m^ = sqrt(w) m, in FP32 with Kahan
// compensation per lane, FP64 across lanes; lnL = -<d|d>/2 + <d|m> - <m|m>/2
// with <d|d> formed once in FP64 from the FP64 data.
//
// One workgroup per (row k2, walker) writes one FP64 partial; a second
// kernel sums each walker's partials in a fixed order (results do not depend
// on how walkers are batched).
#include "internal.hpp"

namespace emri {

constexpr int kLikeThreads = 256;

// ---------------------------------------------------------------------------
// data set
// ---------------------------------------------------------------------------
template <bool MIXED>
__global__ void k_dataset(const double* __restrict__ data, const double* __restrict__ psd,
                          int64_t N, int64_t R1, int64_t R2, double df, void* __restrict__ dsd,
                          void* __restrict__ dsw)
{
    const int64_t half = N / 2, H = N / 2 + 1, hr = R1 / 2;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= half) return;
    const int64_t k2 = b / hr, k1 = b - k2 * hr;
    const int64_t k = k2 + R2 * k1;
    const double S = psd[k];
    const double wk = (k >= 1 && S > 0.0 && isfinite(S)) ? 4.0 * df / S : 0.0;
    const double d0r = data[2 * k], d0i = data[2 * k + 1];
    const double d1r = data[2 * (H + k)], d1i = data[2 * (H + k) + 1];
    if (!MIXED) {
        double2* D = (double2*)dsd;
        D[b] = double2{d0r, d0i};
        D[half + b] = double2{d1r, d1i};
        ((double*)dsw)[b] = wk;
    } else {
        const double sw = sqrt(wk);
        float2* D = (float2*)dsd;
        D[b] = float2{(float)(d0r * sw), (float)(d0i * sw)};
        D[half + b] = float2{(float)(d1r * sw), (float)(d1i * sw)};
        ((float*)dsw)[b] = (float)sw;
    }
}

__device__ inline double block_sum(double v, double* sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) r += sh[i];
    }
    __syncthreads();
    return r;  // valid in lane 0 of the block
}

// <d|d> in FP64 over bins 1..N/2-1 of both channels (one workgroup)
__global__ void __launch_bounds__(1024) k_data_norm(const double* __restrict__ data,
                                                    const double* __restrict__ psd, int64_t N,
                                                    double df, double* __restrict__ out)
{
    __shared__ double sh[16];
    const int64_t H = N / 2 + 1;
    double acc = 0.0;
    for (int64_t k = 1 + threadIdx.x; k < N / 2; k += blockDim.x) {
        const double S = psd[k];
        if (!(S > 0.0 && isfinite(S))) continue;
        const double d0r = data[2 * k], d0i = data[2 * k + 1];
        const double d1r = data[2 * (H + k)], d1i = data[2 * (H + k) + 1];
        acc += (4.0 * df / S) * (d0r * d0r + d0i * d0i + d1r * d1r + d1i * d1i);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[0] = s;
}

hipError_t launch_dataset(const Plan& p, const double* data, const double* psd, void* ds,
                          hipStream_t s)
{
    char* b = (char*)ds;
    const int64_t half = p.N / 2;
    const double df = 1.0 / ((double)p.N * p.dt);
    dim3 grid((unsigned)((half + 255) / 256));
    trace_mark(ST_DATASET, s, true);
    if (p.prec == EMRI_FP64) {
        hipLaunchKernelGGL(k_dataset<false>, grid, dim3(256), 0, s, data, psd, p.N, p.R1, p.R2,
                           df, (void*)(b + p.ds_off_d), (void*)(b + p.ds_off_w));
    } else {
        hipLaunchKernelGGL(k_dataset<true>, grid, dim3(256), 0, s, data, psd, p.N, p.R1, p.R2, df,
                           (void*)(b + p.ds_off_d), (void*)(b + p.ds_off_w));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_data_norm, dim3(1), dim3(1024), 0, s, data, psd, p.N, df,
                           (double*)(b + p.ds_off_norm));
    }
    trace_mark(ST_DATASET, s, false);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// inner product
// ---------------------------------------------------------------------------
__device__ inline void delay_rotation(int64_t k, double phi, double* c, double* s)
{
    // exp(-2 pi i frac(k phi)); the product's rounding error is kept by FMA
    const double kk = (double)k;
    const double p = kk * phi;
    const double err = fma(kk, phi, -p);
    double f = (p - floor(p)) + err;
    f -= floor(f);
    sincospi(-2.0 * f, s, c);
}

template <bool MIXED>
__global__ void __launch_bounds__(kLikeThreads) k_like(const void* __restrict__ zv, int64_t N,
                                                       int64_t R1, int64_t R2, double dt,
                                                       const double* __restrict__ wc,
                                                       const void* __restrict__ dsd,
                                                       const void* __restrict__ dsw,
                                                       double* __restrict__ part)
{
    __shared__ double sh[kLikeThreads / 64];
    const int64_t k2 = blockIdx.x, w = blockIdx.y;
    const double* c = wc + w * WC;
    if (c[WC_VALID] == 0.0) {
        if (threadIdx.x == 0) part[w * R2 + k2] = 0.0;
        return;
    }
    const double scale = c[WC_G] * dt;
    const bool hasdt = c[WC_HASDT] != 0.0;
    const double phi = c[WC_PHI];
    const int64_t half = N / 2, hr = R1 / 2;
    const int64_t prow = (k2 == 0) ? 0 : (R2 - k2);
    double result;
    if (!MIXED) {
        const double2* z = (const double2*)zv + w * N;
        const double2* D = (const double2*)dsd;
        const double* W = (const double*)dsw;
        double acc = 0.0;
        for (int64_t k1 = threadIdx.x; k1 < hr; k1 += kLikeThreads) {
            const int64_t b = k2 * hr + k1;
            const double2 a = z[k2 * R1 + k1];
            const int64_t pc = (k2 == 0) ? ((R1 - k1) & (R1 - 1)) : (R1 - 1 - k1);
            const double2 bb = z[prow * R1 + pc];
            double xr = 0.5 * (a.x + bb.x), xi = 0.5 * (a.y - bb.y);     // X_I
            double yr = 0.5 * (a.y + bb.y), yi = -0.5 * (a.x - bb.x);    // X_II
            if (hasdt) {
                double cr, ci;
                delay_rotation(k2 + R2 * k1, phi, &cr, &ci);
                double t = xr * cr - xi * ci; xi = xr * ci + xi * cr; xr = t;
                t = yr * cr - yi * ci; yi = yr * ci + yi * cr; yr = t;
            }
            const double2 d0 = D[b], d1 = D[half + b];
            const double r0 = d0.x - scale * xr, i0 = d0.y - scale * xi;
            const double r1 = d1.x - scale * yr, i1 = d1.y - scale * yi;
            acc += W[b] * (r0 * r0 + i0 * i0 + r1 * r1 + i1 * i1);
        }
        result = -0.5 * block_sum(acc, sh);
    } else {
        const float2* z = (const float2*)zv + w * N;
        const float2* D = (const float2*)dsd;
        const float* SW = (const float*)dsw;
        float cr_s = 0.f, cr_c = 0.f, mm_s = 0.f, mm_c = 0.f;   // Kahan sums
        const float fs = (float)scale;
        for (int64_t k1 = threadIdx.x; k1 < hr; k1 += kLikeThreads) {
            const int64_t b = k2 * hr + k1;
            const float2 a = z[k2 * R1 + k1];
            const int64_t pc = (k2 == 0) ? ((R1 - k1) & (R1 - 1)) : (R1 - 1 - k1);
            const float2 bb = z[prow * R1 + pc];
            float xr = 0.5f * (a.x + bb.x), xi = 0.5f * (a.y - bb.y);
            float yr = 0.5f * (a.y + bb.y), yi = -0.5f * (a.x - bb.x);
            if (hasdt) {
                double cr, ci;
                delay_rotation(k2 + R2 * k1, phi, &cr, &ci);
                const float fr = (float)cr, fi = (float)ci;
                float t = xr * fr - xi * fi; xi = xr * fi + xi * fr; xr = t;
                t = yr * fr - yi * fi; yi = yr * fi + yi * fr; yr = t;
            }
            const float sc = fs * SW[b];
            xr *= sc; xi *= sc; yr *= sc; yi *= sc;
            const float2 d0 = D[b], d1 = D[half + b];
            const float cross = d0.x * xr + d0.y * xi + d1.x * yr + d1.y * yi;
            const float mm = xr * xr + xi * xi + yr * yr + yi * yi;
            float y = cross - cr_c, t = cr_s + y;
            cr_c = (t - cr_s) - y; cr_s = t;
            y = mm - mm_c; t = mm_s + y;
            mm_c = (t - mm_s) - y; mm_s = t;
        }
        const double lane = ((double)cr_s - (double)cr_c) - 0.5 * ((double)mm_s - (double)mm_c);
        result = block_sum(lane, sh);
    }
    if (threadIdx.x == 0) part[w * R2 + k2] = result;
}

// lnL[w] = base + sum_k2 part[w][k2] (fixed order), -inf for invalid walkers
__global__ void __launch_bounds__(256) k_walker_sum(const double* __restrict__ part, int64_t R2,
                                                    const double* __restrict__ wc,
                                                    const double* __restrict__ norm,
                                                    double* __restrict__ lnL)
{
    __shared__ double sh[4];
    const int64_t w = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < R2; i += 256) acc += part[w * R2 + i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        const double base = norm ? -0.5 * norm[0] : 0.0;
        const double v = base + s;
        lnL[w] = (wc[w * WC + WC_VALID] != 0.0 && !isnan(v)) ? v : -INFINITY;
    }
}

hipError_t launch_likelihood(const Plan& p, int64_t B, const void* ds, void* ws, double* lnL,
                             hipStream_t s)
{
    char* base = (char*)ws;
    const char* db = (const char*)ds;
    const double* wc = (const double*)(base + p.off_wc);
    double* part = (double*)(base + p.off_part);
    dim3 grid((unsigned)p.R2, (unsigned)B);
    trace_mark(ST_LIKE, s, true);
    if (p.prec == EMRI_FP64)
        hipLaunchKernelGGL(k_like<false>, grid, dim3(kLikeThreads), 0, s,
                           (const void*)(base + p.off_z), p.N, p.R1, p.R2, p.dt, wc,
                           (const void*)(db + p.ds_off_d), (const void*)(db + p.ds_off_w), part);
    else
        hipLaunchKernelGGL(k_like<true>, grid, dim3(kLikeThreads), 0, s,
                           (const void*)(base + p.off_z), p.N, p.R1, p.R2, p.dt, wc,
                           (const void*)(db + p.ds_off_d), (const void*)(db + p.ds_off_w), part);
    trace_mark(ST_LIKE, s, false);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double* norm = (p.prec == EMRI_FP64) ? nullptr : (const double*)(db + p.ds_off_norm);
    trace_mark(ST_WALKER_SUM, s, true);
    hipLaunchKernelGGL(k_walker_sum, dim3((unsigned)B), dim3(256), 0, s, part, p.R2, wc, norm,
                       lnL);
    trace_mark(ST_WALKER_SUM, s, false);
    return hipGetLastError();
}

}  // namespace emri
