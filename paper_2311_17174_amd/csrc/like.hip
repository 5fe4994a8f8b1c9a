// like.hip -- stage (d): noise-weighted inner product and the walker sum.
//
// lnL = -1/2 sum_{I,II} sum_{k=1}^{N/2-1} w_k |d_k - m_k|^2,  w_k = 4 df / S_k,
// m_k = g dt exp(-2 pi i k phi) X_k,  g = 1/(Xi d_L), phi = Delta T/(N dt),
// where X is the unnormalised DFT of each channel (Eq. (8) with Eqs. (4)-(6)).
//
// The FFT leaves the packed spectrum Z = X_I + i X_II in transposed order
// z[k2 R1 + k1] = Z[k2 + R2 k1].  The channels of bin k come from Z_k and
// Z_{N-k} (X_I = (Z_k + conj Z_{N-k})/2, X_II = (Z_k - conj Z_{N-k})/(2i)),
// but the likelihood needs them only in sums over k, and there
//   |X_I|^2 + |X_II|^2 = (|Z_k|^2 + |Z_{N-k}|^2) / 2,
// while the data term is linear in Z_k and conj Z_{N-k}: every packed bin j
// can be weighed on its own against a data array that folds both channels
// (k_dataset_bins).  So lnL = -<d|d>/2 + sum_j [Re(x_j q_j) - |x_j|^2 / 2]
// with x_j = (g dt) sqrt(v_j) P_j Z_j, over all bins j of the row-wise pass
// (k_row_like), and <d|d> formed once in FP64 from the FP64 data.
// FP64 path: the sums in FP64.  Mixed path: FP32 per-bin arrays and FP32
// lane sums with Kahan compensation, FP64 across lanes.
//
// The row FFT of the second pass is fused here: one workgroup per (row,
// tile of walkers) transforms the row in registers and LDS and consumes its
// bins directly, so the spectrum is never written to HBM.  Each (row,
// walker) gives one FP64 partial; a second kernel sums each walker's
// partials in a fixed order (results do not depend on how walkers are
// batched).
//
// The frequency-dependent propagation keeps the paired pass (k_rows_like,
// k_rows_like16): its per-bin factor costs a power series and three
// transcendentals, which the pairing of bin k with N - k evaluates once for
// both.  The data set stores data and weights for it at index
// b = k2 (R1/2) + k1 (bins below N/2, which are those with k1 < R1/2).
#include "fft_lds.hpp"

namespace emri {

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

// Per-bin arrays of the row-wise inner product, in the transform's output
// order b = k2 R1 + k1 for the packed bin j = k2 + R2 k1 (j = 0 .. N-1):
// with k = j below N/2 and k = N - j above it, and v = w_k / 2,
//   s[b] = sqrt(v),
//   q[b] = sqrt(v) (conj d_I(k) - i conj d_II(k))   (j < N/2)
//          sqrt(v) (d_I(k) - i d_II(k))             (j > N/2),
// zero at j = 0 and j = N/2.  For the packed spectrum Z = X_I + i X_II the
// two channels' sums over bins 1..N/2-1 are then sums over all bins j:
//   sum_k w_k (|X_I|^2 + |X_II|^2) = sum_j v_j |Z_j|^2,
//   sum_k w_k Re(conj(d_I) P X_I + conj(d_II) P X_II) = sum_j Re(P_j Z_j q_j sqrt(v_j)),
// with P_j the bin's propagation rotation (its conjugate above N/2), so that
// every bin is used on its own, without the bin N - j it was packed with.
template <typename R>
__global__ void k_dataset_bins(const double* __restrict__ data, const double* __restrict__ psd,
                               int64_t N, int64_t R1, int64_t R2, double df,
                               typename C2<R>::T* __restrict__ q, R* __restrict__ sv)
{
    const int64_t H = N / 2 + 1, half = N / 2;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= N) return;
    const int64_t k2 = b / R1, k1 = b - k2 * R1;
    const int64_t j = k2 + R2 * k1;
    const int64_t k = j < half ? j : N - j;
    const double S = psd[k];
    const bool use = j != 0 && j != half && S > 0.0 && isfinite(S);
    const double r = use ? sqrt(2.0 * df / S) : 0.0;     // sqrt(w_k / 2)
    const double d0r = data[2 * k], d0i = data[2 * k + 1];
    const double d1r = data[2 * (H + k)], d1i = data[2 * (H + k) + 1];
    double qr, qi;
    if (j < half) { qr = d0r - d1i; qi = -d0i - d1r; }
    else { qr = d0r + d1i; qi = d0i - d1r; }
    q[b] = typename C2<R>::T{(R)(r * qr), (R)(r * qi)};
    sv[b] = (R)r;
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

// <d|d> in FP64 over bins 1..N/2-1 of both channels: kNormParts workgroups
// write partials, one workgroup adds them in a fixed order
__global__ void __launch_bounds__(256) k_data_norm_part(const double* __restrict__ data,
                                                        const double* __restrict__ psd, int64_t N,
                                                        double df, double* __restrict__ part)
{
    __shared__ double sh[4];
    const int64_t H = N / 2 + 1;
    double acc = 0.0;
    for (int64_t k = 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N / 2;
         k += (int64_t)gridDim.x * blockDim.x) {
        const double S = psd[k];
        if (!(S > 0.0 && isfinite(S))) continue;
        const double d0r = data[2 * k], d0i = data[2 * k + 1];
        const double d1r = data[2 * (H + k)], d1i = data[2 * (H + k) + 1];
        acc += (4.0 * df / S) * (d0r * d0r + d0i * d0i + d1r * d1r + d1i * d1i);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_data_norm_sum(const double* __restrict__ part,
                                                       double* __restrict__ out)
{
    __shared__ double sh[4];
    const double s = block_sum(part[threadIdx.x], sh);
    if (threadIdx.x == 0) out[0] = s;
}

hipError_t launch_dataset(const Plan& p, const double* data, const double* psd, void* ds,
                          hipStream_t s)
{
    char* b = (char*)ds;
    const int64_t half = p.N / 2;
    const double df = 1.0 / ((double)p.N * p.dt);
    dim3 grid((unsigned)((half + 255) / 256));
    const dim3 gridN((unsigned)((p.N + 255) / 256));
    trace_mark(ST_DATASET, s, true);
    if (p.prec == EMRI_FP64) {
        hipLaunchKernelGGL(k_dataset<false>, grid, dim3(256), 0, s, data, psd, p.N, p.R1, p.R2,
                           df, (void*)(b + p.ds_off_d), (void*)(b + p.ds_off_w));
        hipLaunchKernelGGL(k_dataset_bins<double>, gridN, dim3(256), 0, s, data, psd, p.N, p.R1,
                           p.R2, df, (double2*)(b + p.ds_off_q), (double*)(b + p.ds_off_v));
    } else {
        hipLaunchKernelGGL(k_dataset<true>, grid, dim3(256), 0, s, data, psd, p.N, p.R1, p.R2, df,
                           (void*)(b + p.ds_off_d), (void*)(b + p.ds_off_w));
        hipLaunchKernelGGL(k_dataset_bins<float>, gridN, dim3(256), 0, s, data, psd, p.N, p.R1,
                           p.R2, df, (float2*)(b + p.ds_off_q), (float*)(b + p.ds_off_v));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_data_norm_part, dim3(kNormParts), dim3(256), 0, s, data, psd, p.N, df,
                       (double*)(b + p.ds_off_npart));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_data_norm_sum, dim3(1), dim3(kNormParts), 0, s,
                       (const double*)(b + p.ds_off_npart), (double*)(b + p.ds_off_norm));
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

// Propagation factor of one walker per bin k, as a rotation (cr, ci) of the
// unit-distance spectrum (the walker's g dt is applied separately).
// Constant alpha_M, alpha_T (Eqs. (4)-(6)): exp(-2 pi i k phi), or nothing
// when Delta T = 0.
struct PropConst {
    bool hasdt;
    double phi;
    __device__ __forceinline__ bool rot(int64_t k, double* cr, double* ci) const
    {
        if (!hasdt) return false;
        delay_rotation(k, phi, cr, ci);
        return true;
    }
};

// Per-lane sums of the row-wise inner product: x = (scale sv) z,
// cross += Re(x q), mm += |x|^2; the lane's value is cross - mm/2.
template <typename R, bool MIXED> struct BinSum;
template <typename R> struct BinSum<R, false> {
    double cross = 0.0, mm = 0.0;
    __device__ __forceinline__ void add(R zr, R zi, double scale, R sv,
                                        const typename C2<R>::T& q)
    {
        const double f = scale * (double)sv;
        const double xr = f * (double)zr, xi = f * (double)zi;
        cross += xr * (double)q.x - xi * (double)q.y;
        mm += xr * xr + xi * xi;
    }
    __device__ __forceinline__ double lane_sum() const { return cross - 0.5 * mm; }
};
template <typename R> struct BinSum<R, true> {
    float cr_s = 0.f, cr_c = 0.f, mm_s = 0.f, mm_c = 0.f;   // Kahan sums
    __device__ __forceinline__ void add(R zr, R zi, double scale, R sv,
                                        const typename C2<R>::T& q)
    {
        const float f = (float)scale * (float)sv;
        const float xr = f * (float)zr, xi = f * (float)zi;
        const float cross = xr * (float)q.x - xi * (float)q.y;
        const float mm = xr * xr + xi * xi;
        float y = cross - cr_c, u = cr_s + y;
        cr_c = (u - cr_s) - y; cr_s = u;
        y = mm - mm_c; u = mm_s + y;
        mm_c = (u - mm_s) - y; mm_s = u;
    }
    __device__ __forceinline__ double lane_sum() const
    {
        return ((double)cr_s - (double)cr_c) - 0.5 * ((double)mm_s - (double)mm_c);
    }
};

// Frequency-dependent alpha_M, alpha_T (the variant of Sec. 2 "Waveform
// propagation", power series in x = f/f* with coefficients constant in z):
// amplitude (1 + z)^(-alpha_M(f)/2), delay dT(f) = (1/c_T(f) - 1) chi with
// c_T(f)^2 = 1 + alpha_T(row) + sum t_n x^n, phase exp(-2 pi i f dT(f)).
// 1 + alpha_T <= 0 gives NaN, which the walker sum turns into lnL = -inf;
// the DC and Nyquist bins (weight 0) take the factor 1.
struct PropFmg {
    const double* cm;     // m_0..m_{P-1}, then t_0..t_{P-1}
    int P;
    double xs;            // df / f*
    double hl;            // -ln(1 + z) / 2
    double at0;           // alpha_T of the parameter row
    double cdf;           // chi df: f dT(f) = k cdf (1/c_T - 1)
    int64_t half;         // N / 2
    __device__ __forceinline__ bool rot(int64_t k, double* cr, double* ci) const
    {
        if (k == 0 || k == half) {
            *cr = 1.0;
            *ci = 0.0;
            return true;
        }
        const double x = (double)k * xs;
        double am = 0.0, at = 0.0;
        for (int n = P - 1; n >= 0; --n) {
            am = fma(am, x, cm[n]);
            at = fma(at, x, cm[P + n]);
        }
        at += at0;
        const double amp = exp(hl * am);
        const double ct = sqrt(1.0 + at);
        double cyc = (double)k * cdf * (-at / (ct * (1.0 + ct)));
        cyc -= floor(cyc);
        double sn, cs;
        sincospi(-2.0 * cyc, &sn, &cs);
        *cr = amp * cs;
        *ci = amp * sn;
        return true;
    }
};

// Per-lane accumulation of the inner product over the lane's bins.  A bin
// is given by its packed value z = Z_k and the value m = Z_{N-k} it pairs
// with; X_I = (z + conj m)/2, X_II = (z - conj m)/(2i), times the propagation
// factor (g dt) e^{-2 pi i k phi}, weighed against the data of bin b.
// FP64: -1/2 W |d - x|^2 summed in FP64.  Mixed: whitened FP32 data d~ and
// sqrt(W); Kahan sums of <d~|x~> and |x~|^2, combined in FP64.
template <typename R, bool MIXED> struct BinAcc;

template <typename R> struct BinAcc<R, false> {
    double acc = 0.0;
    template <typename Prop>
    __device__ __forceinline__ void add(R zr, R zi, R mr, R mi, int64_t k, int64_t b,
                                        double scale, const Prop& pr,
                                        const typename C2<R>::T* __restrict__ D,
                                        const R* __restrict__ Wt, int64_t half)
    {
        double xr = 0.5 * (zr + mr), xi = 0.5 * (zi - mi);     // X_I
        double yr = 0.5 * (zi + mi), yi = -0.5 * (zr - mr);    // X_II
        double cr, ci;
        if (pr.rot(k, &cr, &ci)) {
            double u = xr * cr - xi * ci; xi = xr * ci + xi * cr; xr = u;
            u = yr * cr - yi * ci; yi = yr * ci + yi * cr; yr = u;
        }
        const typename C2<R>::T d0 = D[b], d1 = D[half + b];
        const double r0 = d0.x - scale * xr, i0 = d0.y - scale * xi;
        const double r1 = d1.x - scale * yr, i1 = d1.y - scale * yi;
        acc += Wt[b] * (r0 * r0 + i0 * i0 + r1 * r1 + i1 * i1);
        asm volatile("" ::: "memory");   // keep the bins' loads from piling up
    }
    __device__ __forceinline__ double lane_sum() const { return -0.5 * acc; }
};

template <typename R> struct BinAcc<R, true> {
    float cr_s = 0.f, cr_c = 0.f, mm_s = 0.f, mm_c = 0.f;   // Kahan sums
    template <typename Prop>
    __device__ __forceinline__ void add(R zr, R zi, R mr, R mi, int64_t k, int64_t b,
                                        double scale, const Prop& pr,
                                        const typename C2<R>::T* __restrict__ D,
                                        const R* __restrict__ Wt, int64_t half)
    {
        float xr = 0.5f * (zr + mr), xi = 0.5f * (zi - mi);
        float yr = 0.5f * (zi + mi), yi = -0.5f * (zr - mr);
        double cr, ci;
        if (pr.rot(k, &cr, &ci)) {
            const float fr = (float)cr, fi = (float)ci;
            float u = xr * fr - xi * fi; xi = xr * fi + xi * fr; xr = u;
            u = yr * fr - yi * fi; yi = yr * fi + yi * fr; yr = u;
        }
        const typename C2<R>::T d0 = D[b], d1 = D[half + b];
        const float sc = (float)scale * (float)Wt[b];
        xr *= sc; xi *= sc; yr *= sc; yi *= sc;
        const float cross = (float)d0.x * xr + (float)d0.y * xi +
                            (float)d1.x * yr + (float)d1.y * yi;
        const float mm = xr * xr + xi * xi + yr * yr + yi * yi;
        float y = cross - cr_c, u = cr_s + y;
        cr_c = (u - cr_s) - y; cr_s = u;
        y = mm - mm_c; u = mm_s + y;
        mm_c = (u - mm_s) - y; mm_s = u;
        asm volatile("" ::: "memory");
    }
    __device__ __forceinline__ double lane_sum() const
    {
        return ((double)cr_s - (double)cr_c) - 0.5 * ((double)mm_s - (double)mm_c);
    }
};

// the propagation factor of walker w (constants c = wc + w WC)
template <bool FMG>
__device__ __forceinline__ auto walker_prop(const double* c, int64_t w, int64_t N,
                                            const double* fcoef, int fP, double fxs, double dt)
{
    if constexpr (FMG) {
        const double z = c[WC_Z];
        const double df = 1.0 / ((double)N * dt);
        return PropFmg{fcoef + w * 2 * fP, fP, fxs, -0.5 * log1p(z), c[WC_AT],
                       c[WC_D] / (1.0 + z) * df, N / 2};
    } else {
        return PropConst{c[WC_HASDT] != 0.0, c[WC_PHI]};
    }
}

// Fused pass B + inner product.  Workgroup (g, walker tile): rows g and
// R2 - g of the column-transformed signal (rows 0 and R2/2 pair with
// themselves), L = R1 points each, L/8 lanes.  For each walker of the tile:
// row A is transformed with its first and last stages in registers, and lane
// t keeps its 8 values (positions p = t + i L/8) there; row B is transformed
// into LDS; then
// lane t owns the bins (A, p) for p < L/2, paired with (B, L-1-p), and the
// bins (B, L-1-p) for p >= L/2, paired with (A, p).  Data and weights of the
// lane's bins are read once per walker; the walker tiles of a row pair run
// together on one XCD (see the mapping below), so they hit that XCD's L2.
// One FP64 partial per (g, walker).  Register budget 128 (4 waves per SIMD,
// two workgroups per CU): occupancy matters more here than the few spills
// it costs the FP64 variant.  The frequency-dependent propagation keeps its
// per-bin series and transcendentals live as well: at 128 registers it
// spills heavily, so it takes 256 (one workgroup per CU, no spills), which
// measured 13.8 ms against 18.5 ms at config 2.
template <typename R, bool MIXED, int MAXT, bool FMG>
__global__ void __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(FMG ? 2 : 4)))
k_rows_like(const typename C2<R>::T* __restrict__ z,
                                                    int64_t N, int L, int lgL, int64_t R2,
                                                    double dt, const double* __restrict__ wc,
                                                    const void* __restrict__ dsd,
                                                    const void* __restrict__ dsw,
                                                    const typename C2<R>::T* __restrict__ twL,
                                                    double* __restrict__ part, int64_t B, int WT,
                                                    const double* __restrict__ fcoef, int fP,
                                                    double fxs)
{
    using T2 = typename C2<R>::T;
    extern __shared__ unsigned char smem_raw[];
    __shared__ double sh[16];
    R* sre = (R*)smem_raw;
    R* sim = sre + padded_len<R>(L);
    // workgroup -> (row pair g, walker tile): the hardware deals consecutive
    // workgroups to the 8 XCDs in turn; XCD x takes the row pairs g = x mod 8
    // and, for each, all walker tiles one after the other, so the tiles of a
    // row pair run together on one XCD and share its data through that L2
    const int64_t nparts = R2 / 2 + 1;
    const int64_t ntiles = (B + WT - 1) / WT;
    const int64_t lid = blockIdx.x >> 3;
    const int64_t g = (int64_t)(blockIdx.x & 7) + 8 * (lid / ntiles);
    const int64_t tile = lid % ntiles;
    if (g >= nparts) return;
    const bool self = (g == 0) || (g == R2 / 2);
    const int64_t rowA = g, rowB = self ? g : R2 - g;
    const int t0 = threadIdx.x;
    const int L8 = L / 8, hL = L / 2;
    const int64_t half = N / 2;
    const int nown = self ? 4 : 8;

    // Lane t owns, for i < 4, the bin (A, p) with p = t + i L/8 < L/2, and for
    // i >= 4 the bin (B, L-1-p); own_row/own_col give that bin, mirror() the
    // position of the value it pairs with (in row B, or row A itself when the
    // row pairs with itself).
    int t = t0;
    auto own_row = [&](int i) -> int64_t { return i < 4 ? rowA : rowB; };
    auto own_col = [&](int i) -> int { const int p = t + i * L8; return i < 4 ? p : L - 1 - p; };
    auto mirror = [&](int i) -> int {
        const int p = t + i * L8;
        if (i >= 4) return L - 1 - p;        // the bin's own value in row B
        if (self && g == 0) return (L - p) & (L - 1);
        return L - 1 - p;
    };
    // data and weights (FP64: d, 4 df/S; mixed: whitened d, sqrt(4 df/S)) are
    // read per walker: the tile's walkers share them through the cache
    const T2* D = (const T2*)dsd;
    const R* Wt = (const R*)dsw;

    for (int wi = 0; wi < WT; ++wi) {
        const int64_t w = tile * WT + wi;
        if (w >= B) break;
        // opaque per iteration: keeps the per-bin index arithmetic inside the
        // loop instead of holding it in registers across the transforms
        t = t0;
        asm volatile("" : "+v"(t));
        const double* c = wc + w * WC;
        if (c[WC_VALID] == 0.0) {
            if (t == 0) part[w * nparts + g] = 0.0;
            continue;
        }
        const T2* zw = z + w * N;
        // row A: lane t loads positions t + i L/8 into registers; a row that
        // pairs with another leaves its transform in registers, a self-paired
        // row leaves it in LDS (its mirror values are read from there)
        R ar[8], ai[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const T2 v = zw[rowA * L + t + i * L8];
            ar[i] = v.x;
            ai[i] = v.y;
        }
        if (!self) {
            fft_regs<R, true>(sre, sim, L, lgL, t, twL, ar, ai);
            __syncthreads();
            if constexpr (sizeof(R) == 8) {
                // FP64: row B goes through LDS from the start; holding its 8
                // values in registers beside row A's costs more in spills
                // than the LDS round trip it saves
                for (int q = t; q < L; q += L8) {
                    const T2 v = zw[rowB * L + q];
                    sre[px<R>(q)] = v.x;
                    sim[px<R>(q)] = v.y;
                }
                __syncthreads();
                lds_fft<R>(sre, sim, L, lgL, t, twL);
            } else {
                R br[8], bi[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const T2 v = zw[rowB * L + t + i * L8];
                    br[i] = v.x;
                    bi[i] = v.y;
                }
                fft_regs<R, false>(sre, sim, L, lgL, t, twL, br, bi);
            }
        } else {
            fft_regs<R, false>(sre, sim, L, lgL, t, twL, ar, ai);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                ar[i] = sre[px<R>(t + i * L8)];
                ai[i] = sim[px<R>(t + i * L8)];
            }
        }
        const double scale = c[WC_G] * dt;
        const auto pr = walker_prop<FMG>(c, w, N, fcoef, fP, fxs, dt);
        BinAcc<R, MIXED> acc;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (i >= nown) continue;
            R zr, zi, mr, mi;                 // bin value and its mirror
            const int mp = px<R>(mirror(i));
            if (i < 4) { zr = ar[i]; zi = ai[i]; mr = sre[mp]; mi = sim[mp]; }
            else { zr = sre[mp]; zi = sim[mp]; mr = ar[i]; mi = ai[i]; }
            acc.add(zr, zi, mr, mi, own_row(i) + R2 * own_col(i), own_row(i) * hL + own_col(i),
                    scale, pr, D, Wt, half);
        }
        const double lane_sum = acc.lane_sum();
        const double s = block_sum(lane_sum, sh);
        if (t == 0) part[w * nparts + g] = s;
        // block_sum ends with a barrier: LDS may be overwritten by the next walker
    }
}

// The same with 16 values per lane (L/16 lanes; radix-16 transforms with two
// LDS exchanges per row): both rows stay in registers through their
// transforms, so it suits FP32; row B's spectrum (row A's for a row that
// pairs with itself) is then written to LDS for the mirror reads.  Lane t
// holds positions p = t + slot_pos16(s) L/16; it owns (A, p) for p < L/2 and
// (B, L-1-p) for p >= L/2 (only p < L/2 in a self-paired row).  Register
// budget 128 (4 waves per SIMD, four workgroups per CU): faster than the
// spill-free 156 registers at three.  With the frequency-dependent
// propagation the balance turns: 168 registers at three waves (13 spills
// instead of 76) measured 6.3 ms against 10.6 ms at config 2 (and 7.6 ms at
// two waves without spills).
template <typename R, bool MIXED, int MAXT, bool FMG>
__global__ void __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(FMG ? 3 : 4)))
k_rows_like16(const typename C2<R>::T* __restrict__ z, int64_t N, int L, int lgL, int64_t R2,
              double dt, const double* __restrict__ wc, const void* __restrict__ dsd,
              const void* __restrict__ dsw, const typename C2<R>::T* __restrict__ twL,
              double* __restrict__ part, int64_t B, int WT, const double* __restrict__ fcoef,
              int fP, double fxs)
{
    using T2 = typename C2<R>::T;
    extern __shared__ unsigned char smem_raw[];
    __shared__ double sh[16];
    R* sre = (R*)smem_raw;
    R* sim = sre + padded_len<R>(L);
    // workgroup -> (row pair g, walker tile), XCD-grouped as in k_rows_like
    const int64_t nparts = R2 / 2 + 1;
    const int64_t ntiles = (B + WT - 1) / WT;
    const int64_t lid = blockIdx.x >> 3;
    const int64_t g = (int64_t)(blockIdx.x & 7) + 8 * (lid / ntiles);
    const int64_t tile = lid % ntiles;
    if (g >= nparts) return;
    const bool self = (g == 0) || (g == R2 / 2);
    const int64_t rowA = g, rowB = self ? g : R2 - g;
    const int t0 = threadIdx.x;
    const int L16 = L / 16, hL = L / 2;
    const int64_t half = N / 2;
    const int RL = last_radix16(lgL);
    const T2* D = (const T2*)dsd;
    const R* Wt = (const R*)dsw;

    for (int wi = 0; wi < WT; ++wi) {
        const int64_t w = tile * WT + wi;
        if (w >= B) break;
        int t = t0;
        asm volatile("" : "+v"(t));
        const double* c = wc + w * WC;
        if (c[WC_VALID] == 0.0) {
            if (t == 0) part[w * nparts + g] = 0.0;
            continue;
        }
        const T2* zw = z + w * N;
        R ar[16], ai[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const T2 v = zw[rowA * L + t + i * L16];
            ar[i] = v.x;
            ai[i] = v.y;
        }
        fft16_regs<R>(sre, sim, L, lgL, t, twL, ar, ai);
        if (!self) {
            R br[16], bi[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const T2 v = zw[rowB * L + t + i * L16];
                br[i] = v.x;
                bi[i] = v.y;
            }
            fft16_regs<R>(sre, sim, L, lgL, t, twL, br, bi);
            __syncthreads();
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const int p = t + slot_pos16(s, RL) * L16;
                sre[px<R>(p)] = br[s];
                sim[px<R>(p)] = bi[s];
            }
        } else {
            __syncthreads();
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const int p = t + slot_pos16(s, RL) * L16;
                sre[px<R>(p)] = ar[s];
                sim[px<R>(p)] = ai[s];
            }
        }
        __syncthreads();
        const double scale = c[WC_G] * dt;
        const auto pr = walker_prop<FMG>(c, w, N, fcoef, fP, fxs, dt);
        BinAcc<R, MIXED> acc;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int p = t + slot_pos16(s, RL) * L16;
            if (p < hL) {
                const int mp = (self && g == 0) ? ((L - p) & (L - 1)) : (L - 1 - p);
                acc.add(ar[s], ai[s], sre[px<R>(mp)], sim[px<R>(mp)], rowA + R2 * p,
                        rowA * hL + p, scale, pr, D, Wt, half);
            } else if (!self) {
                const int q = L - 1 - p;
                acc.add(sre[px<R>(q)], sim[px<R>(q)], ar[s], ai[s], rowB + R2 * q, rowB * hL + q,
                        scale, pr, D, Wt, half);
            }
        }
        const double s = block_sum(acc.lane_sum(), sh);
        if (t == 0) part[w * nparts + g] = s;
        // block_sum ends with a barrier: LDS may be overwritten by the next walker
    }
}

// Fused pass B + inner product, one row at a time: one workgroup per (row
// g, tile of walkers), L/E lanes with E values each (E = 8: radix-8 stages,
// the first and last in registers; E = 16: radix-16 stages, two LDS
// exchanges; FP64 at E = 16 takes up to 256 VGPRs, two waves per SIMD).  After the row's transform lane t holds its bins in
// registers and consumes them with the per-bin arrays of k_dataset_bins, so
// no bin waits for the one it was packed with and rows are independent.
// Per bin j: x = (g dt sqrt(v_j)) P_j Z_j; the lane sums Re(x q_j) and |x|^2
// (FP64, or FP32 with Kahan compensation in the mixed path); one FP64
// partial sum(Re(x q)) - sum(|x|^2)/2 per (row, walker); the walker sum adds
// -<d|d>/2.  The walker tiles of a row run together on one XCD, so the
// row's per-bin arrays are read from HBM once.
template <typename R, bool MIXED, int E, int MAXT>
__global__ void __launch_bounds__(MAXT)
__attribute__((amdgpu_waves_per_eu((sizeof(R) == 8 && E == 16) ? 2 : 4)))
k_row_like(const typename C2<R>::T* __restrict__ z, int64_t N, int L, int lgL, int64_t R2,
           double dt, const double* __restrict__ wc, const typename C2<R>::T* __restrict__ Q,
           const R* __restrict__ SV, const typename C2<R>::T* __restrict__ twL,
           double* __restrict__ part, int64_t B, int WT)
{
    using T2 = typename C2<R>::T;
    extern __shared__ unsigned char smem_raw[];
    __shared__ double shp[32 * 8];   // per (walker of the tile, wave): the wave's sum
    R* sre = (R*)smem_raw;
    R* sim = sre + padded_len<R>(L);
    const int64_t ntiles = (B + WT - 1) / WT;
    const int64_t lid = blockIdx.x >> 3;
    const int64_t g = (int64_t)(blockIdx.x & 7) + 8 * (lid / ntiles);
    const int64_t tile = lid % ntiles;
    if (g >= R2) return;
    const int t0 = threadIdx.x;
    const int LE = L / E;
    const int64_t half = N / 2;
    const int RL = last_radix16(lgL);
    const T2* Qr = Q + g * L;
    const R* Sr = SV + g * L;
    const int nw = (blockDim.x + 63) >> 6;
    int nwk = 0;                       // walkers of this tile

    for (int wi = 0; wi < WT; ++wi) {
        const int64_t w = tile * WT + wi;
        if (w >= B) break;
        nwk = wi + 1;
        int t = t0;
        asm volatile("" : "+v"(t));
        const double* c = wc + w * WC;
        if (c[WC_VALID] == 0.0) {
            if (t < nw) shp[wi * nw + t] = 0.0;
            continue;
        }
        const T2* zr = z + w * N + g * L;
        R xr[E], xi[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const T2 v = zr[t + i * LE];
            xr[i] = v.x;
            xi[i] = v.y;
        }
        if constexpr (E == 8) fft_regs<R, true>(sre, sim, L, lgL, t, twL, xr, xi);
        else fft16_regs<R>(sre, sim, L, lgL, t, twL, xr, xi);
        const double scale = c[WC_G] * dt;
        const bool hasdt = c[WC_HASDT] != 0.0;
        const double phi = c[WC_PHI];
        BinSum<R, MIXED> acc;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int p = t + (E == 8 ? i : slot_pos16(i, RL)) * LE;
            R ar = xr[i], ai = xi[i];
            if (hasdt) {
                const int64_t j = g + R2 * (int64_t)p;
                double cr, ci;
                delay_rotation(j < half ? j : N - j, phi, &cr, &ci);
                if (j > half) ci = -ci;
                const R u = ar * (R)cr - ai * (R)ci;
                ai = ar * (R)ci + ai * (R)cr;
                ar = u;
            }
            acc.add(ar, ai, scale, Sr[p], Qr[p]);
        }
        // the wave's sum; the walker's sum over the waves is formed after
        // the last walker, so no barrier waits on it here (the next
        // walker's first exchange starts with one before LDS is rewritten)
        double v = acc.lane_sum();
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((t & 63) == 0) shp[wi * nw + (t >> 6)] = v;
    }
    __syncthreads();
    if (t0 < nwk) {                    // the waves' sums in a fixed order
        double r = 0.0;
        for (int i = 0; i < nw; ++i) r += shp[t0 * nw + i];
        part[(tile * WT + t0) * R2 + g] = r;
    }
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

// values per lane of the FP64 row-wise pass: 16 (radix 16, 203 VGPRs, two
// waves per SIMD) measured 5.16 ms at config 2 against 5.58 ms for 8
// (radix 8, 128 VGPRs, four waves per SIMD)
constexpr int kRowE64 = 16;

hipError_t launch_likelihood(const Plan& p, int64_t B, const void* ds, void* ws, double* lnL,
                             const FmgArgs* fmg, hipStream_t s)
{
    char* base = (char*)ws;
    const char* db = (const char*)ds;
    const double* wc = (const double*)(base + p.off_wc);
    double* part = (double*)(base + p.off_part);
    const int L = (int)p.R1;
    int WT = (B >= 128) ? 8 : (B >= 16 ? 4 : 1);
    if (p.tn.like_walkers_per_wg >= 1 && p.tn.like_walkers_per_wg <= 32)
        WT = p.tn.like_walkers_per_wg;
    const TwLayout tl = tw_layout(p);
    const char* twb = base + p.off_tw;
    const double* norm = (const double*)(db + p.ds_off_norm);
    if (!fmg) {
        // constant propagation: the row-wise pass
        const bool f64 = p.prec == EMRI_FP64;
        const int E = f64 ? kRowE64 : 16;
        if (L / E > 512 || L / E < 8) return hipErrorInvalidValue;
        const void* kern = f64 ? (E == 8 ? (const void*)k_row_like<double, false, 8, 512>
                                         : (const void*)k_row_like<double, false, 16, 256>)
                               : (const void*)k_row_like<float, true, 16, 256>;
        const size_t lds = f64 ? (size_t)padded_len<double>(L) * 2 * 8
                               : (size_t)padded_len<float>(L) * 2 * 4;
        hipError_t ae = allow_lds(kern, lds);
        if (ae != hipSuccess) return ae;
        const int64_t ntiles = (B + WT - 1) / WT;
        const dim3 grid((unsigned)(((p.R2 + 7) / 8) * 8 * ntiles));
        const void* a_z = (const void*)(base + p.off_z);
        int64_t a_N = p.N, a_R2 = p.R2, a_B = B;
        int a_L = L, a_lgL = p.m1, a_WT = WT;
        double a_dt = p.dt;
        const double* a_wc = wc;
        const void* a_q = (const void*)(db + p.ds_off_q);
        const void* a_v = (const void*)(db + p.ds_off_v);
        const void* a_tw = (const void*)(twb + (f64 ? tl.oB : tl.fB));
        double* a_part = part;
        void* args[] = {&a_z, &a_N, &a_L, &a_lgL, &a_R2, &a_dt, &a_wc, &a_q, &a_v, &a_tw,
                        &a_part, &a_B, &a_WT};
        trace_mark(ST_LIKE, s, true);
        ae = hipLaunchKernel(kern, grid, dim3((unsigned)(L / E)), args, lds, s);
        trace_mark(ST_LIKE, s, false);
        if (ae != hipSuccess) return ae;
        ae = hipGetLastError();
        if (ae != hipSuccess) return ae;
        trace_mark(ST_WALKER_SUM, s, true);
        hipLaunchKernelGGL(k_walker_sum, dim3((unsigned)B), dim3(256), 0, s, part, p.R2, wc,
                           norm, lnL);
        trace_mark(ST_WALKER_SUM, s, false);
        return hipGetLastError();
    }
    const size_t lds = (p.prec == EMRI_FP64) ? (size_t)padded_len<double>(L) * 2 * 8
                                             : (size_t)padded_len<float>(L) * 2 * 4;
    const int64_t nparts = p.R2 / 2 + 1;
    const int64_t ntiles = (B + WT - 1) / WT;
    dim3 grid((unsigned)(((nparts + 7) / 8) * 8 * ntiles));
    // FP32 rows take 16 values per lane; FP64 keeps 8: two rows of 16 FP64
    // values do not fit 128 registers
    const int E = (p.prec == EMRI_FP64) ? 8 : 16;
    const bool f = fmg != nullptr;
    const void* kern =
        (p.prec == EMRI_FP64)
            ? (f ? (const void*)k_rows_like<double, false, 512, true>
                 : (const void*)k_rows_like<double, false, 512, false>)
            : (f ? (const void*)k_rows_like16<float, true, 256, true>
                 : (const void*)k_rows_like16<float, true, 256, false>);
    hipError_t ae = allow_lds(kern, lds);
    if (ae != hipSuccess) return ae;
    if (L / E > 512 || L < 16 * (E / 8)) return hipErrorInvalidValue;   // rows of 2^7 .. 2^12 points
    const dim3 blk((unsigned)(L / E));
    const void* dsd = (const void*)(db + p.ds_off_d);
    const void* dsw = (const void*)(db + p.ds_off_w);
    trace_mark(ST_LIKE, s, true);
    {
        const void* a_z = (const void*)(base + p.off_z);
        int64_t a_N = p.N, a_R2 = p.R2, a_B = B;
        int a_L = L, a_lgL = p.m1, a_WT = WT;
        double a_dt = p.dt;
        const double* a_wc = wc;
        const void* a_tw = (const void*)(twb + (p.prec == EMRI_FP64 ? tl.oB : tl.fB));
        double* a_part = part;
        const double* a_fc = f ? fmg->coef : nullptr;
        int a_fP = f ? fmg->P : 0;
        double a_fxs = f ? 1.0 / ((double)p.N * p.dt * fmg->f_star) : 0.0;
        void* args[] = {&a_z, &a_N, &a_L, &a_lgL, &a_R2, &a_dt, &a_wc, (void*)&dsd,
                        (void*)&dsw, &a_tw, &a_part, &a_B, &a_WT, &a_fc, &a_fP, &a_fxs};
        ae = hipLaunchKernel(kern, grid, blk, args, lds, s);
    }
    trace_mark(ST_LIKE, s, false);
    if (ae != hipSuccess) return ae;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the paired pass sums w |d - m|^2 itself in FP64; the mixed one needs <d|d>
    trace_mark(ST_WALKER_SUM, s, true);
    hipLaunchKernelGGL(k_walker_sum, dim3((unsigned)B), dim3(256), 0, s, part, nparts, wc,
                       (p.prec == EMRI_FP64) ? nullptr : norm, lnL);
    trace_mark(ST_WALKER_SUM, s, false);
    return hipGetLastError();
}

}  // namespace emri
