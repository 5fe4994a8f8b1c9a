// fft.hip -- stage (c): batched FFT of the two-channel waveform.
//
// The two real channels are packed as one complex signal z_j = h_I(t_j) +
// i h_II(t_j); a single N-point complex transform gives both spectra
// (X_I,k = (Z_k + conj Z_{N-k})/2, X_II,k = (Z_k - conj Z_{N-k})/(2i)).
//
// Four-step decomposition N = R1 * R2, j = j1 + R1 j2, k = k2 + R2 k1:
//   pass A  for each column j1: R2-point FFT over j2 (stride R1), times the
//           twiddle W_N^{j1 k2}, stored back in place at k2 R1 + j1; a
//           workgroup owns TA adjacent columns (coalesced runs of TA
//           elements), 16 values per lane, exchanges through LDS
//   pass B  for each row k2: R1-point FFT over j1 (contiguous), in place
// The spectrum is left in "transposed" order: z[k2 R1 + k1] = Z[k2 + R2 k1].
// The likelihood reads it in that order (its data and weights are stored in
// the same order), so no reordering pass is needed on the hot path.
//
// In-LDS transforms are Stockham autosort with radix 8 stages (one radix-4 or
// radix-2 stage for the remainder), L/8 lanes per transform, twiddles from a
// table W_L^e.  All twiddle tables are computed on the device in FP64 with
// sincospi and rounded to FP32 for the mixed path.
#include "fft_lds.hpp"

namespace emri {

TwLayout tw_layout(const Plan& p)
{
    TwLayout t;
    t.nA = p.R2;
    t.nB = p.R1;
    // pass-A output twiddle W_N^{c k2}, k2 = t + i R2/16, as the product
    // Tb[t][c] Ts[i][c] with Tb[t][c] = W_N^{c t}, Ts[i][c] = W_N^{c i R2/16}
    t.nTb = (p.R2 / 16) * p.R1;
    t.nTs = 16 * p.R1;
    size_t o = 0;
    t.oA = o; o += align256(t.nA * 16);
    t.oB = o; o += align256(t.nB * 16);
    t.oTb = o; o += align256(t.nTb * 16);
    t.oTs = o; o += align256(t.nTs * 16);
    t.fA = o; o += align256(t.nA * 8);
    t.fB = o; o += align256(t.nB * 8);
    t.fTb = o; o += align256(t.nTb * 8);
    t.fTs = o; o += align256(t.nTs * 8);
    t.bytes = o;
    return t;
}

// entry i of the concatenated tables: W^{num} = exp(-2 pi i num / den)
__global__ void k_twiddles(int64_t nA, int64_t nB, int64_t nTb, int64_t nTs, int64_t N,
                           int64_t R1, int64_t R2, double2* tA, double2* tB, double2* tTb,
                           double2* tTs, float2* fA, float2* fB, float2* fTb, float2* fTs)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double2* d;
    float2* f;
    double num, den;
    if (i < nA) { d = tA; f = fA; num = (double)i; den = (double)nA; }
    else if ((i -= nA) < nB) { d = tB; f = fB; num = (double)i; den = (double)nB; }
    else if ((i -= nB) < nTb) {
        d = tTb; f = fTb;
        num = (double)((i / R1) * (i % R1)); den = (double)N;        // c t < N
    } else if ((i -= nTb) < nTs) {
        d = tTs; f = fTs;
        num = (double)((i / R1) * (R2 / 16) * (i % R1)); den = (double)N;   // < N
    } else return;
    double s, c;
    sincospi(-2.0 * num / den, &s, &c);
    d[i] = double2{c, s};
    f[i] = float2{(float)c, (float)s};
}

hipError_t launch_twiddles(const Plan& p, void* ws, hipStream_t s)
{
    const TwLayout t = tw_layout(p);
    char* b = (char*)ws + p.off_tw;
    const int64_t n = t.nA + t.nB + t.nTb + t.nTs;
    trace_mark(ST_TWIDDLE, s, true);
    hipLaunchKernelGGL(k_twiddles, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t.nA,
                       t.nB, t.nTb, t.nTs, p.N, p.R1, p.R2, (double2*)(b + t.oA),
                       (double2*)(b + t.oB), (double2*)(b + t.oTb), (double2*)(b + t.oTs),
                       (float2*)(b + t.fA), (float2*)(b + t.fB), (float2*)(b + t.fTb),
                       (float2*)(b + t.fTs));
    trace_mark(ST_TWIDDLE, s, false);
    return hipGetLastError();
}

// column stride (per re/im array) of a pass-A tile: a padded column plus a
// skew.  Lanes run column-fastest (TA columns, then L/16 positions), so the
// 16 lanes that share one 128-byte LDS access cycle (FP64; 32 for FP32) cover
// TA columns times 16/TA (32/TA) consecutive positions: a skew of that many
// slots puts the columns in disjoint banks.
template <typename R>
__host__ __device__ inline int col_stride(int L, int TA)
{
    return padded_len<R>(L) + (TA > 1 ? (int)(128 / sizeof(R)) / TA : 0);
}

// LDS bytes of a pass-A tile of TA columns of R2 points (re and im arrays)
size_t cols_lds_bytes(int prec, int64_t R2, int TA)
{
    if (prec == EMRI_FP64) return (size_t)TA * col_stride<double>((int)R2, TA) * 2 * 8;
    return (size_t)TA * col_stride<float>((int)R2, TA) * 2 * 4;
}

// XCD-aware tile order: the hardware hands consecutive workgroups to the 8
// XCDs in turn; remap so that each XCD receives a contiguous run of tiles
// (adjacent column tiles share 128-byte lines and one XCD's L2).
__device__ inline int64_t xcd_tile(int64_t bid, int64_t nb)
{
    if (nb & 7) return bid;
    return (bid & 7) * (nb >> 3) + (bid >> 3);
}

// pass A: TA columns per workgroup, TA * L / 16 lanes, lane (col, t) =
// (tid mod TA, tid / TA) loads the positions t + i L/16 of its column
// straight into registers (runs of TA adjacent columns per row: coalesced),
// runs the first radix-16 stage there, exchanges through LDS, and keeps the
// last stage's outputs in registers, from which it applies the four-step
// twiddle (two table factors, one cache line per wave per load) and
// stores.  in and out may alias (the tile's read and write sets coincide,
// and every read precedes the first barrier).
// With walker constants wc, the input of walker w is known to vanish from
// sample nv_w = min(K_w 2^cl, Nv) on (0 for an invalid walker): those samples
// are taken as zero and not read, so the synthesis need not write them.
template <typename R, int MAXT>
__global__ void __launch_bounds__(MAXT) k_fft_cols16(const typename C2<R>::T* in,
                                                     typename C2<R>::T* out, int64_t N,
                                                     int64_t R1, int L, int lgL, int TA,
                                                     const typename C2<R>::T* __restrict__ twL,
                                                     const typename C2<R>::T* __restrict__ tTb,
                                                     const typename C2<R>::T* __restrict__ tTs,
                                                     const double* __restrict__ wc, int64_t Nv,
                                                     int cl)
{
    using T2 = typename C2<R>::T;
    extern __shared__ unsigned char smem_raw[];
    R* sre = (R*)smem_raw;
    const int LP = col_stride<R>(L, TA);
    R* sim = sre + TA * LP;
    const int64_t w = blockIdx.y;
    const int64_t c0 = xcd_tile(blockIdx.x, gridDim.x) * TA;
    const T2* src = in + w * N;
    T2* dst = out + w * N;
    int tsh = 0;
    while ((1 << tsh) < TA) ++tsh;
    const int col = threadIdx.x & (TA - 1), t = threadIdx.x >> tsh;
    const int L16 = L / 16;
    const int64_t cg = c0 + col;
    int64_t nv = N;
    if (wc) {
        const double* c = wc + w * WC;
        const int64_t kv = c[WC_VALID] == 0.0 ? 0 : (int64_t)c[WC_KW];
        nv = (kv << cl) < Nv ? (kv << cl) : Nv;
    }
    R xr[16], xi[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int64_t n = cg + R1 * (int64_t)(t + i * L16);
        const T2 v = n < nv ? src[n] : T2{R(0), R(0)};
        xr[i] = v.x;
        xi[i] = v.y;
    }
    const T2 bt = tTb[(int64_t)t * R1 + cg];        // W_N^{cg t}
    fft16_regs<R>(sre + col * LP, sim + col * LP, L, lgL, t, twL, xr, xi);
    const int RL = last_radix16(lgL);
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int i = slot_pos16(s, RL);
        const T2 st = tTs[(int64_t)i * R1 + cg];     // W_N^{cg i L/16}
        const R wr = bt.x * st.x - bt.y * st.y, wi = bt.x * st.y + bt.y * st.x;
        R yr = xr[s], yi = xi[s];
        cmul(yr, yi, wr, wi);
        dst[cg + R1 * (int64_t)(t + i * L16)] = T2{yr, yi};
    }
}

// pass B: one row of length L (= R1) per workgroup, L / 8 lanes, in place;
// lane t keeps the positions t + i L/8 in registers for the first and last
// radix stages
template <typename R, int MAXT>
__global__ void __launch_bounds__(MAXT) k_fft_rows(typename C2<R>::T* z, int64_t N, int L,
                                                   int lgL,
                                                   const typename C2<R>::T* __restrict__ twL)
{
    using T2 = typename C2<R>::T;
    extern __shared__ unsigned char smem_raw[];
    R* sre = (R*)smem_raw;
    R* sim = sre + padded_len<R>(L);
    const int64_t w = blockIdx.y;
    T2* row = z + w * N + (int64_t)blockIdx.x * L;
    const int t = threadIdx.x, L8 = L / 8;
    R xr[8], xi[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const T2 v = row[t + i * L8];
        xr[i] = v.x;
        xi[i] = v.y;
    }
    fft_regs<R, true>(sre, sim, L, lgL, t, twL, xr, xi);
#pragma unroll
    for (int i = 0; i < 8; ++i) row[t + i * L8] = T2{xr[i], xi[i]};
}

template <typename R>
static hipError_t fft_typed(const Plan& p, int64_t B, const void* in, void* ws, bool rows,
                           bool known_tail, hipStream_t s)
{
    using T2 = typename C2<R>::T;
    char* base = (char*)ws;
    const TwLayout t = tw_layout(p);
    const char* twb = base + p.off_tw;
    const bool f64 = sizeof(R) == 8;
    const T2* tA = (const T2*)(twb + (f64 ? t.oA : t.fA));
    const T2* tB = (const T2*)(twb + (f64 ? t.oB : t.fB));
    const T2* tTb = (const T2*)(twb + (f64 ? t.oTb : t.fTb));
    const T2* tTs = (const T2*)(twb + (f64 ? t.oTs : t.fTs));
    T2* z = (T2*)(base + p.off_z);
    const int LA = (int)p.R2, LB = (int)p.R1;
    const size_t ldsA = cols_lds_bytes(p.prec, p.R2, p.TA);
    const size_t ldsB = (size_t)padded_len<R>(LB) * 2 * sizeof(R);
    const int ntA = p.TA * LA / 16, ntB = LB / 8;
    if (ntA > 1024 || ntB > 512 || LA < 16) return hipErrorInvalidValue;
    const bool big = ntA > 512;
    hipError_t ae = big ? allow_lds((const void*)k_fft_cols16<R, 1024>, ldsA)
                        : allow_lds((const void*)k_fft_cols16<R, 512>, ldsA);
    if (ae == hipSuccess && rows) ae = allow_lds((const void*)k_fft_rows<R, 512>, ldsB);
    if (ae != hipSuccess) return ae;
    const T2* src = (const T2*)(in ? in : z);
    const double* wc = known_tail ? (const double*)(base + p.off_wc) : nullptr;
    const dim3 gA((unsigned)(p.R1 / p.TA), (unsigned)B), bA((unsigned)ntA);
    trace_mark(ST_FFT_COLS, s, true);
    if (big)
        hipLaunchKernelGGL((k_fft_cols16<R, 1024>), gA, bA, ldsA, s, src, z, p.N, p.R1, LA, p.m2,
                           p.TA, tA, tTb, tTs, wc, p.Nv, p.cl);
    else
        hipLaunchKernelGGL((k_fft_cols16<R, 512>), gA, bA, ldsA, s, src, z, p.N, p.R1, LA, p.m2,
                           p.TA, tA, tTb, tTs, wc, p.Nv, p.cl);
    trace_mark(ST_FFT_COLS, s, false);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !rows) return e;
    trace_mark(ST_FFT_ROWS, s, true);
    hipLaunchKernelGGL((k_fft_rows<R, 512>), dim3((unsigned)p.R2, (unsigned)B), dim3((unsigned)ntB),
                       ldsB, s, z, p.N, LB, p.m1, tB);
    trace_mark(ST_FFT_ROWS, s, false);
    return hipGetLastError();
}

hipError_t launch_fft_from(const Plan& p, int64_t B, const void* in, void* ws, hipStream_t s)
{
    if (p.prec == EMRI_FP64) return fft_typed<double>(p, B, in, ws, true, false, s);
    return fft_typed<float>(p, B, in, ws, true, false, s);
}

hipError_t launch_fft_cols(const Plan& p, int64_t B, void* ws, hipStream_t s)
{
    if (p.prec == EMRI_FP64) return fft_typed<double>(p, B, nullptr, ws, false, true, s);
    return fft_typed<float>(p, B, nullptr, ws, false, true, s);
}

hipError_t launch_fft(const Plan& p, int64_t B, void* ws, hipStream_t s)
{
    if (p.prec == EMRI_FP64) return fft_typed<double>(p, B, nullptr, ws, true, true, s);
    return fft_typed<float>(p, B, nullptr, ws, true, true, s);
}

// unpack: transposed packed spectrum -> hf[B][2][N/2+1], scaled by dt and,
// when wc is given, by the propagation factor 1/(Xi d_L) exp(-2 pi i k phi)
template <typename R>
__global__ void k_unpack(const typename C2<R>::T* __restrict__ z, typename C2<R>::T* __restrict__ hf,
                         int64_t N, int64_t R1, int64_t R2, double dt,
                         const double* __restrict__ wc)
{
    using T2 = typename C2<R>::T;
    const int64_t H = N / 2 + 1;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w = blockIdx.y;
    if (k >= H) return;
    const T2* zw = z + w * N;
    const int64_t km = (N - k) & (N - 1);
    const T2 a = zw[(k % R2) * R1 + k / R2];
    const T2 b = zw[(km % R2) * R1 + km / R2];
    double sr = 0.5 * dt, si = 0.0;
    if (wc) {
        const double* c = wc + w * WC;
        if (c[WC_VALID] == 0.0) {
            sr = 0.0;
        } else {
            sr *= c[WC_G];
            if (c[WC_HASDT] != 0.0) {
                // exp(-2 pi i frac(k phi)), product rounding kept by FMA
                const double kk = (double)k, phi = c[WC_PHI];
                const double pr = kk * phi;
                double f = (pr - floor(pr)) + fma(kk, phi, -pr);
                f -= floor(f);
                double cs, sn;
                sincospi(-2.0 * f, &sn, &cs);
                si = sr * sn;
                sr *= cs;
            }
        }
    }
    // X_I = (a + conj b)/2, X_II = (a - conj b)/(2i), times (sr + i si)
    const double xr = (double)a.x + (double)b.x, xi = (double)a.y - (double)b.y;
    const double yr = (double)a.y + (double)b.y, yi = -((double)a.x - (double)b.x);
    hf[(w * 2 + 0) * H + k] = T2{(R)(sr * xr - si * xi), (R)(sr * xi + si * xr)};
    hf[(w * 2 + 1) * H + k] = T2{(R)(sr * yr - si * yi), (R)(sr * yi + si * yr)};
}

static hipError_t unpack_any(const Plan& p, int64_t B, const void* ws, void* hf, bool model,
                             hipStream_t s)
{
    const char* base = (const char*)ws;
    const int64_t H = p.N / 2 + 1;
    const double* wc = model ? (const double*)(base + p.off_wc) : nullptr;
    dim3 grid((unsigned)((H + 255) / 256), (unsigned)B);
    trace_mark(ST_UNPACK, s, true);
    if (p.prec == EMRI_FP64)
        hipLaunchKernelGGL(k_unpack<double>, grid, dim3(256), 0, s,
                           (const double2*)(base + p.off_z), (double2*)hf, p.N, p.R1, p.R2, p.dt,
                           wc);
    else
        hipLaunchKernelGGL(k_unpack<float>, grid, dim3(256), 0, s,
                           (const float2*)(base + p.off_z), (float2*)hf, p.N, p.R1, p.R2, p.dt,
                           wc);
    trace_mark(ST_UNPACK, s, false);
    return hipGetLastError();
}

hipError_t launch_unpack(const Plan& p, int64_t B, const void* ws, void* hf, hipStream_t s)
{
    return unpack_any(p, B, ws, hf, false, s);
}

hipError_t launch_model_unpack(const Plan& p, int64_t B, const void* ws, void* mf, hipStream_t s)
{
    return unpack_any(p, B, ws, mf, true, s);
}

// one-sided LISA noise PSD (instrumental noise of Barack & Cutler 2004)
// galactic confusion noise shape (alpha, beta, kappa, gamma, f_knee) for 0.5,
// 1, 2 and 4 years of observation (Robson, Cornish & Liu 2019)
struct Confusion { double al, be, ka, ga, fk; };
__constant__ Confusion kConfusion[4] = {
    {0.133, 243.0, 482.0, 917.0, 0.00258},
    {0.171, 292.0, 1020.0, 1680.0, 0.00215},
    {0.165, 299.0, 611.0, 1340.0, 0.00173},
    {0.138, -221.0, 521.0, 1680.0, 0.00113},
};

// model 0: BC04 instrumental noise; model 1: the sky-averaged sensitivity of
// Robson, Cornish & Liu 2019 (arm L = 2.5 Gm, transfer frequency
// f* = c / (2 pi L), optical-metrology and acceleration noise); models 2..5:
// the same plus galactic confusion noise for 0.5, 1, 2, 4 years
__global__ void k_noise_psd(int64_t H, double df, int model, double* __restrict__ psd)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= H) return;
    const double f = (double)k * df;
    if (k == 0) {
        psd[k] = INFINITY;
        return;
    }
    if (model == 0) {
        const double f2 = f * f;
        psd[k] = 9.18e-52 / (f2 * f2) + 1.59e-41 + 9.18e-38 * f2;
        return;
    }
    const double L = 2.5e9, fs = kLightSpeed / (2.0 * kPi * L);
    const double a = 2e-3 / f, b = 0.4e-3 / f, c = f / 8e-3;
    const double poms = 1.5e-11 * 1.5e-11 * (1.0 + (a * a) * (a * a));
    const double pacc = 3e-15 * 3e-15 * (1.0 + b * b) * (1.0 + (c * c) * (c * c));
    const double cs = cos(f / fs);
    const double w = 2.0 * kPi * f, w2 = w * w;
    const double x = f / fs;
    double sn = 10.0 / (3.0 * L * L) * (poms + 2.0 * (1.0 + cs * cs) * pacc / (w2 * w2)) *
                (1.0 + 0.6 * x * x);
    if (model >= 2) {
        const Confusion t = kConfusion[model - 2];
        sn += 9e-45 * pow(f, -7.0 / 3.0) * exp(-pow(f, t.al) + t.be * f * sin(t.ka * f)) *
              (1.0 + tanh(t.ga * (t.fk - f)));
    }
    psd[k] = sn;
}

hipError_t launch_noise_psd(int model, int64_t N, double dt, double* psd, hipStream_t s)
{
    const int64_t H = N / 2 + 1;
    trace_mark(ST_PSD, s, true);
    hipLaunchKernelGGL(k_noise_psd, dim3((unsigned)((H + 255) / 256)), dim3(256), 0, s, H,
                       1.0 / ((double)N * dt), model, psd);
    trace_mark(ST_PSD, s, false);
    return hipGetLastError();
}

}  // namespace emri
