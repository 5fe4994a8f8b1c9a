// internal.hpp -- shared declarations of the HIP implementation of libemri.
//
// Layout of the per-call workspace (all arrays [B][...] for the walkers of one
// chunk, 256-byte aligned):
//   tw      FFT twiddle tables (see fft.hip)
//   wc      [B][WC] fp64 walker constants (scalars + geometry), see WC_*
//   orb     [B][K+1][10] fp64 orbit nodes: Y_k = (Phi, nu, gamma~, e, alpha)
//           then dY/dt at t_k = k h
//   nv      [B][K+1][n_harm][6] fp64 amplitude values and time derivatives
//           at the orbit nodes
//   co      [B][K][16] fp64 power-basis Hermite coefficients of Phi, nu,
//           gamma~, alpha on each coarse interval (u = (t - t_k)/h in [0,1])
//   ch      [B][K][n_harm][12] harmonic coefficients (fp64, or fp32 for the
//           mixed path): for each n the cubic in u of A n P_n, A n Q_n and
//           2 A J_n(ne) (4 coefficients each)
//   z       [B][N] complex: packed signal h_I + i h_II; the FFT runs in
//           place and leaves the spectrum in transposed order
//   part    [B][R2] fp64 partial sums of the likelihood, per row (or per row
//           pair in the frequency-dependent pass)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/emri.h"

namespace emri {

// ---- walker-constant slots (fp64) ---------------------------------------
enum {
    WC_VALID = 0,   // 1: physical walker, 0: lnL = -inf
    WC_MS = 1,      // M in seconds
    WC_MUS = 2,     // mu in seconds
    WC_A = 3,       // spin a = S/M^2
    WC_CL = 4,      // cos(lambda)
    WC_SL = 5,      // sin(lambda)
    WC_G = 6,       // 1/(Xi d_L) with d_L in seconds
    WC_PHI = 7,     // Delta T / (N dt) reduced to [0, 1)
    WC_NX = 8, WC_NY = 9, WC_NZ = 10,          // source direction N
    WC_SX = 11, WC_SY = 12, WC_SZ = 13,        // spin direction S
    WC_E1X = 14, WC_E1Y = 15, WC_E1Z = 16,     // e1 = (z - S cos th_K)/sin th_K
    WC_E2X = 17, WC_E2Y = 18,                  // e2 = S x z / sin th_K (z comp 0)
    WC_NS = 19,     // N . S
    WC_CTS = 20, WC_STS = 21, WC_CPS = 22, WC_SPS = 23,  // cos/sin theta_S, phi_S
    WC_DOP = 24,    // 2 pi R sin(theta_S), R = 1 AU / c
    WC_KW = 25,     // index of the last orbit node before the LSO
    WC_Z = 26, WC_XI = 27, WC_DT = 28, WC_D = 29,
    WC_HASDT = 30,  // 1 if Delta T != 0
    WC_AT = 31,     // alpha_T of the parameter row
    WC_KSEG = 32,   // 16 slots: K_w as known after orbit segment i (the
                    // segment's end when the orbit is still before the LSO)
    // adaptive integrator state between orbit segments (emri_cfg.ode = DP5, RK78)
    WC_OT = 48,     // time of the state
    WC_OY = 49,     // 5 slots: the state Y
    WC_OF = 54,     // 5 slots: f(Y) (first stage of the next step)
    WC_OH = 59,     // proposed next step
    WC_ONODE = 60,  // next coarse node to fill
    WC_OATT = 61,   // step attempts so far
    WC_OREJ = 62,   // 1: the last attempt was rejected
    WC_ODONE = 63,  // 1: the orbit has ended (window end or LSO)
    WC = 64
};

// partial sums of the data norm <d|d> (mixed path data set)
constexpr int kNormParts = 256;

// ---- physical constants (this library's own copy) -----------------------
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kSunSeconds = 4.925490947641267e-6;      // G Msun / c^3
constexpr double kLightSpeed = 299792458.0;                // m/s
constexpr double kParsecM = 3.0856775814913673e16;         // m
constexpr double kAuSeconds = 1.495978707e11 / 299792458.0;
constexpr double kYearSeconds = 365.25 * 86400.0;          // Julian year
constexpr double kHubble = 67.66;                           // km/s/Mpc
constexpr double kOmegaM = 0.3111;

// ---- launch-plan overrides (emri_tuning_set); 0 = automatic -------------
struct Tuning {
    int orbit_segments;    // 1..kMaxSeg
    int fft_row_log2;      // 7..12
    int fft_col_run_bytes; // 8..256, a power of two
    int like_walkers_per_wg;  // 1..32
};
// one consistent copy of the process-wide overrides
Tuning tuning_now();

// ---- plan: sizes and workspace offsets ----------------------------------
struct Plan {
    Tuning tn;             // overrides this plan was made with
    // problem
    double T_obs, dt;
    int64_t N, Nv;         // transform length, valid samples
    int m;                 // log2 N
    int nh;                // harmonics
    int prec;              // emri_precision
    int cl;                // coarse_log2
    int ic;                // emri_cfg.ic: initial conditions at t = 0 or at the LSO
    int ode;               // emri_cfg.ode: RK4, adaptive DP5 or RK78
    double rtol, atol;     // DP5 tolerances
    int64_t L;             // samples per coarse interval, 2^cl
    int64_t K;             // coarse intervals covering N_valid
    // FFT: N = R1 * R2; pass A: R2-point column FFTs (stride R1), T per WG;
    // pass B: R1-point row FFTs
    int m1, m2;
    int64_t R1, R2;
    int TA;                // columns per pass-A workgroup
    size_t esz;            // bytes per complex element (16 or 8)
    size_t hsz;            // bytes per harmonic coefficient (8 or 4)
    // workspace (bytes, for B walkers)
    int64_t B;
    size_t off_tw, off_wc, off_orb, off_co, off_az, off_ch, off_hb, off_hx, off_z, off_part, total;
    // dataset buffer
    size_t ds_off_d, ds_off_w, ds_off_q, ds_off_v, ds_off_norm, ds_off_npart, ds_total;
};

// fills p with the overrides tn; returns EMRI_OK or an error (message in err)
emri_status make_plan(const emri_cfg* cfg, int64_t B, const Tuning& tn, Plan* p,
                      const char** err);

// twiddle table layout inside the tw region (complex fp64 then fp32 copies)
struct TwLayout {
    int64_t nA, nB;               // W_R2^e, W_R1^e
    int64_t nTb, nTs;             // pass-A four-step factors
    size_t oA, oB, oTb, oTs;      // fp64 tables (double2)
    size_t fA, fB, fTb, fTs;      // fp32 tables (float2)
    size_t bytes;
};
TwLayout tw_layout(const Plan& p);
// LDS bytes of a pass-A tile of TA columns of R2 points
size_t cols_lds_bytes(int prec, int64_t R2, int TA);

// ---- launchers (return hipSuccess or the launch error) -------------------
// the orbit is integrated in segments [k_i, k_{i+1}) of coarse steps so that
// the amplitude tables and synthesis of finished segments overlap the rest
// of the integration; kMaxSeg bounds their number
constexpr int kMaxSeg = 16;
// walker constants and orbit segment 0: nodes 0 .. k1 (with the state at
// the LSO, integrated backward: nodes K .. k1)
hipError_t launch_walker_setup(const Plan& p, const double* params, int64_t B, void* ws,
                               int64_t k1, hipStream_t s);
// orbit segment seg >= 1 from the stored node k0: nodes up to k1 (backward
// from the LSO: down to k1 < k0)
hipError_t launch_walker_resume(const Plan& p, int64_t B, void* ws, int64_t k0, int64_t k1,
                                int seg, hipStream_t s);
// node amplitudes and interval tables of segment seg (intervals [k0, k1))
// the orbit nodes of the workspace to a caller's [B][K+1][10] array (zero
// after K_w and for invalid walkers) and K_w to kw[B]
hipError_t launch_orbit_out(const Plan& p, int64_t B, const void* ws, double* orb, int32_t* kw,
                            hipStream_t s);
hipError_t launch_tables(const Plan& p, int64_t B, void* ws, int64_t k0, int64_t k1, int seg,
                         hipStream_t s);
// samples of the intervals [k0, k1) (k1 may reach N / L: zero tail); with
// zfill false, intervals past a walker's plunge or N_valid are not written
// (for consumers that take the samples from nv_w = min(K_w L, N_valid) on
// as zero: launch_fft_cols, launch_fft)
hipError_t launch_synth(const Plan& p, int64_t B, void* ws, void* out, int64_t k0, int64_t k1,
                        int seg, bool zfill, hipStream_t s);
hipError_t launch_twiddles(const Plan& p, void* ws, hipStream_t s);
// detector azimuth at the start of each coarse interval (read by the synthesis)
hipError_t launch_azimuth(const Plan& p, void* ws, hipStream_t s);
// ensemble sampler step (sampler.hip); the prior box by value
struct PriorBox {
    int32_t D;
    int32_t idx[EMRI_NPAR];
    double lo[EMRI_NPAR], hi[EMRI_NPAR];
};
hipError_t launch_stretch_propose(const double* X, int64_t W, int h, const PriorBox& pr, double a,
                                  const double* u, double* Y, double* lnz, double* lpr,
                                  hipStream_t s);
hipError_t launch_stretch_accept(double* X, double* lnp, int64_t W, int h, const double* Y,
                                 const double* lpr, const double* lnL, const double* lnz,
                                 const double* u, int32_t* acc, hipStream_t s);
hipError_t launch_add_box_prior(const double* X, int64_t n, const PriorBox& pr, double* lnp,
                                hipStream_t s);
// z -> z (transposed); the signal in z is read below nv_w only (walker
// constants of the same batch in the workspace)
hipError_t launch_fft(const Plan& p, int64_t B, void* ws, hipStream_t s);
// FFT reading `in` ([B][N] complex, all of it), result in z
hipError_t launch_fft_from(const Plan& p, int64_t B, const void* in, void* ws, hipStream_t s);
// pass A only (column FFTs with the four-step twiddle), in place on z, read
// below nv_w only as launch_fft
hipError_t launch_fft_cols(const Plan& p, int64_t B, void* ws, hipStream_t s);
hipError_t launch_unpack(const Plan& p, int64_t B, const void* ws, void* hf, hipStream_t s);
hipError_t launch_dataset(const Plan& p, const double* data, const double* psd, void* ds,
                          hipStream_t s);
// frequency-dependent propagation: P series terms per walker, coef [B][2][P]
// (alpha_M coefficients, then alpha_T's) of the walkers of this launch
struct FmgArgs {
    int P;
    double f_star;
    const double* coef;
};
// fused pass B + inner product + per-walker sum; expects pass A done on z;
// fmg NULL: constant propagation
hipError_t launch_likelihood(const Plan& p, int64_t B, const void* ds, void* ws, double* lnL,
                             const FmgArgs* fmg, hipStream_t s);

hipError_t launch_model_unpack(const Plan& p, int64_t B, const void* ws, void* mf,
                               hipStream_t s);  // unpack with 1/(Xi d_L) and delay
hipError_t launch_noise_psd(int model, int64_t N, double dt, double* psd, hipStream_t s);

// ---- per-stage event tracing (see emri_trace_enable) ---------------------
enum Stage {
    ST_SETUP = 0, ST_TABLES, ST_SYNTH, ST_TWIDDLE, ST_FFT_COLS, ST_FFT_ROWS, ST_UNPACK,
    ST_DATASET, ST_LIKE, ST_WALKER_SUM, ST_PSD, ST_SAMPLER, ST_COUNT
};
void trace_mark(int stage, hipStream_t s, bool begin);

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// allow a kernel `bytes` of dynamic LDS (needed above 64 KiB); the attribute
// is set once per kernel and size, so captured launch sequences make no
// attribute calls after the first eager use
hipError_t allow_lds(const void* kernel, size_t bytes);

// create the orbit pipeline's auxiliary stream and events for caller stream
// s now (not capturing), so that later captures on s can use them
emri_status prepare_pipe(hipStream_t s);

// record `msg` as the calling thread's last error and return `st`
emri_status set_error(emri_status st, const char* msg);
// while on, this thread's launches record no trace events (graph capture)
void trace_suppress(bool on);

}  // namespace emri
