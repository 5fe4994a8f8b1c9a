/*
 * emri.h -- C ABI of the MI355X batched EMRI log-likelihood library (libemri).
 *
 * The library evaluates, for a batch of MCMC walkers, the log-likelihood of
 * Saltas & Oliveri, "emri_mc" (arXiv:2311.17174): each walker's Analytic
 * Kludge waveform is generated from the orbital ODE system (Eq. (1)) and the
 * harmonic sum (Eq. (2)), projected on the two low-frequency LISA channels,
 * Fourier transformed (Sec. 3, "Waveform computation"), damped by 1/Xi and
 * delayed by the GW-speed term (Eqs. (4)-(6)), and weighted by the noise
 * curve against the data (Eq. (8)).
 *
 * Conventions for every entry point:
 *  - Array pointers are DEVICE pointers owned by the caller, unless stated.
 *    The library never allocates or frees device memory.  Scratch memory is
 *    the caller's workspace `ws` of `ws_bytes` bytes (size it with
 *    emri_workspace_bytes); its contents are undefined after a call.
 *  - Every call is asynchronous on `stream` (0 = the null stream).  Inputs
 *    must stay valid, and outputs must not be read, until the stream has
 *    reached the call's end.  Calls that share a workspace must be ordered.
 *    Waveform generation may also run on an auxiliary stream the library
 *    keeps per (device, caller stream), created on the first call made while
 *    `stream` is not capturing; it is forked from and joined back into
 *    `stream` by events within the call (also under stream capture), so
 *    `stream` alone orders the call.  A call on a capturing stream that has
 *    no auxiliary stream yet creates none and runs on `stream` alone (same
 *    results).  The auxiliary streams are the only resources the library
 *    keeps.  Calls on
 *    one stream must come from one host thread at a time (as for any
 *    stream); calls on different streams may run concurrently.
 *  - Call-level errors (null pointer, bad configuration, workspace too
 *    small, launch failure) return a negative status and launch nothing new;
 *    emri_last_error() then describes the error (per host thread).
 *  - Per-walker errors are not call errors: a walker outside the physical
 *    domain gets lnL = -infinity (the log-prior convention of the paper's
 *    sampler, Sec. 3 file list) and the call returns EMRI_OK.
 *  - No NaN and no exception crosses the ABI.
 *  - A parameter row is 17 doubles (EMRI_NPAR), row-major [B][17]:
 *      0 M [Msun]   1 mu [Msun]   2 a = S/M^2 in [0,1]   3 e0 in [0,1)
 *      4 nu0 [Hz], 0 < nu0 < nu_LSO(e0)   5 Phi0   6 gamma~0   7 alpha0
 *      8 cos(lambda)   9 theta_S   10 phi_S   11 theta_K   12 phi_K [rad]
 *      13 d_L [Gpc] > 0   14 Xi0   15 n (Eq. (6))
 *      16 alpha_T > -1: constant GW-speed parameter, c_T^2 = 1 + alpha_T
 *         (Eq. (3)); 0 is General Relativity.
 *    With cfg->ic = EMRI_IC_LSO, entries 3, 5, 6, 7 are the state at the
 *    last stable orbit and entry 4 is unused (see emri_cfg).
 *    The first three entries are the masses and spin, as in the paper's
 *    parameter-vector convention (Sec. 3).  The state Y = (Phi, nu, gamma~,
 *    e, alpha) of Eq. (1) starts at t = 0 from entries 3..7.
 */
#ifndef EMRI_H
#define EMRI_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EMRI_NPAR 17
#define EMRI_ABI_VERSION 8

typedef enum {
    EMRI_OK = 0,
    EMRI_EINVAL = -1,        /* bad argument or configuration              */
    EMRI_EWORKSPACE = -2,    /* workspace or dataset buffer too small      */
    EMRI_EDEVICE = -3,       /* HIP launch or device error                 */
    EMRI_EUNSUPPORTED = -4   /* valid request outside the supported range  */
} emri_status;

/* Accuracy.  EMRI_FP64 follows the FP64 reference computation (the same
 * orbit integrator, node interpolation and transform definition) to
 * rounding, except that the harmonic amplitudes between orbit nodes come
 * from cubic tables per coarse interval, whose error falls as the fourth
 * power of the coarse step.  Where the orbit evolves over many coarse steps
 * (every configuration of the tests: 30 days to 2 years, 16-40 harmonics)
 * lnL agrees to 1e-10 relative and its signal part to 1e-10 <m|m>; within a
 * few coarse steps of a plunge the table error reaches ~1e-7 of max|h| at
 * coarse_log2 = 10, and each unit less of coarse_log2 divides it by 16.
 * EMRI_MIXED: lnL to 1e-4 relative and the signal part to 1e-5 <m|m>; its
 * synthesis leaves out harmonics and cubic amplitude terms below 2^-30 of
 * the interval's largest harmonic, under FP32 rounding. */
typedef enum {
    EMRI_FP64 = 0,  /* every stage in FP64                                   */
    EMRI_MIXED = 1  /* FP64 orbit, phases and final reduction; FP32 harmonic
                       sum, response, FFT and products with compensated sums */
} emri_precision;

/* Problem configuration (host struct, passed by pointer).
 *  T_obs        observation time [s] > 0; N_valid = round(T_obs/dt) samples
 *  dt           sampling interval [s] > 0 (the paper uses 0.1 Hz, Sec. 3)
 *  N            transform length, a power of two, 2^12 <= N <= 2^24,
 *               N >= N_valid; samples N_valid..N-1 are zero padding
 *  n_harm       number of harmonics n_max of Eq. (2), 1..64
 *  precision    emri_precision
 *  coarse_log2  the orbit is integrated with step h = dt * 2^coarse_log2
 *               (8..12) and read between nodes by cubic Hermite interpolation
 *  ic           where the parameter row's orbital state applies:
 *               EMRI_IC_START: at t = 0, nu0 = p[4], integrated forward to the
 *               LSO (samples after it are zero);
 *               EMRI_IC_LSO: the paper's convention (Sec. 3 "Waveform
 *               computation"): e = p[3], Phi = p[5], gamma~ = p[6],
 *               alpha = p[7] at the last stable orbit, nu = nu_LSO(e) (p[4]
 *               unused), integrated backward; the LSO is the last coarse
 *               node, t = K h with K = ceil(N_valid / 2^coarse_log2), so the
 *               window ends within one coarse step of the plunge.  A walker
 *               whose backward history leaves 0 <= e < 1, nu > 0 is invalid.
 *  ode          the integrator of Eq. (1) (Sec. 3 "Waveform computation" and
 *               "Computational overhead": a standard adaptive Runge-Kutta
 *               solver, the method's main cost):
 *               EMRI_ODE_RK4: classical RK4 with step h on the coarse nodes;
 *               EMRI_ODE_DP5: the embedded Dormand-Prince 5(4) pair with
 *               step-size control (Hairer, Norsett & Wanner, Solving ODEs I,
 *               Sec. II.4: RMS error norm over the five components, safety
 *               0.9, step factors in [0.2, 5], no growth right after a
 *               rejection; first step h; the last step cut to end on the
 *               window) and its order-4 continuous extension evaluated at the
 *               coarse nodes, whose derivatives are the right-hand side at
 *               the interpolated state.  The nodes reach the waveform step in
 *               the same layout as with RK4.  A walker that needs more than
 *               4 K + 64 step attempts is invalid (lnL = -inf; its
 *               time-domain rows then hold whatever was synthesised before
 *               that was found).
 *               EMRI_ODE_RK78: the paper's "7th-order Runge-Kutta scheme",
 *               read as Fehlberg's embedded 7(8) pair (NASA TR R-287,
 *               1968; 13 stages), the order-7 solution kept and the order-8
 *               one used for the error estimate alone, stepped node to node:
 *               a step never passes the next coarse node (it is cut to end
 *               on it), so every node is a step end of the method and no
 *               interpolation enters.  Step control as for DP5 with the
 *               exponent 1/8; the orbit stops at the first step end past the
 *               LSO (forward) or outside 0 <= e < 1, nu > 0 (backward:
 *               invalid); the same step budget.
 *  reserved     0
 *  ode_rtol     EMRI_ODE_DP5, EMRI_ODE_RK78: relative tolerance, 1e-13 .. 1e-3
 *  ode_atol     EMRI_ODE_DP5, EMRI_ODE_RK78: absolute tolerance >= 0 for Phi,
 *               gamma~ and alpha [rad] and e; nu is held to ode_rtol relative
 *               alone.  Both are ignored with EMRI_ODE_RK4. */
typedef enum { EMRI_IC_START = 0, EMRI_IC_LSO = 1 } emri_ic;
typedef enum { EMRI_ODE_RK4 = 0, EMRI_ODE_DP5 = 1, EMRI_ODE_RK78 = 2 } emri_ode;
typedef struct {
    double T_obs;
    double dt;
    int64_t N;
    int32_t n_harm;
    int32_t precision;
    int32_t coarse_log2;
    int32_t ic;                  /* emri_ic */
    int32_t ode;                 /* emri_ode */
    int32_t reserved;            /* 0 */
    double ode_rtol;
    double ode_atol;
} emri_cfg;

/* Library ABI version (EMRI_ABI_VERSION). */
int emri_abi_version(void);

/* Launch-plan overrides (process-wide), for measurement and tests.  Each
 * field 0 means automatic.  A call plans with one consistent copy of the
 * overrides taken when it starts; changing them while calls run is safe but
 * the running calls keep their plan.  Workspace sizes follow the overrides
 * (size workspaces after setting them).  Results are bitwise independent of
 * orbit_segments and like_walkers_per_wg; fft_row_log2 and
 * fft_col_run_bytes change the transform's factorisation and so its
 * rounding, within the precision's tolerance.
 *  orbit_segments       orbit segments pipelined against the synthesis, 1..16
 *                       (automatic: about 384 coarse steps each, at most 8)
 *  fft_row_log2         log2 of the FFT's row length (the fused likelihood
 *                       pass), 7..12, applied where both passes support it
 *  fft_col_run_bytes    bytes of adjacent columns per column-pass row read,
 *                       a power of two in 8..256 (automatic: 128 FP64, 64 FP32)
 *  like_walkers_per_wg  walkers per workgroup of the likelihood pass, 1..32
 * emri_tuning_set(NULL) restores automatic plans.  Out-of-range fields:
 * EMRI_EINVAL and nothing changes. */
typedef struct {
    int32_t orbit_segments;
    int32_t fft_row_log2;
    int32_t fft_col_run_bytes;
    int32_t like_walkers_per_wg;
    int32_t reserved;            /* 0 */
} emri_tuning;
emri_status emri_tuning_set(const emri_tuning* t);
emri_status emri_tuning_get(emri_tuning* t);

/* Message for the last non-OK status returned on this host thread. */
const char* emri_last_error(void);

/* Workspace bytes for B walkers processed at once (0 if cfg is invalid).
 * The waveform, FFT and likelihood entry points all accept this size. */
size_t emri_workspace_bytes(const emri_cfg* cfg, int64_t B);

/* The orbit of each walker alone (Eq. (1), integrated as emri_cfg.ode
 * selects; Sec. 3 "Waveform computation"): the coarse nodes that the
 * amplitude tables and the synthesis read.
 *  params  [B][17] fp64
 *  orb     [B][K+1][10] fp64, K = ceil(N_valid / 2^coarse_log2): at node
 *          t_k = k dt 2^coarse_log2 the state (Phi, nu, gamma~, e, alpha),
 *          then its time derivative (the right-hand side of Eq. (1) at the
 *          node state); zero after node kw and for an invalid walker
 *  kw      [B] int32: the last node before the LSO (forward), K (backward
 *          from the LSO), -1 for an invalid walker
 *  ws      workspace of at least emri_workspace_bytes(cfg, B) bytes
 * Same precision for every emri_cfg.precision: the orbit is FP64. */
emri_status emri_orbit_batch(const double* params, int64_t B, const emri_cfg* cfg, double* orb,
                             int32_t* kw, void* ws, size_t ws_bytes, hipStream_t stream);

/* Time-domain waveforms (Eqs. (1)-(2) with the LISA response and Doppler
 * phase), at unit distance and without propagation effects -- the paper's
 * waveform() excludes the distance factor (Sec. 3 file list).
 *  params  [B][17] fp64
 *  ht      [B][N][2] real, channel-interleaved (I, II) per sample; fp64 for
 *          EMRI_FP64, fp32 for EMRI_MIXED; zero after N_valid and after the
 *          plunge (the last orbital node before nu reaches nu_LSO(e));
 *          an invalid walker's rows are all zero
 *  ws      workspace of at least emri_workspace_bytes(cfg, B) bytes */
emri_status emri_waveform_batch(const double* params, int64_t B, const emri_cfg* cfg, void* ht,
                                void* ws, size_t ws_bytes, hipStream_t stream);

/* Fourier transform of time-domain waveforms (Sec. 3, "appropriate
 * normalisation" read as h~(f_k) = dt sum_j h_j exp(-2 pi i j k / N)).
 *  ht   [B][N][2] real, as written by emri_waveform_batch (fp64 or fp32)
 *  hf   [B][2][N/2+1] complex (re, im interleaved), bins f_k = k/(N dt),
 *       channel I then II; fp64 or fp32 following cfg->precision
 *  ht and hf must not overlap the workspace. */
emri_status emri_fft_batch(const void* ht, int64_t B, const emri_cfg* cfg, void* hf, void* ws,
                           size_t ws_bytes, hipStream_t stream);

/* Log-likelihood per walker (Eq. (8), read as -1/2 <d - m | d - m>):
 *   lnL_w = -1/2 sum_{I,II} sum_{k=1}^{N/2-1} (4 df / S_k) |d_k - m_k|^2,
 *   m_k = exp(-2 pi i f_k DeltaT) h~_k / (Xi d_L)      (Eqs. (4)-(6))
 * with df = 1/(N dt); DC and Nyquist bins are excluded.
 *  data  [2][N/2+1] complex fp64 (re, im interleaved), channel I then II
 *  psd   [N/2+1] fp64 one-sided noise PSD S_k [1/Hz]; psd[0] is ignored;
 *        every other entry must be positive (checked on the device: a
 *        non-positive entry gives that bin weight 0)
 *  T_obs, dt  must equal cfg->T_obs and cfg->dt
 *  lnL   [B] fp64 output
 *  ws    at least emri_dataset_bytes(cfg) + emri_workspace_bytes(cfg, 1)
 *        bytes; walkers are processed in as many chunks as the workspace
 *        requires (all at once with dataset + workspace_bytes(cfg, B)) */
emri_status emri_loglike_batch(const double* params, int64_t B, const double* data,
                               const double* psd, double T_obs, double dt, const emri_cfg* cfg,
                               double* lnL, void* ws, size_t ws_bytes, hipStream_t stream);

/* Resident data sets for repeated likelihood calls (the serving loop).
 * emri_dataset_init writes, into the caller's buffer `ds`, the data and
 * noise weights in the orders the likelihood kernels read them: per bin of
 * the packed two-channel spectrum, the data combined with the square root
 * of half the weight (so that each bin enters on its own), and per positive
 * frequency the data and weights as given (the frequency-dependent pass);
 * FP32 copies for EMRI_MIXED; and the FP64 data norm <d|d>.  The buffer is
 * valid for the cfg it was made with (same N, dt, precision). */
size_t emri_dataset_bytes(const emri_cfg* cfg);
emri_status emri_dataset_init(const double* data, const double* psd, const emri_cfg* cfg,
                              void* ds, size_t ds_bytes, hipStream_t stream);

/* As emri_loglike_batch, on a resident data set made by emri_dataset_init.
 *  ws  at least emri_workspace_bytes(cfg, 1) bytes; chunked as needed. */
emri_status emri_loglike_dataset(const double* params, int64_t B, const void* ds,
                                 const emri_cfg* cfg, double* lnL, void* ws, size_t ws_bytes,
                                 hipStream_t stream);

/* As emri_loglike_dataset, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  No workspace argument: the call works in a device array of
 * EMRI_NOALLOC_SCRATCH_BYTES (512 MiB) inside the library, which every GPU
 * the library runs on holds until the process ends.  The call itself
 * allocates nothing (no device memory, streams or events; the orbit runs in
 * one segment unless an earlier ordinary call on `stream` set up its
 * pipeline).  Walkers are processed in as many chunks as the array holds;
 * a cfg whose emri_workspace_bytes(cfg, 1) exceeds the array gets
 * EMRI_EWORKSPACE and nothing is launched (every N <= 2^23, and 2^24 at
 * up to about 40 harmonics, fits).  Results are bitwise those of
 * emri_loglike_dataset.  All calls on one GPU share its array and it keeps
 * the last call's contents: calls that overlap on one GPU (concurrent
 * streams or threads) race and must be serialised by the caller. */
#define EMRI_NOALLOC_SCRATCH_BYTES ((size_t)512 << 20)
emri_status emri_loglike_dataset_noalloc(const double* params, int64_t B, const void* ds,
                                         const emri_cfg* cfg, double* lnL, hipStream_t stream);

/* ---- frequency-dependent propagation --------------------------------------
 * The variant of Sec. 2 "Waveform propagation" in which alpha_M and alpha_T
 * depend on the GW frequency, written as power series in x = f / f_star with
 * coefficients constant in z:
 *   alpha_M(f) = sum_{n<P} m_n x^n,   alpha_T(f) = p[16] + sum_{n<P} t_n x^n.
 * The friction integral of Eq. (5) then gives the extra amplitude factor
 * (1 + z)^(-alpha_M(f)/2) on top of Eq. (6), and the speed the delay
 * Delta T(f) = (1/c_T(f) - 1) chi / c with c_T(f)^2 = 1 + alpha_T(f) (chi the
 * comoving distance), applied as exp(-2 pi i f Delta T(f)) bin by bin.  A
 * walker with 1 + alpha_T(f) <= 0 in any bin 1..N/2-1 gets lnL = -inf. */
#define EMRI_FMG_MAX 8
typedef struct {
    int32_t order;               /* P, 0..EMRI_FMG_MAX (0: the constant propagation, with the
                                    delay evaluated bin by bin) */
    int32_t reserved;            /* 0 */
    double f_star;               /* pivot frequency [Hz], > 0 */
} emri_fmg;                      /* a HOST struct, read during the call */

/* As emri_loglike_dataset, with the series coefficients coef[B][2][P]
 * (device; per walker m_0..m_{P-1} then t_0..t_{P-1}; may be NULL when
 * P = 0).  Errors: order outside 0..8, f_star not positive and finite, or a
 * NULL pointer: EMRI_EINVAL before anything is launched. */
emri_status emri_loglike_dataset_fmg(const double* params, int64_t B, const double* coef,
                                     const emri_fmg* fmg, const void* ds, const emri_cfg* cfg,
                                     double* lnL, void* ws, size_t ws_bytes, hipStream_t stream);

/* Frequency-domain model of each walker, the quantity the likelihood
 * compares with the data (Eqs. (4)-(6) applied to the transformed waveform):
 *   m_k = exp(-2 pi i f_k DeltaT) h~_k / (Xi d_L),  k = 0..N/2
 *  mf   [B][2][N/2+1] complex (re, im interleaved), fp64 or fp32 following
 *       cfg->precision; an invalid walker's rows are zero
 *  ws   at least emri_workspace_bytes(cfg, B) bytes
 * With a noise draw added, the model at the injection is the mock data set
 * (the paper's fiducial h[theta_0](f), Sec. 3 "Overview"). */
emri_status emri_model_batch(const double* params, int64_t B, const emri_cfg* cfg, void* mf,
                             void* ws, size_t ws_bytes, hipStream_t stream);

/* One-sided LISA noise PSD on the frequency grid f_k = k/(N dt), k = 0..N/2
 * (the paper's get_noise(), Sec. 3, which has two noise models), in 1/Hz;
 * psd[0] = +infinity.
 *  model 0: instrumental noise of Barack & Cutler 2004,
 *           S(f) = 9.18e-52 f^-4 + 1.59e-41 + 9.18e-38 f^2;
 *  model 1: the sky-averaged sensitivity of Robson, Cornish & Liu 2019,
 *           10/(3 L^2) [P_OMS + 2 (1 + cos^2(f/f*)) P_acc/(2 pi f)^4]
 *           (1 + 0.6 (f/f*)^2), L = 2.5e9 m, f* = c/(2 pi L);
 *  models 2..5: model 1 plus their galactic confusion noise for 0.5, 1, 2
 *           and 4 years of observation.
 * Other models: EMRI_EUNSUPPORTED.
 *  psd  [N/2+1] fp64 device output */
emri_status emri_noise_psd(int model, int64_t N, double dt, double* psd, hipStream_t stream);

/* Per-stage device timing (profiling).  While enabled, every kernel launch
 * of the library is bracketed by HIP events on the stream it runs on; with
 * the auxiliary stream, stages overlap and their sum exceeds the call's
 * duration.
 * emri_trace_read synchronises the recorded events, writes for each stage i
 * (0 <= i < n) the summed duration in ms and the number of launches since the
 * previous read, and returns the number of stages.  Stage names come from
 * emri_trace_stage_name.  Host-thread safe only if one thread traces. */
emri_status emri_trace_enable(int on);
int emri_trace_read(double* ms, int64_t* launches, int n);
const char* emri_trace_stage_name(int i);

/* ---- serving loop ------------------------------------------------------
 * A persistent request loop for many concurrent MCMC chains (the paper's
 * vectorised walker matrix, Sec. 3, served to several chains at once).
 * Requests of W walkers against a resident data set are packed with other
 * pending requests of the same data set into batches (continuous batching:
 * a request that arrives while others run joins the next batch that has a
 * free stream and HBM), each batch is admitted only when its device block
 * (parameters, results and workspace) fits in the caller's arena (admission
 * by HBM footprint), and each batch runs as one hipGraph replay (captured
 * once per device block and reused).  Batches run concurrently on several
 * streams.  Per-walker results do not depend on how requests were batched. */
typedef struct emri_server emri_server;

typedef struct {
    void* arena;          /* device memory owned by the caller: the HBM budget */
    size_t arena_bytes;
    int32_t n_streams;    /* batches in flight at once, 1..16 */
    int32_t max_batch;    /* walkers per batch, multiple of 32, 32..4096;
                             requests are at most this large */
    int32_t use_graphs;   /* 1: launch batches as captured hipGraphs */
    int32_t reserved;     /* must be 0 */
} emri_server_cfg;

typedef struct {
    int64_t submitted, completed, rejected;
    int64_t batches, graph_launches, graph_captures;
    int64_t walkers, padded_walkers;  /* evaluated for requests / as padding */
    size_t arena_in_use, arena_peak;
} emri_server_stats;

/* Starts the scheduler thread on the current device. */
emri_status emri_server_create(const emri_server_cfg* cfg, emri_server** out);
/* Finishes in-flight batches, fails pending requests, frees host resources. */
emri_status emri_server_destroy(emri_server* s);
/* Copies a data set (device data [2][N/2+1] complex fp64, psd [N/2+1]) into
 * the arena in the likelihood's order; blocks until the copy is done. */
emri_status emri_server_add_dataset(emri_server* s, const emri_cfg* cfg, const double* data,
                                    const double* psd, int32_t* dataset_id);
/* Queues W walkers: params is HOST memory [W][17], copied before the call
 * returns; lnL is HOST memory [W], written when the request completes.
 * EMRI_EWORKSPACE if the request could never fit in the arena. */
emri_status emri_server_submit(emri_server* s, int32_t dataset_id, const double* params,
                               int64_t W, double* lnL, uint64_t* ticket);
/* Waits for a request (timeout_s < 0: forever).  On EMRI_OK lnL is written
 * and *latency_s (if non-NULL) is the time from submit to completion; the
 * ticket is then released.  EMRI_EINVAL for an unknown ticket; a timeout
 * returns EMRI_EDEVICE with the request still queued. */
emri_status emri_server_wait(emri_server* s, uint64_t ticket, double timeout_s,
                             double* latency_s);
emri_status emri_server_stats_get(emri_server* s, emri_server_stats* out);

/* ---- ensemble sampler step -------------------------------------------------
 * The affine-invariant stretch move of Goodman & Weare (2010), which the
 * paper's sampler applies to the walker matrix (Sec. 1 iii; Sec. 3
 * "Posterior sampling"), in its parallel form: the ensemble of 2W walkers
 * (rows of X, EMRI_NPAR doubles each) is split into halves [0, W) and
 * [W, 2W), updated in turn, each against the other.  For walker k of half h
 * a partner j of the other half is drawn, a stretch z with density
 * proportional to 1/sqrt(z) on [1/a, a], and the proposal
 * Y = X_j + z (X_k - X_j) on the free coordinates (the others are kept) is
 * accepted with probability min(1, z^(D-1) p(Y) / p(X_k)).  The log-posterior
 * is a flat prior on a box of the free coordinates (-inf outside) plus the
 * log-likelihood against a resident data set (emri_dataset_init).
 * The random numbers are inputs (u, in [0, 1)), so that a step is a
 * deterministic function of them: u[h][k][0] picks the partner
 * (j = floor(u0 W)), u[h][k][1] the stretch (z = ((a-1) u1 + 1)^2 / a),
 * u[h][k][2] the acceptance (accept if ln u2 < (D-1) ln z + lnp(Y) - lnp(X_k);
 * a proposal at -inf is rejected, a walker at -inf takes any finite one). */
typedef struct {
    int32_t n_free;              /* D, 1..EMRI_NPAR */
    int32_t idx[EMRI_NPAR];      /* parameter indices of the free coordinates (first D) */
    double lo[EMRI_NPAR];        /* prior box: lo[d] <= p[idx[d]] <= hi[d] */
    double hi[EMRI_NPAR];
} emri_prior;                    /* a HOST struct, read during the call */

/* Workspace of emri_stretch_step for 2W walkers evaluated in one chunk
 * (smaller workspaces down to the proposals plus emri_workspace_bytes(cfg, 1)
 * work in chunks). */
size_t emri_sampler_workspace_bytes(const emri_cfg* cfg, int64_t W);

/* lnp[n] = log-prior (box) + log-likelihood of the n walkers X[n][17]
 * against the resident data set ds.  ws as emri_loglike_dataset. */
emri_status emri_ensemble_lnprob(const double* X, int64_t n, const emri_prior* prior,
                                 const void* ds, const emri_cfg* cfg, double* lnp, void* ws,
                                 size_t ws_bytes, hipStream_t stream);

/* One step of the ensemble X[2W][17] (device, updated in place) with
 * log-posteriors lnp[2W] (device, in/out, e.g. from emri_ensemble_lnprob);
 * a > 1 is the stretch scale (2 is the usual choice); u[2][W][3] device
 * uniforms; accepted[2W] (device, may be NULL) receives 1 where the walker
 * moved.  Errors: W < 1, a <= 1, a prior with D outside 1..17, an index
 * outside 0..16 or repeated, lo > hi: EMRI_EINVAL; workspace smaller than the
 * proposals plus emri_workspace_bytes(cfg, 1): EMRI_EWORKSPACE. */
emri_status emri_stretch_step(double* X, double* lnp, int64_t W, const emri_prior* prior,
                              double a, const double* u, const void* ds, const emri_cfg* cfg,
                              int32_t* accepted, void* ws, size_t ws_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* EMRI_H */
