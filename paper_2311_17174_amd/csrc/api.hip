// api.hip -- the C ABI of libemri (declared in include/emri.h): argument
// checks, workspace planning, chunking and the launch sequence of the hot
// path.  Every arithmetic step runs in the kernels of walker.hip, synth.hip,
// fft.hip and like.hip.
#include "internal.hpp"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

namespace emri {

static thread_local std::string g_err;

// ---- event tracing ---------------------------------------------------------
static const char* const kStageNames[ST_COUNT] = {
    "walker_setup", "amplitude_tables", "synthesis", "twiddles", "fft_columns",
    "fft_rows", "unpack", "dataset", "inner_product", "walker_sum", "noise_psd", "sampler"};

struct TraceRec { int stage; hipEvent_t a, b; };
static std::mutex g_trace_mu;
static bool g_trace_on = false;
static std::vector<hipEvent_t> g_events;   // pool, reused after each read
static size_t g_next_event = 0;
static std::vector<TraceRec> g_recs;

static hipEvent_t next_event()
{
    if (g_next_event == g_events.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_events.push_back(e);
    }
    return g_events[g_next_event++];
}

static thread_local bool g_trace_suppress = false;

void trace_suppress(bool on) { g_trace_suppress = on; }

void trace_mark(int stage, hipStream_t s, bool begin)
{
    if (!g_trace_on || g_trace_suppress) return;
    std::lock_guard<std::mutex> lk(g_trace_mu);
    hipEvent_t e = next_event();
    if (!e) return;
    if (hipEventRecord(e, s) != hipSuccess) return;
    if (begin) {
        g_recs.push_back(TraceRec{stage, e, nullptr});
    } else {
        for (size_t i = g_recs.size(); i-- > 0;)
            if (g_recs[i].stage == stage && g_recs[i].b == nullptr) { g_recs[i].b = e; break; }
    }
}

static emri_status fail(emri_status st, const char* msg)
{
    g_err = msg ? msg : "";
    return st;
}

emri_status set_error(emri_status st, const char* msg) { return fail(st, msg); }

static std::mutex g_lds_mu;
static std::vector<std::pair<const void*, size_t>> g_lds_set;

hipError_t allow_lds(const void* kernel, size_t bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_lds_mu);
    for (auto& kv : g_lds_set)
        if (kv.first == kernel && kv.second >= bytes) return hipSuccess;
    const hipError_t e =
        hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) g_lds_set.emplace_back(kernel, bytes);
    return e;
}

static emri_status fail_hip(hipError_t e, const char* where)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    g_err = buf;
    return EMRI_EDEVICE;
}

// ---- launch-plan overrides --------------------------------------------------
// Set only through emri_tuning_set; a call takes one copy under the lock and
// plans with it throughout, so a concurrent change never mixes two plans.
static std::mutex g_tuning_mu;
static Tuning g_tuning = {0, 0, 0, 0};

Tuning tuning_now()
{
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    return g_tuning;
}

emri_status make_plan(const emri_cfg* cfg, int64_t B, const Tuning& tn, Plan* p,
                      const char** err)
{
    *err = nullptr;
    if (!cfg) { *err = "cfg is NULL"; return EMRI_EINVAL; }
    if (!(cfg->T_obs > 0.0) || !isfinite(cfg->T_obs)) { *err = "T_obs must be positive"; return EMRI_EINVAL; }
    if (!(cfg->dt > 0.0) || !isfinite(cfg->dt)) { *err = "dt must be positive"; return EMRI_EINVAL; }
    if (cfg->N <= 0 || (cfg->N & (cfg->N - 1))) { *err = "N must be a power of two"; return EMRI_EINVAL; }
    if (cfg->N < ((int64_t)1 << 12) || cfg->N > ((int64_t)1 << 24)) {
        *err = "N must be in [2^12, 2^24]";
        return EMRI_EUNSUPPORTED;
    }
    const double nvd = cfg->T_obs / cfg->dt;
    if (!(nvd < 9.0e18)) { *err = "T_obs/dt too large"; return EMRI_EINVAL; }
    const int64_t Nv = (int64_t)llround(nvd);
    if (Nv < 1 || Nv > cfg->N) { *err = "need 1 <= round(T_obs/dt) <= N"; return EMRI_EINVAL; }
    if (cfg->n_harm < 1 || cfg->n_harm > 64) { *err = "n_harm must be in [1, 64]"; return EMRI_EINVAL; }
    if (cfg->precision != EMRI_FP64 && cfg->precision != EMRI_MIXED) {
        *err = "unknown precision";
        return EMRI_EINVAL;
    }
    if (cfg->coarse_log2 < 8 || cfg->coarse_log2 > 12) {
        *err = "coarse_log2 must be in [8, 12]";
        return EMRI_EUNSUPPORTED;
    }
    if (cfg->ic != EMRI_IC_START && cfg->ic != EMRI_IC_LSO) {
        *err = "ic must be EMRI_IC_START or EMRI_IC_LSO";
        return EMRI_EINVAL;
    }
    if (cfg->ode != EMRI_ODE_RK4 && cfg->ode != EMRI_ODE_DP5 && cfg->ode != EMRI_ODE_RK78) {
        *err = "ode must be EMRI_ODE_RK4, EMRI_ODE_DP5 or EMRI_ODE_RK78";
        return EMRI_EINVAL;
    }
    if (cfg->reserved != 0) { *err = "reserved must be 0"; return EMRI_EINVAL; }
    if (cfg->ode != EMRI_ODE_RK4 &&
        !(cfg->ode_rtol >= 1e-13 && cfg->ode_rtol <= 1e-3 && cfg->ode_atol >= 0.0 &&
          isfinite(cfg->ode_atol))) {
        *err = "adaptive tolerances: need 1e-13 <= ode_rtol <= 1e-3 and a finite ode_atol >= 0";
        return EMRI_EINVAL;
    }
    if (B < 0) { *err = "B must be >= 0"; return EMRI_EINVAL; }

    Plan& q = *p;
    memset(&q, 0, sizeof q);
    q.tn = tn;
    q.T_obs = cfg->T_obs;
    q.ic = cfg->ic;
    q.ode = cfg->ode;
    q.rtol = cfg->ode_rtol;
    q.atol = cfg->ode_atol;
    q.dt = cfg->dt;
    q.N = cfg->N;
    q.Nv = Nv;
    int m = 0;
    while (((int64_t)1 << m) < q.N) ++m;
    q.m = m;
    q.nh = cfg->n_harm;
    q.prec = cfg->precision;
    q.cl = cfg->coarse_log2;
    q.L = (int64_t)1 << q.cl;
    q.K = (Nv + q.L - 1) / q.L;
    // FFT split: rows (pass B, contiguous, fused with the likelihood) up to
    // 2^12 so a row transform has 512 lanes; columns the rest (up to 2^12)
    q.m1 = (m + 1) / 2 + 1;
    if (q.m1 > 12) q.m1 = 12;
    // an override of the row length 2^m1 applies where both passes support it
    if (tn.fft_row_log2) {
        const int v = tn.fft_row_log2;
        if (v >= 7 && v <= 12 && m - v >= 4 && m - v <= 12) q.m1 = v;
    }
    q.m2 = m - q.m1;
    q.R1 = (int64_t)1 << q.m1;
    q.R2 = (int64_t)1 << q.m2;
    q.esz = (q.prec == EMRI_FP64) ? 16 : 8;
    q.hsz = (q.prec == EMRI_FP64) ? 8 : 4;
    // pass-A workgroup: TA columns in rows of TA * esz = 128 bytes (FP64) or
    // 64 bytes (FP32) (or the override), within 1024 lanes (16 values each)
    // and the 160 KiB of LDS a workgroup may hold
    size_t run_bytes = (q.prec == EMRI_FP64) ? 128 : 64;
    if (tn.fft_col_run_bytes) run_bytes = (size_t)tn.fft_col_run_bytes;
    int ta = (int)(run_bytes / q.esz);
    if (ta < 1) ta = 1;
    while (ta > 16) ta /= 2;
    while (ta > 1 && (ta * q.R2 / 16 > 1024 || cols_lds_bytes(q.prec, q.R2, ta) > 160 * 1024))
        ta /= 2;
    q.TA = ta;

    q.B = B;
    size_t o = 0;
    const TwLayout tl = tw_layout(q);
    q.off_tw = o; o += align256(tl.bytes);
    q.off_wc = o; o += align256((size_t)B * WC * 8);
    q.off_orb = o; o += align256((size_t)B * (q.K + 1) * 10 * 8);
    q.off_co = o; o += align256((size_t)B * q.K * 16 * 8);
    q.off_az = o; o += align256((size_t)q.K * 16);
    q.off_ch = o; o += align256((size_t)B * q.K * q.nh * 12 * q.hsz);
    // mixed path: per (walker, interval, harmonic) the bound of the
    // harmonic's amplitudes and of their cubic coefficients (float2), and
    // per (walker, interval) the harmonics to sum and the cubic flag (int2)
    q.off_hb = o; o += (q.prec == EMRI_MIXED) ? align256((size_t)B * q.K * q.nh * 8) : 0;
    q.off_hx = o; o += (q.prec == EMRI_MIXED) ? align256((size_t)B * q.K * 8) : 0;
    q.off_z = o; o += align256((size_t)B * q.N * q.esz);
    q.off_part = o; o += align256((size_t)B * q.R2 * 8);
    q.total = o;

    size_t d = 0;
    const int64_t half = q.N / 2;
    q.ds_off_d = d; d += align256((size_t)2 * half * q.esz);
    q.ds_off_w = d; d += align256((size_t)half * (q.prec == EMRI_FP64 ? 8 : 4));
    q.ds_off_q = d; d += align256((size_t)q.N * q.esz);
    q.ds_off_v = d; d += align256((size_t)q.N * (q.prec == EMRI_FP64 ? 8 : 4));
    q.ds_off_norm = d; d += 256;
    q.ds_off_npart = d; d += align256((size_t)kNormParts * 8);
    q.ds_total = d;
    return EMRI_OK;
}

static emri_status check_launch(hipError_t e, const char* where)
{
    if (e != hipSuccess) return fail_hip(e, where);
    return EMRI_OK;
}

// ---- orbit-segment pipeline -------------------------------------------------
// The orbit integration is sequential in time and runs one lane per walker:
// alone it would leave the GPU nearly idle.  It is cut into S segments of
// coarse steps; the caller's stream integrates them in turn and builds each
// finished segment's tables while an auxiliary stream synthesises the
// samples of the segments already tabulated.  One auxiliary stream
// (non-blocking, default priority) and its events per (device, caller
// stream), created on first use and kept until the process ends.  Every wait refers to an event recorded earlier in
// host order, and the caller's stream waits for the auxiliary stream before
// returning, so the pair behaves as one stream to the caller (also under
// stream capture, where the auxiliary stream joins and leaves the capture).
struct Pipe {
    hipStream_t aux = nullptr;
    hipEvent_t seg[kMaxSeg] = {};
    hipEvent_t join = nullptr;
};
static std::mutex g_pipe_mu;
static std::map<std::pair<int, hipStream_t>, Pipe> g_pipes;
// set on a thread for the duration of a call that must create nothing
static thread_local bool g_pipe_no_create = false;

// the auxiliary stream and events of caller stream s on the current device:
// found, or created when s is not capturing; *out = nullptr (and EMRI_OK)
// when s is capturing and has none, so that nothing is created inside a
// capture (the call then runs its orbit in one segment on s alone), and
// likewise inside a call that allocates nothing
static emri_status get_pipe(hipStream_t s, Pipe** out)
{
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "pipeline: hipGetDevice");
    std::lock_guard<std::mutex> lk(g_pipe_mu);
    auto it = g_pipes.find({dev, s});
    if (it != g_pipes.end()) {
        *out = &it->second;
        return EMRI_OK;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    e = hipStreamIsCapturing(s, &cs);
    if (e != hipSuccess) return fail_hip(e, "pipeline: hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone || g_pipe_no_create) return EMRI_OK;
    Pipe q;
    e = hipStreamCreateWithFlags(&q.aux, hipStreamNonBlocking);
    for (int i = 0; i < kMaxSeg && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&q.seg[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&q.join, hipEventDisableTiming);
    if (e != hipSuccess) {
        for (int i = 0; i < kMaxSeg; ++i)
            if (q.seg[i]) (void)hipEventDestroy(q.seg[i]);
        if (q.join) (void)hipEventDestroy(q.join);
        if (q.aux) (void)hipStreamDestroy(q.aux);
        return fail_hip(e, "pipeline: stream/event creation");
    }
    *out = &g_pipes.emplace(std::make_pair(dev, s), q).first->second;
    return EMRI_OK;
}

emri_status prepare_pipe(hipStream_t s)
{
    Pipe* pp = nullptr;
    const emri_status st = get_pipe(s, &pp);
    if (st == EMRI_OK && !pp) return fail(EMRI_EINVAL, "pipeline: stream is capturing");
    return st;
}

// number of orbit segments: about 384 coarse steps each, at most 8 (the
// override: 1 .. 16)
static int orbit_segments(const Plan& p, bool zero_tail)
{
    // From the LSO the orbit is integrated backward and the segments run in
    // reverse time order.  A walker found invalid in a later segment would
    // leave samples of the earlier ones in time-domain output, so there the
    // backward orbit runs as one segment; the likelihood and model paths
    // take their samples only from valid walkers.
    if (p.ic == EMRI_IC_LSO && zero_tail) return 1;
    int64_t S = p.K / 384;
    if (p.tn.orbit_segments) S = p.tn.orbit_segments;
    else if (S > 8) S = 8;
    if (S > kMaxSeg) S = kMaxSeg;
    if (S > p.K) S = p.K;
    return S < 1 ? 1 : (int)S;
}

// walkers [0, B) of params, workspace planned for at least B walkers.  With
// zero_tail false the samples from nv_w = min(K_w L, N_valid) on are left
// unwritten (the FFT's pass A takes them as zero)
static emri_status run_waveforms(const Plan& p, const double* params, int64_t B, void* ws,
                                 void* out, bool zero_tail, hipStream_t s)
{
    int S = orbit_segments(p, zero_tail);
    const bool back = p.ic == EMRI_IC_LSO;
    // synthesis intervals: with the zero tail up to N / L, else those covering N_valid
    const int64_t KT = zero_tail ? p.N / p.L : p.K;
    // segment bounds in integration order: the first segment (integrated
    // before anything else can start) is a quarter of the others
    auto kb = [&](int i) -> int64_t {
        if (i <= 0) return 0;
        if (i >= S) return p.K;
        return p.K * (int64_t)(1 + 4 * (i - 1)) / (int64_t)(1 + 4 * (S - 1));
    };
    // segment i covers the intervals [lo(i), hi(i)): forward [kb(i), kb(i+1)),
    // backward from the LSO [K - kb(i+1), K - kb(i))
    auto lo = [&](int i) -> int64_t { return back ? p.K - kb(i + 1) : kb(i); };
    auto hi = [&](int i) -> int64_t { return back ? p.K - kb(i) : kb(i + 1); };
    emri_status st;
    if ((st = check_launch(launch_azimuth(p, ws, s), "azimuth table"))) return st;
    Pipe* pp = nullptr;
    if (S > 1) {
        if ((st = get_pipe(s, &pp))) return st;
        if (!pp) S = 1;   // first use of s inside a capture: one segment
    }
    if (S == 1) {
        if ((st = check_launch(launch_walker_setup(p, params, B, ws, back ? 0 : p.K, s),
                               "walker setup")))
            return st;
        if ((st = check_launch(launch_tables(p, B, ws, 0, p.K, 0, s), "amplitude tables")))
            return st;
        return check_launch(launch_synth(p, B, ws, out, 0, KT, 0, zero_tail, s), "synthesis");
    }
    // the first segment's last node: kb(1) forward, K - kb(1) backward
    st = check_launch(launch_walker_setup(p, params, B, ws, back ? lo(0) : hi(0), s),
                      "walker setup");
    bool forked = false;
    // the caller's stream integrates segment i and builds its tables (small
    // kernels that fill the issue slots the synthesis leaves); the auxiliary
    // stream synthesises segment i meanwhile
    for (int i = 0; i < S && st == EMRI_OK; ++i) {
        // resume from the previous segment's last node: forward from lo(i)
        // up to hi(i), backward from hi(i) down to lo(i)
        if (i > 0 &&
            (st = check_launch(back ? launch_walker_resume(p, B, ws, hi(i), lo(i), i, s)
                                    : launch_walker_resume(p, B, ws, lo(i), hi(i), i, s),
                               "orbit")))
            break;
        if ((st = check_launch(launch_tables(p, B, ws, lo(i), hi(i), i, s), "amplitude tables")))
            break;
        if ((st = check_launch(hipEventRecord(pp->seg[i], s), "pipeline: event record"))) break;
        if ((st = check_launch(hipStreamWaitEvent(pp->aux, pp->seg[i], 0), "pipeline: wait")))
            break;
        forked = true;
        // forward, the last segment also takes the zero tail past K
        const int64_t sh = (!back && i == S - 1) ? KT : hi(i);
        if ((st = check_launch(launch_synth(p, B, ws, out, lo(i), sh, i, zero_tail, pp->aux),
                               "synthesis")))
            break;
    }
    if (forked) {   // join, also after a failed launch
        const hipError_t e1 = hipEventRecord(pp->join, pp->aux);
        const hipError_t e2 = (e1 == hipSuccess) ? hipStreamWaitEvent(s, pp->join, 0) : e1;
        if (st == EMRI_OK) st = check_launch(e2, "pipeline: join");
    }
    return st;
}

// largest chunk <= B whose plan fits in `bytes`
static int64_t fit_chunk(const emri_cfg* cfg, int64_t B, size_t bytes, const Tuning& tn)
{
    Plan p;
    const char* err;
    int64_t lo = 0, hi = B;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        make_plan(cfg, mid, tn, &p, &err);
        if (p.total <= bytes) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace emri

using namespace emri;

extern "C" {

int emri_abi_version(void) { return EMRI_ABI_VERSION; }

emri_status emri_tuning_set(const emri_tuning* t)
{
    Tuning v = {0, 0, 0, 0};
    if (t) {
        if (t->orbit_segments < 0 || t->orbit_segments > kMaxSeg)
            return fail(EMRI_EINVAL, "tuning: orbit_segments must be 0 (automatic) or 1..16");
        if (t->fft_row_log2 != 0 && (t->fft_row_log2 < 7 || t->fft_row_log2 > 12))
            return fail(EMRI_EINVAL, "tuning: fft_row_log2 must be 0 (automatic) or 7..12");
        const int rb = t->fft_col_run_bytes;
        if (rb != 0 && (rb < 8 || rb > 256 || (rb & (rb - 1))))
            return fail(EMRI_EINVAL,
                        "tuning: fft_col_run_bytes must be 0 (automatic) or a power of two in 8..256");
        if (t->like_walkers_per_wg < 0 || t->like_walkers_per_wg > 32)
            return fail(EMRI_EINVAL, "tuning: like_walkers_per_wg must be 0 (automatic) or 1..32");
        if (t->reserved != 0) return fail(EMRI_EINVAL, "tuning: reserved must be 0");
        v = Tuning{t->orbit_segments, t->fft_row_log2, rb, t->like_walkers_per_wg};
    }
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    g_tuning = v;
    return EMRI_OK;
}

emri_status emri_tuning_get(emri_tuning* t)
{
    if (!t) return fail(EMRI_EINVAL, "null pointer argument");
    const Tuning v = tuning_now();
    t->orbit_segments = v.orbit_segments;
    t->fft_row_log2 = v.fft_row_log2;
    t->fft_col_run_bytes = v.fft_col_run_bytes;
    t->like_walkers_per_wg = v.like_walkers_per_wg;
    t->reserved = 0;
    return EMRI_OK;
}

const char* emri_last_error(void) { return g_err.c_str(); }

size_t emri_workspace_bytes(const emri_cfg* cfg, int64_t B)
{
    Plan p;
    const char* err;
    if (make_plan(cfg, B < 1 ? 1 : B, tuning_now(), &p, &err) != EMRI_OK) return 0;
    return p.total;
}

size_t emri_dataset_bytes(const emri_cfg* cfg)
{
    Plan p;
    const char* err;
    if (make_plan(cfg, 1, tuning_now(), &p, &err) != EMRI_OK) return 0;
    return p.ds_total;
}

emri_status emri_waveform_batch(const double* params, int64_t B, const emri_cfg* cfg, void* ht,
                                void* ws, size_t ws_bytes, hipStream_t stream)
{
    Plan p;
    const char* err;
    emri_status st = make_plan(cfg, B, tuning_now(), &p, &err);
    if (st != EMRI_OK) return fail(st, err);
    if (B == 0) return EMRI_OK;
    if (!params || !ht || !ws) return fail(EMRI_EINVAL, "null pointer argument");
    if (ws_bytes < p.total) return fail(EMRI_EWORKSPACE, "workspace smaller than emri_workspace_bytes(cfg, B)");
    return run_waveforms(p, params, B, ws, ht, true, stream);
}

emri_status emri_orbit_batch(const double* params, int64_t B, const emri_cfg* cfg, double* orb,
                             int32_t* kw, void* ws, size_t ws_bytes, hipStream_t stream)
{
    Plan p;
    const char* err;
    emri_status st = make_plan(cfg, B, tuning_now(), &p, &err);
    if (st != EMRI_OK) return fail(st, err);
    if (B == 0) return EMRI_OK;
    if (!params || !orb || !kw || !ws) return fail(EMRI_EINVAL, "null pointer argument");
    if (ws_bytes < p.total) return fail(EMRI_EWORKSPACE, "workspace smaller than emri_workspace_bytes(cfg, B)");
    // the whole orbit as one segment: forward up to node K, backward down to 0
    const bool back = p.ic == EMRI_IC_LSO;
    if ((st = check_launch(launch_walker_setup(p, params, B, ws, back ? 0 : p.K, stream),
                           "walker setup")))
        return st;
    return check_launch(launch_orbit_out(p, B, ws, orb, kw, stream), "orbit copy");
}

emri_status emri_fft_batch(const void* ht, int64_t B, const emri_cfg* cfg, void* hf, void* ws,
                           size_t ws_bytes, hipStream_t stream)
{
    Plan p;
    const char* err;
    emri_status st = make_plan(cfg, B, tuning_now(), &p, &err);
    if (st != EMRI_OK) return fail(st, err);
    if (B == 0) return EMRI_OK;
    if (!ht || !hf || !ws) return fail(EMRI_EINVAL, "null pointer argument");
    if (ws_bytes < p.total) return fail(EMRI_EWORKSPACE, "workspace smaller than emri_workspace_bytes(cfg, B)");
    if ((st = check_launch(launch_twiddles(p, ws, stream), "twiddles"))) return st;
    if ((st = check_launch(launch_fft_from(p, B, ht, ws, stream), "fft"))) return st;
    return check_launch(launch_unpack(p, B, ws, hf, stream), "unpack");
}

static emri_status loglike_chunks(const emri_cfg* cfg, const double* params, int64_t B,
                                  const void* ds, double* lnL, void* ws, size_t ws_bytes,
                                  hipStream_t stream, const emri_fmg* fmg = nullptr,
                                  const double* coef = nullptr)
{
    const Tuning tn = tuning_now();
    Plan p1;
    const char* err;
    emri_status st = make_plan(cfg, 1, tn, &p1, &err);
    if (st != EMRI_OK) return fail(st, err);
    if (ws_bytes < p1.total) return fail(EMRI_EWORKSPACE, "workspace smaller than emri_workspace_bytes(cfg, 1)");
    const int64_t chunk = fit_chunk(cfg, B, ws_bytes, tn);
    Plan p;
    make_plan(cfg, chunk, tn, &p, &err);
    if ((st = check_launch(launch_twiddles(p, ws, stream), "twiddles"))) return st;
    for (int64_t w0 = 0; w0 < B; w0 += chunk) {
        const int64_t nb = (B - w0 < chunk) ? (B - w0) : chunk;
        if ((st = run_waveforms(p, params + w0 * EMRI_NPAR, nb, ws,
                                (char*)ws + p.off_z, false, stream)))
            return st;
        if ((st = check_launch(launch_fft_cols(p, nb, ws, stream), "fft columns"))) return st;
        FmgArgs fa{fmg ? fmg->order : 0, fmg ? fmg->f_star : 0.0,
                   coef ? coef + w0 * 2 * (fmg ? fmg->order : 0) : nullptr};
        if ((st = check_launch(launch_likelihood(p, nb, ds, ws, lnL + w0, fmg ? &fa : nullptr,
                                                 stream),
                               "likelihood")))
            return st;
    }
    return EMRI_OK;
}

emri_status emri_loglike_batch(const double* params, int64_t B, const double* data,
                               const double* psd, double T_obs, double dt, const emri_cfg* cfg,
                               double* lnL, void* ws, size_t ws_bytes, hipStream_t stream)
{
    Plan p;
    const char* err;
    emri_status st = make_plan(cfg, 1, tuning_now(), &p, &err);
    if (st != EMRI_OK) return fail(st, err);
    if (T_obs != cfg->T_obs || dt != cfg->dt) return fail(EMRI_EINVAL, "T_obs and dt must equal cfg->T_obs and cfg->dt");
    if (B < 0) return fail(EMRI_EINVAL, "B must be >= 0");
    if (B == 0) return EMRI_OK;
    if (!params || !data || !psd || !lnL || !ws) return fail(EMRI_EINVAL, "null pointer argument");
    const size_t dsb = align256(p.ds_total);
    if (ws_bytes < dsb + p.total) return fail(EMRI_EWORKSPACE, "workspace smaller than emri_dataset_bytes(cfg) + emri_workspace_bytes(cfg, 1)");
    if ((st = check_launch(launch_dataset(p, data, psd, ws, stream), "dataset"))) return st;
    return loglike_chunks(cfg, params, B, ws, lnL, (char*)ws + dsb, ws_bytes - dsb, stream);
}

emri_status emri_dataset_init(const double* data, const double* psd, const emri_cfg* cfg,
                              void* ds, size_t ds_bytes, hipStream_t stream)
{
    Plan p;
    const char* err;
    emri_status st = make_plan(cfg, 1, tuning_now(), &p, &err);
    if (st != EMRI_OK) return fail(st, err);
    if (!data || !psd || !ds) return fail(EMRI_EINVAL, "null pointer argument");
    if (ds_bytes < p.ds_total) return fail(EMRI_EWORKSPACE, "dataset buffer smaller than emri_dataset_bytes(cfg)");
    return check_launch(launch_dataset(p, data, psd, ds, stream), "dataset");
}

emri_status emri_loglike_dataset(const double* params, int64_t B, const void* ds,
                                 const emri_cfg* cfg, double* lnL, void* ws, size_t ws_bytes,
                                 hipStream_t stream)
{
    Plan p;
    const char* err;
    emri_status st = make_plan(cfg, 1, tuning_now(), &p, &err);
    if (st != EMRI_OK) return fail(st, err);
    if (B < 0) return fail(EMRI_EINVAL, "B must be >= 0");
    if (B == 0) return EMRI_OK;
    if (!params || !ds || !lnL || !ws) return fail(EMRI_EINVAL, "null pointer argument");
    return loglike_chunks(cfg, params, B, ds, lnL, ws, ws_bytes, stream);
}

}  // extern "C"

// ---- likelihood without allocation ---------------------------------------------
// For callers that cannot allocate device memory, a file-scope device array
// stands in for the caller's workspace.  Each device holds its own copy for
// the life of the process.  In host code the array's name is only a host
// stand-in: its device address is taken with hipGetSymbolAddress, once per
// device with that device current, and only that address is handed to
// kernels.  No kernel of the likelihood path needs the workspace to start at
// zero (every value is written before it is read), so nothing is cleared.
namespace emri {
static __device__ __align__(256) unsigned char scratch[EMRI_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;

static emri_status scratch_address(void** out)
{
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "scratch: hipGetDevice");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return EMRI_OK;
    }
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return fail_hip(e, "scratch: hipGetSymbolAddress");
    g_scratch_ptr[dev] = ptr;
    *out = ptr;
    return EMRI_OK;
}
}  // namespace emri

extern "C" {

emri_status emri_loglike_dataset_noalloc(const double* params, int64_t B, const void* ds,
                                         const emri_cfg* cfg, double* lnL, hipStream_t stream)
{
    Plan p;
    const char* err;
    emri_status st = make_plan(cfg, 1, tuning_now(), &p, &err);
    if (st != EMRI_OK) return fail(st, err);
    if (B < 0) return fail(EMRI_EINVAL, "B must be >= 0");
    if (B == 0) return EMRI_OK;
    if (!params || !ds || !lnL) return fail(EMRI_EINVAL, "null pointer argument");
    if (p.total > (size_t)EMRI_NOALLOC_SCRATCH_BYTES)
        return fail(EMRI_EWORKSPACE,
                    "one walker's workspace (emri_workspace_bytes(cfg, 1)) exceeds "
                    "EMRI_NOALLOC_SCRATCH_BYTES");
    void* ws = nullptr;
    if ((st = scratch_address(&ws))) return st;
    // neither pipeline streams nor trace events are created inside this call
    const bool pipe_prev = g_pipe_no_create, trace_prev = g_trace_suppress;
    g_pipe_no_create = true;
    g_trace_suppress = true;
    st = loglike_chunks(cfg, params, B, ds, lnL, ws, EMRI_NOALLOC_SCRATCH_BYTES, stream);
    g_pipe_no_create = pipe_prev;
    g_trace_suppress = trace_prev;
    return st;
}

emri_status emri_loglike_dataset_fmg(const double* params, int64_t B, const double* coef,
                                     const emri_fmg* fmg, const void* ds, const emri_cfg* cfg,
                                     double* lnL, void* ws, size_t ws_bytes, hipStream_t stream)
{
    Plan p;
    const char* err;
    emri_status st = make_plan(cfg, 1, tuning_now(), &p, &err);
    if (st != EMRI_OK) return fail(st, err);
    if (!fmg) return fail(EMRI_EINVAL, "null fmg descriptor");
    if (fmg->order < 0 || fmg->order > EMRI_FMG_MAX)
        return fail(EMRI_EINVAL, "fmg: order must be in 0..8");
    if (!(fmg->f_star > 0.0) || !isfinite(fmg->f_star))
        return fail(EMRI_EINVAL, "fmg: f_star must be positive and finite");
    if (B < 0) return fail(EMRI_EINVAL, "B must be >= 0");
    if (B == 0) return EMRI_OK;
    if (!params || !ds || !lnL || !ws || (fmg->order > 0 && !coef))
        return fail(EMRI_EINVAL, "null pointer argument");
    return loglike_chunks(cfg, params, B, ds, lnL, ws, ws_bytes, stream, fmg, coef);
}

// ---- ensemble sampler step ---------------------------------------------------
static emri_status check_prior(const emri_prior* pr, PriorBox* out)
{
    if (!pr) return fail(EMRI_EINVAL, "null prior");
    if (pr->n_free < 1 || pr->n_free > EMRI_NPAR)
        return fail(EMRI_EINVAL, "prior: n_free must be in 1..17");
    bool seen[EMRI_NPAR] = {};
    out->D = pr->n_free;
    for (int d = 0; d < EMRI_NPAR; ++d) {
        out->idx[d] = 0;
        out->lo[d] = out->hi[d] = 0.0;
    }
    for (int d = 0; d < pr->n_free; ++d) {
        const int i = pr->idx[d];
        if (i < 0 || i >= EMRI_NPAR || seen[i])
            return fail(EMRI_EINVAL, "prior: free indices must be distinct, in 0..16");
        seen[i] = true;
        if (!(pr->lo[d] <= pr->hi[d])) return fail(EMRI_EINVAL, "prior: lo > hi (or NaN)");
        out->idx[d] = i;
        out->lo[d] = pr->lo[d];
        out->hi[d] = pr->hi[d];
    }
    return EMRI_OK;
}

// proposals of W walkers at the head of the workspace
static size_t sampler_head_bytes(int64_t W)
{
    return align256((size_t)W * EMRI_NPAR * 8) + 3 * align256((size_t)W * 8);
}


emri_status emri_model_batch(const double* params, int64_t B, const emri_cfg* cfg, void* mf,
                             void* ws, size_t ws_bytes, hipStream_t stream)
{
    Plan p;
    const char* err;
    emri_status st = make_plan(cfg, B, tuning_now(), &p, &err);
    if (st != EMRI_OK) return fail(st, err);
    if (B == 0) return EMRI_OK;
    if (!params || !mf || !ws) return fail(EMRI_EINVAL, "null pointer argument");
    if (ws_bytes < p.total) return fail(EMRI_EWORKSPACE, "workspace smaller than emri_workspace_bytes(cfg, B)");
    if ((st = run_waveforms(p, params, B, ws, (char*)ws + p.off_z, false, stream))) return st;
    if ((st = check_launch(launch_twiddles(p, ws, stream), "twiddles"))) return st;
    if ((st = check_launch(launch_fft(p, B, ws, stream), "fft"))) return st;
    return check_launch(launch_model_unpack(p, B, ws, mf, stream), "unpack");
}

emri_status emri_noise_psd(int model, int64_t N, double dt, double* psd, hipStream_t stream)
{
    if (model < 0 || model > 5)
        return fail(EMRI_EUNSUPPORTED, "noise models are 0 (BC04) and 1..5 (Robson-Cornish-Liu)");
    if (N < 2 || (N & (N - 1)) || !(dt > 0.0) || !isfinite(dt))
        return fail(EMRI_EINVAL, "N must be a power of two >= 2 and dt positive");
    if (!psd) return fail(EMRI_EINVAL, "null pointer argument");
    return check_launch(launch_noise_psd(model, N, dt, psd, stream), "noise psd");
}

emri_status emri_trace_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_trace_mu);
    g_trace_on = on != 0;
    return EMRI_OK;
}

int emri_trace_read(double* ms, int64_t* launches, int n)
{
    std::lock_guard<std::mutex> lk(g_trace_mu);
    for (int i = 0; i < n && i < ST_COUNT; ++i) {
        if (ms) ms[i] = 0.0;
        if (launches) launches[i] = 0;
    }
    for (const TraceRec& r : g_recs) {
        if (!r.b) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) continue;
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) continue;
        if (r.stage < n) {
            if (ms) ms[r.stage] += t;
            if (launches) launches[r.stage] += 1;
        }
    }
    g_recs.clear();
    g_next_event = 0;
    return ST_COUNT;
}

const char* emri_trace_stage_name(int i)
{
    return (i >= 0 && i < ST_COUNT) ? kStageNames[i] : "";
}


size_t emri_sampler_workspace_bytes(const emri_cfg* cfg, int64_t W)
{
    if (W < 1) W = 1;
    const size_t w = emri_workspace_bytes(cfg, W);
    return w ? sampler_head_bytes(W) + w : 0;
}

emri_status emri_ensemble_lnprob(const double* X, int64_t n, const emri_prior* prior,
                                 const void* ds, const emri_cfg* cfg, double* lnp, void* ws,
                                 size_t ws_bytes, hipStream_t stream)
{
    PriorBox pb;
    emri_status st = check_prior(prior, &pb);
    if (st != EMRI_OK) return st;
    if (n < 0) return fail(EMRI_EINVAL, "n must be >= 0");
    if (n == 0) return EMRI_OK;
    if ((st = emri_loglike_dataset(X, n, ds, cfg, lnp, ws, ws_bytes, stream))) return st;
    return check_launch(launch_add_box_prior(X, n, pb, lnp, stream), "prior");
}

emri_status emri_stretch_step(double* X, double* lnp, int64_t W, const emri_prior* prior,
                              double a, const double* u, const void* ds, const emri_cfg* cfg,
                              int32_t* accepted, void* ws, size_t ws_bytes, hipStream_t stream)
{
    PriorBox pb;
    emri_status st = check_prior(prior, &pb);
    if (st != EMRI_OK) return st;
    if (W < 1) return fail(EMRI_EINVAL, "W must be >= 1");
    if (!(a > 1.0) || !isfinite(a)) return fail(EMRI_EINVAL, "stretch scale a must be > 1");
    if (!X || !lnp || !u || !ds || !ws) return fail(EMRI_EINVAL, "null pointer argument");
    Plan p1;
    const char* err;
    if ((st = make_plan(cfg, 1, tuning_now(), &p1, &err)) != EMRI_OK) return fail(st, err);
    const size_t head = sampler_head_bytes(W);
    if (ws_bytes < head + p1.total)
        return fail(EMRI_EWORKSPACE, "workspace smaller than the proposals plus emri_workspace_bytes(cfg, 1)");
    char* b = (char*)ws;
    double* Y = (double*)b;
    double* lnz = (double*)(b + align256((size_t)W * EMRI_NPAR * 8));
    double* lpr = (double*)((char*)lnz + align256((size_t)W * 8));
    double* lnL = (double*)((char*)lpr + align256((size_t)W * 8));
    for (int h = 0; h < 2; ++h) {
        const double* uh = u + (int64_t)h * W * 3;
        if ((st = check_launch(launch_stretch_propose(X, W, h, pb, a, uh, Y, lnz, lpr, stream),
                               "stretch proposals")))
            return st;
        if ((st = loglike_chunks(cfg, Y, W, ds, lnL, b + head, ws_bytes - head, stream)))
            return st;
        if ((st = check_launch(launch_stretch_accept(X, lnp, W, h, Y, lpr, lnL, lnz, uh, accepted,
                                                     stream),
                               "stretch acceptance")))
            return st;
    }
    return EMRI_OK;
}

}  // extern "C"
