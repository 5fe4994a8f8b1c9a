// server.hip -- persistent request loop over the likelihood (emri_server_*).
//
// Host-side runtime, no kernels of its own.  The scheduling core
// (server_core.hpp: arena, request queue, continuous batching, admission by
// HBM footprint, the scheduler thread) is host-only C++; this file gives it
// its device side: a batch is admitted when a stream is free and its device
// block fits in the caller's arena, and runs as one replay of a hipGraph
// captured for that block (parameters H2D, the likelihood kernels, results
// D2H); results go to the requests when the batch's event completes.  Blocks
// are cached per (data set, padded batch size) so graphs are reused; idle
// blocks are evicted when a new batch needs the memory.
#include "internal.hpp"
#include "server_core.hpp"

#include <string.h>

#include <vector>

namespace emri {

static_assert(serve::kOk == EMRI_OK && serve::kEinval == EMRI_EINVAL &&
                  serve::kEworkspace == EMRI_EWORKSPACE && serve::kEdevice == EMRI_EDEVICE,
              "status values of the serving core");
static_assert(serve::kNpar == EMRI_NPAR, "parameter row length");

// the device side of the serving core: one HIP stream and completion event
// per slot, pinned staging per block, one captured graph per block
struct HipDevice {
    struct DsInfo {
        emri_cfg cfg;
    };
    struct Extra {
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    using Block = serve::Scheduler<HipDevice>::Block;

    int device = 0;
    bool use_graphs = true;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;

    size_t block_bytes(const DsInfo& d, int64_t bucket, size_t* ws_bytes)
    {
        const size_t ws = emri_workspace_bytes(&d.cfg, bucket);
        if (ws_bytes) *ws_bytes = ws;
        if (!ws) return 0;
        return align256((size_t)bucket * EMRI_NPAR * 8) + align256((size_t)bucket * 8) + ws;
    }

    bool block_init(Block& b)
    {
        return hipHostMalloc((void**)&b.h_params, (size_t)b.bucket * EMRI_NPAR * 8,
                             hipHostMallocDefault) == hipSuccess &&
               hipHostMalloc((void**)&b.h_lnL, (size_t)b.bucket * 8, hipHostMallocDefault) ==
                   hipSuccess;
    }

    void block_release(Block& b)
    {
        if (b.x.exec) (void)hipGraphExecDestroy(b.x.exec);
        if (b.x.graph) (void)hipGraphDestroy(b.x.graph);
        if (b.h_params) (void)hipHostFree(b.h_params);
        if (b.h_lnL) (void)hipHostFree(b.h_lnL);
        b.x = Extra{};
        b.h_params = b.h_lnL = nullptr;
    }

    // the batch's work on s: parameters in, likelihood, results out
    static emri_status enqueue(Block& b, const DsInfo& d, const void* ds, hipStream_t s)
    {
        if (hipMemcpyAsync(b.d_params, b.h_params, (size_t)b.bucket * EMRI_NPAR * 8,
                           hipMemcpyHostToDevice, s) != hipSuccess)
            return EMRI_EDEVICE;
        emri_status st = emri_loglike_dataset(b.d_params, b.bucket, ds, &d.cfg, b.d_lnL, b.ws,
                                              b.ws_bytes, s);
        if (st != EMRI_OK) return st;
        if (hipMemcpyAsync(b.h_lnL, b.d_lnL, (size_t)b.bucket * 8, hipMemcpyDeviceToHost, s) !=
            hipSuccess)
            return EMRI_EDEVICE;
        return EMRI_OK;
    }

    // the first use of a block runs eagerly (kernel attributes are set
    // outside any capture); its graph is captured at the second use and
    // replayed afterwards
    int launch(Block& b, const DsInfo& d, const void* ds, int slot, serve::Stats& st)
    {
        hipStream_t s = streams[(size_t)slot];
        if (use_graphs && b.uses >= 1) {
            if (!b.x.exec) {
                trace_suppress(true);
                if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                    trace_suppress(false);
                    return EMRI_EDEVICE;
                }
                const emri_status e = enqueue(b, d, ds, s);
                hipGraph_t g = nullptr;
                const hipError_t ec = hipStreamEndCapture(s, &g);
                trace_suppress(false);
                if (e != EMRI_OK || ec != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    return e != EMRI_OK ? e : EMRI_EDEVICE;
                }
                if (hipGraphInstantiate(&b.x.exec, g, nullptr, nullptr, 0) != hipSuccess) {
                    (void)hipGraphDestroy(g);
                    b.x.exec = nullptr;
                    return EMRI_EDEVICE;
                }
                b.x.graph = g;
                st.graph_captures++;
            }
            if (hipGraphLaunch(b.x.exec, s) != hipSuccess) return EMRI_EDEVICE;
            st.graph_launches++;
        } else {
            const emri_status e = enqueue(b, d, ds, s);
            if (e != EMRI_OK) return e;
        }
        return hipEventRecord(events[(size_t)slot], s) == hipSuccess ? EMRI_OK : EMRI_EDEVICE;
    }

    int query(int slot)
    {
        const hipError_t q = hipEventQuery(events[(size_t)slot]);
        if (q == hipErrorNotReady) return 1;
        return q == hipSuccess ? 0 : -1;
    }

    void drain(int slot) { (void)hipStreamSynchronize(streams[(size_t)slot]); }

    void thread_start() { (void)hipSetDevice(device); }
};

}  // namespace emri

struct emri_server {
    emri::HipDevice dev;
    std::unique_ptr<emri::serve::Scheduler<emri::HipDevice>> core;
};

using namespace emri;

extern "C" {

emri_status emri_server_create(const emri_server_cfg* cfg, emri_server** out)
{
    if (!cfg || !out) return set_error(EMRI_EINVAL, "null pointer argument");
    *out = nullptr;
    if (!cfg->arena || cfg->arena_bytes < 4096) return set_error(EMRI_EINVAL, "arena missing or too small");
    if (cfg->n_streams < 1 || cfg->n_streams > 16) return set_error(EMRI_EINVAL, "n_streams must be in [1, 16]");
    if (cfg->max_batch < 32 || cfg->max_batch > 4096 || cfg->max_batch % 32)
        return set_error(EMRI_EINVAL, "max_batch must be a multiple of 32 in [32, 4096]");
    if (cfg->reserved != 0) return set_error(EMRI_EINVAL, "reserved must be 0");
    auto S = new emri_server();
    S->dev.use_graphs = cfg->use_graphs != 0;
    if (hipGetDevice(&S->dev.device) != hipSuccess) { delete S; return set_error(EMRI_EDEVICE, "no device"); }
    auto cleanup = [&]() {
        for (auto x : S->dev.streams) (void)hipStreamDestroy(x);
        for (auto x : S->dev.events) (void)hipEventDestroy(x);
        delete S;
    };
    for (int i = 0; i < cfg->n_streams; ++i) {
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            cleanup();
            return set_error(EMRI_EDEVICE, "stream creation failed");
        }
        S->dev.streams.push_back(s);
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            cleanup();
            return set_error(EMRI_EDEVICE, "event creation failed");
        }
        S->dev.events.push_back(e);
        // the orbit pipeline's auxiliary stream and events of this stream,
        // made now so that captures on it never create any
        const emri_status st = prepare_pipe(s);
        if (st != EMRI_OK) {
            cleanup();
            return st;
        }
    }
    S->core.reset(new serve::Scheduler<HipDevice>(S->dev, cfg->arena, cfg->arena_bytes,
                                                  cfg->n_streams, cfg->max_batch));
    S->core->start();
    *out = S;
    return EMRI_OK;
}

emri_status emri_server_destroy(emri_server* S)
{
    if (!S) return set_error(EMRI_EINVAL, "null server");
    S->core->stop();
    S->core.reset();
    for (auto x : S->dev.streams) (void)hipStreamDestroy(x);
    for (auto x : S->dev.events) (void)hipEventDestroy(x);
    delete S;
    return EMRI_OK;
}

emri_status emri_server_add_dataset(emri_server* S, const emri_cfg* cfg, const double* data,
                                    const double* psd, int32_t* id)
{
    if (!S || !cfg || !data || !psd || !id) return set_error(EMRI_EINVAL, "null pointer argument");
    const size_t n = emri_dataset_bytes(cfg);
    if (!n) return set_error(EMRI_EINVAL, "invalid configuration");
    void* p = S->core->reserve_dataset(n);
    if (!p) return set_error(EMRI_EWORKSPACE, "arena too small for the data set");
    // the copy runs on a stream of its own creation's lifetime: the slots'
    // streams belong to the scheduler thread
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        S->core->unreserve_dataset(p, n);
        return set_error(EMRI_EDEVICE, "stream creation failed");
    }
    const emri_status st = emri_dataset_init(data, psd, cfg, p, n, s);
    const hipError_t se = hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    if (st != EMRI_OK || se != hipSuccess) {
        S->core->unreserve_dataset(p, n);
        return st != EMRI_OK ? st : set_error(EMRI_EDEVICE, "data set copy failed");
    }
    *id = S->core->commit_dataset(HipDevice::DsInfo{*cfg}, p, n);
    return EMRI_OK;
}

emri_status emri_server_submit(emri_server* S, int32_t dataset_id, const double* params, int64_t W,
                               double* lnL, uint64_t* ticket)
{
    if (!S || !params || !lnL || !ticket) return set_error(EMRI_EINVAL, "null pointer argument");
    const char* err = nullptr;
    const int st = S->core->submit(dataset_id, params, W, lnL, ticket, &err);
    return st == EMRI_OK ? EMRI_OK : set_error((emri_status)st, err);
}

emri_status emri_server_wait(emri_server* S, uint64_t ticket, double timeout_s, double* latency_s)
{
    if (!S) return set_error(EMRI_EINVAL, "null server");
    const char* err = nullptr;
    const int st = S->core->wait(ticket, timeout_s, latency_s, &err);
    return st == EMRI_OK ? EMRI_OK : set_error((emri_status)st, err);
}

emri_status emri_server_stats_get(emri_server* S, emri_server_stats* out)
{
    if (!S || !out) return set_error(EMRI_EINVAL, "null pointer argument");
    serve::Stats st;
    size_t in_use = 0, peak = 0;
    S->core->stats(&st, &in_use, &peak);
    out->submitted = st.submitted;
    out->completed = st.completed;
    out->rejected = st.rejected;
    out->batches = st.batches;
    out->graph_launches = st.graph_launches;
    out->graph_captures = st.graph_captures;
    out->walkers = st.walkers;
    out->padded_walkers = st.padded_walkers;
    out->arena_in_use = in_use;
    out->arena_peak = peak;
    return EMRI_OK;
}

}  // extern "C"
