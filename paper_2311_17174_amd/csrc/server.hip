// server.hip -- persistent request loop over the likelihood (emri_server_*).
//
// Host-side runtime, no kernels of its own: a scheduler thread packs pending
// requests of the same resident data set into batches (continuous batching),
// admits a batch when a stream is free and its device block fits in the
// caller's arena (admission by HBM footprint), launches it as one replay of a
// hipGraph captured for that block (parameters H2D, the likelihood kernels,
// results D2H), and scatters results to the requests when the batch's event
// completes.  Blocks are cached per (data set, padded batch size) so graphs
// are reused; idle blocks are evicted when a new batch needs the memory.
//
// Batch sizes are rounded up to a multiple of 32 walkers; padding rows repeat
// the batch's first walker and their results are discarded.  Per-walker
// results do not depend on the batch (every reduction is per walker and in a
// fixed order), so a request gives the same lnL alone and in any mix.
#include "internal.hpp"

#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

namespace emri {

using Clock = std::chrono::steady_clock;

// first-fit allocator over the caller's arena, with coalescing
struct Arena {
    char* base = nullptr;
    size_t bytes = 0, in_use = 0, peak = 0;
    std::map<size_t, size_t> free_;   // offset -> size

    void init(void* b, size_t n)
    {
        base = (char*)b;
        bytes = n & ~(size_t)255;
        free_.clear();
        if (bytes) free_[0] = bytes;
    }
    void* alloc(size_t n)
    {
        n = align256(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, rem = it->second - n;
            free_.erase(it);
            if (rem) free_[off + n] = rem;
            in_use += n;
            if (in_use > peak) peak = in_use;
            return base + off;
        }
        return nullptr;
    }
    void release(void* p, size_t n)
    {
        n = align256(n);
        size_t off = (size_t)((char*)p - base);
        in_use -= n;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }
};

struct Dataset {
    emri_cfg cfg;
    void* ds;
    size_t bytes;
};

struct Request {
    uint64_t ticket;
    int32_t ds;
    int64_t W;
    std::vector<double> params;   // host copy [W][17]
    double* lnL;                  // caller's host output
    Clock::time_point t_submit, t_done;
    bool done = false;
    emri_status status = EMRI_OK;
};

struct Block {                    // device block of one (data set, batch size)
    int32_t ds = 0;
    int64_t bucket = 0;
    void* dev = nullptr;
    size_t bytes = 0;
    double* d_params = nullptr;
    double* d_lnL = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    double* h_params = nullptr;   // pinned staging
    double* h_lnL = nullptr;
    int uses = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct Batch {
    std::shared_ptr<Block> blk;
    std::vector<std::shared_ptr<Request>> reqs;
    int slot;
};

}  // namespace emri

struct emri_server {
    emri_server_cfg cfg{};
    int device = 0;
    emri::Arena arena;
    size_t dataset_bytes = 0;
    std::vector<emri::Dataset> datasets;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<bool> busy;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<std::shared_ptr<emri::Request>> pending;
    std::unordered_map<uint64_t, std::shared_ptr<emri::Request>> live;
    std::multimap<std::pair<int32_t, int64_t>, std::shared_ptr<emri::Block>> idle;
    std::vector<emri::Batch> inflight;
    uint64_t next_ticket = 1;
    bool stop = false;
    emri_server_stats st{};
    std::thread th;
};

namespace emri {

static int64_t bucket_of(int64_t W) { return (W + 31) / 32 * 32; }

static size_t block_bytes(const emri_cfg& cfg, int64_t bucket, size_t* ws_bytes)
{
    const size_t ws = emri_workspace_bytes(&cfg, bucket);
    if (ws_bytes) *ws_bytes = ws;
    if (!ws) return 0;
    return align256((size_t)bucket * EMRI_NPAR * 8) + align256((size_t)bucket * 8) + ws;
}

static void destroy_block(emri_server* S, Block& b)
{
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    if (b.h_params) (void)hipHostFree(b.h_params);
    if (b.h_lnL) (void)hipHostFree(b.h_lnL);
    if (b.dev) S->arena.release(b.dev, b.bytes);
    b = Block{};
}

// a block for (ds, bucket): cached, or new from the arena (evicting idle
// blocks of other shapes if needed); nullptr if it does not fit now
static std::shared_ptr<Block> get_block(emri_server* S, int32_t ds, int64_t bucket)
{
    auto key = std::make_pair(ds, bucket);
    auto it = S->idle.find(key);
    if (it != S->idle.end()) {
        auto b = it->second;
        S->idle.erase(it);
        return b;
    }
    size_t wsb = 0;
    const size_t need = block_bytes(S->datasets[ds].cfg, bucket, &wsb);
    void* p = S->arena.alloc(need);
    while (!p && !S->idle.empty()) {
        auto victim = S->idle.begin();
        destroy_block(S, *victim->second);
        S->idle.erase(victim);
        p = S->arena.alloc(need);
    }
    if (!p) return nullptr;
    auto b = std::make_shared<Block>();
    b->ds = ds;
    b->bucket = bucket;
    b->dev = p;
    b->bytes = need;
    char* c = (char*)p;
    b->d_params = (double*)c;
    c += align256((size_t)bucket * EMRI_NPAR * 8);
    b->d_lnL = (double*)c;
    c += align256((size_t)bucket * 8);
    b->ws = c;
    b->ws_bytes = wsb;
    if (hipHostMalloc((void**)&b->h_params, (size_t)bucket * EMRI_NPAR * 8, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void**)&b->h_lnL, (size_t)bucket * 8, hipHostMallocDefault) != hipSuccess) {
        destroy_block(S, *b);
        return nullptr;
    }
    return b;
}

// the batch's work on `s`: parameters in, likelihood, results out
static emri_status enqueue_batch(emri_server* S, Block& b, hipStream_t s)
{
    const Dataset& d = S->datasets[b.ds];
    if (hipMemcpyAsync(b.d_params, b.h_params, (size_t)b.bucket * EMRI_NPAR * 8,
                       hipMemcpyHostToDevice, s) != hipSuccess)
        return EMRI_EDEVICE;
    emri_status st = emri_loglike_dataset(b.d_params, b.bucket, d.ds, &d.cfg, b.d_lnL, b.ws,
                                          b.ws_bytes, s);
    if (st != EMRI_OK) return st;
    if (hipMemcpyAsync(b.h_lnL, b.d_lnL, (size_t)b.bucket * 8, hipMemcpyDeviceToHost, s) !=
        hipSuccess)
        return EMRI_EDEVICE;
    return EMRI_OK;
}

static emri_status launch_batch(emri_server* S, Batch& bt)
{
    Block& b = *bt.blk;
    hipStream_t s = S->streams[bt.slot];
    // pack the requests' walkers, pad with copies of the first walker
    int64_t off = 0;
    for (auto& r : bt.reqs) {
        memcpy(b.h_params + off * EMRI_NPAR, r->params.data(), (size_t)r->W * EMRI_NPAR * 8);
        off += r->W;
    }
    for (int64_t i = off; i < b.bucket; ++i)
        memcpy(b.h_params + i * EMRI_NPAR, b.h_params, EMRI_NPAR * 8);
    S->st.walkers += off;
    S->st.padded_walkers += b.bucket - off;
    emri_status st = EMRI_OK;
    // first use of a block runs eagerly (sets up kernels and attributes);
    // the graph is captured at the second use and replayed afterwards
    if (S->cfg.use_graphs && b.uses >= 1) {
        if (!b.exec) {
            trace_suppress(true);
            if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                trace_suppress(false);
                return EMRI_EDEVICE;
            }
            st = enqueue_batch(S, b, s);
            hipGraph_t g = nullptr;
            const hipError_t ec = hipStreamEndCapture(s, &g);
            trace_suppress(false);
            if (st != EMRI_OK || ec != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return st != EMRI_OK ? st : EMRI_EDEVICE;
            }
            if (hipGraphInstantiate(&b.exec, g, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGraphDestroy(g);
                return EMRI_EDEVICE;
            }
            b.graph = g;
            S->st.graph_captures++;
        }
        if (hipGraphLaunch(b.exec, s) != hipSuccess) return EMRI_EDEVICE;
        S->st.graph_launches++;
    } else {
        st = enqueue_batch(S, b, s);
        if (st != EMRI_OK) return st;
    }
    b.uses++;
    if (hipEventRecord(S->events[bt.slot], s) != hipSuccess) return EMRI_EDEVICE;
    S->st.batches++;
    return EMRI_OK;
}

static void finish_batch(emri_server* S, Batch& bt, bool ok)
{
    const auto now = Clock::now();
    int64_t off = 0;
    for (auto& r : bt.reqs) {
        if (ok) memcpy(r->lnL, bt.blk->h_lnL + off, (size_t)r->W * 8);
        off += r->W;
        r->status = ok ? EMRI_OK : EMRI_EDEVICE;
        r->t_done = now;
        r->done = true;
        S->st.completed++;
    }
    S->busy[bt.slot] = false;
    if (ok) S->idle.emplace(std::make_pair(bt.blk->ds, bt.blk->bucket), bt.blk);
    else destroy_block(S, *bt.blk);
    S->cv_done.notify_all();
}

// admit as many batches as free streams and memory allow (lock held)
static void admit(emri_server* S)
{
    for (;;) {
        int slot = -1;
        for (int i = 0; i < (int)S->busy.size(); ++i)
            if (!S->busy[i]) { slot = i; break; }
        if (slot < 0 || S->pending.empty()) return;
        bool launched = false;
        std::set<int32_t> tried;
        for (size_t i = 0; i < S->pending.size() && !launched; ++i) {
            const int32_t d = S->pending[i]->ds;
            if (!tried.insert(d).second) continue;
            // oldest requests of data set d, up to max_batch walkers and a
            // block that fits in the arena's batch capacity (every single
            // request does: submit checks it)
            const size_t capacity = S->arena.bytes - S->dataset_bytes;
            std::vector<size_t> pick;
            int64_t total = 0;
            for (size_t j = i; j < S->pending.size(); ++j) {
                const auto& r = S->pending[j];
                if (r->ds != d || total + r->W > S->cfg.max_batch) continue;
                if (!pick.empty() &&
                    block_bytes(S->datasets[d].cfg, bucket_of(total + r->W), nullptr) > capacity)
                    continue;
                pick.push_back(j);
                total += r->W;
            }
            auto blk = get_block(S, d, bucket_of(total));
            if (!blk) continue;   // does not fit now; try another data set
            Batch bt;
            bt.blk = blk;
            bt.slot = slot;
            for (size_t k = 0; k < pick.size(); ++k) bt.reqs.push_back(S->pending[pick[k]]);
            for (size_t k = pick.size(); k-- > 0;) S->pending.erase(S->pending.begin() + pick[k]);
            S->busy[slot] = true;
            const emri_status st = launch_batch(S, bt);
            if (st != EMRI_OK) {
                finish_batch(S, bt, false);
            } else {
                S->inflight.push_back(std::move(bt));
            }
            launched = true;
        }
        if (!launched) return;
    }
}

static void scheduler(emri_server* S)
{
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        for (size_t i = 0; i < S->inflight.size();) {
            const hipError_t q = hipEventQuery(S->events[S->inflight[i].slot]);
            if (q == hipErrorNotReady) { ++i; continue; }
            finish_batch(S, S->inflight[i], q == hipSuccess);
            S->inflight.erase(S->inflight.begin() + i);
        }
        if (S->stop && S->inflight.empty()) break;
        if (!S->stop) admit(S);
        if (S->inflight.empty()) {
            if (!S->pending.empty()) {   // nothing admissible (host allocation failed): back off
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::milliseconds(1));
                lk.lock();
                continue;
            }
            S->cv_sched.wait(lk, [&] { return S->stop || !S->pending.empty(); });
        } else {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        }
    }
}

}  // namespace emri

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
    S->cfg = *cfg;
    if (hipGetDevice(&S->device) != hipSuccess) { delete S; return set_error(EMRI_EDEVICE, "no device"); }
    S->arena.init(cfg->arena, cfg->arena_bytes);
    for (int i = 0; i < cfg->n_streams; ++i) {
        hipStream_t s;
        hipEvent_t e;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            for (auto x : S->streams) (void)hipStreamDestroy(x);
            for (auto x : S->events) (void)hipEventDestroy(x);
            delete S;
            return set_error(EMRI_EDEVICE, "stream or event creation failed");
        }
        S->streams.push_back(s);
        S->events.push_back(e);
        S->busy.push_back(false);
    }
    S->th = std::thread(scheduler, S);
    *out = S;
    return EMRI_OK;
}

emri_status emri_server_destroy(emri_server* S)
{
    if (!S) return set_error(EMRI_EINVAL, "null server");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (auto& r : S->pending) {
            r->status = EMRI_EDEVICE;
            r->done = true;
        }
        S->pending.clear();
        S->cv_sched.notify_all();
        S->cv_done.notify_all();
    }
    S->th.join();
    for (auto& kv : S->idle) destroy_block(S, *kv.second);
    S->idle.clear();
    for (auto x : S->streams) (void)hipStreamDestroy(x);
    for (auto x : S->events) (void)hipEventDestroy(x);
    delete S;
    return EMRI_OK;
}

emri_status emri_server_add_dataset(emri_server* S, const emri_cfg* cfg, const double* data,
                                    const double* psd, int32_t* id)
{
    if (!S || !cfg || !data || !psd || !id) return set_error(EMRI_EINVAL, "null pointer argument");
    const size_t n = emri_dataset_bytes(cfg);
    if (!n) return set_error(EMRI_EINVAL, "invalid configuration");
    std::lock_guard<std::mutex> lk(S->mu);
    void* p = S->arena.alloc(n);
    if (!p) return set_error(EMRI_EWORKSPACE, "arena too small for the data set");
    const emri_status st = emri_dataset_init(data, psd, cfg, p, n, S->streams[0]);
    if (st != EMRI_OK || hipStreamSynchronize(S->streams[0]) != hipSuccess) {
        S->arena.release(p, n);
        return st != EMRI_OK ? st : set_error(EMRI_EDEVICE, "data set copy failed");
    }
    S->datasets.push_back(Dataset{*cfg, p, n});
    S->dataset_bytes += align256(n);
    *id = (int32_t)S->datasets.size() - 1;
    return EMRI_OK;
}

emri_status emri_server_submit(emri_server* S, int32_t dataset_id, const double* params, int64_t W,
                               double* lnL, uint64_t* ticket)
{
    if (!S || !params || !lnL || !ticket) return set_error(EMRI_EINVAL, "null pointer argument");
    std::lock_guard<std::mutex> lk(S->mu);
    if (dataset_id < 0 || dataset_id >= (int32_t)S->datasets.size())
        return set_error(EMRI_EINVAL, "unknown data set");
    if (W < 1 || W > S->cfg.max_batch) return set_error(EMRI_EINVAL, "W must be in [1, max_batch]");
    if (S->stop) return set_error(EMRI_EINVAL, "server is stopping");
    const size_t need = block_bytes(S->datasets[dataset_id].cfg, bucket_of(W), nullptr);
    if (need == 0 || need > S->arena.bytes - S->dataset_bytes) {
        S->st.rejected++;
        return set_error(EMRI_EWORKSPACE, "request exceeds the server's HBM budget");
    }
    auto r = std::make_shared<Request>();
    r->ticket = S->next_ticket++;
    r->ds = dataset_id;
    r->W = W;
    r->params.assign(params, params + W * EMRI_NPAR);
    r->lnL = lnL;
    r->t_submit = Clock::now();
    S->pending.push_back(r);
    S->live[r->ticket] = r;
    S->st.submitted++;
    *ticket = r->ticket;
    S->cv_sched.notify_one();
    return EMRI_OK;
}

emri_status emri_server_wait(emri_server* S, uint64_t ticket, double timeout_s, double* latency_s)
{
    if (!S) return set_error(EMRI_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->live.find(ticket);
    if (it == S->live.end()) return set_error(EMRI_EINVAL, "unknown ticket");
    auto r = it->second;
    if (timeout_s < 0) {
        S->cv_done.wait(lk, [&] { return r->done; });
    } else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                    [&] { return r->done; })) {
        return set_error(EMRI_EDEVICE, "timeout: request still queued or running");
    }
    S->live.erase(ticket);
    if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    if (r->status != EMRI_OK) return set_error(r->status, "request failed (device error or server stopped)");
    return EMRI_OK;
}

emri_status emri_server_stats_get(emri_server* S, emri_server_stats* out)
{
    if (!S || !out) return set_error(EMRI_EINVAL, "null pointer argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->arena_in_use = S->arena.in_use;
    out->arena_peak = S->arena.peak;
    return EMRI_OK;
}

}  // extern "C"
