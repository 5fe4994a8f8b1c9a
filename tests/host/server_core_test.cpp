// Host test of the serving core (paper_2311_17174_amd/csrc/server_core.hpp)
// on a simulated device, built with the address and undefined-behaviour
// sanitizers and, separately, the thread sanitizer (tests/test_host_sanitizers.py).
//
// The simulated device keeps "device memory" in host memory: the arena is a
// malloc'd buffer; a launch copies the parameters into the block's arena
// range and hands the batch to a worker thread, which computes a known
// function of every row after a short random delay, copies the results to
// the block's staging buffer and marks the slot done.  The checks:
//  - arena: random allocations, pinned allocations and releases against a
//    byte map (no overlap, exact accounting, full coalescing, largest gap);
//  - every served result equals the function of its own row (so batching,
//    padding and scattering are right), from several client threads;
//  - no two batches in flight share arena bytes;
//  - failed launches fail their requests (after the slot drained) and the
//    server goes on;
//  - admission: an arena that holds one block at a time serves everything;
//    a request larger than any range between data sets is rejected at
//    submit, also when a data set added after blocks existed split the
//    arena (the case that once left such a request queued forever);
//  - stopping with queued requests fails them and returns.
#include "server_core.hpp"

#include <assert.h>
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <random>

using emri::serve::Arena;
using emri::serve::Scheduler;
using emri::serve::Stats;
using emri::serve::align256;
using emri::serve::kEdevice;
using emri::serve::kEworkspace;
using emri::serve::kNpar;
using emri::serve::kOk;

#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            abort();                                                           \
        }                                                                      \
    } while (0)

static double row_value(const double* p, double ds_value)
{
    double v = ds_value;
    for (int j = 0; j < kNpar; ++j) v += p[j] * (double)(j + 1);
    return v;
}

struct SimDevice {
    struct DsInfo {
        size_t bytes_per_walker;
        double value;
    };
    struct Extra {
        int launches;
    };
    using Block = Scheduler<SimDevice>::Block;

    struct Slot {
        std::atomic<int> state{0};   // 0 idle, 1 queued, 2 done, 3 failed
        bool fail_at_end = false;
        Block* b = nullptr;
        double value = 0;
        int delay_us = 0;
    };

    explicit SimDevice(int n, uint64_t seed, double fail_rate)
        : slots(n), rng(seed), fail_rate(fail_rate)
    {
        worker = std::thread([this] { work(); });
    }
    ~SimDevice()
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            quit = true;
        }
        cv.notify_all();
        worker.join();
    }

    size_t block_bytes(const DsInfo& d, int64_t bucket, size_t* ws_bytes)
    {
        const size_t ws = (size_t)bucket * d.bytes_per_walker + 4096;
        if (ws_bytes) *ws_bytes = ws;
        return align256((size_t)bucket * kNpar * 8) + align256((size_t)bucket * 8) + ws;
    }
    bool block_init(Block& b)
    {
        std::lock_guard<std::mutex> lk(mu);
        if (fail_init_next) {
            fail_init_next = false;
            return false;
        }
        b.h_params = (double*)malloc((size_t)b.bucket * kNpar * 8);
        b.h_lnL = (double*)malloc((size_t)b.bucket * 8);
        return b.h_params && b.h_lnL;
    }
    void block_release(Block& b)
    {
        free(b.h_params);
        free(b.h_lnL);
        b.h_params = b.h_lnL = nullptr;
    }
    int launch(Block& b, const DsInfo& d, const void* ds, int slot, Stats& st)
    {
        CHECK(ds != nullptr);
        std::unique_lock<std::mutex> lk(mu);
        Slot& s = slots[(size_t)slot];
        CHECK(s.state.load() != 1);
        // no batch in flight may share arena bytes with this one
        const char* lo = (const char*)b.dev;
        const char* hi = lo + b.bytes;
        for (auto& o : slots)
            if (o.state.load() == 1 && o.b) {
                const char* ol = (const char*)o.b->dev;
                CHECK(hi <= ol || ol + o.b->bytes <= lo);
            }
        std::uniform_real_distribution<double> U(0.0, 1.0);
        const bool fail = U(rng) < fail_rate;
        // "H2D": the parameters into the block's arena range, and scribble
        // over its workspace as the kernels would
        memcpy(b.d_params, b.h_params, (size_t)b.bucket * kNpar * 8);
        memset(b.ws, 0xA5, b.ws_bytes);
        b.x.launches++;
        if (b.uses >= 1) st.graph_launches++;
        if (fail) {
            // a partly enqueued batch: work was queued before the failure
            s.b = &b;
            s.value = d.value;
            s.delay_us = 50;
            s.state.store(1);
            launches_failed++;
            lk.unlock();
            cv.notify_all();
            return kEdevice;
        }
        s.b = &b;
        s.value = d.value;
        s.delay_us = (int)(U(rng) * 200.0);
        s.fail_at_end = fail_next_completion;
        fail_next_completion = false;
        s.state.store(1);
        lk.unlock();
        cv.notify_all();
        return kOk;
    }
    int query(int slot)
    {
        const int s = slots[(size_t)slot].state.load();
        if (s == 1) return 1;
        return s == 3 ? -1 : 0;
    }
    void set_hold(bool h)
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            hold = h;
        }
        cv.notify_all();
    }
    void drain(int slot)
    {
        while (slots[(size_t)slot].state.load() == 1) std::this_thread::yield();
    }
    void thread_start() {}

    void work()
    {
        for (;;) {
            Slot* job = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] {
                    if (quit) return true;
                    if (hold) return false;
                    for (auto& s : slots)
                        if (s.state.load() == 1) return true;
                    return false;
                });
                if (quit) return;
                for (auto& s : slots)
                    if (s.state.load() == 1) { job = &s; break; }
            }
            std::this_thread::sleep_for(std::chrono::microseconds(job->delay_us));
            std::lock_guard<std::mutex> lk(mu);
            Block& b = *job->b;
            for (int64_t i = 0; i < b.bucket; ++i)
                b.d_lnL[i] = row_value(b.d_params + i * kNpar, job->value);
            memcpy(b.h_lnL, b.d_lnL, (size_t)b.bucket * 8);   // "D2H"
            job->b = nullptr;
            job->state.store(job->fail_at_end ? 3 : 2);
            job->fail_at_end = false;
        }
    }

    std::vector<Slot> slots;
    std::mt19937_64 rng;
    double fail_rate;
    bool fail_init_next = false;
    bool fail_next_completion = false;
    bool hold = false;
    int launches_failed = 0;
    std::mutex mu;
    std::condition_variable cv;
    bool quit = false;
    std::thread worker;
};

// ---------------------------------------------------------------- arena
static void test_arena(uint64_t seed)
{
    const size_t bytes = 1 << 20;
    std::vector<char> mem(bytes);
    Arena a;
    a.init(mem.data(), bytes);
    std::vector<int> owner(bytes / 256, -1);
    struct Live { void* p; size_t n; bool pinned; };
    std::vector<Live> live;
    std::mt19937_64 r(seed);
    for (int it = 0; it < 20000; ++it) {
        const int op = (int)(r() % 10);
        if (op < 5 || live.empty()) {
            const size_t n = 1 + r() % (bytes / 16);
            const bool pin = (r() % 8) == 0;
            void* p = pin ? a.alloc_pinned(n) : a.alloc(n);
            if (!p) continue;
            const size_t off = (size_t)((char*)p - mem.data());
            CHECK(off % 256 == 0 && off + align256(n) <= bytes);
            for (size_t k = off / 256; k < (off + align256(n)) / 256; ++k) {
                CHECK(owner[k] == -1);
                owner[k] = (int)live.size();
            }
            live.push_back(Live{p, n, pin});
        } else {
            const size_t i = r() % live.size();
            const Live L = live[i];
            const size_t off = (size_t)((char*)L.p - mem.data());
            if (L.pinned) a.pinned_.erase(off);
            a.release(L.p, L.n);
            for (size_t k = off / 256; k < (off + align256(L.n)) / 256; ++k) owner[k] = -1;
            live[i] = live.back();
            live.pop_back();
            for (size_t k = 0; k < owner.size(); ++k)
                if (owner[k] == (int)live.size()) owner[k] = (int)i;
        }
        // accounting and the largest range between pinned allocations
        size_t used = 0;
        for (auto& L : live) used += align256(L.n);
        CHECK(a.in_use == used);
        if (it % 97 == 0) {
            size_t best = 0, run = 0;
            for (size_t k = 0; k < owner.size(); ++k) {
                const bool pinned = owner[k] >= 0 && live[(size_t)owner[k]].pinned;
                run = pinned ? 0 : run + 256;
                if (run > best) best = run;
            }
            CHECK(a.largest_gap() == best);
            // free ranges are disjoint, sorted, not adjacent (coalesced) and free
            size_t end = 0;
            bool first = true;
            for (auto& kv : a.free_) {
                CHECK(first || kv.first > end);
                for (size_t k = kv.first / 256; k < (kv.first + kv.second) / 256; ++k)
                    CHECK(owner[k] == -1);
                end = kv.first + kv.second;
                first = false;
            }
        }
    }
    for (auto& L : live) {
        if (L.pinned) a.pinned_.erase((size_t)((char*)L.p - mem.data()));
        a.release(L.p, L.n);
    }
    CHECK(a.in_use == 0 && a.free_.size() == 1 && a.free_.begin()->second == bytes);
    CHECK(a.largest_gap() == bytes);
}

// ---------------------------------------------------------------- scheduler
struct Server {
    SimDevice dev;
    std::vector<char> arena;
    Scheduler<SimDevice> core;
    Server(size_t arena_bytes, int slots, int64_t max_batch, uint64_t seed, double fail_rate)
        : dev(slots, seed, fail_rate), arena(arena_bytes),
          core(dev, arena.data(), arena_bytes, slots, max_batch)
    {
        core.start();
    }
    int32_t add(size_t bytes, double value, size_t per_walker)
    {
        void* p = core.reserve_dataset(bytes);
        CHECK(p != nullptr);
        return core.commit_dataset(SimDevice::DsInfo{per_walker, value}, p, bytes);
    }
};

static std::vector<double> rows(int64_t W, uint64_t seed)
{
    std::mt19937_64 r(seed);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    std::vector<double> p((size_t)W * kNpar);
    for (auto& x : p) x = U(r);
    return p;
}

static void test_mixed_clients(uint64_t seed, double fail_rate)
{
    Server S(64 << 20, 3, 256, seed, fail_rate);
    const double vals[3] = {1.5, -2.0, 7.25};
    int32_t ids[3];
    for (int d = 0; d < 3; ++d) ids[d] = S.add(1 << 20, vals[d], 1024 * (d + 1));
    std::atomic<int> ok{0}, failed{0};
    std::vector<std::thread> clients;
    for (int c = 0; c < 6; ++c) {
        clients.emplace_back([&, c] {
            std::mt19937_64 r(seed * 31 + (uint64_t)c);
            for (int q = 0; q < 60; ++q) {
                const int d = (int)(r() % 3);
                const int64_t W = 1 + (int64_t)(r() % 256);
                const auto P = rows(W, r());
                std::vector<double> out((size_t)W, 0.0);
                uint64_t t = 0;
                CHECK(S.core.submit(ids[d], P.data(), W, out.data(), &t, nullptr) == kOk);
                double lat = -1;
                const int st = S.core.wait(t, 60.0, &lat, nullptr);
                if (st == kOk) {
                    for (int64_t i = 0; i < W; ++i)
                        CHECK(out[(size_t)i] == row_value(&P[(size_t)i * kNpar], vals[d]));
                    CHECK(lat >= 0);
                    ok++;
                } else {
                    CHECK(st == kEdevice);
                    failed++;
                }
            }
        });
    }
    for (auto& t : clients) t.join();
    Stats st;
    size_t in_use = 0, peak = 0;
    S.core.stats(&st, &in_use, &peak);
    CHECK(st.submitted == 360 && st.completed == 360);
    CHECK(ok + failed == 360);
    if (fail_rate == 0.0) CHECK(failed == 0);
    CHECK(st.batches < 360);   // requests were batched together
    CHECK(peak <= S.arena.size());
    S.core.stop();
    printf("mixed clients (fail rate %.2f): ok %d failed %d batches %lld peak %zu\n", fail_rate,
           ok.load(), failed.load(), (long long)st.batches, peak);
}

static void test_admission(uint64_t seed)
{
    // data set of 1 MiB; blocks of 32 walkers take ~36 KiB + 4 KiB
    SimDevice::DsInfo info{1024, 3.0};
    SimDevice probe(1, seed, 0.0);
    const size_t one = probe.block_bytes(info, 32, nullptr);
    const size_t arena = (1 << 20) + one + one / 2;
    Server S(arena, 4, 64, seed, 0.0);
    const int32_t d = S.add(1 << 20, 3.0, 1024);
    // a 64-walker block never fits: rejected at submit
    {
        const auto P = rows(64, 1);
        std::vector<double> out(64);
        uint64_t t = 0;
        const char* err = nullptr;
        CHECK(S.core.submit(d, P.data(), 64, out.data(), &t, &err) == kEworkspace);
    }
    // requests of <= 32 walkers: one block at a time, all served
    std::vector<std::vector<double>> Ps, outs(5);
    std::vector<uint64_t> ts(5);
    const int64_t Ws[5] = {4, 20, 31, 9, 16};
    for (int i = 0; i < 5; ++i) {
        Ps.push_back(rows(Ws[i], 100 + (uint64_t)i));
        outs[(size_t)i].resize((size_t)Ws[i]);
        CHECK(S.core.submit(d, Ps[(size_t)i].data(), Ws[i], outs[(size_t)i].data(), &ts[(size_t)i],
                            nullptr) == kOk);
    }
    for (int i = 0; i < 5; ++i) {
        CHECK(S.core.wait(ts[(size_t)i], 60.0, nullptr, nullptr) == kOk);
        for (int64_t k = 0; k < Ws[i]; ++k)
            CHECK(outs[(size_t)i][(size_t)k] == row_value(&Ps[(size_t)i][(size_t)k * kNpar], 3.0));
    }
    Stats st;
    size_t in_use = 0, peak = 0;
    S.core.stats(&st, &in_use, &peak);
    CHECK(st.rejected == 1 && st.completed == 5 && peak <= arena);
    S.core.stop();
}

// A data set added while blocks exist can land between them and split the
// arena.  A request whose block fits the total free bytes but no range
// between data sets must be rejected at submit (it once stayed queued
// forever); requests that fit a range still run, evicting idle blocks.
static void wait_batches(Scheduler<SimDevice>& core, int64_t n)
{
    for (int i = 0; i < 100000; ++i) {
        Stats st;
        size_t a = 0, b = 0;
        core.stats(&st, &a, &b);
        if (st.batches >= n) return;
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    CHECK(!"batches were not launched");
}

static void test_split_arena(uint64_t seed)
{
    const size_t pw = 4096, dsz = 65536, small = 63488;
    SimDevice::DsInfo info{pw, 0.5};
    SimDevice probe(1, seed, 0.0);
    const size_t b32 = probe.block_bytes(info, 32, nullptr);
    const size_t b64 = probe.block_bytes(info, 64, nullptr);
    // the top range left above two blocks is too small for the second data
    // set, the range of a released block is not
    CHECK(small < dsz && dsz <= b32);
    const size_t arena = 2 * b32 + small + dsz;
    Server S(arena, 2, 64, seed, 0.0);
    const int32_t d0 = S.add(dsz, 0.5, pw);
    // two batches in flight: block A at the bottom (its batch fails at the
    // end, which releases A) and block B above it
    S.dev.set_hold(true);
    {
        std::lock_guard<std::mutex> lk(S.dev.mu);
        S.dev.fail_next_completion = true;
    }
    const auto P1 = rows(32, 7), P2 = rows(32, 8);
    std::vector<double> o1(32), o2(32);
    uint64_t t1 = 0, t2 = 0;
    CHECK(S.core.submit(d0, P1.data(), 32, o1.data(), &t1, nullptr) == kOk);
    wait_batches(S.core, 1);
    CHECK(S.core.submit(d0, P2.data(), 32, o2.data(), &t2, nullptr) == kOk);
    wait_batches(S.core, 2);
    S.dev.set_hold(false);
    CHECK(S.core.wait(t1, 60.0, nullptr, nullptr) == kEdevice);
    CHECK(S.core.wait(t2, 60.0, nullptr, nullptr) == kOk);
    CHECK(o2[31] == row_value(&P2[31 * kNpar], 0.5));
    // the second data set goes into A's range, below B: the arena is split
    void* p1 = S.core.reserve_dataset(dsz);
    CHECK(p1 != nullptr);
    CHECK((size_t)((char*)p1 - S.arena.data()) == b32 - dsz);
    const int32_t d1 = S.core.commit_dataset(SimDevice::DsInfo{pw, 0.25}, p1, dsz);
    // a 64-walker block fits the free bytes once B is evicted, but no range
    // between the data sets
    Stats st;
    size_t in_use = 0, peak = 0;
    S.core.stats(&st, &in_use, &peak);
    CHECK(b64 <= arena - 2 * dsz && b64 > b32 + small && b64 > b32 - dsz);
    const auto P = rows(64, 9);
    std::vector<double> out(64);
    uint64_t t = 0;
    CHECK(S.core.submit(d0, P.data(), 64, out.data(), &t, nullptr) == kEworkspace);
    // 32-walker requests of both data sets run (the second evicts B)
    for (int k = 0; k < 4; ++k) {
        const auto Q = rows(32, 20 + (uint64_t)k);
        std::vector<double> o(32);
        uint64_t tk = 0;
        CHECK(S.core.submit(k % 2 ? d1 : d0, Q.data(), 32, o.data(), &tk, nullptr) == kOk);
        CHECK(S.core.wait(tk, 60.0, nullptr, nullptr) == kOk);
        CHECK(o[31] == row_value(&Q[31 * kNpar], k % 2 ? 0.25 : 0.5));
    }
    S.core.stop();
}

// host staging that cannot be allocated fails the batch's requests
static void test_staging_failure(uint64_t seed)
{
    Server S(16 << 20, 1, 64, seed, 0.0);
    const int32_t d = S.add(1 << 16, 1.0, 512);
    {
        std::lock_guard<std::mutex> lk(S.dev.mu);
        S.dev.fail_init_next = true;
    }
    const auto P = rows(10, 3);
    std::vector<double> out(10);
    uint64_t t = 0;
    CHECK(S.core.submit(d, P.data(), 10, out.data(), &t, nullptr) == kOk);
    CHECK(S.core.wait(t, 60.0, nullptr, nullptr) == kEdevice);
    CHECK(S.core.submit(d, P.data(), 10, out.data(), &t, nullptr) == kOk);
    CHECK(S.core.wait(t, 60.0, nullptr, nullptr) == kOk);
    CHECK(out[9] == row_value(&P[9 * kNpar], 1.0));
    S.core.stop();
}

// stop with requests still queued: they fail, waits return
static void test_stop_with_pending(uint64_t seed)
{
    auto S = std::make_unique<Server>(16 << 20, 1, 64, seed, 0.0);
    const int32_t d = S->add(1 << 16, 1.0, 512);
    std::vector<std::vector<double>> outs(40, std::vector<double>(64));
    std::vector<uint64_t> ts(40);
    const auto P = rows(64, 5);
    for (int i = 0; i < 40; ++i)
        CHECK(S->core.submit(d, P.data(), 64, outs[(size_t)i].data(), &ts[(size_t)i], nullptr) == kOk);
    S->core.stop();
    int ok = 0, bad = 0;
    for (int i = 0; i < 40; ++i) {
        const int st = S->core.wait(ts[(size_t)i], 10.0, nullptr, nullptr);
        if (st == kOk) ok++;
        else { CHECK(st == kEdevice); bad++; }
    }
    CHECK(ok + bad == 40);
    S.reset();
}

int main(int argc, char** argv)
{
    const uint64_t seed = argc > 1 ? strtoull(argv[1], nullptr, 10) : 1;
    test_arena(seed);
    printf("arena ok\n");
    test_mixed_clients(seed, 0.0);
    test_mixed_clients(seed + 1, 0.1);
    test_admission(seed);
    printf("admission ok\n");
    test_split_arena(seed);
    printf("split arena ok\n");
    test_staging_failure(seed);
    printf("staging failure ok\n");
    test_stop_with_pending(seed);
    printf("stop ok\n");
    printf("ALL OK\n");
    return 0;
}
