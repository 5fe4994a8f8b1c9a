// server_core.hpp -- host-only core of the serving loop (emri_server_*):
// the arena allocator, the request queue, continuous batching, admission by
// HBM footprint and the scheduler thread.
//
// Nothing here calls HIP.  The device side is a policy class `Dev` (the HIP
// streams, events, graphs and pinned staging of server.hip; a simulated
// device in the host tests, which build this file with the address,
// undefined-behaviour and thread sanitizers).  `Dev` provides:
//
//   struct DsInfo;                         per data set (its configuration)
//   struct Extra;                          per block device state
//   size_t block_bytes(const DsInfo&, int64_t bucket, size_t* ws_bytes);
//                                          arena bytes of a block (0: invalid)
//   bool block_init(Block&);               host staging for h_params/h_lnL
//   void block_release(Block&);            frees what block_init and launch made
//   int  launch(Block&, const DsInfo&, const void* ds, int slot, Stats&);
//        parameters in, likelihood, results out, then the slot's completion
//        marker; returns kOk or a negative status
//   int  query(int slot);                  0 done, 1 running, < 0 failed
//   void drain(int slot);                  waits until the slot's work ended
//   void thread_start();                   called first on the scheduler thread
//
// Batches are rounded up to a multiple of 32 walkers; padding rows repeat
// the batch's first walker and their results are dropped.  Every reduction
// of the likelihood is per walker and in a fixed order, so a request gives
// the same lnL alone and in any mix.
#pragma once

#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

namespace emri {
namespace serve {

// status values (the same numbers as emri_status)
enum { kOk = 0, kEinval = -1, kEworkspace = -2, kEdevice = -3 };
constexpr int kNpar = 17;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline int64_t bucket_of(int64_t W) { return (W + 31) / 32 * 32; }

// First-fit allocator over the caller's arena with coalescing of free
// ranges.  Data sets are pinned for the server's lifetime and placed at the
// top of the highest free range that holds them; blocks come first-fit from
// the bottom.  largest_gap() is the largest range between pinned data sets,
// which is free whenever no block exists: a block of at most that size can
// always be placed once the blocks in use have been released.
struct Arena {
    char* base = nullptr;
    size_t bytes = 0, in_use = 0, peak = 0;
    std::map<size_t, size_t> free_;     // offset -> size
    std::map<size_t, size_t> pinned_;   // offset -> size (data sets)

    void init(void* b, size_t n)
    {
        base = (char*)b;
        bytes = n & ~(size_t)255;
        free_.clear();
        pinned_.clear();
        in_use = peak = 0;
        if (bytes) free_[0] = bytes;
    }
    void take(std::map<size_t, size_t>::iterator it, size_t off, size_t n)
    {
        const size_t fo = it->first, fs = it->second;
        free_.erase(it);
        if (off > fo) free_[fo] = off - fo;
        if (off + n < fo + fs) free_[off + n] = fo + fs - (off + n);
        in_use += n;
        if (in_use > peak) peak = in_use;
    }
    void* alloc(size_t n)
    {
        n = align256(n);
        if (n == 0) return nullptr;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first;
            take(it, off, n);
            return base + off;
        }
        return nullptr;
    }
    void* alloc_pinned(size_t n)
    {
        n = align256(n);
        if (n == 0) return nullptr;
        for (auto it = free_.rbegin(); it != free_.rend(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first + it->second - n;
            take(std::prev(it.base()), off, n);
            pinned_[off] = n;
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
    size_t largest_gap() const
    {
        size_t best = 0, at = 0;
        for (const auto& kv : pinned_) {
            if (kv.first - at > best) best = kv.first - at;
            at = kv.first + kv.second;
        }
        if (bytes - at > best) best = bytes - at;
        return best;
    }
};

struct Stats {
    int64_t submitted = 0, completed = 0, rejected = 0;
    int64_t batches = 0, graph_launches = 0, graph_captures = 0;
    int64_t walkers = 0, padded_walkers = 0;
};

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    int32_t ds = 0;
    int64_t W = 0;
    std::vector<double> params;   // host copy [W][17]
    double* lnL = nullptr;        // caller's host output
    Clock::time_point t_submit, t_done;
    bool done = false;
    int status = kOk;
};

template <class Dev>
class Scheduler {
public:
    struct Block {                // device block of one (data set, batch size)
        int32_t ds = 0;
        int64_t bucket = 0;
        void* dev = nullptr;      // arena range: params, results, workspace
        size_t bytes = 0;
        double* d_params = nullptr;
        double* d_lnL = nullptr;
        void* ws = nullptr;
        size_t ws_bytes = 0;
        double* h_params = nullptr;   // host staging (Dev::block_init)
        double* h_lnL = nullptr;
        int uses = 0;
        typename Dev::Extra x{};
    };
    struct Dataset {
        typename Dev::DsInfo info;
        void* ptr;
        size_t bytes;
    };

    Scheduler(Dev& dev, void* arena, size_t arena_bytes, int n_slots, int64_t max_batch)
        : dev_(dev), busy_((size_t)n_slots, false), max_batch_(max_batch)
    {
        arena_.init(arena, arena_bytes);
    }
    ~Scheduler() { stop(); }

    void start() { th_ = std::thread([this] { loop(); }); }

    // finishes in-flight batches, fails pending requests, releases blocks
    void stop()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (stopped_) return;
            stop_ = true;
            for (auto& r : pending_) {
                r->status = kEdevice;
                r->done = true;
                r->t_done = Clock::now();
            }
            pending_.clear();
            cv_sched_.notify_all();
            cv_done_.notify_all();
        }
        if (th_.joinable()) th_.join();
        std::lock_guard<std::mutex> lk(mu_);
        for (auto& kv : idle_) release_block(*kv.second);
        idle_.clear();
        stopped_ = true;
    }

    // arena range for a data set of n bytes (nullptr: does not fit); the
    // caller fills it and then calls commit_dataset, or gives it back
    void* reserve_dataset(size_t n)
    {
        std::lock_guard<std::mutex> lk(mu_);
        return arena_.alloc_pinned(n);
    }
    void unreserve_dataset(void* p, size_t n)
    {
        std::lock_guard<std::mutex> lk(mu_);
        arena_.pinned_.erase((size_t)((char*)p - arena_.base));
        arena_.release(p, n);
    }
    int32_t commit_dataset(const typename Dev::DsInfo& info, void* p, size_t n)
    {
        std::lock_guard<std::mutex> lk(mu_);
        datasets_.push_back(Dataset{info, p, n});
        return (int32_t)datasets_.size() - 1;
    }

    int submit(int32_t ds, const double* params, int64_t W, double* lnL, uint64_t* ticket,
               const char** err)
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (ds < 0 || ds >= (int32_t)datasets_.size()) return fail(err, kEinval, "unknown data set");
        if (W < 1 || W > max_batch_) return fail(err, kEinval, "W must be in [1, max_batch]");
        if (stop_) return fail(err, kEinval, "server is stopping");
        const size_t need = dev_.block_bytes(datasets_[ds].info, bucket_of(W), nullptr);
        if (need == 0 || align256(need) > arena_.largest_gap()) {
            st_.rejected++;
            return fail(err, kEworkspace, "request exceeds the server's HBM budget");
        }
        auto r = std::make_shared<Request>();
        r->ticket = next_ticket_++;
        r->ds = ds;
        r->W = W;
        r->params.assign(params, params + W * kNpar);
        r->lnL = lnL;
        r->t_submit = Clock::now();
        pending_.push_back(r);
        live_[r->ticket] = r;
        st_.submitted++;
        *ticket = r->ticket;
        cv_sched_.notify_one();
        return kOk;
    }

    // timeout_s < 0: forever
    int wait(uint64_t ticket, double timeout_s, double* latency_s, const char** err)
    {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = live_.find(ticket);
        if (it == live_.end()) return fail(err, kEinval, "unknown ticket");
        auto r = it->second;
        if (timeout_s < 0) {
            cv_done_.wait(lk, [&] { return r->done; });
        } else {
            // the deadline is on the steady clock; the waits themselves are
            // short slices on the system clock (a clock step moves one slice)
            const double t = timeout_s < 1e9 ? timeout_s : 1e9;
            const auto deadline =
                Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                   std::chrono::duration<double>(t));
            while (!r->done) {
                if (Clock::now() >= deadline)
                    return fail(err, kEdevice, "timeout: request still queued or running");
                cv_done_.wait_until(lk, std::chrono::system_clock::now() +
                                            std::chrono::milliseconds(20));
            }
        }
        live_.erase(ticket);
        if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
        if (r->status != kOk)
            return fail(err, r->status, "request failed (device error or server stopped)");
        return kOk;
    }

    void stats(Stats* s, size_t* in_use, size_t* peak)
    {
        std::lock_guard<std::mutex> lk(mu_);
        *s = st_;
        *in_use = arena_.in_use;
        *peak = arena_.peak;
    }

private:
    static int fail(const char** err, int st, const char* msg)
    {
        if (err) *err = msg;
        return st;
    }

    void release_block(Block& b)
    {
        dev_.block_release(b);
        if (b.dev) arena_.release(b.dev, b.bytes);
        b = Block{};
    }

    // a block for (ds, bucket): cached, or new from the arena (evicting idle
    // blocks if needed).  nullptr with *hard false: it does not fit until
    // running batches end; with *hard true: host staging failed
    std::shared_ptr<Block> get_block(int32_t ds, int64_t bucket, bool* hard)
    {
        *hard = false;
        auto key = std::make_pair(ds, bucket);
        auto it = idle_.find(key);
        if (it != idle_.end()) {
            auto b = it->second;
            idle_.erase(it);
            return b;
        }
        size_t wsb = 0;
        const size_t need = dev_.block_bytes(datasets_[ds].info, bucket, &wsb);
        void* p = arena_.alloc(need);
        while (!p && !idle_.empty()) {
            auto victim = idle_.begin();
            release_block(*victim->second);
            idle_.erase(victim);
            p = arena_.alloc(need);
        }
        if (!p) return nullptr;
        auto b = std::make_shared<Block>();
        b->ds = ds;
        b->bucket = bucket;
        b->dev = p;
        b->bytes = need;
        char* c = (char*)p;
        b->d_params = (double*)c;
        c += align256((size_t)bucket * kNpar * 8);
        b->d_lnL = (double*)c;
        c += align256((size_t)bucket * 8);
        b->ws = c;
        b->ws_bytes = wsb;
        if (!dev_.block_init(*b)) {
            release_block(*b);
            *hard = true;
            return nullptr;
        }
        return b;
    }

    struct Batch {
        std::shared_ptr<Block> blk;
        std::vector<std::shared_ptr<Request>> reqs;
        int slot = -1;
    };

    int launch_batch(Batch& bt)
    {
        Block& b = *bt.blk;
        int64_t off = 0;
        for (auto& r : bt.reqs) {
            memcpy(b.h_params + off * kNpar, r->params.data(), (size_t)r->W * kNpar * 8);
            off += r->W;
        }
        for (int64_t i = off; i < b.bucket; ++i)
            memcpy(b.h_params + i * kNpar, b.h_params, kNpar * 8);
        st_.walkers += off;
        st_.padded_walkers += b.bucket - off;
        const int st = dev_.launch(b, datasets_[b.ds].info, datasets_[b.ds].ptr, bt.slot, st_);
        if (st == kOk) {
            b.uses++;
            st_.batches++;
        }
        return st;
    }

    void finish(std::vector<std::shared_ptr<Request>>& reqs, const double* h_lnL, int status)
    {
        const auto now = Clock::now();
        int64_t off = 0;
        for (auto& r : reqs) {
            if (status == kOk) memcpy(r->lnL, h_lnL + off, (size_t)r->W * 8);
            off += r->W;
            r->status = status;
            r->t_done = now;
            r->done = true;
            st_.completed++;
        }
        cv_done_.notify_all();
    }

    void finish_batch(Batch& bt, bool ok)
    {
        if (!ok) dev_.drain(bt.slot);   // nothing of the batch may still run
        finish(bt.reqs, bt.blk->h_lnL, ok ? kOk : kEdevice);
        busy_[(size_t)bt.slot] = false;
        if (ok) idle_.emplace(std::make_pair(bt.blk->ds, bt.blk->bucket), bt.blk);
        else release_block(*bt.blk);
    }

    // admit as many batches as free slots and memory allow (lock held)
    void admit()
    {
        for (;;) {
            int slot = -1;
            for (size_t i = 0; i < busy_.size(); ++i)
                if (!busy_[i]) { slot = (int)i; break; }
            if (slot < 0 || pending_.empty()) return;
            bool progressed = false;
            std::set<int32_t> tried;
            const size_t capacity = arena_.largest_gap();
            for (size_t i = 0; i < pending_.size() && !progressed; ++i) {
                const int32_t d = pending_[i]->ds;
                if (!tried.insert(d).second) continue;
                // oldest requests of data set d, up to max_batch walkers and a
                // block no larger than any block could be (every single
                // request fits: submit checks it)
                std::vector<size_t> pick;
                int64_t total = 0;
                for (size_t j = i; j < pending_.size(); ++j) {
                    const auto& r = pending_[j];
                    if (r->ds != d || total + r->W > max_batch_) continue;
                    if (!pick.empty() &&
                        align256(dev_.block_bytes(datasets_[d].info, bucket_of(total + r->W),
                                                  nullptr)) > capacity)
                        continue;
                    pick.push_back(j);
                    total += r->W;
                }
                bool hard = false;
                auto blk = get_block(d, bucket_of(total), &hard);
                Batch bt;
                for (size_t k = 0; k < pick.size(); ++k) bt.reqs.push_back(pending_[pick[k]]);
                if (!blk && !hard) continue;   // does not fit now; try another data set
                for (size_t k = pick.size(); k-- > 0;) pending_.erase(pending_.begin() + (long)pick[k]);
                progressed = true;
                if (!blk) {                     // host staging failed: fail the requests
                    finish(bt.reqs, nullptr, kEdevice);
                    continue;
                }
                bt.blk = blk;
                bt.slot = slot;
                busy_[(size_t)slot] = true;
                if (launch_batch(bt) != kOk) finish_batch(bt, false);
                else inflight_.push_back(std::move(bt));
            }
            if (!progressed) return;
        }
    }

    void loop()
    {
        dev_.thread_start();
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            for (size_t i = 0; i < inflight_.size();) {
                const int q = dev_.query(inflight_[i].slot);
                if (q == 1) { ++i; continue; }
                finish_batch(inflight_[i], q == 0);
                inflight_.erase(inflight_.begin() + (long)i);
            }
            if (stop_ && inflight_.empty()) break;
            if (!stop_) admit();
            if (inflight_.empty()) {
                // With nothing running every block is idle and evictable, so
                // admit() has placed or failed every request it could see;
                // any left cannot run: fail them rather than spin.
                if (!pending_.empty()) {
                    std::vector<std::shared_ptr<Request>> left(pending_.begin(), pending_.end());
                    pending_.clear();
                    finish(left, nullptr, kEdevice);
                }
                cv_sched_.wait(lk, [&] { return stop_ || !pending_.empty(); });
            } else {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            }
        }
    }

    Dev& dev_;
    Arena arena_;
    std::vector<Dataset> datasets_;
    std::vector<bool> busy_;
    int64_t max_batch_;
    std::mutex mu_;
    std::condition_variable cv_sched_, cv_done_;
    std::deque<std::shared_ptr<Request>> pending_;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> live_;
    std::multimap<std::pair<int32_t, int64_t>, std::shared_ptr<Block>> idle_;
    std::vector<Batch> inflight_;
    uint64_t next_ticket_ = 1;
    bool stop_ = false, stopped_ = false;
    Stats st_;
    std::thread th_;
};

}  // namespace serve
}  // namespace emri
