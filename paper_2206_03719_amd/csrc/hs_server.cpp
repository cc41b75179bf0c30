// hs_server.cpp -- continuous-batching request loop.
//
// The server owns a caller-provided device pool (the HBM budget).  Requests
// queue in arrival order; an idle slot admits, among the queued requests
// whose workspace fits the free pool, the one with the least estimated work,
// so small requests do not wait behind large ones -- but a request is passed
// at most 2 x slots times, after which the slots wait for it.
// Requests that arrive while others run start as slots and memory free up.
// Every slot is a host worker thread with its own HIP stream (default
// priority).  The path and Gram kernels of admitted requests run side by side
// on the device; a backward sweep whose workgroups wait on each other (the
// cluster sweep) runs while no other such sweep does, so that all its
// workgroups can be resident.  Each request's device interval (HIP events on
// its stream against one reference event) is kept, and the statistics report
// how many requests were on the device at once.  A request's plan depends
// only on the request, and every kernel reduction has a fixed order, so its
// results are bit-identical alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/hs_api.h"
#include "hs_plan.hpp"
#include "hs_run.hpp"

namespace hs {

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, size) in 256-byte units; host bookkeeping only.
class PoolAlloc {
public:
    explicit PoolAlloc(size_t size) : size_(size & ~size_t(255)) { free_[0] = size_; }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                if (used_ > peak_) peak_ = used_;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) & ~size_t(255);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest_free() const
    {
        size_t m = 0;
        for (const auto& f : free_) m = std::max(m, f.second);
        return m;
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t size() const { return size_; }

private:
    size_t size_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

enum class St { Queued, Running, Done, Cancelled };

struct Item {
    uint64_t ticket = 0;
    Request q;
    size_t ws = 0;
    size_t ws_min = 0;  // the least workspace it runs in (more passes)
    St state = St::Queued;
    hs_status status = HS_OK;
    std::string error;
    RunResult res;
    Clock::time_point t_submit, t_done;
    int passed = 0;  // admissions of later requests while this one was queued
    double work = 0.0;  // estimated device work: path-steps x (scenarios + path tasks)
};

// Times (seconds) a request's work was on the device, from the reference event.
struct Interval {
    double start, end;
};

}  // namespace
}  // namespace hs

struct hs_server {
    int device = 0;
    unsigned char* pool = nullptr;
    hs::PoolAlloc alloc{0};
    std::mutex mu;
    std::condition_variable cv;
    std::deque<hs::Item*> queue;
    std::map<uint64_t, std::unique_ptr<hs::Item>> items;
    std::vector<std::thread> workers;
    uint64_t next_ticket = 1;
    bool stop = false;
    int64_t submitted = 0, completed = 0, cancelled = 0, failed = 0, running = 0;
    double path_steps = 0.0;
    int max_slots = 1;
    hipEvent_t ref = nullptr;  // device-time origin of the request intervals
    std::vector<hs::Interval> intervals;
    static constexpr size_t kQueueCap = 4096;
};

namespace hs {
namespace {

// Admission (caller holds s->mu): the queued request with the least
// estimated work whose workspace the free pool holds, reserving it at *off;
// every older request it passes counts one more pass.  A request passed
// 2 x slots times goes next: the oldest such request is admitted as soon as
// the pool holds it, and nothing passes it meanwhile (bounded waiting).
std::deque<Item*>::iterator admit(hs_server* s, size_t* off)
{
    auto& q = s->queue;
    const int limit = 2 * s->max_slots;
    for (auto it = q.begin(); it != q.end(); ++it)
        if ((*it)->passed >= limit) {
            // it may shrink to the largest free block (at least its minimum):
            // it runs in more passes, with the same results, instead of
            // holding every slot until its full workspace frees up
            const size_t fb = s->alloc.largest_free() & ~size_t(255);
            if (fb < (*it)->ws && fb >= (*it)->ws_min) (*it)->ws = fb;
            return s->alloc.alloc((*it)->ws, off) ? it : q.end();
        }
    std::vector<std::deque<Item*>::iterator> order;
    order.reserve(q.size());
    for (auto it = q.begin(); it != q.end(); ++it) order.push_back(it);
    std::stable_sort(order.begin(), order.end(),
                     [](const auto& a, const auto& b) { return (*a)->work < (*b)->work; });
    for (auto it : order)
        if (s->alloc.alloc((*it)->ws, off)) {
            for (auto o = q.begin(); o != it; ++o) ++(*o)->passed;
            return it;
        }
    return q.end();
}

void worker_main(hs_server* s)
{
    (void)hipSetDevice(s->device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
        (void)hipStreamDestroy(st);
        st = nullptr;
    }
    for (;;) {
        Item* it = nullptr;
        size_t off = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            std::deque<Item*>::iterator pick;
            s->cv.wait(lk, [&] {
                if (s->stop) return true;
                pick = admit(s, &off);
                return pick != s->queue.end();
            });
            if (s->stop) break;
            it = *pick;
            s->queue.erase(pick);
            it->state = St::Running;
            ++s->running;
        }
        RunResult res;
        hs_status rc = HS_EDEVICE;
        std::string err;
        Interval iv{0.0, 0.0};
        if (st) {
            (void)hipEventRecord(e0, st);
            rc = run_greek_set(it->q, s->pool + off, it->ws, st, res, nullptr, true);
            if (rc != HS_OK) err = hs_last_error();
            float a = 0.f, b = 0.f;
            if (hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                hipEventElapsedTime(&a, s->ref, e0) == hipSuccess &&
                hipEventElapsedTime(&b, s->ref, e1) == hipSuccess)
                iv = Interval{a * 1e-3, b * 1e-3};
        } else {
            err = "could not create a HIP stream for this slot";
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->alloc.release(off, it->ws);
            --s->running;
            it->res = std::move(res);
            it->status = rc;
            it->error = err;
            it->state = St::Done;
            it->t_done = Clock::now();
            if (rc == HS_OK) {
                ++s->completed;
                s->path_steps += static_cast<double>(it->res.price.size()) *
                                 static_cast<double>(it->q.P) * it->q.n;
                if (iv.end > iv.start) s->intervals.push_back(iv);
            } else {
                ++s->failed;
            }
        }
        s->cv.notify_all();
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
}

// The most requests on the device at once, and the seconds during which at
// least two were, over the completed requests' device intervals.
void overlap_of(const std::vector<Interval>& iv, int* most, double* overlap_s)
{
    std::vector<std::pair<double, int>> ev;
    ev.reserve(iv.size() * 2);
    for (const Interval& i : iv) {
        ev.emplace_back(i.start, +1);
        ev.emplace_back(i.end, -1);
    }
    std::sort(ev.begin(), ev.end());  // an end before a start at equal times
    int cur = 0, hi = 0;
    double t_prev = 0.0, both = 0.0;
    for (const auto& e : ev) {
        if (cur >= 2) both += e.first - t_prev;
        cur += e.second;
        hi = std::max(hi, cur);
        t_prev = e.first;
    }
    *most = hi;
    *overlap_s = both;
}

}  // namespace
}  // namespace hs

using namespace hs;

extern "C" {

hs_status hs_server_create(int device, void* d_pool, size_t pool_bytes, int32_t max_slots,
                           hs_server** out)
{
    if (!out || !d_pool || pool_bytes < 4096 || max_slots < 1 || max_slots > 64 ||
        reinterpret_cast<uintptr_t>(d_pool) % 256 != 0) {
        set_error("hs_server_create: need a 256-byte aligned pool of >= 4 KiB and 1..64 slots");
        return HS_EINVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        set_error("hs_server_create: device %d not available", device);
        return HS_EDEVICE;
    }
    auto* s = new hs_server();
    s->device = device;
    s->pool = static_cast<unsigned char*>(d_pool);
    s->alloc = PoolAlloc(pool_bytes);
    s->max_slots = max_slots;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess ||
        hipEventCreate(&s->ref) != hipSuccess || hipEventRecord(s->ref, nullptr) != hipSuccess ||
        hipEventSynchronize(s->ref) != hipSuccess) {
        set_error("hs_server_create: could not record the reference event");
        if (s->ref) (void)hipEventDestroy(s->ref);
        (void)hipSetDevice(prev);
        delete s;
        return HS_EDEVICE;
    }
    (void)hipSetDevice(prev);
    for (int i = 0; i < max_slots; ++i) s->workers.emplace_back(worker_main, s);
    *out = s;
    return HS_OK;
}

hs_status hs_submit(hs_server* s, const hs_request* r, uint64_t* ticket)
{
    if (!s || !r || !ticket) {
        set_error("hs_submit: null argument");
        return HS_EINVAL;
    }
    auto it = std::make_unique<Item>();
    hs_status rc = copy_request(&r->model, r->corr, &r->option, r->n_paths, r->n_steps, &r->bumps,
                                &r->opts, it->q);
    if (rc != HS_OK) return rc;
    rc = validate(it->q);
    if (rc != HS_OK) return rc;
    {
        std::vector<Scenario> sc;  // catches non-SPD bumped correlations now
        rc = expand_scenarios(it->q, sc);
        if (rc != HS_OK) return rc;
        // work estimate for admission order: every scenario's sweep and
        // Gram reads, and the base path and every path task
        double units = static_cast<double>(sc.size() + it->q.N);
        for (const Scenario& x : sc) units += x.hi - x.lo;
        it->work = units * static_cast<double>(it->q.P) * static_cast<double>(it->q.n);
    }
    const size_t full = workspace_bound(it->q, false);
    const size_t mn = workspace_bound(it->q, true);
    const size_t cap = s->alloc.size();
    if (mn > cap) {
        set_error("hs_submit: request needs at least %zu bytes, the pool has %zu", mn, cap);
        return HS_ENOMEM;
    }
    // a request larger than the pool runs in passes in half of it (or its
    // minimum), so that it leaves room for others; results do not depend on
    // the workspace size
    it->ws = full <= cap ? full : std::max(mn, cap / 2);
    it->ws_min = mn;
    it->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->queue.size() >= hs_server::kQueueCap) {
            set_error("hs_submit: queue full");
            return HS_EBUSY;
        }
        it->ticket = s->next_ticket++;
        *ticket = it->ticket;
        s->queue.push_back(it.get());
        s->items[it->ticket] = std::move(it);
        ++s->submitted;
    }
    s->cv.notify_all();
    return HS_OK;
}

hs_status hs_poll(hs_server* s, uint64_t ticket, hs_greeks* out, int32_t* done, double* latency_s)
{
    if (!s || !done) {
        set_error("hs_poll: null argument");
        return HS_EINVAL;
    }
    std::unique_ptr<Item> fin;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto f = s->items.find(ticket);
        if (f == s->items.end()) {
            set_error("hs_poll: unknown or retired ticket %llu",
                      static_cast<unsigned long long>(ticket));
            return HS_ENOTFOUND;
        }
        Item* it = f->second.get();
        if (it->state == St::Queued || it->state == St::Running) {
            *done = 0;
            return HS_OK;
        }
        fin = std::move(f->second);
        s->items.erase(f);
    }
    *done = 1;
    if (latency_s)
        *latency_s = std::chrono::duration<double>(fin->t_done - fin->t_submit).count();
    if (fin->state == St::Cancelled) {
        set_error("hs_poll: request %llu was cancelled", static_cast<unsigned long long>(ticket));
        return HS_ECANCELLED;
    }
    if (fin->status != HS_OK) {
        set_error("%s", fin->error.c_str());
        return fin->status;
    }
    if (out) fill_greeks(fin->q, fin->res, out);
    return HS_OK;
}

hs_status hs_cancel(hs_server* s, uint64_t ticket)
{
    if (!s) {
        set_error("hs_cancel: null server");
        return HS_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    auto f = s->items.find(ticket);
    if (f == s->items.end()) {
        set_error("hs_cancel: unknown ticket");
        return HS_ENOTFOUND;
    }
    Item* it = f->second.get();
    if (it->state != St::Queued) {
        set_error("hs_cancel: request already %s", it->state == St::Running ? "running" : "finished");
        return HS_EBUSY;
    }
    for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
        if (*q == it) {
            s->queue.erase(q);
            break;
        }
    it->state = St::Cancelled;
    it->t_done = Clock::now();
    ++s->cancelled;
    s->cv.notify_all();
    return HS_OK;
}

hs_status hs_server_get_stats(hs_server* s, hs_server_stats* out)
{
    if (!s || !out) {
        set_error("hs_server_get_stats: null argument");
        return HS_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->cancelled = s->cancelled;
    out->failed = s->failed;
    out->running = s->running;
    out->queued = static_cast<int64_t>(s->queue.size());
    out->pool_bytes = s->alloc.size();
    out->pool_in_use = s->alloc.used();
    out->pool_peak = s->alloc.peak();
    out->path_steps_done = s->path_steps;
    int most = 0;
    double both = 0.0;
    overlap_of(s->intervals, &most, &both);
    out->device_max_concurrent = most;
    out->device_overlap_s = both;
    out->slots = s->max_slots;
    return HS_OK;
}

void hs_server_destroy(hs_server* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (Item* it : s->queue) {
            it->state = St::Cancelled;
            ++s->cancelled;
        }
        s->queue.clear();
    }
    s->cv.notify_all();
    for (auto& t : s->workers) t.join();
    if (s->ref) (void)hipEventDestroy(s->ref);
    delete s;
}

}  // extern "C"
