// Serving loop for KKT solves of several patterns (the C ABI in kkt.h, "Serving"): pattern
// registry, resident solver slots carved from one device pool (admission by HBM footprint),
// a FIFO queue that lets later requests overtake one that does not fit yet, and worker
// threads that each drive a batch of same-pattern requests on their own HIP stream: one
// refactorization launch for the batch (kkt_refactor_batch), replayed from a HIP graph
// captured once per set of slots, then the batch's FGMRES-IR solves.
#include "kkt.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// First-fit allocator over [0, size) in 256-byte units; neighbours merge on release.
class PoolAllocator {
public:
    explicit PoolAllocator(size_t size) { free_[0] = size; }
    bool take(size_t bytes, size_t *off) {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, start = it->first + bytes;
            free_.erase(it);
            if (rest) free_[start] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }

private:
    std::map<size_t, size_t> free_;  // offset -> bytes
    size_t used_ = 0;
};

struct Pattern {
    kkt_handle_t proto = nullptr;  // analysed, never bound; slots are clones
    size_t slot_bytes = 0;
};

struct Slot {
    int32_t pattern = -1;
    kkt_handle_t h = nullptr;
    size_t off = 0, bytes = 0;
    bool busy = false;
    uint64_t last_used = 0;
};

struct Request {
    int64_t ticket = 0;
    int32_t pattern = 0;
    const double *values = nullptr, *b = nullptr;
    double *x = nullptr;
    double tol = 0.0;
    Clock::time_point submitted, started, finished;
    bool done = false;
    kkt_status_t status = KKT_OK;
    kkt_solve_info_t info{};
    int32_t slot = -1, new_slot = 0;
};

}  // namespace

struct kkt_server_s {
    int device = 0;
    int max_batch = 4;
    bool use_graphs = true;
    int64_t batches = 0, batched_requests = 0, graph_launches = 0;
    char *pool = nullptr;
    size_t pool_bytes = 0;
    std::unique_ptr<PoolAllocator> alloc;
    std::vector<Pattern> patterns;
    std::vector<Slot> slots;  // entries with h == nullptr are unused
    std::deque<std::shared_ptr<Request>> queue;
    std::map<int64_t, std::shared_ptr<Request>> tickets;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable work_cv, done_cv;
    bool stopping = false;
    int64_t next_ticket = 1;
    uint64_t clock = 0;
    int64_t completed = 0, created = 0, evicted = 0;

    // Picks the first queued request that can start now, reserving (or carving) its slot.
    // Called with mu held.  Returns nullptr when none can.
    // With only >= 0, only requests of that pattern are considered (growing a batch).
    std::shared_ptr<Request> admit(int32_t *slot_index, bool *fresh, int32_t only = -1) {
        for (auto it = queue.begin(); it != queue.end(); ++it) {
            const int32_t p = (*it)->pattern;
            if (only >= 0 && p != only) continue;
            int32_t found = -1;
            for (size_t s = 0; s < slots.size(); ++s)
                if (slots[s].h && !slots[s].busy && slots[s].pattern == p) {
                    found = (int32_t)s;
                    break;
                }
            bool carved = false;
            if (found < 0) {
                size_t off = 0;
                bool ok = alloc->take(patterns[p].slot_bytes, &off);
                while (!ok) {  // evict the least recently used idle slot of another pattern
                    int32_t victim = -1;
                    for (size_t s = 0; s < slots.size(); ++s)
                        if (slots[s].h && !slots[s].busy && slots[s].pattern != p &&
                            (victim < 0 || slots[s].last_used < slots[victim].last_used))
                            victim = (int32_t)s;
                    if (victim < 0) break;
                    kkt_release(slots[victim].h);
                    alloc->give(slots[victim].off, slots[victim].bytes);
                    slots[victim] = Slot();
                    ++evicted;
                    ok = alloc->take(patterns[p].slot_bytes, &off);
                }
                if (!ok) continue;  // does not fit yet: later requests may go ahead
                kkt_handle_t h = nullptr;
                if (kkt_clone(patterns[p].proto, &h) != KKT_OK) {
                    alloc->give(off, patterns[p].slot_bytes);
                    continue;
                }
                Slot sl;
                sl.pattern = p;
                sl.h = h;
                sl.off = off;
                sl.bytes = patterns[p].slot_bytes;
                auto free_it = std::find_if(slots.begin(), slots.end(), [](const Slot &x) { return !x.h; });
                if (free_it == slots.end()) {
                    slots.push_back(sl);
                    found = (int32_t)slots.size() - 1;
                } else {
                    *free_it = sl;
                    found = (int32_t)(free_it - slots.begin());
                }
                carved = true;
                ++created;
            }
            slots[found].busy = true;
            slots[found].last_used = ++clock;
            std::shared_ptr<Request> r = *it;
            queue.erase(it);
            *slot_index = found;
            *fresh = carved;
            return r;
        }
        return nullptr;
    }

    void worker_main() {
        (void)hipSetDevice(device);
        hipStream_t stream = nullptr;
        const bool have_stream = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
        for (;;) {
            struct Item {
                std::shared_ptr<Request> r;
                int32_t si;
                bool fresh;
                kkt_handle_t h;
                size_t off, bytes;
            };
            std::vector<Item> batch;
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    int32_t si = -1;
                    bool fresh = false;
                    std::shared_ptr<Request> r = admit(&si, &fresh);
                    if (r) {
                        batch.push_back({r, si, fresh, slots[si].h, slots[si].off, slots[si].bytes});
                        break;
                    }
                    if (stopping && queue.empty()) break;
                    work_cv.wait(lk);
                }
                if (batch.empty()) break;
                // queued requests of the same pattern join the batch while slots are free or fit
                while ((int)batch.size() < max_batch) {
                    int32_t si = -1;
                    bool fresh = false;
                    std::shared_ptr<Request> r = admit(&si, &fresh, batch[0].r->pattern);
                    if (!r) break;
                    batch.push_back({r, si, fresh, slots[si].h, slots[si].off, slots[si].bytes});
                }
                if (batch.size() > 1) {
                    ++batches;
                    batched_requests += (int64_t)batch.size();
                }
            }
            const auto started = Clock::now();
            std::vector<kkt_status_t> st(batch.size(), have_stream ? KKT_OK : KKT_EDEVICE);
            std::vector<kkt_handle_t> hs;
            std::vector<const double *> vals;
            for (size_t b = 0; b < batch.size(); ++b) {
                batch[b].r->started = started;
                if (st[b] == KKT_OK && batch[b].fresh)
                    st[b] = kkt_bind_workspace(batch[b].h, pool + batch[b].off, batch[b].bytes, stream);
                if (st[b] == KKT_OK) {
                    hs.push_back(batch[b].h);
                    vals.push_back(batch[b].r->values);
                }
            }
            kkt_status_t sr = KKT_OK;
            if (!hs.empty()) {
                sr = use_graphs ? kkt_refactor_batch_graph(hs.data(), vals.data(), (int32_t)hs.size(), stream)
                                : kkt_refactor_batch(hs.data(), vals.data(), (int32_t)hs.size(), stream);
                if (sr == KKT_OK && use_graphs) {
                    std::lock_guard<std::mutex> lk(mu);
                    ++graph_launches;
                }
            }
            for (size_t b = 0; b < batch.size(); ++b) {
                Request &r = *batch[b].r;
                if (st[b] == KKT_OK) st[b] = sr;
                if (st[b] == KKT_OK) st[b] = kkt_solve(batch[b].h, r.b, r.x, r.tol, &r.info, stream);
                if (have_stream && hipStreamSynchronize(stream) != hipSuccess && st[b] == KKT_OK) st[b] = KKT_EDEVICE;
                r.finished = Clock::now();
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                for (size_t b = 0; b < batch.size(); ++b) {
                    Request &r = *batch[b].r;
                    const int32_t si = batch[b].si;
                    r.status = st[b];
                    r.slot = si;
                    r.new_slot = batch[b].fresh ? 1 : 0;
                    r.done = true;
                    // a slot whose handle failed, or that re-pivoted (its analysis now differs
                    // from the pattern's), is retired: every request is served by a slot on the
                    // pattern's own analysis, so a result does not depend on the slot's history
                    if (st[b] == KKT_EDEVICE || r.info.repivoted) {
                        kkt_release(slots[si].h);
                        alloc->give(slots[si].off, slots[si].bytes);
                        slots[si] = Slot();
                    } else {
                        slots[si].busy = false;
                    }
                    ++completed;
                }
            }
            done_cv.notify_all();
            work_cv.notify_all();
        }
        if (have_stream) (void)hipStreamDestroy(stream);
    }
};

extern "C" {

kkt_status_t kkt_server_create(void *dev_pool, size_t pool_bytes, int32_t workers, kkt_server_t *out) {
    if (!out) return KKT_EINVAL;
    *out = nullptr;
    if (!dev_pool || pool_bytes < 256 || workers < 1 || ((uintptr_t)dev_pool & 255) != 0) return KKT_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return KKT_EDEVICE;
    kkt_server_s *s = nullptr;
    try {
        s = new kkt_server_s();
        s->device = dev;
        s->pool = (char *)dev_pool;
        s->pool_bytes = pool_bytes & ~size_t(255);
        s->alloc.reset(new PoolAllocator(s->pool_bytes));
        for (int w = 0; w < workers; ++w) s->workers.emplace_back([s] { s->worker_main(); });
    } catch (...) {
        if (s) {
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->stopping = true;
            }
            s->work_cv.notify_all();
            for (auto &t : s->workers) t.join();
            delete s;
        }
        return KKT_ENOMEM;
    }
    *out = s;
    return KKT_OK;
}

kkt_status_t kkt_server_add_pattern(kkt_server_t s, const kkt_opts_t *opts, int64_t n, const int64_t *rowptr,
                                    const int32_t *colidx, const double *values_first, int32_t *pattern_id) {
    if (!s || !pattern_id) return KKT_EINVAL;
    kkt_handle_t h = nullptr;
    kkt_status_t st = kkt_analyze(opts, n, rowptr, colidx, values_first, &h);
    if (st != KKT_OK) return st;
    size_t bytes = 0;
    st = kkt_workspace_size(h, 1, &bytes);
    if (st != KKT_OK) {
        kkt_release(h);
        return st;
    }
    // room for a re-pivoted factorization with more fill
    bytes = bytes + bytes / 2 + (size_t(1) << 20);
    if (((bytes + 255) & ~size_t(255)) > s->pool_bytes) {  // could never be admitted
        kkt_release(h);
        return KKT_ENOMEM;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    Pattern p;
    p.proto = h;
    p.slot_bytes = bytes;
    s->patterns.push_back(p);
    *pattern_id = (int32_t)s->patterns.size() - 1;
    return KKT_OK;
}

kkt_status_t kkt_server_submit(kkt_server_t s, int32_t pattern_id, const double *dev_values, const double *dev_b,
                               double *dev_x, double tol, int64_t *ticket) {
    if (!s || !ticket || !dev_values || !dev_b || !dev_x || dev_b == dev_x) return KKT_EINVAL;
    auto r = std::make_shared<Request>();
    r->pattern = pattern_id;
    r->values = dev_values;
    r->b = dev_b;
    r->x = dev_x;
    r->tol = tol;
    r->submitted = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (pattern_id < 0 || pattern_id >= (int32_t)s->patterns.size() || s->stopping) return KKT_EINVAL;
        r->ticket = s->next_ticket++;
        s->tickets[r->ticket] = r;
        s->queue.push_back(r);
        *ticket = r->ticket;
    }
    s->work_cv.notify_one();
    return KKT_OK;
}

kkt_status_t kkt_server_wait(kkt_server_t s, int64_t ticket, kkt_solve_info_t *info, kkt_request_times_t *times) {
    if (!s) return KKT_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return KKT_EINVAL;
    std::shared_ptr<Request> r = it->second;
    s->done_cv.wait(lk, [&] { return r->done; });
    s->tickets.erase(ticket);
    if (info) *info = r->info;
    if (times) {
        times->queued_ms = ms_between(r->submitted, r->started);
        times->service_ms = ms_between(r->started, r->finished);
        times->latency_ms = ms_between(r->submitted, r->finished);
        times->slot = r->slot;
        times->new_slot = r->new_slot;
    }
    return r->status;
}

kkt_status_t kkt_server_poll(kkt_server_t s, int64_t ticket, int32_t *done) {
    if (!s || !done) return KKT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return KKT_EINVAL;
    *done = it->second->done ? 1 : 0;
    return KKT_OK;
}

kkt_status_t kkt_server_stats(kkt_server_t s, int64_t *completed, int64_t *slots_created, int64_t *slots_evicted,
                              int64_t *pool_in_use) {
    if (!s) return KKT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (completed) *completed = s->completed;
    if (slots_created) *slots_created = s->created;
    if (slots_evicted) *slots_evicted = s->evicted;
    if (pool_in_use) *pool_in_use = (int64_t)s->alloc->used();
    return KKT_OK;
}

kkt_status_t kkt_server_configure(kkt_server_t s, int32_t max_batch, int32_t use_graphs) {
    if (!s || max_batch < 1 || max_batch > 8 || (use_graphs != 0 && use_graphs != 1)) return KKT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    s->max_batch = max_batch;
    s->use_graphs = use_graphs != 0;
    return KKT_OK;
}

kkt_status_t kkt_server_batch_stats(kkt_server_t s, int64_t *batches, int64_t *batched_requests,
                                    int64_t *graph_launches) {
    if (!s) return KKT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (batches) *batches = s->batches;
    if (batched_requests) *batched_requests = s->batched_requests;
    if (graph_launches) *graph_launches = s->graph_launches;
    return KKT_OK;
}

kkt_status_t kkt_server_destroy(kkt_server_t s) {
    if (!s) return KKT_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->work_cv.notify_all();
    for (auto &t : s->workers) t.join();
    for (auto &sl : s->slots)
        if (sl.h) kkt_release(sl.h);
    for (auto &p : s->patterns) kkt_release(p.proto);
    delete s;
    return KKT_OK;
}

}  // extern "C"
