// tj_serve.cpp - the serving loop (tj_server_*): requests admitted against a
// device arena and run concurrently on per-slot HIP streams.
//
// Admission is first-come first-served over two queues: re-admissions (phase 2
// of a join materialisation, after its count) go ahead of new requests. A
// request is admitted when a slot is idle and the arena has room for its
// workspace; the arena holds nothing else, so every admitted request finishes
// and frees what it took, and the queue always drains.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "tj.h"

namespace {

constexpr uint64_t kAlign = 256;
constexpr uint64_t kMaxRows = (1ull << 31) - 1;

inline uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// First-fit allocator over the arena; free blocks are kept sorted by offset
// and merged with their neighbours on release. Guarded by the server mutex.
class Arena {
public:
    void init(char* base, uint64_t bytes)
    {
        base_ = base;
        bytes_ = bytes;
        free_.clear();
        free_[0] = bytes;
    }
    // nullptr when no free block holds `bytes`
    char* take(uint64_t bytes)
    {
        bytes = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const uint64_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            live_[off] = bytes;
            return base_ + off;
        }
        return nullptr;
    }
    void give(char* p)
    {
        if (!p) return;
        const uint64_t off = (uint64_t)(p - base_);
        auto lv = live_.find(off);
        if (lv == live_.end()) return;
        uint64_t len = lv->second, start = off;
        live_.erase(lv);
        used_ -= len;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && next->first == off + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
    }
    uint64_t bytes() const { return bytes_; }
    const char* base() const { return base_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }

private:
    char* base_ = nullptr;
    uint64_t bytes_ = 0, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;  // offset -> length
    std::map<uint64_t, uint64_t> live_;  // offset -> length
};

struct Job {
    uint64_t ticket = 0;
    tj_request_t req{};
    int phase = 0;                 // materialise: 1 count, 2 write pairs
    uint64_t count = 0;            // known after phase 1
    char* ws = nullptr;            // arena block held while running
    uint64_t ws_bytes = 0;
    Clock::time_point submitted, admitted;
    double run_ms = 0;
    bool done = false;
    bool waited = false;           // a thread is in tj_server_wait for it
    tj_result_t res{};
};

}  // namespace

struct tj_server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    Arena arena;
    int device = 0;
    int slots = 0;
    bool stopping = false;
    uint64_t next_ticket = 1;
    std::deque<Job*> fresh, again;      // new requests; phase-2 re-admissions
    std::map<uint64_t, Job*> jobs;      // every ticket not yet waited for
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;

    // Workspace for a call of this shape: the full plan if it fits the arena,
    // else the minimum; 0 if even that does not fit.
    uint64_t ws_for(int op, int kt, uint64_t n_r, uint64_t n_s)
    {
        uint64_t mn = 0, full = 0;
        if (tj_workspace_query(op, kt, n_r, n_s, &mn, &full) != TJ_OK) return 0;
        if (align_up(full) <= arena.bytes()) return full;
        if (align_up(mn) <= arena.bytes()) return mn;
        return 0;
    }

    // Tries to reserve the workspace of `j`'s next phase; false if the arena
    // has no room now. A job that can never fit is admitted as a failure.
    bool reserve(Job* j)
    {
        const tj_request_t& r = j->req;
        const int op = r.op == TJ_OP_JOIN_MATERIALIZE && j->phase == 1 ? TJ_OP_JOIN_COUNT : r.op;
        const uint64_t ws = ws_for(op, r.key_type, r.n_r, r.op == TJ_OP_SORT ? 0 : r.n_s);
        if (ws == 0) {
            j->res.status = TJ_E_WORKSPACE;
            return true;  // completes without running
        }
        char* a = arena.take(ws);
        if (!a) return false;
        j->ws = a;
        j->ws_bytes = ws;
        return true;
    }

    // Next job a worker may start (lock held): phase-2 jobs first, each queue in order.
    Job* admit()
    {
        for (std::deque<Job*>* q : {&again, &fresh}) {
            if (q->empty()) continue;
            Job* j = q->front();
            if (!reserve(j)) return nullptr;  // the head waits for memory; nothing overtakes it
            q->pop_front();
            return j;
        }
        return nullptr;
    }

    void run(Job* j, hipStream_t st)
    {
        const tj_request_t& r = j->req;
        tj_options_t opt{};
        opt.partitioner = r.partitioner;
        tj_stats_t stats{};
        int rc = j->res.status;
        if (rc == TJ_OK) {
            if (r.op == TJ_OP_SORT) {
                rc = tj_sort_ex(r.key_type, r.r_keys, r.r_rids, r.n_r, r.out0, r.out1, j->ws, j->ws_bytes, st, &opt,
                                &stats);
                j->count = r.n_r;
            } else if (r.op == TJ_OP_JOIN_COUNT || j->phase == 1) {
                uint64_t cnt = 0;
                rc = tj_join_count_ex(r.key_type, r.r_keys, r.n_r, r.s_keys, r.n_s, &cnt, j->ws, j->ws_bytes, st, &opt,
                                      &stats);
                j->count = cnt;
            } else {
                uint64_t cnt = 0;
                rc = tj_join_materialize_ex(r.key_type, r.r_keys, r.r_rids, r.n_r, r.s_keys, r.s_rids, r.n_s,
                                            (int32_t*)r.out0, r.out1, r.capacity, &cnt, j->ws, j->ws_bytes, st, &opt,
                                            &stats);
                if ((rc == TJ_OK || rc == TJ_E_CAPACITY) && cnt != j->count) rc = TJ_E_INTERNAL;
            }
        }
        j->res.status = rc;
        j->res.learned = stats.learned;
        j->res.key_ranges = stats.key_ranges;
    }

    void worker(int slot)
    {
        (void)hipSetDevice(device);
        hipStream_t st = streams[slot];
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            Job* j = nullptr;
            cv_work.wait(lk, [&] { return (j = admit()) != nullptr || (stopping && fresh.empty() && again.empty()); });
            if (!j) return;
            j->admitted = Clock::now();
            lk.unlock();
            run(j, st);
            const auto end = Clock::now();
            lk.lock();
            j->run_ms += ms_between(j->admitted, end);
            arena.give(j->ws);
            j->ws = nullptr;
            bool phase1 = j->req.op == TJ_OP_JOIN_MATERIALIZE && j->phase == 1 && j->res.status == TJ_OK;
            if (phase1 && j->count > j->req.capacity) {
                j->res.status = TJ_E_CAPACITY;  // nothing to write: the pairs would not fit
                phase1 = false;
            }
            if (phase1) {
                j->phase = 2;
                again.push_back(j);
            } else {
                const int st_ = j->res.status;
                j->res.op = j->req.op;
                j->res.count = st_ == TJ_OK || st_ == TJ_E_CAPACITY ? j->count : 0;
                j->res.run_ms = j->run_ms;
                j->res.total_ms = ms_between(j->submitted, end);
                j->res.queue_ms = j->res.total_ms - j->run_ms;
                j->done = true;
                cv_done.notify_all();
            }
            cv_work.notify_all();  // memory was freed: the queue head may fit now
        }
    }
};

extern "C" {

int tj_server_create(void* arena, uint64_t arena_bytes, int slots, tj_server_t** server)
{
    if (!arena || !server || slots < 1 || slots > 64) return TJ_E_ARG;
    if ((uintptr_t)arena % kAlign || arena_bytes < (64ull << 10)) return TJ_E_WORKSPACE;
    tj_server* s = new (std::nothrow) tj_server();
    if (!s) return TJ_E_INTERNAL;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return TJ_E_HIP;
    }
    s->arena.init((char*)arena, arena_bytes / kAlign * kAlign);
    s->slots = slots;
    for (int i = 0; i < slots; i++) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
            delete s;
            return TJ_E_HIP;
        }
        s->streams.push_back(st);
    }
    try {
        for (int i = 0; i < slots; i++) s->workers.emplace_back([s, i] { s->worker(i); });
    } catch (...) {  // no thread could be started: stop the ones that were
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stopping = true;
        }
        s->cv_work.notify_all();
        for (std::thread& t : s->workers) t.join();
        for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
        delete s;
        return TJ_E_INTERNAL;
    }
    *server = s;
    return TJ_OK;
}

int tj_server_submit(tj_server_t* s, const tj_request_t* req, uint64_t* ticket)
{
    if (!s || !req || !ticket) return TJ_E_ARG;
    const tj_request_t& r = *req;
    if (r.key_type != TJ_KEY_I32 && r.key_type != TJ_KEY_I64) return TJ_E_ARG;
    if (r.partitioner != TJ_PART_RADIX && r.partitioner != TJ_PART_LEARNED && r.partitioner != TJ_PART_AUTO)
        return TJ_E_ARG;
    if (r.n_r > kMaxRows || r.n_s > kMaxRows) return TJ_E_TOO_LARGE;
    const uint64_t kb = (uint64_t)r.key_type;
    auto overlap = [](const void* a, uint64_t an, const void* b, uint64_t bn) {
        if (!a || !b || !an || !bn) return false;
        const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
        return x < y + bn && y < x + an;
    };
    const void* outs[2] = {r.out0, r.out1};
    uint64_t osz[2] = {0, 0};
    switch (r.op) {
    case TJ_OP_SORT:
        if (r.n_r && (!r.r_keys || !r.r_rids || !r.out0 || !r.out1)) return TJ_E_ARG;
        osz[0] = r.n_r * kb;
        osz[1] = r.n_r * 4;
        break;
    case TJ_OP_JOIN_COUNT:
        if ((r.n_r && !r.r_keys) || (r.n_s && !r.s_keys)) return TJ_E_ARG;
        break;
    case TJ_OP_JOIN_MATERIALIZE:
        if ((r.n_r && (!r.r_keys || !r.r_rids)) || (r.n_s && (!r.s_keys || !r.s_rids))) return TJ_E_ARG;
        if (r.capacity && (!r.out0 || !r.out1)) return TJ_E_ARG;
        osz[0] = osz[1] = r.capacity * 4;
        break;
    default: return TJ_E_ARG;
    }
    {
        const void* ins[4] = {r.r_keys, r.r_rids, r.s_keys, r.s_rids};
        const uint64_t isz[4] = {r.n_r * kb, r.n_r * 4, r.n_s * kb, r.n_s * 4};
        std::lock_guard<std::mutex> lk(s->mu);
        for (int o = 0; o < 2; o++) {
            for (int i = 0; i < 4; i++)
                if (overlap(outs[o], osz[o], ins[i], isz[i])) return TJ_E_ALIAS;
            if (overlap(outs[o], osz[o], s->arena.base(), s->arena.bytes())) return TJ_E_ALIAS;
        }
        if (overlap(outs[0], osz[0], outs[1], osz[1])) return TJ_E_ALIAS;
    }
    Job* j = new (std::nothrow) Job();
    if (!j) return TJ_E_INTERNAL;
    j->req = r;
    j->phase = r.op == TJ_OP_JOIN_MATERIALIZE ? 1 : 0;
    j->submitted = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) {
            delete j;
            return TJ_E_ARG;
        }
        j->ticket = s->next_ticket++;
        s->jobs[j->ticket] = j;
        s->fresh.push_back(j);
        *ticket = j->ticket;
    }
    s->cv_work.notify_one();
    return TJ_OK;
}

int tj_server_wait(tj_server_t* s, uint64_t ticket, tj_result_t* result)
{
    if (!s || !result) return TJ_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return TJ_E_ARG;
    Job* j = it->second;
    if (j->waited) return TJ_E_ARG;  // one wait per ticket
    j->waited = true;
    s->cv_done.wait(lk, [&] { return j->done; });
    *result = j->res;
    s->jobs.erase(ticket);
    delete j;
    return TJ_OK;
}

int tj_server_memory(tj_server_t* s, uint64_t* in_use, uint64_t* peak)
{
    if (!s || !in_use || !peak) return TJ_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *in_use = s->arena.used();
    *peak = s->arena.peak();
    return TJ_OK;
}

int tj_server_destroy(tj_server_t* s)
{
    if (!s) return TJ_E_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    for (std::thread& t : s->workers) t.join();
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    for (auto& kv : s->jobs) delete kv.second;
    delete s;
    return TJ_OK;
}

}  // extern "C"
