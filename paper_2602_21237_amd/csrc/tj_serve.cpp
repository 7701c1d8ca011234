// tj_serve.cpp - the serving loop (tj_server_*): requests admitted against a
// device arena and run concurrently on per-slot HIP streams.
//
// Admission is first-come first-served. A request is admitted when a slot is
// idle and the arena has room for its workspace; the arena holds nothing else,
// so every admitted request finishes and frees what it took, and the queue
// always drains. A join materialisation is one call: it writes its pairs when
// they fit the caller's capacity and otherwise reports TJ_E_CAPACITY with the
// count, so no separate count pass is needed.
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

#include "tj_internal.h"

namespace tj {
void release_thread_staging();  // frees the calling thread's pinned staging (tj_abi.cpp)
}

namespace {

constexpr uint64_t kAlign = 256;
constexpr uint64_t kMaxRows = (1ull << 31) - 1;
constexpr uint64_t kFuseDefaultRows = 1ull << 16;  // rows of a request the server fuses by default
constexpr uint32_t kFuseDefaultRequests = 32;      // requests per fused call by default
constexpr uint32_t kFuseMaxRequests = 256;
constexpr size_t kFuseLookahead = 256;             // queue positions searched for partners

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
    uint64_t count = 0;
    uint32_t fused = 1;            // requests of the call that served this one
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
    std::deque<Job*> fresh;             // requests in arrival order
    std::map<uint64_t, Job*> jobs;      // every ticket not yet waited for
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    uint64_t fuse_rows = kFuseDefaultRows;       // 0: no fusion
    uint32_t fuse_requests = kFuseDefaultRequests;

    // Rows a request brings (both sides of a join).
    static uint64_t rows_of(const tj_request_t& r) { return r.n_r + (r.op == TJ_OP_SORT ? 0 : r.n_s); }

    bool fusable(const Job* j) const
    {
        const tj_request_t& r = j->req;
        return fuse_rows && fuse_requests > 1 && j->res.status == TJ_OK && r.partitioner == TJ_PART_RADIX &&
               (r.op == TJ_OP_SORT || r.op == TJ_OP_JOIN_MATERIALIZE) && rows_of(r) <= fuse_rows;
    }

    // Arena bytes of a fused call over `b`: the combined columns, the
    // composite call's outputs and its full workspace, the descriptors and
    // the pair boundaries.
    uint64_t fused_bytes(const std::vector<Job*>& b)
    {
        const tj_request_t& r0 = b[0]->req;
        const uint64_t kb = (uint64_t)r0.key_type;
        uint64_t nr = 0, ns = 0, cap = 0;
        for (const Job* j : b) {
            nr += j->req.n_r;
            ns += j->req.op == TJ_OP_SORT ? 0 : j->req.n_s;
            cap += j->req.op == TJ_OP_SORT ? 0 : j->req.capacity;
        }
        const int types[2] = {TJ_KEY_I32, r0.key_type};
        uint64_t mws = 0;
        if (tj_multi_workspace_query(r0.op, 2, types, nr, ns, &mws) != TJ_OK) return ~0ull;
        uint64_t bytes = mws + align_up(b.size() * sizeof(tj::FuseDesc)) + align_up((b.size() + 1) * 8);
        if (r0.op == TJ_OP_SORT) bytes += 2 * (2 * align_up(nr * 4) + align_up(nr * kb));
        else bytes += 2 * align_up(nr * 4) + align_up(nr * kb) + 2 * align_up(ns * 4) + align_up(ns * kb) +
                      2 * align_up(cap * 4);
        return bytes;
    }

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
        const uint64_t ws = ws_for(r.op, r.key_type, r.n_r, r.op == TJ_OP_SORT ? 0 : r.n_s);
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

    // Next work a worker may start (lock held), in arrival order: the head of
    // the queue, with the queued requests it can be fused with (same op and
    // key type, small) when the arena holds the fused call; the first job of
    // a fused batch holds the batch's arena block.
    bool admit(std::vector<Job*>& batch)
    {
        batch.clear();
        if (fresh.empty()) return false;
        Job* j = fresh.front();
        if (fusable(j)) {
            batch.push_back(j);
            uint64_t rows = rows_of(j->req);
            const uint64_t max_rows = fuse_rows * 16;
            for (size_t i = 1; i < fresh.size() && i < kFuseLookahead && batch.size() < fuse_requests; i++) {
                Job* k = fresh[i];
                if (!fusable(k) || k->req.op != j->req.op || k->req.key_type != j->req.key_type) continue;
                if (rows + rows_of(k->req) > max_rows) continue;
                batch.push_back(k);
                rows += rows_of(k->req);
            }
            while (batch.size() > 1) {
                const uint64_t need = fused_bytes(batch);
                char* a = need <= arena.bytes() ? arena.take(need) : nullptr;
                if (a) {
                    j->ws = a;
                    j->ws_bytes = need;
                    for (Job* k : batch) fresh.erase(std::find(fresh.begin(), fresh.end(), k));
                    return true;
                }
                batch.pop_back();  // fewer partners: a smaller fused call
            }
            batch.clear();
        }
        if (!reserve(j)) return false;  // the head waits for memory; nothing overtakes it
        fresh.pop_front();
        batch.push_back(j);
        return true;
    }

    // One fused call over `b` (b.size() >= 2) in the arena block of b[0];
    // every job's status and count are set. A join batch whose pairs exceed
    // the summed capacities (some request's own capacity is too small) runs
    // its requests one by one in the same block instead.
    void run_fused(std::vector<Job*>& b, hipStream_t st)
    {
        const tj_request_t& r0 = b[0]->req;
        const int kt = r0.key_type;
        const uint64_t kb = (uint64_t)kt;
        const bool sort = r0.op == TJ_OP_SORT;
        const uint32_t nreq = (uint32_t)b.size();
        std::vector<tj::FuseDesc> desc(nreq);
        uint64_t nr = 0, ns = 0, cap = 0, maxr = 0, maxs = 0;
        for (uint32_t i = 0; i < nreq; i++) {
            const tj_request_t& r = b[i]->req;
            tj::FuseDesc& d = desc[i];
            d.r_keys = r.r_keys;
            d.r_rids = r.r_rids;
            d.s_keys = sort ? nullptr : r.s_keys;
            d.s_rids = sort ? nullptr : r.s_rids;
            d.out0 = r.out0;
            d.out1 = r.out1;
            d.n_r = r.n_r;
            d.n_s = sort ? 0 : r.n_s;
            d.off_r = nr;
            d.off_s = ns;
            d.capacity = sort ? 0 : r.capacity;
            nr += d.n_r;
            ns += d.n_s;
            cap += d.capacity;
            maxr = std::max(maxr, d.n_r);
            maxs = std::max(maxs, d.n_s);
        }
        char* p = b[0]->ws;
        auto take = [&](uint64_t bytes) {
            char* q = p;
            p += align_up(bytes);
            return q;
        };
        tj::FuseDesc* d_desc = (tj::FuseDesc*)take(nreq * sizeof(tj::FuseDesc));
        uint64_t* d_bounds = (uint64_t*)take((nreq + 1) * 8);
        const int types[2] = {TJ_KEY_I32, kt};
        tj_stats_t stats{};
        int rc = TJ_OK;
        auto ck = [&](hipError_t e) {
            if (e != hipSuccess && rc == TJ_OK) rc = TJ_E_HIP;
        };
        ck(hipMemcpyAsync(d_desc, desc.data(), nreq * sizeof(tj::FuseDesc), hipMemcpyHostToDevice, st));
        if (sort) {
            int32_t* item = (int32_t*)take(nr * 4);
            void* keys = take(nr * kb);
            int32_t* rids = (int32_t*)take(nr * 4);
            int32_t* oitem = (int32_t*)take(nr * 4);
            void* okeys = take(nr * kb);
            int32_t* orids = (int32_t*)take(nr * 4);
            char* mws = p;
            const uint64_t mws_bytes = (uint64_t)(b[0]->ws + b[0]->ws_bytes - p);
            if (rc == TJ_OK) ck(tj::launch_fuse_gather(kt, d_desc, nreq, maxr, 0, 0, item, keys, rids, st));
            if (rc == TJ_OK) {
                const void* kin[2] = {item, keys};
                void* kout[2] = {oitem, okeys};
                rc = tj_sort_multi(2, types, kin, rids, nr, kout, orids, mws, mws_bytes, st, &stats);
            }
            if (rc == TJ_OK) ck(tj::launch_fuse_scatter_sort(kt, d_desc, nreq, maxr, okeys, orids, st));
            if (rc == TJ_OK) ck(hipStreamSynchronize(st));
            for (Job* j : b) {
                j->res.status = rc;
                j->count = j->req.n_r;
            }
        } else {
            int32_t* item_r = (int32_t*)take(nr * 4);
            void* keys_r = take(nr * kb);
            int32_t* pos_r = (int32_t*)take(nr * 4);
            int32_t* item_s = (int32_t*)take(ns * 4);
            void* keys_s = take(ns * kb);
            int32_t* pos_s = (int32_t*)take(ns * 4);
            int32_t* pr = (int32_t*)take(cap * 4);
            int32_t* ps = (int32_t*)take(cap * 4);
            char* mws = p;
            const uint64_t mws_bytes = (uint64_t)(b[0]->ws + b[0]->ws_bytes - p);
            if (rc == TJ_OK) ck(tj::launch_fuse_gather(kt, d_desc, nreq, maxr, 0, 1, item_r, keys_r, pos_r, st));
            if (rc == TJ_OK) ck(tj::launch_fuse_gather(kt, d_desc, nreq, maxs, 1, 1, item_s, keys_s, pos_s, st));
            uint64_t cnt = 0;
            if (rc == TJ_OK) {
                const void* rk[2] = {item_r, keys_r};
                const void* sk[2] = {item_s, keys_s};
                rc = tj_join_materialize_multi(2, types, rk, pos_r, nr, sk, pos_s, ns, cap ? pr : nullptr,
                                               cap ? ps : nullptr, cap, &cnt, mws, mws_bytes, st, &stats);
            }
            if (rc == TJ_E_CAPACITY) {
                // some request's pairs exceed its capacity: serve them one by one
                for (Job* j : b) {
                    const tj_request_t& r = j->req;
                    tj_options_t opt{};
                    uint64_t c = 0;
                    j->res.status = tj_join_materialize_ex(r.key_type, r.r_keys, r.r_rids, r.n_r, r.s_keys, r.s_rids,
                                                           r.n_s, (int32_t*)r.out0, r.out1, r.capacity, &c, b[0]->ws,
                                                           b[0]->ws_bytes, st, &opt, &stats);
                    j->count = c;
                    j->fused = 1;
                }
                return;
            }
            std::vector<uint64_t> bounds(nreq + 1, 0);
            if (rc == TJ_OK) ck(tj::launch_fuse_bounds(pr, item_r, cnt, nreq, d_bounds, st));
            if (rc == TJ_OK) ck(tj::launch_fuse_scatter_pairs(d_desc, nreq, d_bounds, pr, ps, cnt, st));
            if (rc == TJ_OK) ck(hipMemcpyAsync(bounds.data(), d_bounds, (nreq + 1) * 8, hipMemcpyDeviceToHost, st));
            if (rc == TJ_OK) ck(hipStreamSynchronize(st));
            for (uint32_t i = 0; i < nreq; i++) {
                Job* j = b[i];
                j->count = rc == TJ_OK ? bounds[i + 1] - bounds[i] : 0;
                j->res.status = rc != TJ_OK ? rc : (j->count > j->req.capacity ? TJ_E_CAPACITY : TJ_OK);
            }
        }
        for (Job* j : b) {
            j->res.learned = 0;
            j->res.key_ranges = stats.key_ranges;
            j->res.windows = stats.windows;
        }
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
            } else if (r.op == TJ_OP_JOIN_COUNT) {
                uint64_t cnt = 0;
                rc = tj_join_count_ex(r.key_type, r.r_keys, r.n_r, r.s_keys, r.n_s, &cnt, j->ws, j->ws_bytes, st, &opt,
                                      &stats);
                j->count = cnt;
            } else {
                uint64_t cnt = 0;
                rc = tj_join_materialize_ex(r.key_type, r.r_keys, r.r_rids, r.n_r, r.s_keys, r.s_rids, r.n_s,
                                            (int32_t*)r.out0, r.out1, r.capacity, &cnt, j->ws, j->ws_bytes, st, &opt,
                                            &stats);
                j->count = cnt;
            }
        }
        j->res.status = rc;
        j->res.learned = stats.learned;
        j->res.key_ranges = stats.key_ranges;
        j->res.windows = stats.windows;
    }

    void worker(int slot)
    {
        (void)hipSetDevice(device);
        hipStream_t st = streams[slot];
        std::unique_lock<std::mutex> lk(mu);
        std::vector<Job*> batch;
        for (;;) {
            bool got = false;
            cv_work.wait(lk, [&] { return (got = admit(batch)) || (stopping && fresh.empty()); });
            if (!got) {
                lk.unlock();
                tj::release_thread_staging();  // the thread ends: its pinned staging goes with it
                return;
            }
            const auto start = Clock::now();
            for (Job* j : batch) {
                j->admitted = start;
                j->fused = (uint32_t)batch.size();
            }
            lk.unlock();
            if (batch.size() > 1) {
                try {
                    run_fused(batch, st);
                } catch (...) {  // host memory ran out: nothing crosses the C ABI
                    for (Job* j : batch) j->res.status = TJ_E_INTERNAL;
                }
            } else {
                run(batch[0], st);
            }
            const auto end = Clock::now();
            lk.lock();
            arena.give(batch[0]->ws);
            batch[0]->ws = nullptr;
            for (Job* j : batch) {
                j->run_ms += ms_between(j->admitted, end);
                const int st_ = j->res.status;
                j->res.op = j->req.op;
                j->res.count = st_ == TJ_OK || st_ == TJ_E_CAPACITY ? j->count : 0;
                j->res.run_ms = j->run_ms;
                j->res.total_ms = ms_between(j->submitted, end);
                j->res.queue_ms = j->res.total_ms - j->run_ms;
                j->res.fused = j->fused;
                j->done = true;
            }
            cv_done.notify_all();
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

int tj_server_configure(tj_server_t* s, uint64_t fuse_max_rows, uint32_t fuse_max_requests)
{
    if (!s || fuse_max_requests > kFuseMaxRequests || fuse_max_rows > kMaxRows) return TJ_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    s->fuse_rows = fuse_max_rows;
    s->fuse_requests = fuse_max_requests;
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
