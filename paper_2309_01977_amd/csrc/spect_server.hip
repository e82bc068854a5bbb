// spect_server.hip - reconstruction server with continuous (iteration-level)
// batching: requests are admitted as they arrive, by resident count and
// memory footprint, and every resident request advances together, one step
// per tick, through the work-list kernels.
//
// A request is a whole OSEM reconstruction (the computation of
// osem_reconstruct): the sensitivity pass of each subset (which also fills
// the subset's attenuation table), then n_iters x n_subsets subiterations.
// Each of these is one step.  A scheduler thread launches ticks back to back
// on up to four lanes (streams, which run concurrently): a lane's tick takes
// the next step of each of the lane's resident requests (requests at
// different subsets, iterations and geometries alike) and runs them as one
// launch per stage (see tick_build).  Requests queue in arrival order; at
// every tick boundary they are admitted in that order, to the lane with the
// least work left, as soon as fewer than n_slots requests are resident and
// the pool holds a free block of the workspace (a wide request may wait for
// another wide one to finish; see admit()); a request retires once
// the tick holding its last step has finished, freeing its block.  A request's state lives in its
// block laid out as osem_reconstruct's workspace and its steps use
// osem_reconstruct's launch arguments, so its result is osem_reconstruct's,
// bitwise, whatever shares its ticks.  The first tick of a request waits (on
// the device) for an event recorded on the caller's stream at submission.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "spect.h"
#include "spect_internal.h"

using spect_internal::clear_error;
using spect_internal::set_error;

namespace {

struct Request {
    const spect_plan *plan = nullptr;
    float *f = nullptr;
    const float *mu = nullptr, *g = nullptr, *s = nullptr;
    int iters = 0, subsets = 1;
    size_t ws = 0, off = 0;
    hipEvent_t ready = nullptr;  // recorded on the caller's stream at submission
    int state = SPECT_REQ_QUEUED;
    int steps = 0, issued = 0;   // steps of the request, steps launched so far
    double step_work = 0;        // voxel-angles of one step
    int err = SPECT_OK;
    std::string msg;
};

struct Block {
    size_t off, size;
};

// Buffers of one tick's launch tables; reused once the tick has finished.
struct TickSlot {
    char *host = nullptr, *dev = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;      // recorded on the lane after the tick's kernels
    hipEvent_t uploaded = nullptr;  // recorded on the upload stream after the table copy
    std::vector<int64_t> finishing;  // requests whose last step is in this tick
};

constexpr int kRing = 3;
// Scheduler poll interval while ticks are in flight (submissions end a wait
// early).
constexpr int kPollUs = 20;

size_t round256(size_t x) { return (x + 255) & ~size_t(255); }

int failf(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int failf(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(code, buf);
}

}  // namespace

// A lane: a stream with its own ticks over its own resident requests.
// Lanes run concurrently, so the kernels of different lanes overlap on the
// device; within a lane every tick advances all of its requests together.
struct Lane {
    hipStream_t stream = nullptr;
    std::vector<int64_t> resident;  // admitted and unfinished, in admission order
    TickSlot ring[kRing];
    std::deque<int> inflight;       // ring slots in launch order
    std::deque<long> seq;           // global launch number of each in-flight tick
};

constexpr int kMaxLanes = 4;
// A request is wide when one of its steps covers at least this many
// voxel-angles (a 15-angle subset of a 128^3 object is 3.1e7); wide requests
// overlap only while at least kWideBacklog of them are queued.
constexpr double kWideStep = double(1 << 24);
constexpr int kWideBacklog = 4;

struct spect_server {
    int device = 0;
    int max_resident = 1;
    std::vector<Lane> lanes;
    hipStream_t upload = nullptr;  // tick table copies, beside the lanes' kernels
    char *pool = nullptr;
    size_t pool_bytes = 0, in_use = 0;
    std::vector<Block> free_list;  // sorted by offset, coalesced
    std::deque<int64_t> queue;
    std::map<int64_t, Request> reqs;
    int64_t next_id = 1;
    int peak_running = 0;
    long ticks = 0;  // ticks launched
    std::mutex mu;
    std::condition_variable wake;   // submissions and shutdown, for the scheduler
    std::condition_variable done;   // retirements, for waiting callers
    bool stop = false;
    std::thread worker;

    bool alloc(size_t n, size_t *off)
    {
        for (size_t i = 0; i < free_list.size(); ++i)
            if (free_list[i].size >= n) {
                *off = free_list[i].off;
                free_list[i].off += n;
                free_list[i].size -= n;
                if (free_list[i].size == 0) free_list.erase(free_list.begin() + i);
                in_use += n;
                return true;
            }
        return false;
    }

    void release(size_t off, size_t n)
    {
        in_use -= n;
        auto it = std::lower_bound(free_list.begin(), free_list.end(), off,
                                   [](const Block &b, size_t o) { return b.off < o; });
        it = free_list.insert(it, Block{off, n});
        const size_t i = it - free_list.begin();
        if (i + 1 < free_list.size() && free_list[i].off + free_list[i].size == free_list[i + 1].off) {
            free_list[i].size += free_list[i + 1].size;
            free_list.erase(free_list.begin() + i + 1);
        }
        if (i > 0 && free_list[i - 1].off + free_list[i - 1].size == free_list[i].off) {
            free_list[i - 1].size += free_list[i].size;
            free_list.erase(free_list.begin() + i);
        }
    }

    static void drop_ready(Request &r)
    {
        if (r.ready) (void)hipEventDestroy(r.ready);
        r.ready = nullptr;
    }

    int running() const
    {
        int n = 0;
        for (const Lane &l : lanes) n += (int)l.resident.size();
        return n;
    }

    // A resident request leaves: its block returns to the pool.  Called once
    // the stream has passed every tick that used the block.
    void retire(Lane &ln, int64_t id, int state, int err, const std::string &msg)
    {
        Request &r = reqs[id];
        r.state = state;
        r.err = err;
        r.msg = msg;
        release(r.off, r.ws);
        drop_ready(r);
        ln.resident.erase(std::remove(ln.resident.begin(), ln.resident.end(), id), ln.resident.end());
    }

    // work a lane still has to launch: steps left x voxel-angles per step
    double lane_load(const Lane &ln)
    {
        double n = 0;
        for (int64_t id : ln.resident) {
            const Request &r = reqs[id];
            n += (double)(r.steps - r.issued) * r.step_work;
        }
        return n;
    }

    // A wide request's steps fill the device on their own.  Two wide
    // requests resident together share the device and both finish late,
    // where running them in turn finishes the older one first: at light load
    // that ordering gives the shorter latency tail.  So a wide request waits
    // while another wide one is resident, unless a backlog of wide requests
    // is queued (then they overlap for throughput); narrow requests behind a
    // waiting wide one may start first, and run beside the wide ones.
    static bool wide(const Request &r) { return r.step_work >= kWideStep; }

    // Admit in arrival order while a resident place and a pool block are
    // free, with the exception above for waiting wide requests; a request
    // that does not fit in the pool stops admission until blocks return.
    void admit()
    {
        while (!queue.empty() && running() < max_resident) {
            int wide_res = 0, wide_q = 0;
            for (const Lane &ln : lanes)
                for (int64_t rid : ln.resident) wide_res += wide(reqs[rid]) ? 1 : 0;
            for (int64_t qid : queue) wide_q += wide(reqs[qid]) ? 1 : 0;
            const int wide_cap = wide_q >= kWideBacklog ? max_resident : 1;
            auto pick = queue.begin();
            while (pick != queue.end() && wide(reqs[*pick]) && wide_res >= wide_cap) ++pick;
            if (pick == queue.end()) break;
            Request &r = reqs[*pick];
            size_t off = 0;
            if (!alloc(r.ws, &off)) break;
            const int64_t id = *pick;
            queue.erase(pick);
            r.off = off;
            r.issued = 0;
            if (r.iters == 0) {
                // nothing changes f (osem_reconstruct with zero iterations)
                r.state = SPECT_REQ_DONE;
                release(off, r.ws);
                drop_ready(r);
                done.notify_all();
                continue;
            }
            r.state = SPECT_REQ_RUNNING;
            // the lane with the fewest steps left
            Lane *best = &lanes[0];
            for (Lane &ln : lanes)
                if (lane_load(ln) < lane_load(*best)) best = &ln;
            best->resident.push_back(id);
            peak_running = std::max(peak_running, running());
        }
    }

    // Retire the requests of lane ln's oldest tick if it has finished;
    // returns whether it had.  Called with the lock held.
    bool finish_oldest(Lane &ln)
    {
        if (ln.inflight.empty()) return false;
        TickSlot &ts = ln.ring[ln.inflight.front()];
        const hipError_t e = hipEventQuery(ts.done);
        if (e == hipErrorNotReady) return false;
        ln.inflight.pop_front();
        ln.seq.pop_front();
        for (int64_t id : ts.finishing) {
            if (e == hipSuccess)
                retire(ln, id, SPECT_REQ_DONE, SPECT_OK, "");
            else
                retire(ln, id, SPECT_REQ_FAILED, SPECT_EHIP, hipGetErrorString(e));
        }
        ts.finishing.clear();
        if (e != hipSuccess) fail_resident(ln, SPECT_EHIP, hipGetErrorString(e));
        done.notify_all();
        return true;
    }

    // A launch or runtime error: every resident request of the lane fails
    // once its stream has drained.
    void fail_resident(Lane &ln, int err, const std::string &msg)
    {
        (void)hipStreamSynchronize(ln.stream);
        ln.inflight.clear();
        ln.seq.clear();
        for (TickSlot &ts : ln.ring) ts.finishing.clear();
        std::vector<int64_t> ids = ln.resident;
        for (int64_t id : ids) retire(ln, id, SPECT_REQ_FAILED, err, msg);
        done.notify_all();
    }

    // Launch lane ln's next tick: the next step of each of its resident
    // requests with steps left.  Returns false if there was nothing to launch.
    bool launch_tick(Lane &ln, std::unique_lock<std::mutex> &lk)
    {
        std::vector<spect_internal::TickItem> items;
        std::vector<int64_t> ids, first, last;
        for (int64_t id : ln.resident) {
            Request &r = reqs[id];
            if (r.issued >= r.steps) continue;
            const int k = r.issued, M = r.subsets;
            spect_internal::TickItem it{r.plan, r.f, r.mu, r.g, r.s, pool + r.off, M, k < M ? 1 : 0,
                                        k < M ? k : (k - M) % M, k == M ? 1 : 0};
            items.push_back(it);
            ids.push_back(id);
            if (k == 0) first.push_back(id);
            if (k + 1 == r.steps) last.push_back(id);
        }
        if (items.empty()) return false;
        int slot = -1;
        for (int k = 0; k < kRing; ++k)
            if (std::find(ln.inflight.begin(), ln.inflight.end(), k) == ln.inflight.end()) {
                slot = k;
                break;
            }
        TickSlot &ts = ln.ring[slot];
        std::vector<hipEvent_t> waits;
        for (int64_t id : first) waits.push_back(reqs[id].ready);
        lk.unlock();
        // host work and launches without the lock: only this thread changes
        // resident requests, the rings and the streams
        int st = SPECT_OK;
        std::string msg;
        int bst = SPECT_OK;
        spect_internal::TickTables *T = spect_internal::tick_build(items.data(), (int)items.size(), &bst);
        const size_t need = spect_internal::tick_bytes(T);
        if (need > ts.cap) {
            if (ts.host) (void)hipHostFree(ts.host);
            if (ts.dev) (void)hipFree(ts.dev);
            ts.host = ts.dev = nullptr;
            ts.cap = 0;
            const size_t cap = std::max(need + need / 2, size_t(1) << 20);
            if (hipHostMalloc(reinterpret_cast<void **>(&ts.host), cap) != hipSuccess ||
                hipMalloc(reinterpret_cast<void **>(&ts.dev), cap) != hipSuccess) {
                st = SPECT_ENOMEM;
                msg = "tick table allocation failed";
            } else {
                ts.cap = cap;
            }
        }
        for (hipEvent_t ev : waits)
            if (st == SPECT_OK && hipStreamWaitEvent(ln.stream, ev, 0) != hipSuccess) {
                st = SPECT_EHIP;
                msg = "a lane stream could not wait for a submission event";
            }
        if (st == SPECT_OK) {
            st = spect_internal::tick_launch(T, ts.host, ts.dev, ln.stream, upload, ts.uploaded);
            if (st != SPECT_OK) msg = spect_last_error();
        }
        if (st == SPECT_OK && hipEventRecord(ts.done, ln.stream) != hipSuccess) {
            st = SPECT_EHIP;
            msg = "tick event record failed";
        }
        spect_internal::tick_free(T);
        lk.lock();
        if (st != SPECT_OK) {
            fail_resident(ln, st, msg);
            return true;
        }
        for (int64_t id : ids) reqs[id].issued++;
        ts.finishing = last;
        ln.inflight.push_back(slot);
        ln.seq.push_back(ticks++);
        return true;
    }

    void run()
    {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            for (Lane &ln : lanes)
                while (finish_oldest(ln)) {
                }
            if (!stop) admit();
            bool launched = false, busy = false;
            for (Lane &ln : lanes) {
                if ((int)ln.inflight.size() < kRing && launch_tick(ln, lk)) launched = true;
                busy = busy || !ln.inflight.empty();
            }
            if (launched) continue;
            if (busy) {
                // ticks in flight: poll every lane, so that a lane whose
                // ticks are short is refilled while another's long tick runs
                wake.wait_for(lk, std::chrono::microseconds(kPollUs));
                continue;
            }
            if (stop && running() == 0) break;
            wake.wait(lk, [&] { return stop || !queue.empty(); });
        }
    }
};

extern "C" {

int spect_server_create(int32_t n_slots, size_t pool_bytes, spect_server **out)
{
    if (!out) return set_error(SPECT_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_slots < 1 || n_slots > 64) return failf(SPECT_EINVAL, "n_slots = %d outside [1, 64]", n_slots);
    if (pool_bytes < 256) return set_error(SPECT_EINVAL, "pool_bytes must be at least 256");
    spect_server *s = new spect_server();
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return set_error(SPECT_EHIP, "no HIP device");
    }
    s->max_resident = n_slots;
    s->pool_bytes = pool_bytes & ~size_t(255);
    if (hipMalloc(reinterpret_cast<void **>(&s->pool), s->pool_bytes) != hipSuccess) {
        delete s;
        return failf(SPECT_ENOMEM, "hipMalloc of a %zu-byte pool failed", pool_bytes);
    }
    s->free_list.push_back(Block{0, s->pool_bytes});
    s->lanes.resize(std::min(n_slots, kMaxLanes));
    bool okay = true;
    okay = okay && hipStreamCreateWithFlags(&s->upload, hipStreamNonBlocking) == hipSuccess;
    for (Lane &ln : s->lanes) {
        okay = okay && hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) == hipSuccess;
        for (TickSlot &ts : ln.ring) {
            okay = okay && hipEventCreateWithFlags(&ts.done, hipEventDisableTiming) == hipSuccess;
            okay = okay && hipEventCreateWithFlags(&ts.uploaded, hipEventDisableTiming) == hipSuccess;
        }
    }
    if (!okay) {
        spect_server_destroy(s);
        return set_error(SPECT_EHIP, "stream or event creation failed");
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return clear_error();
}

int spect_server_destroy(spect_server *s)
{
    if (!s) return clear_error();
    if (s->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
            for (int64_t id : s->queue) spect_server::drop_ready(s->reqs[id]);
            s->queue.clear();
        }
        s->wake.notify_all();
        s->worker.join();
    }
    for (Lane &ln : s->lanes) {
        if (ln.stream) {
            (void)hipStreamSynchronize(ln.stream);
            (void)hipStreamDestroy(ln.stream);
        }
        for (TickSlot &ts : ln.ring) {
            if (ts.done) (void)hipEventDestroy(ts.done);
            if (ts.uploaded) (void)hipEventDestroy(ts.uploaded);
            if (ts.host) (void)hipHostFree(ts.host);
            if (ts.dev) (void)hipFree(ts.dev);
        }
    }
    if (s->upload) {
        (void)hipStreamSynchronize(s->upload);
        (void)hipStreamDestroy(s->upload);
    }
    for (auto &kv : s->reqs) spect_server::drop_ready(kv.second);
    if (s->pool) (void)hipFree(s->pool);
    delete s;
    return clear_error();
}

int spect_server_submit(spect_server *s, const spect_plan *plan, float *f, const float *mu, const float *g,
                        const float *s_add, int32_t n_iters, int32_t n_subsets, void *stream,
                        int64_t *request_id)
{
    if (!s) return set_error(SPECT_EINVAL, "server is NULL");
    if (!request_id) return set_error(SPECT_EINVAL, "request_id is NULL");
    if (!plan || !f || !g) return set_error(SPECT_EINVAL, "plan, f and g must not be NULL");
    if (n_iters < 0) return failf(SPECT_EINVAL, "n_iters = %d is negative", n_iters);
    size_t ws = 0;
    int st = spect_internal::tick_region_bytes(plan, n_subsets, mu != nullptr, &ws);
    if (st) return st;
    ws = round256(std::max<size_t>(ws, 256));
    if (ws > s->pool_bytes)
        return failf(SPECT_EINVAL, "request needs %zu workspace bytes, the pool has %zu", ws, s->pool_bytes);
    Request r;
    r.plan = plan;
    r.f = f;
    r.mu = mu;
    r.g = g;
    r.s = s_add;
    r.iters = n_iters;
    r.subsets = n_subsets;
    r.steps = n_subsets * (1 + n_iters);
    r.step_work = spect_internal::step_work(plan, n_subsets);
    r.ws = ws;
    if (hipEventCreateWithFlags(&r.ready, hipEventDisableTiming) != hipSuccess)
        return set_error(SPECT_EHIP, "event creation failed");
    if (hipEventRecord(r.ready, static_cast<hipStream_t>(stream)) != hipSuccess) {
        (void)hipEventDestroy(r.ready);
        return set_error(SPECT_EHIP, "could not record the submission event on the caller's stream");
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const int64_t id = s->next_id++;
        s->reqs[id] = r;
        s->queue.push_back(id);
        *request_id = id;
    }
    s->wake.notify_all();
    return clear_error();
}

int spect_server_progress(spect_server *s, int32_t *n_running, int32_t *n_queued)
{
    if (!s) return set_error(SPECT_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (n_running) *n_running = s->running();
    if (n_queued) *n_queued = (int32_t)s->queue.size();
    return clear_error();
}

int spect_server_status(spect_server *s, int64_t request_id, int32_t *state)
{
    if (!s || !state) return set_error(SPECT_EINVAL, "server and state must not be NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end()) return failf(SPECT_EINVAL, "unknown request %lld", (long long)request_id);
    *state = it->second.state;
    if (it->second.state == SPECT_REQ_FAILED) return set_error(it->second.err, it->second.msg.c_str());
    return clear_error();
}

int spect_server_wait(spect_server *s, int64_t request_id)
{
    if (!s) return set_error(SPECT_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end()) return failf(SPECT_EINVAL, "unknown request %lld", (long long)request_id);
    s->done.wait(lk, [&] {
        const int st = s->reqs[request_id].state;
        return st == SPECT_REQ_DONE || st == SPECT_REQ_FAILED;
    });
    const Request &r = s->reqs[request_id];
    if (r.state == SPECT_REQ_FAILED) return set_error(r.err, r.msg.c_str());
    return clear_error();
}

int spect_server_stats(const spect_server *s, int32_t *n_running, int32_t *n_queued, int32_t *peak_running,
                       size_t *pool_in_use)
{
    if (!s) return set_error(SPECT_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(const_cast<spect_server *>(s)->mu);
    if (n_running) *n_running = s->running();
    if (n_queued) *n_queued = (int32_t)s->queue.size();
    if (peak_running) *peak_running = s->peak_running;
    if (pool_in_use) *pool_in_use = s->in_use;
    return clear_error();
}

int spect_server_forget(spect_server *s, int64_t request_id)
{
    if (!s) return set_error(SPECT_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end()) return failf(SPECT_EINVAL, "unknown request %lld", (long long)request_id);
    if (it->second.state != SPECT_REQ_DONE && it->second.state != SPECT_REQ_FAILED)
        return set_error(SPECT_EINVAL, "request is still queued or running");
    s->reqs.erase(it);
    return clear_error();
}

}  // extern "C"
